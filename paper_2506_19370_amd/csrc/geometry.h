// Internal host-side description of subpatch grids and their connectivity.
#pragma once
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace fcs {

enum SideKind { kInternal = 0, kInflow = 1, kOutflow = 2, kSlip = 3, kExact = 4, kNoSlip = 5 };

struct Run {
  int start = 0, len = 0;
  int lo = kInternal, hi = kInternal;  // kinds of the two ends
};

struct BoundaryEntry {
  int j, i, kind, dir;  // dir: 0 = end of a q^1 line, 1 = end of a q^2 line
};

struct Grid {
  int n1 = 0, n2 = 0, type = 0;
  std::vector<double> x, y;
  std::vector<uint8_t> mask;
  int side[4] = {0, 0, 0, 0};  // W, E, S, N
  int notch = kSlip;
  double inflow[4] = {1, 0, 0, 1};

  std::vector<Run> rows, cols;  // rows[j] runs along q^1, cols[i] along q^2
  bool affine = false;
  // metrics and derived per-point data, (n2, n1)
  std::vector<double> t1x, t1y, t2x, t2y, g11, g12, g22, lap1, lap2, hx, depth;
  std::vector<uint8_t> fringe, xfringe;
  std::vector<BoundaryEntry> bnd;
  double bb[4] = {0, 0, 0, 0};  // bounding box of active nodes
  int64_t offset = 0;            // first global point index

  // nearest-node hash
  double h0 = 1, hx0 = 0, hy0 = 0;
  int hnx = 1, hny = 1;
  std::vector<int> hstart, hidx;

  size_t np() const { return static_cast<size_t>(n1) * n2; }
  size_t at(int j, int i) const { return static_cast<size_t>(j) * n1 + i; }
};

// Runs, side kinds, metrics, fringe, boundary points, depth and the spatial
// hash of one subpatch; false with a message on invalid input.
bool build_grid(Grid& g, int d, int C, int n_f, std::string& err);

// build_grid of every subpatch on host threads; on failure the lowest
// failing index and its message.
bool build_grids(std::vector<Grid>& grids, int d, int C, int n_f, std::string& err, int& bad);

// Apply a dense FC operator along the runs of a (n2, n1) field.
void apply_lines(const Grid& g, int d, int C, int kind, int dir, const double* f, double* out);

struct InterpRow {
  int64_t dst;                                  // global point index
  std::vector<std::pair<int64_t, double>> ent;  // global donor index, weight
};

// Interpolation rows of every fringe point (Sec. 3.3).  false with a message
// when a fringe point has no eligible donor.
bool build_fringe_rows(const std::vector<Grid>& grids, std::vector<InterpRow>& rows, std::string& err);

// Rows of the multi-patch viscosity blend (points without a row keep their
// own smoothed value), each in factored form: the point's own value with weight wself,
// plus per overlapping subpatch scale * sum_b wj[b] sum_a wi[a] u(j0 + b,
// i0 + a) over its ni x nj interpolation stencil (ni, nj = 6, or 1 on a
// grid line), the tensor product of the two directions' Lagrange weights.
struct BlendTerm {
  int64_t base;    // global index of node (j0, i0)
  int32_t stride;  // row length n1 of the donor subpatch
  int32_t ni, nj;
  int32_t pad;
  double scale;
  double wi[6], wj[6];
};
struct BlendRow {
  int64_t dst;
  double wself;
  std::vector<BlendTerm> terms;
};
void build_blend_terms(const std::vector<Grid>& grids, int n_v, std::vector<BlendRow>& rows);

}  // namespace fcs
