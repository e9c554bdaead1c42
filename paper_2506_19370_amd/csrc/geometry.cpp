// Subpatch grids and inter-patch connectivity, built once on the host.
//
// Sec. 3 (patch types S, I, C1, C2; subpatch grids, with the L-shaped C1
// corner subpatch given by an activity mask), Sec. 3.3 (n_f-point fringe of
// the internal sides, exchange or interpolation of solution values, donors
// never in a fringe), Sec. 5 item 1 (Jacobian of the inverse mapping), and
// the windowed viscosity blend of Sec. 4.  Readings (not fixed by the
// paper): degree-5 tensor Lagrange interpolation with a stencil centred on
// the donor cell and clamped into the index box, Newton inversion of the
// donor mapping interpolated the same way, coordinates within 1e-9 of a grid
// line snapped to it, donor = the eligible subpatch in which the point lies
// deepest (index distance to internal sides), ties to the lowest index;
// blend windows rising smoothly from 0 at internal sides to 1 at depth 2 n_v.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <limits>

#include <atomic>
#include <thread>

#include "fc_builder.h"

namespace fcs {

namespace {

constexpr double kSnap = 1e-9;
// Newton steps below this (index units) end the donor inversion: with O(1)
// coordinates and spacings down to 1e-4 the rounding floor of a step is a
// few 1e-12, and the snap to grid lines (kSnap) is coarser anyway.
constexpr double kNewtonTol = 1e-10;
constexpr int kOrder = 6;
constexpr double kInf = std::numeric_limits<double>::infinity();

bool runs_of(const uint8_t* mask, int nlines, int len, int stride_line, int stride_pt,
             std::vector<Run>& out, std::string& err) {
  out.assign(nlines, Run());
  for (int l = 0; l < nlines; ++l) {
    int first = -1, last = -1, count = 0;
    for (int s = 0; s < len; ++s) {
      if (mask[static_cast<size_t>(l) * stride_line + static_cast<size_t>(s) * stride_pt]) {
        if (first < 0) first = s;
        last = s;
        ++count;
      }
    }
    if (count == 0) continue;
    if (last - first + 1 != count) {
      err = "a grid line holds more than one run of active points";
      return false;
    }
    out[l].start = first;
    out[l].len = count;
  }
  return true;
}

void lagrange(double u, double* w) {
  for (int k = 0; k < kOrder; ++k) {
    double v = 1.0;
    for (int m = 0; m < kOrder; ++m)
      if (m != k) v *= (u - m) / static_cast<double>(k - m);
    w[k] = v;
  }
}

void dlagrange(double u, double* dw) {
  for (int k = 0; k < kOrder; ++k) {
    double acc = 0.0;
    for (int m = 0; m < kOrder; ++m) {
      if (m == k) continue;
      double term = 1.0 / static_cast<double>(k - m);
      for (int l = 0; l < kOrder; ++l)
        if (l != k && l != m) term = term * (u - l) / static_cast<double>(k - l);
      acc += term;
    }
    dw[k] = acc;
  }
}

int stencil_start(double xi, int n) {
  int s = static_cast<int>(std::floor(xi)) - 2;
  return std::max(0, std::min(s, n - kOrder));
}

void build_hash(Grid& g) {
  double xmin = kInf, xmax = -kInf, ymin = kInf, ymax = -kInf;
  for (size_t k = 0; k < g.np(); ++k) {
    xmin = std::min(xmin, g.x[k]);
    xmax = std::max(xmax, g.x[k]);
    ymin = std::min(ymin, g.y[k]);
    ymax = std::max(ymax, g.y[k]);
  }
  double area = std::max((xmax - xmin) * (ymax - ymin), 1e-300);
  g.h0 = std::max(std::sqrt(area / static_cast<double>(g.np())) * 2.0, 1e-300);
  g.hx0 = xmin;
  g.hy0 = ymin;
  g.hnx = std::max(1, static_cast<int>((xmax - xmin) / g.h0) + 1);
  g.hny = std::max(1, static_cast<int>((ymax - ymin) / g.h0) + 1);
  std::vector<int> count(static_cast<size_t>(g.hnx) * g.hny + 1, 0);
  auto cell = [&](size_t k) {
    int cx = std::min(g.hnx - 1, static_cast<int>((g.x[k] - g.hx0) / g.h0));
    int cy = std::min(g.hny - 1, static_cast<int>((g.y[k] - g.hy0) / g.h0));
    return static_cast<size_t>(cy) * g.hnx + cx;
  };
  for (size_t k = 0; k < g.np(); ++k) count[cell(k) + 1]++;
  for (size_t c = 1; c < count.size(); ++c) count[c] += count[c - 1];
  g.hstart = count;
  g.hidx.assign(g.np(), 0);
  std::vector<int> fill(count.begin(), count.end() - 1);
  for (size_t k = 0; k < g.np(); ++k) g.hidx[fill[cell(k)]++] = static_cast<int>(k);
}

size_t nearest_node(const Grid& g, double px, double py) {
  int cx = static_cast<int>(std::floor((px - g.hx0) / g.h0));
  int cy = static_cast<int>(std::floor((py - g.hy0) / g.h0));
  cx = std::max(0, std::min(g.hnx - 1, cx));
  cy = std::max(0, std::min(g.hny - 1, cy));
  double best = kInf;
  size_t bk = 0;
  int maxr = std::max(g.hnx, g.hny);
  for (int r = 0; r <= maxr; ++r) {
    for (int yy = cy - r; yy <= cy + r; ++yy) {
      if (yy < 0 || yy >= g.hny) continue;
      for (int xx = cx - r; xx <= cx + r; ++xx) {
        if (xx < 0 || xx >= g.hnx) continue;
        if (std::max(std::abs(xx - cx), std::abs(yy - cy)) != r) continue;
        size_t c = static_cast<size_t>(yy) * g.hnx + xx;
        for (int q = g.hstart[c]; q < g.hstart[c + 1]; ++q) {
          size_t k = g.hidx[q];
          double d2 = (g.x[k] - px) * (g.x[k] - px) + (g.y[k] - py) * (g.y[k] - py);
          if (d2 < best || (d2 == best && k < bk)) {
            best = d2;
            bk = k;
          }
        }
      }
    }
    // every node outside ring r is farther than (r) * h0 from the query cell
    if (best < kInf && std::sqrt(best) <= r * g.h0) break;
  }
  return bk;
}

// Newton inversion of the interpolated donor mapping (see header comment).
bool invert(const Grid& g, double px, double py, double& xi, double& eta) {
  size_t k0 = nearest_node(g, px, py);
  xi = static_cast<double>(k0 % g.n1);
  eta = static_cast<double>(k0 / g.n1);
  double scale = std::max({g.bb[1] - g.bb[0], g.bb[3] - g.bb[2], 1e-300});
  bool ok = false;
  double wu[kOrder], wv[kOrder], du[kOrder], dv[kOrder];
  for (int it = 0; it < 40; ++it) {
    int i0 = stencil_start(xi, g.n1), j0 = stencil_start(eta, g.n2);
    lagrange(xi - i0, wu);
    lagrange(eta - j0, wv);
    dlagrange(xi - i0, du);
    dlagrange(eta - j0, dv);
    double fx = 0, fy = 0, xa = 0, xb = 0, ya = 0, yb = 0;
    for (int b = 0; b < kOrder; ++b)
      for (int a = 0; a < kOrder; ++a) {
        size_t k = g.at(j0 + b, i0 + a);
        fx += wv[b] * wu[a] * g.x[k];
        fy += wv[b] * wu[a] * g.y[k];
        xa += wv[b] * du[a] * g.x[k];
        xb += dv[b] * wu[a] * g.x[k];
        ya += wv[b] * du[a] * g.y[k];
        yb += dv[b] * wu[a] * g.y[k];
      }
    fx -= px;
    fy -= py;
    double det = xa * yb - xb * ya;
    if (!(std::abs(det) > 0)) return false;
    double dxi = (yb * fx - xb * fy) / det;
    double deta = (-ya * fx + xa * fy) / det;
    xi = std::max(-3.0, std::min(g.n1 + 2.0, xi - dxi));
    eta = std::max(-3.0, std::min(g.n2 + 2.0, eta - deta));
    ok = (std::abs(dxi) < kNewtonTol && std::abs(deta) < kNewtonTol) || std::hypot(fx, fy) < 1e-15 * scale;
    if (ok) break;
  }
  double rx = std::nearbyint(xi), ry = std::nearbyint(eta);
  if (std::abs(xi - rx) < kSnap) xi = rx;
  if (std::abs(eta - ry) < kSnap) eta = ry;
  return ok;
}

bool inside(const Grid& g, double xi, double eta) {
  if (!(xi >= -kSnap && xi <= g.n1 - 1 + kSnap && eta >= -kSnap && eta <= g.n2 - 1 + kSnap)) return false;
  int j = std::max(0, std::min(g.n2 - 1, static_cast<int>(std::nearbyint(eta))));
  int i = std::max(0, std::min(g.n1 - 1, static_cast<int>(std::nearbyint(xi))));
  const Run& r = g.rows[j];
  if (r.len == 0 || !(r.start - kSnap <= xi && xi <= r.start + r.len - 1 + kSnap)) return false;
  const Run& c = g.cols[i];
  if (c.len == 0 || !(c.start - kSnap <= eta && eta <= c.start + c.len - 1 + kSnap)) return false;
  return true;
}

double depth_at(const Grid& g, double xi, double eta) {
  int j = std::max(0, std::min(g.n2 - 1, static_cast<int>(std::nearbyint(eta))));
  int i = std::max(0, std::min(g.n1 - 1, static_cast<int>(std::nearbyint(xi))));
  double best = kInf;
  const Run& r = g.rows[j];
  if (r.len) {
    if (r.lo == kInternal) best = std::min(best, xi - r.start);
    if (r.hi == kInternal) best = std::min(best, r.start + r.len - 1 - xi);
  }
  const Run& c = g.cols[i];
  if (c.len) {
    if (c.lo == kInternal) best = std::min(best, eta - c.start);
    if (c.hi == kInternal) best = std::min(best, c.start + c.len - 1 - eta);
  }
  return best;
}

struct Entry {
  int j, i;
  double w;
};

// First nodes of the 6-point stencil along one direction, most preferred
// first: the centred start clamped into the index box, then that start
// moved by +1, -1, +2, -2 while it stays in the box and its span still
// holds the point.  A coordinate on a grid line uses the node itself (-1).
int stencil_starts(double xi, int n, int* out) {
  if (xi == std::nearbyint(xi)) {
    out[0] = -1;
    return 1;
  }
  const int c = stencil_start(xi, n), shift[5] = {0, 1, -1, 2, -2};
  int cnt = 0;
  for (int s : shift) {
    int v = c + s;
    if (v >= 0 && v <= n - kOrder && v <= xi && xi <= v + kOrder - 1) out[cnt++] = v;
  }
  return cnt;
}

// Interpolation stencil at (xi, eta) whose nodes all satisfy `ok`: the
// candidate positions are tried by the sum of their ranks along the two
// directions, then by the rank along q^1 (where the centred stencil would
// reach a masked or fringe node, e.g. beside the obstacle quadrant of a
// corner subpatch, the interpolation becomes one-sided).  false if none.
// The stencil in factored form: first nodes (j0, i0), sizes ni x nj and the
// weights of the two directions (the entry weights are wj[b] * wi[a]).
struct Stencil {
  int i0, j0, ni, nj;
  double wi[kOrder], wj[kOrder];
};

template <class Pred>
bool stencil_factored(const Grid& g, double xi, double eta, Pred ok, Stencil& st) {
  int si[5], sj[5];
  const int ni_c = stencil_starts(xi, g.n1, si), nj_c = stencil_starts(eta, g.n2, sj);
  for (int total = 0; total <= ni_c + nj_c - 2; ++total)
    for (int ri = 0; ri <= total; ++ri) {
      const int rj = total - ri;
      if (ri >= ni_c || rj >= nj_c) continue;
      int ii[kOrder], jj[kOrder];
      double wi[kOrder], wj[kOrder];
      int ni = 1, nj = 1;
      if (si[ri] < 0) {
        ii[0] = static_cast<int>(xi);
        wi[0] = 1.0;
      } else {
        ni = kOrder;
        lagrange(xi - si[ri], wi);
        for (int a = 0; a < kOrder; ++a) ii[a] = si[ri] + a;
      }
      if (sj[rj] < 0) {
        jj[0] = static_cast<int>(eta);
        wj[0] = 1.0;
      } else {
        nj = kOrder;
        lagrange(eta - sj[rj], wj);
        for (int b = 0; b < kOrder; ++b) jj[b] = sj[rj] + b;
      }
      bool good = true;
      for (int b = 0; b < nj && good; ++b)
        for (int a = 0; a < ni && good; ++a) good = ok(g.at(jj[b], ii[a]));
      if (!good) continue;
      st.i0 = ii[0];
      st.j0 = jj[0];
      st.ni = ni;
      st.nj = nj;
      for (int a = 0; a < ni; ++a) st.wi[a] = wi[a];
      for (int b = 0; b < nj; ++b) st.wj[b] = wj[b];
      return true;
    }
  return false;
}

template <class Pred>
bool stencil(const Grid& g, double xi, double eta, Pred ok, std::vector<Entry>& out) {
  Stencil st;
  if (!stencil_factored(g, xi, eta, ok, st)) return false;
  out.clear();
  for (int b = 0; b < st.nj; ++b)
    for (int a = 0; a < st.ni; ++a) out.push_back({st.j0 + b, st.i0 + a, st.wj[b] * st.wi[a]});
  return true;
}

bool bbox_candidate(const Grid& s, double px, double py) {
  double tol = 1e-9 * std::max({s.bb[1] - s.bb[0], s.bb[3] - s.bb[2], 1.0});
  return px >= s.bb[0] - tol && px <= s.bb[1] + tol && py >= s.bb[2] - tol && py <= s.bb[3] + tol;
}

double smooth_step(double t) {
  if (t >= 1.0) return 1.0;
  if (!(t > 0.0)) return 0.0;
  double a = std::exp(-1.0 / t), b = std::exp(-1.0 / (1.0 - t));
  return a / (a + b);
}

}  // namespace

void apply_lines(const Grid& g, int d, int C, int kind, int dir, const double* f, double* out) {
  std::fill(out, out + g.np(), 0.0);
  if (dir == 0) {
    for (int j = 0; j < g.n2; ++j) {
      const Run& r = g.rows[j];
      if (!r.len) continue;
      const std::vector<double>& D = *fc_operator(r.len, d, C, kind);
      for (int t = 0; t < r.len; ++t) {
        double s = 0;
        for (int q = 0; q < r.len; ++q) s += D[static_cast<size_t>(t) * r.len + q] * f[g.at(j, r.start + q)];
        out[g.at(j, r.start + t)] = s;
      }
    }
  } else {
    for (int i = 0; i < g.n1; ++i) {
      const Run& r = g.cols[i];
      if (!r.len) continue;
      const std::vector<double>& D = *fc_operator(r.len, d, C, kind);
      for (int t = 0; t < r.len; ++t) {
        double s = 0;
        for (int q = 0; q < r.len; ++q) s += D[static_cast<size_t>(t) * r.len + q] * f[g.at(r.start + q, i)];
        out[g.at(r.start + t, i)] = s;
      }
    }
  }
}

bool build_grid(Grid& g, int d, int C, int n_f, std::string& err) {
  const int n1 = g.n1, n2 = g.n2;
  const size_t np = g.np();
  if (g.mask.empty()) g.mask.assign(np, 1);
  if (!runs_of(g.mask.data(), n2, n1, n1, 1, g.rows, err)) return false;
  if (!runs_of(g.mask.data(), n1, n2, 1, n1, g.cols, err)) return false;
  for (auto& r : g.rows) {
    if (!r.len) continue;
    if (r.len < 2 * d) {
      err = "a q^1 line is shorter than twice the FC matching width";
      return false;
    }
    r.lo = r.start == 0 ? g.side[0] : g.notch;
    r.hi = r.start + r.len == n1 ? g.side[1] : g.notch;
  }
  for (auto& c : g.cols) {
    if (!c.len) continue;
    if (c.len < 2 * d) {
      err = "a q^2 line is shorter than twice the FC matching width";
      return false;
    }
    c.lo = c.start == 0 ? g.side[2] : g.notch;
    c.hi = c.start + c.len == n2 ? g.side[3] : g.notch;
  }
  // metrics (Sec. 5 item 1): Jacobian of the inverse mapping
  std::vector<double> x1(np), x2(np), y1(np), y2(np);
  apply_lines(g, d, C, 0, 0, g.x.data(), x1.data());
  apply_lines(g, d, C, 0, 1, g.x.data(), x2.data());
  apply_lines(g, d, C, 0, 0, g.y.data(), y1.data());
  apply_lines(g, d, C, 0, 1, g.y.data(), y2.data());
  std::vector<double>* met[4] = {&g.t1x, &g.t1y, &g.t2x, &g.t2y};
  for (auto* m : met) m->assign(np, 0.0);
  size_t nact = 0;
  for (size_t k = 0; k < np; ++k) {
    if (!g.mask[k]) continue;
    ++nact;
    double det = x1[k] * y2[k] - x2[k] * y1[k];
    if (!(std::abs(det) > 0)) {
      err = "singular patch mapping";
      return false;
    }
    g.t1x[k] = y2[k] / det;
    g.t1y[k] = -x2[k] / det;
    g.t2x[k] = -y1[k] / det;
    g.t2y[k] = x1[k] / det;
  }
  if (nact == 0) {
    err = "subpatch without active points";
    return false;
  }
  double scale = 0, mean[4] = {0, 0, 0, 0}, dev = 0;
  for (int c = 0; c < 4; ++c)
    for (size_t k = 0; k < np; ++k)
      if (g.mask[k]) {
        scale = std::max(scale, std::abs((*met[c])[k]));
        mean[c] += (*met[c])[k];
      }
  for (int c = 0; c < 4; ++c) mean[c] /= static_cast<double>(nact);
  for (int c = 0; c < 4; ++c)
    for (size_t k = 0; k < np; ++k)
      if (g.mask[k]) dev = std::max(dev, std::abs((*met[c])[k] - mean[c]));
  g.affine = dev <= 1e-6 * scale;
  // an affine subpatch takes the mean metrics, with components below 1e-6 of
  // the largest set to zero (axis-aligned grids are then exactly Cartesian)
  for (int c = 0; c < 4; ++c)
    if (std::abs(mean[c]) <= 1e-6 * scale) mean[c] = 0.0;
  if (g.affine)
    for (int c = 0; c < 4; ++c)
      for (size_t k = 0; k < np; ++k) (*met[c])[k] = g.mask[k] ? mean[c] : 0.0;
  g.g11.assign(np, 0);
  g.g12.assign(np, 0);
  g.g22.assign(np, 0);
  g.lap1.assign(np, 0);
  g.lap2.assign(np, 0);
  for (size_t k = 0; k < np; ++k) {
    g.g11[k] = g.t1x[k] * g.t1x[k] + g.t1y[k] * g.t1y[k];
    g.g12[k] = g.t1x[k] * g.t2x[k] + g.t1y[k] * g.t2y[k];
    g.g22[k] = g.t2x[k] * g.t2x[k] + g.t2y[k] * g.t2y[k];
  }
  if (!g.affine) {
    std::vector<double> a1(np), a2(np), b1(np), b2(np);
    // lap t^k = d/dx (t^k_x) + d/dy (t^k_y)
    const std::vector<double>* mx[2] = {&g.t1x, &g.t2x};
    const std::vector<double>* my[2] = {&g.t1y, &g.t2y};
    std::vector<double>* lap[2] = {&g.lap1, &g.lap2};
    for (int q = 0; q < 2; ++q) {
      apply_lines(g, d, C, 0, 0, mx[q]->data(), a1.data());
      apply_lines(g, d, C, 0, 1, mx[q]->data(), a2.data());
      apply_lines(g, d, C, 0, 0, my[q]->data(), b1.data());
      apply_lines(g, d, C, 0, 1, my[q]->data(), b2.data());
      for (size_t k = 0; k < np; ++k)
        (*lap[q])[k] = g.mask[k] ? (g.t1x[k] * a1[k] + g.t2x[k] * a2[k]) + (g.t1y[k] * b1[k] + g.t2y[k] * b2[k])
                                 : 0.0;
    }
  }
  // local mesh size: 1 / sqrt of the largest eigenvalue of the metric tensor
  // g^{kl} (index units), the distance between neighbouring grid lines along
  // the most compressed direction (on a skewed grid well below the spacing
  // of neighbouring nodes)
  g.hx.assign(np, 0.0);
  for (size_t k = 0; k < np; ++k) {
    if (!g.mask[k]) continue;
    const double half = 0.5 * (g.g11[k] + g.g22[k]);
    const double dif = 0.5 * (g.g11[k] - g.g22[k]);
    const double lam = half + std::sqrt(dif * dif + g.g12[k] * g.g12[k]);
    g.hx[k] = 1.0 / std::sqrt(lam);
  }
  // fringe (Sec. 3.3), exact-data layer, boundary points, depth
  g.fringe.assign(np, 0);
  g.xfringe.assign(np, 0);
  g.depth.assign(np, kInf);
  g.bnd.clear();
  auto end = [&](int kind, int dist, size_t k, int j, int i, int dir, bool at_end) {
    if (kind == kInternal) {
      if (dist < n_f) g.fringe[k] = 1;
      g.depth[k] = std::min(g.depth[k], static_cast<double>(dist));
    } else if (kind == kExact) {
      if (dist < n_f) g.xfringe[k] = 1;
    } else if (at_end) {
      g.bnd.push_back({j, i, kind, dir});
    }
  };
  for (int j = 0; j < n2; ++j) {
    const Run& r = g.rows[j];
    if (!r.len) continue;
    for (int i = r.start; i < r.start + r.len; ++i) {
      end(r.lo, i - r.start, g.at(j, i), j, i, 0, i == r.start);
    }
    for (int i = r.start; i < r.start + r.len; ++i) {
      end(r.hi, r.start + r.len - 1 - i, g.at(j, i), j, i, 0, i == r.start + r.len - 1);
    }
  }
  for (int i = 0; i < n1; ++i) {
    const Run& c = g.cols[i];
    if (!c.len) continue;
    for (int j = c.start; j < c.start + c.len; ++j) end(c.lo, j - c.start, g.at(j, i), j, i, 1, j == c.start);
    for (int j = c.start; j < c.start + c.len; ++j)
      end(c.hi, c.start + c.len - 1 - j, g.at(j, i), j, i, 1, j == c.start + c.len - 1);
  }
  for (size_t k = 0; k < np; ++k) {
    if (!g.mask[k]) {
      g.fringe[k] = g.xfringe[k] = 0;
      g.depth[k] = 0.0;
    } else if (g.fringe[k]) {
      g.xfringe[k] = 0;
    }
  }
  g.bb[0] = g.bb[2] = kInf;
  g.bb[1] = g.bb[3] = -kInf;
  for (size_t k = 0; k < np; ++k)
    if (g.mask[k]) {
      g.bb[0] = std::min(g.bb[0], g.x[k]);
      g.bb[1] = std::max(g.bb[1], g.x[k]);
      g.bb[2] = std::min(g.bb[2], g.y[k]);
      g.bb[3] = std::max(g.bb[3], g.y[k]);
    }
  build_hash(g);
  return true;
}

// The subpatches whose bounding box (widened by the tolerance of
// bbox_candidate) meets that of subpatch p, in ascending order: the only
// ones that can pass bbox_candidate for a point of p.
static std::vector<size_t> box_neighbours(const std::vector<Grid>& grids, size_t p) {
  std::vector<size_t> out;
  const Grid& gp = grids[p];
  for (size_t s = 0; s < grids.size(); ++s) {
    if (s == p) continue;
    const Grid& gs = grids[s];
    const double tol = 1e-9 * std::max({gs.bb[1] - gs.bb[0], gs.bb[3] - gs.bb[2], 1.0});
    if (gp.bb[1] < gs.bb[0] - tol || gp.bb[0] > gs.bb[1] + tol || gp.bb[3] < gs.bb[2] - tol ||
        gp.bb[2] > gs.bb[3] + tol)
      continue;
    out.push_back(s);
  }
  return out;
}

static void fringe_rows_of(const std::vector<Grid>& grids, size_t p, std::vector<InterpRow>& rows, std::string& err);

// Runs fn(p) for p = 0 .. n-1 on up to 16 host threads (subpatches are
// independent: each call reads the grids and writes only its own slot).
template <class Fn>
static void for_each_patch(size_t n, Fn fn) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const size_t nt = std::min<size_t>(hw, n);
  std::atomic<size_t> next{0};
  auto work = [&]() {
    for (size_t p = next++; p < n; p = next++) fn(p);
  };
  std::vector<std::thread> pool;
  for (size_t t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
}

bool build_grids(std::vector<Grid>& grids, int d, int C, int n_f, std::string& err, int& bad) {
  std::vector<std::string> perr(grids.size());
  std::vector<char> ok(grids.size(), 1);
  for_each_patch(grids.size(), [&](size_t p) { ok[p] = build_grid(grids[p], d, C, n_f, perr[p]); });
  for (size_t p = 0; p < grids.size(); ++p)
    if (!ok[p]) {
      err = perr[p];
      bad = static_cast<int>(p);
      return false;
    }
  return true;
}

bool build_fringe_rows(const std::vector<Grid>& grids, std::vector<InterpRow>& rows, std::string& err) {
  rows.clear();
  std::vector<std::vector<InterpRow>> per(grids.size());
  std::vector<std::string> perr(grids.size());
  for_each_patch(grids.size(), [&](size_t p) { fringe_rows_of(grids, p, per[p], perr[p]); });
  for (size_t p = 0; p < grids.size(); ++p)
    if (!perr[p].empty()) {
      err = perr[p];
      return false;
    }
  for (auto& v : per)
    for (auto& r : v) rows.push_back(std::move(r));
  return true;
}

static void fringe_rows_of(const std::vector<Grid>& grids, size_t p, std::vector<InterpRow>& rows, std::string& err) {
  std::vector<Entry> ent;
  {
    const Grid& gp = grids[p];
    const std::vector<size_t> nb = box_neighbours(grids, p);
    for (int j = 0; j < gp.n2; ++j)
      for (int i = 0; i < gp.n1; ++i) {
        size_t k = gp.at(j, i);
        if (!gp.fringe[k]) continue;
        double px = gp.x[k], py = gp.y[k];
        double best = -kInf;
        int bs = -1;
        std::vector<Entry> bent;
        for (size_t s : nb) {
          const Grid& gs = grids[s];
          if (!bbox_candidate(gs, px, py)) continue;
          double xi, eta;
          if (!invert(gs, px, py, xi, eta) || !inside(gs, xi, eta)) continue;
          if (!stencil(gs, xi, eta, [&](size_t kk) { return gs.mask[kk] && !gs.fringe[kk]; }, ent)) continue;
          double dep = depth_at(gs, xi, eta);
          if (dep > best + 1e-9) {
            best = dep;
            bs = static_cast<int>(s);
            bent = ent;
          }
        }
        if (bs < 0) {
          err = "fringe point (" + std::to_string(j) + ", " + std::to_string(i) + ") of subpatch " +
                std::to_string(p) + " has no donor";
          return;
        }
        InterpRow row;
        row.dst = gp.offset + static_cast<int64_t>(k);
        const Grid& gs = grids[bs];
        for (const Entry& e : bent) row.ent.push_back({gs.offset + static_cast<int64_t>(gs.at(e.j, e.i)), e.w});
        rows.push_back(std::move(row));
      }
  }
}

static void blend_terms_of(const std::vector<Grid>& grids, size_t p, int n_v, std::vector<BlendRow>& rows) {
  const Grid& gp = grids[p];
  const std::vector<size_t> nb = box_neighbours(grids, p);
  std::vector<std::pair<double, BlendTerm>> lst;
  for (int j = 0; j < gp.n2; ++j)
    for (int i = 0; i < gp.n1; ++i) {
      size_t k = gp.at(j, i);
      if (!gp.mask[k]) continue;
      double px = gp.x[k], py = gp.y[k];
      lst.clear();
      for (size_t s : nb) {
        const Grid& gs = grids[s];
        if (!bbox_candidate(gs, px, py)) continue;
        double xi, eta;
        if (!invert(gs, px, py, xi, eta) || !inside(gs, xi, eta)) continue;
        double w = smooth_step(depth_at(gs, xi, eta) / (2.0 * n_v));
        if (!(w > 0.0)) continue;
        Stencil st;
        if (!stencil_factored(gs, xi, eta, [&](size_t kk) { return gs.mask[kk] != 0; }, st)) continue;
        BlendTerm t{};
        t.base = gs.offset + static_cast<int64_t>(gs.at(st.j0, st.i0));
        t.stride = gs.n1;
        t.ni = st.ni;
        t.nj = st.nj;
        for (int a = 0; a < st.ni; ++a) t.wi[a] = st.wi[a];
        for (int b = 0; b < st.nj; ++b) t.wj[b] = st.wj[b];
        lst.push_back({w, t});
      }
      if (lst.empty()) continue;
      double wp = smooth_step(gp.depth[k] / (2.0 * n_v));
      double total = wp;
      for (const auto& c : lst) total += c.first;
      BlendRow row;
      row.dst = gp.offset + static_cast<int64_t>(k);
      row.wself = wp > 0 ? wp / total : 0.0;
      for (auto& c : lst) {
        c.second.scale = c.first / total;
        row.terms.push_back(c.second);
      }
      rows.push_back(std::move(row));
    }
}

void build_blend_terms(const std::vector<Grid>& grids, int n_v, std::vector<BlendRow>& rows) {
  rows.clear();
  std::vector<std::vector<BlendRow>> per(grids.size());
  for_each_patch(grids.size(), [&](size_t p) { blend_terms_of(grids, p, n_v, per[p]); });
  for (auto& v : per)
    for (auto& r : v) rows.push_back(std::move(r));
}

}  // namespace fcs
