// C ABI of the solver: context creation (Alg. 2 on one GPU), workspace
// layout, per-step and per-stage launch sequence (Alg. 1, 3, 4, 5), queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/fcsdnn.h"
#include "fc_builder.h"
#include "gemm.h"
#include "geometry.h"
#include "kernels.h"
#include "stage_kernels.h"
#include "window_kernels.h"

using namespace fcs;

namespace {

// SSPRK(5,4), Shu-Osher form (Spiteri & Ruuth); see the stage kernel.
constexpr double kA0 = 0.391752226571890;
constexpr double kB20 = 0.444370493651235, kB21 = 0.555629506348765, kA1 = 0.368410593050371;
constexpr double kB30 = 0.620101851488403, kB32 = 0.379898148511597, kA2 = 0.251891774271694;
constexpr double kB40 = 0.178079954393132, kB43 = 0.821920045606868, kA3 = 0.544974750228521;
constexpr double kC2 = 0.517231671970585, kC3 = 0.096059710526147, kD3 = 0.063692468666290;
constexpr double kC4 = 0.386708617503269, kD4 = 0.226007483236906;

void stage_fractions(double* c) {
  // stage outputs approximate the solution at t + c[s] dt (Butcher abscissae)
  double a1 = kA0;
  double a2[2] = {kB21 * a1, kA1};
  double a3[3] = {kB32 * a2[0], kB32 * a2[1], kA2};
  double a4[4] = {kB43 * a3[0], kB43 * a3[1], kB43 * a3[2], kA3};
  c[0] = a1;
  c[1] = a2[0] + a2[1];
  c[2] = a3[0] + a3[1] + a3[2];
  c[3] = a4[0] + a4[1] + a4[2] + a4[3];
  c[4] = 1.0;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carve {
  size_t used = 0;
  size_t take(size_t bytes) {
    size_t o = used;
    used = align_up(used + std::max<size_t>(bytes, 1));
    return o;
  }
};

// A contraction task before device pointers are known.
struct TaskSpec {
  int src_arr, dst_arr;  // array ids
  int64_t src_off, dst_off;
  int32_t row_stride, s_stride, nrow, ncomp, n, op;
  int32_t act = -1;  // activity entry of row 0 (skippable viscous task), else -1
};

enum ArrayId { A_U0, A_UA, A_UB, A_F, A_DF1, A_DF2, A_W1, A_W2, A_W11, A_W22, A_W12, A_MU, A_MU1, A_MU2, A_IN, A_NARR };

// PH_EULER0: the first stage's contraction, which also takes the viscosity
// gradient (frozen for the step) in the same launch.
enum Phase { PH_EULER, PH_CROSS, PH_MUGRAD, PH_FILT1, PH_FILT2, PH_EULER0, PH_SMEAR1, PH_SMEAR2, PH_N };

}  // namespace

struct fcs_ctx {
  fcs_params prm{};
  std::vector<float> sdnn;  // bf16-rounded weights, FP32 biases
  std::vector<Grid> grids;
  int64_t P = 0, nactive = 0;
  bool visc = false, cross = false;
  // mixed forms store the stage derivatives as FP32 (not with the cross
  // phase, which reads W1 as an FP64 operand)
  bool deriv_f32 = false;
  std::string err;

  // operators (zero-padded tables shared by all precisions)
  OpPack opk;

  std::vector<TaskSpec> phase_tasks[PH_N];
  std::vector<GemmTile> phase_tiles[PH_N];

  // host tables
  std::vector<uint8_t> flags;
  std::vector<int32_t> pid;
  std::vector<int32_t> ij;  // (j << 16) | i of every point
  std::vector<PatchDev> pdev;
  std::vector<int2> rowrun, colrun;
  std::vector<int64_t> copy_pairs, idst, icol;
  std::vector<int32_t> csrc;  // per point: copy donor of a lattice fringe point, else the point itself
  std::vector<int32_t> iptr;
  std::vector<double> ival;
  std::vector<BlendRowDev> brow;    // viscosity blend rows (factored)
  std::vector<BlendTermDev> bterm;
  std::vector<BcEntry> bc;
  std::vector<WallLine> walls;  // lines ending at no-slip adiabatic walls
  std::vector<int32_t> bcidx;  // entry of each boundary point
  std::vector<double> metric_host[10];  // t1x t1y t2x t2y g11 g12 g22 lap1 lap2 hx
  std::vector<double> basis, wdil;
  std::vector<uint8_t> tau_host;
  // activity flags (one per row and column of the lattice subpatches whose
  // viscous derivatives are skipped in a step where mu vanishes along the
  // line), and the flags of each blend row's point
  int32_t nact = 0;
  std::vector<int2> bact;
  std::vector<uint8_t> act_host;

  // device
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  hipStream_t stream = nullptr;
  // second stream of the per-step fork: the filter runs beside the viscosity
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;    // filter chain beside Alg. 3
  hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;  // step size beside the first contraction
  bool bound = false;
  std::map<std::string, size_t> off;
  double* arr[A_NARR] = {};
  GemmTask* d_tasks[PH_N][3] = {};
  GemmTile* d_tiles[PH_N] = {};
  OpTables optab{};
  int dt_blocks = 512;
  GemmVariant var[PH_N];
  size_t tile_cap[PH_N] = {};
  bool tuned = false;
  float tune_ms[16] = {};
  int stage_variant = 0;  // index of var[PH_EULER] among the candidates

  // time stepping
  int stage_in_step = 0;
  int64_t steps = 0, stages = 0;
  // the solution is past t = 0 (a step completed, or fcs_set_time set t > 0):
  // the filter of Alg. 4 applies from then on
  bool past_t0 = false;
  // the initial data have been made to satisfy the boundary conditions (done
  // once before the first step from t = 0; set_state and set_time reset it)
  bool t0_prepared = false;
  double t_host = 0.0;
  double* cur = nullptr;  // buffer that holds the latest state

  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double prof_ms = 0.0, prof_ovh_ms = 0.0;
  int64_t prof_n = 0, prof_ovh_n = 0;
  // useful flops and bytes of the timed launches (lines actually needed)
  double prof_flops = 0.0, prof_bytes = 0.0;
  int64_t prof_fn = 0;

  // graphs: [0] step without filter, [1] with; the profiled copies carry
  // external event-record nodes around each stage contraction
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraphExec_t pgexec[2] = {nullptr, nullptr};
  hipEvent_t pev[2][12] = {};  // stage pairs (stages 1..4 used), then an empty pair (event-node latency)
  bool capturing_prof = false;
  bool in_capture = false;  // a whole step is being captured into a graph
  // the proxy values (PS) hold the current state's: the last stage of a step
  // evaluates them; set_state invalidates them
  bool ps_valid = false;
  int prof_wf = 0, prof_stage = 0;

  template <typename T>
  T* dptr(const char* name) {
    return reinterpret_cast<T*>(ws + off.at(name));
  }
  fcs_status fail(fcs_status s, const std::string& m) {
    err = m;
    return s;
  }
};

namespace {

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return (ctx)->fail(FCS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
float host_bf16_to_f(uint16_t h) {
  uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int op_id(fcs_ctx* c, int n, int kind) {
  return c->opk.add(n, kind);
}

size_t first_active(const Grid& g) {
  for (size_t k = 0; k < g.np(); ++k)
    if (g.mask[k]) return k;
  return 0;
}

// Tasks for all lines of one grid along one direction, grouped by runs.
// span: activity entry of each line (skippable viscous tasks), else null.
void add_line_tasks(fcs_ctx* c, Phase ph, const Grid& g, int dir, int kind, int src_arr, int src_comp0,
                    int dst_arr, int dst_comp0, int ncomp, const int32_t* span = nullptr) {
  const int nl = dir == 0 ? g.n2 : g.n1;
  const std::vector<Run>& runs = dir == 0 ? g.rows : g.cols;
  int l = 0;
  while (l < nl) {
    if (!runs[l].len) {
      ++l;
      continue;
    }
    int l1 = l + 1;
    while (l1 < nl && runs[l1].start == runs[l].start && runs[l1].len == runs[l].len) ++l1;
    TaskSpec t;
    t.src_arr = src_arr;
    t.dst_arr = dst_arr;
    int64_t first = dir == 0 ? (g.offset + static_cast<int64_t>(l) * g.n1 + runs[l].start)
                             : (g.offset + static_cast<int64_t>(runs[l].start) * g.n1 + l);
    t.src_off = static_cast<int64_t>(src_comp0) * c->P + first;
    t.dst_off = static_cast<int64_t>(dst_comp0) * c->P + first;
    t.row_stride = dir == 0 ? g.n1 : 1;
    t.s_stride = dir == 0 ? 1 : g.n1;
    t.nrow = l1 - l;
    t.ncomp = ncomp;
    t.n = runs[l].len;
    t.op = op_id(c, runs[l].len, kind);
    t.act = span ? span[l] : -1;
    c->phase_tasks[ph].push_back(t);
    l = l1;
  }
}

void build_tiles(fcs_ctx* c, int ph) {
  const auto& tasks = c->phase_tasks[ph];
  std::vector<int32_t> n(tasks.size()), nl(tasks.size());
  std::vector<uint8_t> late(tasks.size());
  for (size_t q = 0; q < tasks.size(); ++q) {
    n[q] = tasks[q].n;
    nl[q] = tasks[q].nrow * tasks[q].ncomp;
    late[q] = tasks[q].act >= 0;  // skippable viscous lines
  }
  gemm_build_tiles(c->var[ph], n.data(), nl.data(), tasks.size(), c->phase_tiles[ph], late.data());
}

double exact_flops(const std::vector<TaskSpec>& tasks) {
  double f = 0;
  for (const auto& t : tasks) f += 2.0 * t.n * t.n * static_cast<double>(t.nrow) * t.ncomp;
  return f;
}

// Algorithmic bytes of one line of a stage-contraction task: the operand
// line read once in FP64, the result written once in the precision of its
// array (FP32 stage derivatives in the mixed forms).
double task_bytes(const fcs_ctx* c, const TaskSpec& t) {
  const bool f32 = c->deriv_f32 && t.dst_arr != A_MU1 && t.dst_arr != A_MU2 && !(c->cross && t.dst_arr == A_W1);
  return t.n * (8.0 + (f32 ? 4.0 : 8.0));
}

fcs_status upload(fcs_ctx* c, const char* name, const void* src, size_t bytes) {
  if (!bytes) return FCS_OK;
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off.at(name), src, bytes, hipMemcpyHostToDevice, c->stream));
  return FCS_OK;
}

}  // namespace

extern "C" int fcs_version(void) { return 101; }

extern "C" const char* fcs_last_error(const fcs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" fcs_status fcs_create(const fcs_params* prm, int32_t npatch, const fcs_patch_desc* patches,
                                 fcs_ctx** out) {
  if (!prm || !patches || !out || npatch <= 0) return FCS_EINVAL;
  *out = nullptr;
  std::unique_ptr<fcs_ctx> c(new (std::nothrow) fcs_ctx());
  if (!c) return FCS_ENOMEM;
  c->prm = *prm;
  c->prm.sdnn_weights = nullptr;
  const fcs_params& p = c->prm;
  if (p.fc_d < 1 || p.fc_d > 12 || p.fc_C < 4 || p.fc_C > 64 || p.n_f < 1 || p.n_v < 1 || p.n_v > 64 ||
      p.precision < 0 || p.precision > 3 || p.av_mode < 0 || p.av_mode > 3 || !(p.gamma > 1.0) ||
      !(p.cfl > 0.0)) {
    *out = c.release();
    return (*out)->fail(FCS_EINVAL, "invalid solver parameters");
  }
  c->visc = p.av_mode != FCS_AV_OFF;
  if (p.smear && !c->visc) {
    *out = c.release();
    return (*out)->fail(FCS_EINVAL, "the initial-data smearing needs a smoothness classifier (av_mode)");
  }
  if (p.av_mode == FCS_AV_SDNN) {
    if (!prm->sdnn_weights) {
      *out = c.release();
      return (*out)->fail(FCS_EINVAL, "SDNN viscosity needs weights");
    }
    c->sdnn.assign(prm->sdnn_weights, prm->sdnn_weights + FCS_SDNN_NPARAM);
    // weights rounded to bf16 (the products' precision); biases stay FP32
    const int wsec[3][2] = {{0, 64 * 16}, {64 * 16 + 64, 64 * 64}, {64 * 16 + 64 + 64 * 64 + 64, 3 * 64}};
    for (auto& s : wsec)
      for (int q = s[0]; q < s[0] + s[1]; ++q) c->sdnn[q] = host_bf16_to_f(host_bf16(c->sdnn[q]));
  }
  // grids
  c->grids.resize(npatch);
  int64_t offset = 0;
  std::string err;
  for (int q = 0; q < npatch; ++q) {
    const fcs_patch_desc& d = patches[q];
    Grid& g = c->grids[q];
    if (d.n1 < 2 * p.fc_d || d.n2 < 2 * p.fc_d || d.n1 > 1024 || d.n2 > 1024 || !d.x || !d.y) {
      *out = c.release();
      return (*out)->fail(FCS_EINVAL, "subpatch " + std::to_string(q) + ": bad size or coordinates");
    }
    for (int s = 0; s < 4; ++s)
      if (d.side[s] < 0 || d.side[s] > 5 || d.notch < 0 || d.notch > 5) {
        *out = c.release();
        return (*out)->fail(FCS_EINVAL, "bad side kind");
      }
    g.n1 = d.n1;
    g.n2 = d.n2;
    g.type = d.type;
    size_t np = g.np();
    g.x.assign(d.x, d.x + np);
    g.y.assign(d.y, d.y + np);
    if (d.mask) g.mask.assign(d.mask, d.mask + np);
    for (int s = 0; s < 4; ++s) g.side[s] = d.side[s];
    g.notch = d.notch;
    for (int s = 0; s < 4; ++s) g.inflow[s] = d.inflow[s];
    if (g.type == FCS_PATCH_C1 && !d.mask) {
      *out = c.release();
      return (*out)->fail(FCS_EINVAL, "C1 subpatch without mask");
    }
    g.offset = offset;
    offset += static_cast<int64_t>(np);
  }
  // runs, metrics, fringe and hashes of every subpatch (independent of each
  // other; host threads)
  int bad = -1;
  if (!build_grids(c->grids, p.fc_d, p.fc_C, p.n_f, err, bad)) {
    *out = c.release();
    return (*out)->fail(FCS_EINVAL, "subpatch " + std::to_string(bad) + ": " + err);
  }
  c->P = offset;
  if (offset >= (int64_t{1} << 31)) {  // point indices are stored as int32 in the window table
    *out = c.release();
    return (*out)->fail(FCS_EINVAL, "more than 2^31 - 1 points in one context");
  }
  // per-point tables
  const int64_t P = c->P;
  c->flags.assign(P, 0);
  c->pid.assign(P, 0);
  c->ij.assign(P, 0);
  for (auto& m : c->metric_host) m.assign(P, 0.0);
  int rr = 0, cr = 0;
  for (int q = 0; q < npatch; ++q) {
    const Grid& g = c->grids[q];
    PatchDev pd{};
    pd.offset = g.offset;
    pd.n1 = g.n1;
    pd.n2 = g.n2;
    pd.row_run = rr;
    pd.col_run = cr;
    pd.affine = g.affine;
    pd.act_row = -1;
    pd.act_col = -1;
    if (g.affine) {
      const size_t k0 = first_active(g);
      pd.t1x = g.t1x[k0];
      pd.t1y = g.t1y[k0];
      pd.t2x = g.t2x[k0];
      pd.t2y = g.t2y[k0];
      pd.g11 = g.g11[k0];
      pd.g12 = g.g12[k0];
      pd.g22 = g.g22[k0];
    }
    c->pdev.push_back(pd);
    for (const Run& r : g.rows) c->rowrun.push_back(make_int2(r.start, r.len));
    for (const Run& r : g.cols) c->colrun.push_back(make_int2(r.start, r.len));
    rr += g.n2;
    cr += g.n1;
    const std::vector<double>* src[10] = {&g.t1x, &g.t1y, &g.t2x, &g.t2y, &g.g11, &g.g12, &g.g22, &g.lap1, &g.lap2, &g.hx};
    for (size_t k = 0; k < g.np(); ++k) {
      int64_t gk = g.offset + static_cast<int64_t>(k);
      uint8_t f = 0;
      if (g.mask[k]) {
        f |= kActive;
        ++c->nactive;
      }
      if (g.fringe[k]) f |= kFringe;
      if (g.xfringe[k]) f |= kXFringe;
      if (g.affine) f |= kAffine;
      c->flags[gk] = f;
      c->pid[gk] = q;
      c->ij[gk] = (static_cast<int32_t>(k / g.n1) << 16) | static_cast<int32_t>(k % g.n1);
      for (int m = 0; m < 10; ++m) c->metric_host[m][gk] = (*src[m])[k];
      if (g.mask[k] && g.g12[k] != 0.0) c->cross = true;
    }
    // boundary conditions: one entry per point (slip normal or corner, then
    // inflow or exact-vortex data)
    std::map<int64_t, size_t> at;
    auto entry = [&](int64_t gk) -> BcEntry& {
      auto it = at.find(gk);
      if (it != at.end()) return c->bc[it->second];
      at[gk] = c->bc.size();
      BcEntry e{};
      e.k = gk;
      c->bc.push_back(e);
      return c->bc.back();
    };
    for (const BoundaryEntry& b : g.bnd) {
      size_t k = g.at(b.j, b.i);
      int64_t gk = g.offset + static_cast<int64_t>(k);
      if (b.kind == kSlip) {
        double nx = b.dir == 0 ? g.t1x[k] : g.t2x[k];
        double ny = b.dir == 0 ? g.t1y[k] : g.t2y[k];
        double h = std::hypot(nx, ny);
        BcEntry& e = entry(gk);
        if (e.slip == 0) {
          e.slip = 1;
          e.nx = nx / h;
          e.ny = ny / h;
        } else {
          e.slip = 2;
        }
      }
    }
    for (const BoundaryEntry& b : g.bnd) {
      if (b.kind != kInflow) continue;
      BcEntry& e = entry(g.offset + static_cast<int64_t>(g.at(b.j, b.i)));
      double r = g.inflow[0], u = g.inflow[1], v = g.inflow[2], pr = g.inflow[3];
      e.dirichlet = 1;
      e.e[0] = r;
      e.e[1] = r * u;
      e.e[2] = r * v;
      e.e[3] = pr / (p.gamma - 1.0) + 0.5 * r * (u * u + v * v);
    }
    for (size_t k = 0; k < g.np(); ++k)
      if (g.xfringe[k]) {
        BcEntry& e = entry(g.offset + static_cast<int64_t>(k));
        e.dirichlet = 2;
        e.x = g.x[k];
        e.y = g.y[k];
      }
  }
  // boundary points are flagged so the stage kernel applies their entry
  c->bcidx.assign(P, 0);
  for (size_t q = 0; q < c->bc.size(); ++q) {
    c->bcidx[c->bc[q].k] = static_cast<int32_t>(q);
    c->flags[c->bc[q].k] |= kBoundary;
  }
  // communication tables
  std::vector<InterpRow> rows;
  if (npatch > 1 && !build_fringe_rows(c->grids, rows, err)) {
    *out = c.release();
    return (*out)->fail(FCS_EOVERLAP, err);
  }
  c->iptr.push_back(0);
  c->csrc.resize(P);
  for (int64_t k = 0; k < P; ++k) c->csrc[k] = static_cast<int32_t>(k);
  for (const InterpRow& r : rows) {
    if (r.ent.size() == 1 && r.ent[0].second == 1.0) {
      c->copy_pairs.push_back(r.dst);
      c->copy_pairs.push_back(r.ent[0].first);
      c->csrc[r.dst] = static_cast<int32_t>(r.ent[0].first);
    } else {
      c->idst.push_back(r.dst);
      for (const auto& e : r.ent) {
        c->icol.push_back(e.first);
        c->ival.push_back(e.second);
      }
      c->iptr.push_back(static_cast<int32_t>(c->icol.size()));
    }
  }
  if (c->visc && npatch > 1) {
    std::vector<BlendRow> brows;
    build_blend_terms(c->grids, p.n_v, brows);
    for (const BlendRow& r : brows) {
      BlendRowDev d{};
      d.dst = r.dst;
      d.wself = r.wself;
      d.t0 = static_cast<int32_t>(c->bterm.size());
      for (const BlendTerm& t : r.terms) {
        BlendTermDev e{};
        e.base = t.base;
        e.stride = t.stride;
        e.ni = t.ni;
        e.nj = t.nj;
        e.scale = t.scale;
        for (int a = 0; a < 6; ++a) {
          e.wi[a] = t.wi[a];
          e.wj[a] = t.wj[a];
        }
        c->bterm.push_back(e);
      }
      d.t1 = static_cast<int32_t>(c->bterm.size());
      c->brow.push_back(d);
    }
  }
  // viscosity tables: dilation weights, modal basis
  c->wdil.assign(p.n_v + 1, 0.0);
  for (int o = 0; o < p.n_v; ++o) {
    double t = static_cast<double>(o) / p.n_v;
    c->wdil[o] = std::exp(1.0 - 1.0 / (1.0 - t * t));
  }
  c->basis.assign(256, 0.0);
  modal_basis16(c->basis.data());
  // contraction tasks
  for (int q = 0; q < npatch; ++q) {
    const Grid& g = c->grids[q];
    if (g.affine) {
      // contravariant fluxes a f_x + b f_y with the constant metric terms
      add_line_tasks(c.get(), PH_EULER, g, 0, FCS_OP_D1, A_F, 0, A_DF1, 0, 4);
      add_line_tasks(c.get(), PH_EULER, g, 1, FCS_OP_D1, A_F, 4, A_DF2, 4, 4);
    } else {
      add_line_tasks(c.get(), PH_EULER, g, 0, FCS_OP_D1, A_F, 0, A_DF1, 0, 8);
      add_line_tasks(c.get(), PH_EULER, g, 1, FCS_OP_D1, A_F, 0, A_DF2, 0, 8);
    }
    if (c->visc) {
      // Lattice subpatch (constant metric, g^12 = 0): the derivatives along
      // a row meet only mu and d mu / dq^1 of that row, which vanish exactly
      // where mu vanishes on the whole row (columns likewise), so its lines
      // get activity entries and are skipped in steps where mu is zero on them.
      // (Subpatches with an empty row or column keep every line.)
      std::vector<int32_t> rspan, cspan;
      const int32_t *rs = nullptr, *cs = nullptr;
      bool full = true;
      for (const Run& r : g.rows) full = full && r.len > 0;
      for (const Run& r : g.cols) full = full && r.len > 0;
      if (g.affine && c->pdev[q].g12 == 0.0 && full && !p.visc_all_lines) {
        PatchDev& pd = c->pdev[q];
        pd.act_row = c->nact;
        pd.act_col = c->nact + g.n2;
        c->nact += g.n2 + g.n1;
        for (int l = 0; l < g.n2; ++l) rspan.push_back(pd.act_row + l);
        for (int l = 0; l < g.n1; ++l) cspan.push_back(pd.act_col + l);
        rs = rspan.data();
        cs = cspan.data();
      }
      add_line_tasks(c.get(), PH_EULER, g, 0, FCS_OP_D1, A_IN, 0, A_W1, 0, 4, rs);
      add_line_tasks(c.get(), PH_EULER, g, 0, FCS_OP_D2, A_IN, 0, A_W11, 0, 4, rs);
      add_line_tasks(c.get(), PH_EULER, g, 1, FCS_OP_D1, A_IN, 0, A_W2, 0, 4, cs);
      add_line_tasks(c.get(), PH_EULER, g, 1, FCS_OP_D2, A_IN, 0, A_W22, 0, 4, cs);
      // the mixed derivative of w enters only through g^12: subpatches where
      // g^12 vanishes at every active point need none (their W12 entries
      // keep the workspace's zeros, multiplied by g^12 = 0)
      bool has12 = false;
      for (size_t k = 0; k < g.np() && !has12; ++k) has12 = g.mask[k] && g.g12[k] != 0.0;
      if (c->cross && has12) add_line_tasks(c.get(), PH_CROSS, g, 1, FCS_OP_D1, A_W1, 0, A_W12, 0, 4);
      add_line_tasks(c.get(), PH_MUGRAD, g, 0, FCS_OP_D1, A_MU, 0, A_MU1, 0, 1);
      add_line_tasks(c.get(), PH_MUGRAD, g, 1, FCS_OP_D1, A_MU, 0, A_MU2, 0, 1);
    }
    if (p.filter) {
      add_line_tasks(c.get(), PH_FILT1, g, 0, FCS_OP_FILTER, A_F, 0, A_DF1, 0, 4);
      add_line_tasks(c.get(), PH_FILT2, g, 1, FCS_OP_FILTER, A_DF1, 0, A_DF2, 0, 4);
    }
    if (p.smear) {
      add_line_tasks(c.get(), PH_SMEAR1, g, 0, FCS_OP_SMEAR, A_F, 0, A_DF1, 0, 4);
      add_line_tasks(c.get(), PH_SMEAR2, g, 1, FCS_OP_SMEAR, A_DF1, 0, A_DF2, 0, 4);
    }
  }
  // activity flags of the row and the column of each blend row's point
  if (c->nact)
    for (const BlendRowDev& br : c->brow) {
      const int64_t k = br.dst;
      const PatchDev& pd = c->pdev[c->pid[k]];
      const int32_t j = c->ij[k] >> 16, i = c->ij[k] & 0xFFFF;
      c->bact.push_back(pd.act_row >= 0 ? make_int2(pd.act_row + j, pd.act_col + i) : make_int2(-1, -1));
    }
  // no-slip adiabatic walls: the lines ending there (Sec. 7 obstacle
  // conditions; a node ending two such lines uses the line along q^2)
  for (const Grid& g : c->grids) {
    std::map<std::pair<int, int>, int> dir_of;  // (j, i) -> line direction
    for (const BoundaryEntry& b : g.bnd)
      if (b.kind == kNoSlip) {
        auto key = std::make_pair(b.j, b.i);
        auto it = dir_of.find(key);
        dir_of[key] = it == dir_of.end() ? b.dir : std::max(it->second, b.dir);
      }
    std::map<std::pair<int, int>, std::vector<int>> line_pos;  // (dir, line) -> wall positions
    for (const auto& kv : dir_of) {
      const int j = kv.first.first, i = kv.first.second, dir = kv.second;
      const Run& r = dir == 0 ? g.rows[j] : g.cols[i];
      line_pos[std::make_pair(dir, dir == 0 ? j : i)].push_back((dir == 0 ? i : j) - r.start);
    }
    for (auto& kv : line_pos) {
      const int dir = kv.first.first, l = kv.first.second;
      const Run& r = dir == 0 ? g.rows[l] : g.cols[l];
      std::vector<int>& ps = kv.second;
      std::sort(ps.begin(), ps.end());
      WallLine w{};
      w.first = g.offset + (dir == 0 ? static_cast<int64_t>(l) * g.n1 + r.start
                                     : static_cast<int64_t>(r.start) * g.n1 + l);
      w.stride = dir == 0 ? 1 : g.n1;
      w.n = r.len;
      w.op = op_id(c.get(), r.len, FCS_OP_D1);
      w.pos[0] = ps[0];
      w.pos[1] = ps.size() > 1 ? ps[1] : -1;
      // a wall node that also carries Dirichlet data (an inflow side
      // meeting the wall) keeps them: it is solved for with the line but not
      // written
      for (int q = 0; q < 2; ++q) {
        w.keep[q] = 0;
        if (w.pos[q] < 0) continue;
        const int jj = dir == 0 ? l : r.start + w.pos[q], ii = dir == 0 ? r.start + w.pos[q] : l;
        for (const BoundaryEntry& b : g.bnd)
          if (b.j == jj && b.i == ii && (b.kind == kInflow || b.kind == kExact)) w.keep[q] = 1;
        if (g.xfringe[g.at(jj, ii)]) w.keep[q] = 1;
      }
      c->walls.push_back(w);
    }
  }
  // mixed forms store the stage derivatives in FP32 (their precision); with
  // cross derivatives W1 stays FP64, the operand of the cross contraction
  c->deriv_f32 = p.precision != FCS_PREC_FP64;
  if (c->visc) {
    c->phase_tasks[PH_EULER0] = c->phase_tasks[PH_EULER];
    c->phase_tasks[PH_EULER0].insert(c->phase_tasks[PH_EULER0].end(), c->phase_tasks[PH_MUGRAD].begin(),
                                     c->phase_tasks[PH_MUGRAD].end());
  }
  for (int ph = 0; ph < PH_N; ++ph) {
    // room for the tile list of every candidate shape the autotuner may pick
    size_t cap = 0;
    if (ph == PH_EULER || ph == PH_CROSS || ph == PH_EULER0) {
      int nv = 0;
      const GemmVariant* cand = gemm_variants(p.precision, &nv);
      for (int q = 0; q < nv; ++q) {
        c->var[ph] = cand[q];
        build_tiles(c.get(), ph);
        cap = std::max(cap, c->phase_tiles[ph].size());
      }
      c->var[ph] = GemmVariant{};
    }
    if ((ph == PH_FILT1 || ph == PH_FILT2) && p.precision == FCS_PREC_BF16X3) {
      // the split-BF16 filter in the line-stationary shape (one tile per 64
      // lines, fewer than the default shape's tiles)
      GemmVariant v;
      v.kc = 32;
      v.line = true;
      c->var[ph] = v;
    }
    build_tiles(c.get(), ph);
    c->tile_cap[ph] = std::max(cap, c->phase_tiles[ph].size());
  }
  // workspace layout
  Carve cv;
  auto& o = c->off;
  const size_t D = sizeof(double);
  for (const char* n : {"U0", "UA", "UB", "ACC"}) o[n] = cv.take(4 * P * D);
  for (const char* n : {"F", "DF1", "DF2"}) o[n] = cv.take(8 * P * D);
  if (c->visc) {
    for (const char* n : {"W1", "W2", "W11", "W22"}) o[n] = cv.take(4 * P * D);
    o["W12"] = cv.take((c->cross ? 4 * P : 1) * D);
    for (const char* n : {"MU", "MU1", "MU2", "MUHAT", "MUT", "TMP"}) o[n] = cv.take(P * D);
    o["PS"] = cv.take(2 * P * D);  // proxy and wave speed, interleaved
    o["TAU"] = cv.take(2 * P);
    o["WGEO"] = cv.take(P * 16);  // window geometry of every point (int4)
    o["LACT"] = cv.take(c->nact);
    o["BACT"] = cv.take(c->bact.size() * sizeof(int2));
  }
  for (int m = 0; m < 10; ++m) o["MET" + std::to_string(m)] = cv.take(P * D);
  o["FLAGS"] = cv.take(P);
  o["PID"] = cv.take(P * 4);
  o["IJ"] = cv.take(P * 4);
  o["PATCH"] = cv.take(c->pdev.size() * sizeof(PatchDev));
  o["ROWRUN"] = cv.take(c->rowrun.size() * sizeof(int2));
  o["COLRUN"] = cv.take(c->colrun.size() * sizeof(int2));
  o["OPOFF"] = cv.take(c->opk.off.size() * 8);
  o["OPROFF"] = cv.take(c->opk.roff.size() * 8);
  o["OPLD"] = cv.take(c->opk.ld.size() * 4);
  o["OPF64"] = cv.take(c->opk.elems * D);
  o["OPROW"] = cv.take(c->opk.rows * D);
  if (p.precision == FCS_PREC_FP32) o["OPF32"] = cv.take(c->opk.elems * 4);
  if (p.precision == FCS_PREC_BF16X3 || p.precision == FCS_PREC_BF16X6) {
    o["OPBHI"] = cv.take(c->opk.elems * 2);
    o["OPBLO"] = cv.take(c->opk.elems * 2);
  }
  if (p.precision == FCS_PREC_BF16X6) o["OPBMID"] = cv.take(c->opk.elems * 2);
  for (int ph = 0; ph < PH_N; ++ph) {
    for (int v = 0; v < 3; ++v)
      o["TASK" + std::to_string(ph) + "_" + std::to_string(v)] = cv.take(c->phase_tasks[ph].size() * sizeof(GemmTask));
    o["TILE" + std::to_string(ph)] = cv.take(c->tile_cap[ph] * sizeof(GemmTile));
  }
  o["COPY"] = cv.take(c->copy_pairs.size() * 8);
  o["CSRC"] = cv.take(P * 4);
  o["IDST"] = cv.take(c->idst.size() * 8);
  o["IPTR"] = cv.take(c->iptr.size() * 4);
  o["ICOL"] = cv.take(c->icol.size() * 8);
  o["IVAL"] = cv.take(c->ival.size() * D);
  o["BROW"] = cv.take(c->brow.size() * sizeof(BlendRowDev));
  o["BTERM"] = cv.take(c->bterm.size() * sizeof(BlendTermDev));
  o["BC"] = cv.take(c->bc.size() * sizeof(BcEntry));
  o["WALL"] = cv.take(c->walls.size() * sizeof(WallLine));
  o["WTH"] = cv.take(c->walls.size() * 2 * D);
  o["SDNNF"] = cv.take(64 * 84 * 4);  // classifier fragment table
  o["BCIDX"] = cv.take(P * 4);
  o["GCTR"] = cv.take(kGemmCounters * PH_N * 4);  // tile counters of the persistent contractions
  o["SDNN"] = cv.take(FCS_SDNN_NPARAM * 4);
  o["BASIS"] = cv.take(256 * D);
  o["WDIL"] = cv.take((p.n_v + 1) * D);
  o["SCAL"] = cv.take(8 * D);  // t, dt, last_dt, bad flag
  o["DTPART"] = cv.take(c->dt_blocks * D);
  c->ws_need = cv.used;
  c->tau_host.assign(2 * P, 0);
  *out = c.release();
  return FCS_OK;
}

extern "C" fcs_status fcs_workspace_size(const fcs_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return FCS_EINVAL;
  *bytes = ctx->ws_need;
  return FCS_OK;
}

namespace {
ViscArgs visc_args(fcs_ctx* c);
}  // namespace

extern "C" fcs_status fcs_bind(fcs_ctx* c, void* workspace, size_t bytes, void* stream) {
  if (!c || !workspace) return FCS_EINVAL;
  if (bytes < c->ws_need) return c->fail(FCS_ENOMEM, "workspace smaller than fcs_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return c->fail(FCS_EINVAL, "workspace not 256-byte aligned");
  c->ws = static_cast<char*>(workspace);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(stream);
  HIPCHK(c, hipMemsetAsync(c->ws, 0, c->ws_need, c->stream));
  const int64_t P = c->P;
  // operators in every precision the context uses
  std::vector<double> f64, rows;
  if (!c->opk.fill(c->prm.fc_d, c->prm.fc_C, f64, rows)) return c->fail(FCS_EINVAL, "unsupported operator length");
  fcs_status st;
  if ((st = upload(c, "OPF64", f64.data(), f64.size() * 8)) != FCS_OK) return st;
  if ((st = upload(c, "OPROW", rows.data(), rows.size() * 8)) != FCS_OK) return st;
  if ((st = upload(c, "OPOFF", c->opk.off.data(), c->opk.off.size() * 8)) != FCS_OK) return st;
  if ((st = upload(c, "OPROFF", c->opk.roff.data(), c->opk.roff.size() * 8)) != FCS_OK) return st;
  if ((st = upload(c, "OPLD", c->opk.ld.data(), c->opk.ld.size() * 4)) != FCS_OK) return st;
  std::vector<float> f32;
  std::vector<uint16_t> bhi, blo, bmid;
  if (c->prm.precision == FCS_PREC_FP32) {
    f32.assign(f64.begin(), f64.end());
    if ((st = upload(c, "OPF32", f32.data(), f32.size() * 4)) != FCS_OK) return st;
  }
  if (c->prm.precision == FCS_PREC_BF16X3) {
    split_bf16(f64, bhi, blo);
    if ((st = upload(c, "OPBHI", bhi.data(), bhi.size() * 2)) != FCS_OK) return st;
    if ((st = upload(c, "OPBLO", blo.data(), blo.size() * 2)) != FCS_OK) return st;
  }
  if (c->prm.precision == FCS_PREC_BF16X6) {
    split_bf16x3(f64, bhi, bmid, blo);
    if ((st = upload(c, "OPBHI", bhi.data(), bhi.size() * 2)) != FCS_OK) return st;
    if ((st = upload(c, "OPBMID", bmid.data(), bmid.size() * 2)) != FCS_OK) return st;
    if ((st = upload(c, "OPBLO", blo.data(), blo.size() * 2)) != FCS_OK) return st;
  }
  c->optab.off = c->dptr<int64_t>("OPOFF");
  c->optab.ld = c->dptr<int32_t>("OPLD");
  c->optab.roff = c->dptr<int64_t>("OPROFF");
  c->optab.f64 = c->dptr<double>("OPF64");
  c->optab.rowsum = c->dptr<double>("OPROW");
  c->optab.f32 = c->prm.precision == FCS_PREC_FP32 ? c->dptr<float>("OPF32") : nullptr;
  const bool split = c->prm.precision == FCS_PREC_BF16X3 || c->prm.precision == FCS_PREC_BF16X6;
  c->optab.bhi = split ? c->dptr<uint16_t>("OPBHI") : nullptr;
  c->optab.blo = split ? c->dptr<uint16_t>("OPBLO") : nullptr;
  c->optab.bmid = c->prm.precision == FCS_PREC_BF16X6 ? c->dptr<uint16_t>("OPBMID") : nullptr;
  // arrays
  c->arr[A_U0] = c->dptr<double>("U0");
  c->arr[A_UA] = c->dptr<double>("UA");
  c->arr[A_UB] = c->dptr<double>("UB");
  c->arr[A_F] = c->dptr<double>("F");
  c->arr[A_DF1] = c->dptr<double>("DF1");
  c->arr[A_DF2] = c->dptr<double>("DF2");
  if (c->visc) {
    c->arr[A_W1] = c->dptr<double>("W1");
    c->arr[A_W2] = c->dptr<double>("W2");
    c->arr[A_W11] = c->dptr<double>("W11");
    c->arr[A_W22] = c->dptr<double>("W22");
    c->arr[A_W12] = c->dptr<double>("W12");
    c->arr[A_MU] = c->dptr<double>("MU");
    c->arr[A_MU1] = c->dptr<double>("MU1");
    c->arr[A_MU2] = c->dptr<double>("MU2");
  }
  // tasks: three variants by the stage input buffer (U0, UA, UB)
  std::vector<GemmTask> staging_tasks[PH_N][3];
  for (int ph = 0; ph < PH_N; ++ph)
    for (int v = 0; v < 3; ++v) {
      std::vector<GemmTask>& dt = staging_tasks[ph][v];
      dt.clear();
      for (const TaskSpec& s : c->phase_tasks[ph]) {
        GemmTask t{};
        t.act = s.act;
        double* sbase = s.src_arr == A_IN ? c->arr[A_U0 + v] : c->arr[s.src_arr];
        t.src = sbase + s.src_off;
        const bool f32 = c->deriv_f32 && (ph == PH_EULER || ph == PH_EULER0 || ph == PH_CROSS) &&
                         s.dst_arr != A_MU1 && s.dst_arr != A_MU2 && !(c->cross && s.dst_arr == A_W1);
        // element offsets count in the stored type
        t.dst = f32 ? static_cast<void*>(reinterpret_cast<float*>(c->arr[s.dst_arr]) + s.dst_off)
                    : static_cast<void*>(c->arr[s.dst_arr] + s.dst_off);
        t.comp_stride = P;
        t.row_stride = s.row_stride;
        t.s_stride = s.s_stride;
        t.nrow = s.nrow;
        t.ncomp = s.ncomp;
        t.n = s.n;
        t.op = s.op;
        t.out_f32 = f32 ? 1 : 0;
        dt.push_back(t);
      }
      std::string name = "TASK" + std::to_string(ph) + "_" + std::to_string(v);
      if ((st = upload(c, name.c_str(), dt.data(), dt.size() * sizeof(GemmTask))) != FCS_OK) return st;
      c->d_tasks[ph][v] = c->dptr<GemmTask>(name.c_str());
    }
  for (int ph = 0; ph < PH_N; ++ph) {
    std::string name = "TILE" + std::to_string(ph);
    if ((st = upload(c, name.c_str(), c->phase_tiles[ph].data(), c->phase_tiles[ph].size() * sizeof(GemmTile))) !=
        FCS_OK)
      return st;
    c->d_tiles[ph] = c->dptr<GemmTile>(name.c_str());
  }
  for (int m = 0; m < 10; ++m) {
    std::string name = "MET" + std::to_string(m);
    if ((st = upload(c, name.c_str(), c->metric_host[m].data(), P * 8)) != FCS_OK) return st;
  }
  struct {
    const char* n;
    const void* p;
    size_t b;
  } ups[] = {
      {"FLAGS", c->flags.data(), c->flags.size()},
      {"PID", c->pid.data(), c->pid.size() * 4},
      {"IJ", c->ij.data(), c->ij.size() * 4},
      {"PATCH", c->pdev.data(), c->pdev.size() * sizeof(PatchDev)},
      {"ROWRUN", c->rowrun.data(), c->rowrun.size() * sizeof(int2)},
      {"COLRUN", c->colrun.data(), c->colrun.size() * sizeof(int2)},
      {"COPY", c->copy_pairs.data(), c->copy_pairs.size() * 8},
      {"CSRC", c->csrc.data(), c->csrc.size() * 4},
      {"IDST", c->idst.data(), c->idst.size() * 8},
      {"IPTR", c->iptr.data(), c->iptr.size() * 4},
      {"ICOL", c->icol.data(), c->icol.size() * 8},
      {"IVAL", c->ival.data(), c->ival.size() * 8},
      {"BROW", c->brow.data(), c->brow.size() * sizeof(BlendRowDev)},
      {"BTERM", c->bterm.data(), c->bterm.size() * sizeof(BlendTermDev)},
      {"BC", c->bc.data(), c->bc.size() * sizeof(BcEntry)},
      {"WALL", c->walls.data(), c->walls.size() * sizeof(WallLine)},
      {"BCIDX", c->bcidx.data(), c->bcidx.size() * 4},
      {"SDNN", c->sdnn.data(), c->sdnn.size() * 4},
      {"BASIS", c->basis.data(), c->basis.size() * 8},
      {"WDIL", c->wdil.data(), c->wdil.size() * 8},
      {"BACT", c->bact.data(), c->bact.size() * sizeof(int2)},
  };
  for (auto& u : ups)
    if ((st = upload(c, u.n, u.p, u.b)) != FCS_OK) return st;
  if (c->visc && c->prm.av_mode == FCS_AV_SDNN)
    HIPCHK(c, launch_sdnn_pack(c->dptr<float>("SDNN"), c->dptr<uint32_t>("SDNNF"), c->stream));
  if (c->visc) HIPCHK(c, launch_window_geo(visc_args(c), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& v : staging_tasks)
    for (auto& w : v) std::vector<GemmTask>().swap(w);
  c->bound = true;
  c->cur = c->arr[A_U0];
  double scal0[5] = {c->t_host, 0.0, 0.0, 0.0, c->t_host};
  HIPCHK(c, hipMemcpyAsync(c->dptr<double>("SCAL"), scal0, sizeof(scal0), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->stream && !c->stream2) {
    // default priority, like the caller's stream
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork2, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_join2, hipEventDisableTiming));
  }
  return FCS_OK;
}

namespace {

// Adds an event-record node to the graph being captured on the context's
// stream, after everything captured so far, and makes it the new frontier.
fcs_status record_in_capture(fcs_ctx* c, hipEvent_t ev) {
  hipStreamCaptureStatus cs;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  HIPCHK(c, hipStreamGetCaptureInfo_v2(c->stream, &cs, nullptr, &g, &deps, &nd));
  if (cs != hipStreamCaptureStatusActive) return c->fail(FCS_EHIP, "event node requested outside a capture");
  hipGraphNode_t node;
  HIPCHK(c, hipGraphAddEventRecordNode(&node, g, deps, nd, ev));
  HIPCHK(c, hipStreamUpdateCaptureDependencies(c->stream, &node, 1, hipStreamSetCaptureDependencies));
  return FCS_OK;
}

fcs_status run_gemm(fcs_ctx* c, int ph, int variant, int precision, bool timed, hipStream_t s = nullptr) {
  if (!s) s = c->stream;
  if (c->phase_tiles[ph].empty()) return FCS_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed && c->capturing_prof) {
    // inside a profiled graph: one event pair per stage, recorded as graph nodes
    e0 = c->pev[c->prof_wf][2 * c->prof_stage];
    e1 = c->pev[c->prof_wf][2 * c->prof_stage + 1];
    fcs_status st = record_in_capture(c, e0);
    if (st != FCS_OK) return st;
  } else if (timed && c->prof && c->ev_used + 2 <= c->ev.size()) {
    e0 = c->ev[c->ev_used++];
    e1 = c->ev[c->ev_used++];
    HIPCHK(c, hipEventRecord(e0, c->stream));
  }
  // the stage phases in their tuned shape; the once-per-step phases in the
  // default shape, through the stage kernels in the mixed forms and through
  // k_gemm_step (FP64, its own name in profiles) otherwise
  if (ph == PH_EULER || ph == PH_CROSS || ph == PH_EULER0 || precision != FCS_PREC_FP64)
    HIPCHK(c, launch_gemm(precision, c->var[ph], c->d_tasks[ph][variant], c->d_tiles[ph],
                          static_cast<int>(c->phase_tiles[ph].size()), c->optab, c->dptr<int>("GCTR") + kGemmCounters * ph,
                          s));
  else
    HIPCHK(c, launch_gemm_step(c->d_tasks[ph][variant], c->d_tiles[ph], static_cast<int>(c->phase_tiles[ph].size()),
                               c->optab, s));
  if (e1) {
    if (c->capturing_prof) {
      fcs_status st = record_in_capture(c, e1);
      if (st != FCS_OK) return st;
    } else
      HIPCHK(c, hipEventRecord(e1, c->stream));
  }
  return FCS_OK;
}

// Device arguments of the viscosity kernels (Alg. 3 and the blend).
ViscArgs visc_args(fcs_ctx* c) {
  const int64_t P = c->P;
  const fcs_params& p = c->prm;
  ViscArgs v{};
  v.P = P;
  v.U = c->arr[A_U0];
  v.flags = c->dptr<uint8_t>("FLAGS");
  v.pid = c->dptr<int32_t>("PID");
  v.patches = c->dptr<PatchDev>("PATCH");
  v.rowrun = c->dptr<int2>("ROWRUN");
  v.colrun = c->dptr<int2>("COLRUN");
  v.ps = c->dptr<double2>("PS");
  v.ij = c->dptr<int32_t>("IJ");
  v.hx = c->dptr<double>("MET9");
  v.tau = c->dptr<uint8_t>("TAU");
  v.muhat = c->dptr<double>("MUHAT");
  v.tmp = c->dptr<double>("TMP");
  v.mut = c->dptr<double>("MUT");
  v.mu = c->arr[A_MU];
  v.mode = p.av_mode;
  v.weights = c->dptr<float>("SDNN");
  v.sdnn_table = c->dptr<uint32_t>("SDNNF");
  v.basis = c->dptr<double>("BASIS");
  v.c_mu = p.c_mu;
  v.gamma = p.gamma;
  v.nv = p.n_v;
  v.wdil = c->dptr<double>("WDIL");
  v.nblend = static_cast<int>(c->brow.size());
  v.brow = c->dptr<BlendRowDev>("BROW");
  v.bterm = c->dptr<BlendTermDev>("BTERM");
  v.act = c->nact ? c->dptr<uint8_t>("LACT") : nullptr;
  v.bact = c->nact ? c->dptr<int2>("BACT") : nullptr;
  v.wgeo = c->dptr<int4>("WGEO");
  return v;
}

// Alg. 3 + blend + gradient of mu and the filter (Alg. 4); the adaptive
// step size follows in the first stage.
fcs_status per_step(fcs_ctx* c) {
  const int64_t P = c->P;
  const fcs_params& p = c->prm;
  double* U0 = c->arr[A_U0];
  fcs_status st;
  ViscArgs v{};
  if (c->visc) {
    v = visc_args(c);
    // a captured step relies on the previous step's last stage (or on the
    // proxy launch that precedes the graph's first replay)
    if (!c->in_capture && !c->ps_valid) HIPCHK(c, launch_proxy(v, c->stream));
  }
  // Alg. 4 (filter) reads and rewrites the state, which after the proxy
  // kernel no part of Alg. 3 reads: with a second stream the two run side by
  // side and join before the step size is taken.
  const bool filt = p.filter && c->past_t0;
  const bool fork = filt && c->visc && c->stream2 != nullptr;
  if (filt) {
    hipStream_t fs = c->stream;
    if (fork) {
      HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
      HIPCHK(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
      fs = c->stream2;
    }
    HIPCHK(c, launch_filter_pre(U0, c->arr[A_F], c->dptr<uint8_t>("FLAGS"), P, p.gamma, fs));
    // the filter's contractions in the precision mode (Alg. 4 on the FP64
    // state; outputs FP64)
    if ((st = run_gemm(c, PH_FILT1, 0, p.precision, false, fs)) != FCS_OK) return st;
    if ((st = run_gemm(c, PH_FILT2, 0, p.precision, false, fs)) != FCS_OK) return st;
    const double* met[4] = {c->dptr<double>("MET0"), c->dptr<double>("MET1"), c->dptr<double>("MET2"),
                            c->dptr<double>("MET3")};
    FluxOut fo{c->arr[A_F], met[0], met[1], met[2], met[3], p.gamma - 1.0, c->dptr<int32_t>("PID"),
               c->dptr<PatchDev>("PATCH")};
    HIPCHK(c, launch_filter_post(c->arr[A_DF2], U0, c->dptr<uint8_t>("FLAGS"), P, fo, fs));
    if (fork) HIPCHK(c, hipEventRecord(c->ev_join, c->stream2));
  }
  if (c->visc) {
    HIPCHK(c, launch_viscosity(v, c->stream));
    // which viscous contraction tiles this step needs (mu is frozen for it;
    // the viscosity kernels have left the line activity flags)
    if (c->nact)
      HIPCHK(c, launch_tile_activity(c->d_tasks[PH_EULER][0], c->d_tiles[PH_EULER],
                                     static_cast<int>(c->phase_tiles[PH_EULER].size()), c->d_tasks[PH_EULER0][0],
                                     c->d_tiles[PH_EULER0], static_cast<int>(c->phase_tiles[PH_EULER0].size()),
                                     v.act, c->stream));
  }
  if (fork) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  if (p.smear && !c->past_t0) {
    // Alg. 4 at t = 0 (after the viscosity, which Alg. 1 evaluates first):
    // the window from this step's classes, the strongly filtered rho, rho u,
    // rho v, theta (FCS_OP_SMEAR along q^1 then q^2) and the blend.  The
    // indicator and the window are held in the first stage's output buffer,
    // not yet written in this step: mu-hat stays this step's, and the
    // viscous derivative arrays hold nothing but derivatives (the stage
    // kernel multiplies their values on skipped lines by exact zeros, so
    // they must stay finite: FP64 window values read as FP32 pairs in the
    // mixed forms are not)
    const uint8_t* flags = c->dptr<uint8_t>("FLAGS");
    double* ind = c->arr[A_UA];
    double* w = c->arr[A_UA] + P;
    HIPCHK(c, launch_smear_window(v, ind, w, c->stream));
    HIPCHK(c, launch_filter_pre(U0, c->arr[A_F], flags, P, p.gamma, c->stream));
    if ((st = run_gemm(c, PH_SMEAR1, 0, FCS_PREC_FP64, false)) != FCS_OK) return st;
    if ((st = run_gemm(c, PH_SMEAR2, 0, FCS_PREC_FP64, false)) != FCS_OK) return st;
    HIPCHK(c, launch_smear_post(c->arr[A_DF2], c->arr[A_F], w, U0, flags, P, c->stream));
  }
  return FCS_OK;  // the step size is taken by the first stage (one_stage)
}

fcs_status apply_walls(fcs_ctx* c, double* U, const FluxOut& fo, double2* ps);

fcs_status one_stage(fcs_ctx* c, int s) {
  const int64_t P = c->P;
  const fcs_params& p = c->prm;
  static const int in_buf[5] = {A_U0, A_UA, A_UB, A_UA, A_UB};
  static const int out_buf[5] = {A_UA, A_UB, A_UA, A_UB, A_U0};
  double* in = c->arr[in_buf[s]];
  double* outp = c->arr[out_buf[s]];
  const int variant = in_buf[s] - A_U0;
  const uint8_t* flags = c->dptr<uint8_t>("FLAGS");
  const double* met[10];
  for (int m = 0; m < 10; ++m) met[m] = c->dptr<double>(("MET" + std::to_string(m)).c_str());
  // fluxes of the stage input: computed here at the first stage of a step
  // (after the filter); later stages receive them from the previous stage's
  // update and fringe fill
  FluxOut fo{c->arr[A_F], met[0], met[1], met[2], met[3], p.gamma - 1.0, c->dptr<int32_t>("PID"),
             c->dptr<PatchDev>("PATCH")};
  // after the filter (every step but the first) the filter's last kernel has
  // already stored the fluxes of the stage input
  if (s == 0 && !(p.filter && c->past_t0)) HIPCHK(c, launch_flux(in, flags, fo, P, c->stream));
  // The step size (CFL and viscous limits) reads only the filtered state and
  // mu: it runs on the second stream beside the first stage's contraction
  // and joins before the stage update that uses it.
  const bool dt_side = s == 0 && c->stream2 != nullptr;
  if (s == 0) {
    hipStream_t ds = c->stream;
    if (dt_side) {
      HIPCHK(c, hipEventRecord(c->ev_fork2, c->stream));
      HIPCHK(c, hipStreamWaitEvent(c->stream2, c->ev_fork2, 0));
      ds = c->stream2;
    }
    HIPCHK(c, launch_dt(in, flags, met[9], c->visc ? c->arr[A_MU] : nullptr, c->dptr<double>("DTPART"),
                        c->dt_blocks, P, p.gamma, p.cfl, p.dt_fixed, c->dptr<double>("SCAL"), ds));
    if (dt_side) HIPCHK(c, hipEventRecord(c->ev_join2, c->stream2));
  }
  fcs_status st;
  c->prof_stage = s;
  // the first stage's launch also differentiates mu (PH_EULER0); the later
  // stages' launches carry the stage tasks only and are the ones timed
  const int eph = (s == 0 && c->visc) ? PH_EULER0 : PH_EULER;
  if ((st = run_gemm(c, eph, variant, p.precision, s > 0)) != FCS_OK) return st;
  if (c->visc && c->cross)
    if ((st = run_gemm(c, PH_CROSS, 0, p.precision, false)) != FCS_OK) return st;
  if (dt_side) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join2, 0));
  StageArgs a{};
  a.P = P;
  a.stage = s;
  switch (s) {
    case 0: a.c[0] = kA0; break;
    case 1: a.c[1] = kB20; a.c[2] = kB21; a.c[3] = kA1; break;
    case 2: a.c[1] = kB30; a.c[2] = kB32; a.c[3] = kA2; a.c[4] = kC2; break;
    case 3: a.c[1] = kB40; a.c[2] = kB43; a.c[3] = kA3; a.c[4] = kC3; a.c[5] = kD3; break;
    default: a.c[4] = kC4; a.c[5] = kD4; break;
  }
  a.gm1 = p.gamma - 1.0;
  a.flags = flags;
  a.in = in;
  a.U0 = c->arr[A_U0];
  a.out = outp;
  a.acc = c->dptr<double>("ACC");
  a.DF1 = c->arr[A_DF1];
  a.DF2 = c->arr[A_DF2];
  a.t1x = met[0];
  a.t1y = met[1];
  a.t2x = met[2];
  a.t2y = met[3];
  a.visc = c->visc;
  if (c->visc) {
    a.mu = c->arr[A_MU];
    a.mu1 = c->arr[A_MU1];
    a.mu2 = c->arr[A_MU2];
    a.g11 = met[4];
    a.g12 = met[5];
    a.g22 = met[6];
    a.lap1 = met[7];
    a.lap2 = met[8];
    a.W1 = c->arr[A_W1];
    a.W2 = c->arr[A_W2];
    a.W11 = c->arr[A_W11];
    a.W22 = c->arr[A_W22];
    a.W12 = c->cross ? c->arr[A_W12] : nullptr;
  }
  a.deriv_f32 = c->deriv_f32;
  a.w1_f64 = c->deriv_f32 && c->cross;
  a.pid = c->dptr<int32_t>("PID");
  a.patches = c->dptr<PatchDev>("PATCH");
  double* scal = c->dptr<double>("SCAL");
  a.dt = scal + 1;
  a.bad_flag = reinterpret_cast<int*>(scal + 3);
  double frac[5];
  stage_fractions(frac);
  a.bcs.bc = c->dptr<BcEntry>("BC");
  a.bcs.bcidx = c->dptr<int32_t>("BCIDX");
  a.bcs.gamma = p.gamma;
  a.bcs.t = scal;
  a.bcs.frac = frac[s];
  a.bcs.vortex = VortexArgs{p.vortex[0], p.vortex[1], p.vortex[2], p.vortex[3], p.vortex[4]};
  // the last stage's output starts the next step, whose fluxes follow the filter
  FluxOut next = fo;
  if (s == 4) next.F = nullptr;
  a.flux = next;
  // copy fringe points are updated inside the stage kernel (from their
  // donors); the fringe kernel evaluates the interpolation rows only.  With
  // no-slip walls every point takes its own update first: the wall
  // temperature's FC-Neumann condition reads whole grid lines, fringe points
  // included, before the fringe fill; the copies follow the walls.
  a.csrc = c->walls.empty() ? c->dptr<int32_t>("CSRC") : nullptr;
  // the last stage also leaves the next step's proxy values
  a.ps = (s == 4 && c->visc) ? c->dptr<double2>("PS") : nullptr;
  HIPCHK(c, launch_stage(a, c->stream));
  // no-slip walls need the whole stage output; the copy fringe points are
  // filled after them
  if ((st = apply_walls(c, outp, next, a.ps)) != FCS_OK) return st;
  const int ncopy = c->walls.empty() ? 0 : static_cast<int>(c->copy_pairs.size() / 2);
  HIPCHK(c, launch_fringe(outp, flags, c->dptr<int64_t>("COPY"), ncopy, c->dptr<int64_t>("IDST"),
                          c->dptr<int32_t>("IPTR"), c->dptr<int64_t>("ICOL"), c->dptr<double>("IVAL"),
                          static_cast<int>(c->idst.size()), P, next, a.ps, p.gamma, c->stream));
  if (s == 4) c->ps_valid = c->visc;
  c->cur = outp;
  return FCS_OK;
}

// No-slip adiabatic walls of a state (after its other boundary conditions,
// before the fringe fill): fluxes and proxy values of the corrected points
// through fo / ps when set.
fcs_status apply_walls(fcs_ctx* c, double* U, const FluxOut& fo, double2* ps) {
  if (c->walls.empty()) return FCS_OK;
  HIPCHK(c, launch_walls(U, c->dptr<WallLine>("WALL"), static_cast<int>(c->walls.size()), c->optab,
                         c->dptr<double>("WTH"), c->dptr<uint8_t>("FLAGS"), c->P, c->prm.gamma, fo, ps, c->stream));
  return FCS_OK;
}

// Before the first step from t = 0: the initial data are made to satisfy
// the boundary conditions (walls, inflow, exact data), as the solution does
// after every stage; the first step's viscosity then sees the jumps that
// the walls impose.
fcs_status prepare_t0(fcs_ctx* c) {
  const fcs_params& p = c->prm;
  double* U0 = c->arr[A_U0];
  const uint8_t* flags = c->dptr<uint8_t>("FLAGS");
  BcArgs b{};
  b.bc = c->dptr<BcEntry>("BC");
  b.bcidx = c->dptr<int32_t>("BCIDX");
  b.gamma = p.gamma;
  b.vortex = VortexArgs{p.vortex[0], p.vortex[1], p.vortex[2], p.vortex[3], p.vortex[4]};
  if (!c->bc.empty()) HIPCHK(c, launch_bc_state(U0, flags, b, c->t_host, c->P, c->stream));
  FluxOut none{};
  none.F = nullptr;
  fcs_status st;
  if ((st = apply_walls(c, U0, none, nullptr)) != FCS_OK) return st;
  // the fringe points keep the data's own (pointwise) values: interpolating
  // discontinuous initial data would overshoot; the first stage's fringe
  // fill follows the smearing
  (void)flags;
  c->ps_valid = false;
  c->t0_prepared = true;
  return FCS_OK;
}

fcs_status full_step_eager(fcs_ctx* c) {
  fcs_status st;
  if ((st = per_step(c)) != FCS_OK) return st;
  for (int s = 0; s < 5; ++s)
    if ((st = one_stage(c, s)) != FCS_OK) return st;
  return FCS_OK;
}

// Useful flops and bytes of one stage contraction of the last step (a
// viscous line counts only if that step needed it).  Synchronizes.
fcs_status stage_work(fcs_ctx* c, double* flops, double* bytes) {
  if (c->nact) {
    c->act_host.resize(c->nact);
    HIPCHK(c, hipMemcpyAsync(c->act_host.data(), c->dptr<uint8_t>("LACT"), c->nact, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  double f = 0, b = 0;
  for (const TaskSpec& t : c->phase_tasks[PH_EULER]) {
    double lines = static_cast<double>(t.nrow) * t.ncomp;
    if (t.act >= 0) {
      int live = 0;
      for (int r = 0; r < t.nrow; ++r) live += c->act_host[t.act + r] != 0;
      lines = static_cast<double>(live) * t.ncomp;
    }
    f += 2.0 * t.n * t.n * lines;
    b += task_bytes(c, t) * lines;
  }
  *flops = f;
  *bytes = b;
  return FCS_OK;
}

// Profile mode: accumulates the useful work of `launches` stage contractions
// of the step just run.
fcs_status prof_account(fcs_ctx* c, int launches) {
  double f = 0, b = 0;
  fcs_status st = stage_work(c, &f, &b);
  if (st != FCS_OK) return st;
  c->prof_flops += launches * f;
  c->prof_bytes += launches * b;
  c->prof_fn += launches;
  return FCS_OK;
}

fcs_status check_bad(fcs_ctx* c) {
  int bad = 0;
  HIPCHK(c, hipMemcpyAsync(&bad, c->dptr<double>("SCAL") + 3, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (bad) return c->fail(FCS_ENONFINITE, "non-finite or non-physical state (rho <= 0 or p <= 0)");
  return FCS_OK;
}

}  // namespace

extern "C" fcs_status fcs_set_state(fcs_ctx* c, int32_t patch, int32_t vars, const double* src,
                                    int32_t src_on_device) {
  if (!c || !src) return FCS_EINVAL;
  if (!c->bound) return c->fail(FCS_ESTATE, "fcs_set_state before fcs_bind");
  if (patch < 0 || patch >= static_cast<int32_t>(c->grids.size())) return c->fail(FCS_EINVAL, "bad patch index");
  // the state lives in U0 at step boundaries only
  if (c->stage_in_step != 0) return c->fail(FCS_ESTATE, "fcs_set_state inside a step: advance to a step boundary first");
  if (vars != FCS_VARS_CONS && vars != FCS_VARS_PRIM) return c->fail(FCS_EINVAL, "bad variable kind");
  c->ps_valid = false;
  c->t0_prepared = false;
  const Grid& g = c->grids[patch];
  const size_t np = g.np();
  std::vector<double> h(4 * np);
  if (src_on_device) {
    HIPCHK(c, hipMemcpyAsync(h.data(), src, 4 * np * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::copy(src, src + 4 * np, h.begin());
  }
  const double gm = c->prm.gamma;
  std::vector<double> e(4 * np, 0.0);
  for (size_t k = 0; k < np; ++k) {
    if (!g.mask[k]) continue;
    if (vars == FCS_VARS_PRIM) {
      double r = h[k], u = h[np + k], v = h[2 * np + k], pr = h[3 * np + k];
      e[k] = r;
      e[np + k] = r * u;
      e[2 * np + k] = r * v;
      e[3 * np + k] = pr / (gm - 1.0) + 0.5 * r * (u * u + v * v);
    } else {
      for (int q = 0; q < 4; ++q) e[q * np + k] = h[q * np + k];
    }
  }
  for (int q = 0; q < 4; ++q)
    HIPCHK(c, hipMemcpyAsync(c->arr[A_U0] + q * c->P + g.offset, e.data() + q * np, np * 8, hipMemcpyHostToDevice,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->cur = c->arr[A_U0];
  return FCS_OK;
}

extern "C" fcs_status fcs_set_time(fcs_ctx* c, double t) {
  if (!c || !std::isfinite(t)) return FCS_EINVAL;
  if (c->stage_in_step != 0) return c->fail(FCS_ESTATE, "fcs_set_time inside a step: advance to a step boundary first");
  c->t_host = t;
  c->past_t0 = t != 0.0;
  c->t0_prepared = false;
  if (c->bound) {
    HIPCHK(c, hipMemcpyAsync(c->dptr<double>("SCAL"), &c->t_host, 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dptr<double>("SCAL") + 4, &c->t_host, 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return FCS_OK;
}

extern "C" fcs_status fcs_set_tau(fcs_ctx* c, int32_t patch, const uint8_t* tau) {
  if (!c || !tau) return FCS_EINVAL;
  if (!c->bound || !c->visc) return c->fail(FCS_ESTATE, "fcs_set_tau needs a bound context with viscosity");
  if (patch < 0 || patch >= static_cast<int32_t>(c->grids.size())) return c->fail(FCS_EINVAL, "bad patch index");
  const Grid& g = c->grids[patch];
  for (int dir = 0; dir < 2; ++dir) {
    for (size_t k = 0; k < g.np(); ++k) {
      if (tau[dir * g.np() + k] > 2) return c->fail(FCS_EINVAL, "tau values must be 0, 1 or 2");
    }
    HIPCHK(c, hipMemcpyAsync(c->dptr<uint8_t>("TAU") + dir * c->P + g.offset, tau + dir * g.np(), g.np(),
                             hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FCS_OK;
}

namespace {

fcs_status capture_step(fcs_ctx* c, int with_filter, bool profiled) {
  hipGraphExec_t* slot = profiled ? &c->pgexec[with_filter] : &c->gexec[with_filter];
  if (*slot) return FCS_OK;
  if (profiled)
    for (auto& e : c->pev[with_filter])
      if (!e) HIPCHK(c, hipEventCreate(&e));
  hipGraph_t graph;
  const bool saved = c->past_t0;
  c->past_t0 = with_filter != 0;
  bool saved_prof = c->prof;
  const bool saved_ps = c->ps_valid;
  c->prof = false;
  c->capturing_prof = profiled;
  c->in_capture = true;
  c->prof_wf = with_filter;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  fcs_status st = FCS_OK;
  if (profiled && (st = record_in_capture(c, c->pev[with_filter][10])) == FCS_OK)
    st = record_in_capture(c, c->pev[with_filter][11]);
  if (st == FCS_OK) st = full_step_eager(c);
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  c->past_t0 = saved;
  c->prof = saved_prof;
  c->capturing_prof = false;
  c->in_capture = false;
  c->ps_valid = saved_ps;
  if (st != FCS_OK) return st;
  if (e != hipSuccess) return c->fail(FCS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(slot, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return c->fail(FCS_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return FCS_OK;
}

}  // namespace

namespace {

// Autotuner of the contraction tile shape: times every candidate variant on
// the stage contraction (current state, stage-0 operands) with HIP events
// and keeps the fastest for the stage and cross-derivative launches.  With
// skippable viscous lines the candidates run on the tiles the current
// state's viscosity needs, as a step from this state would.
fcs_status autotune(fcs_ctx* c) {
  constexpr int kTuneReps = 10;  // timed launches per candidate
  c->tuned = true;
  if (!c->prm.autotune || c->phase_tiles[PH_EULER].empty()) return FCS_OK;
  int nv = 0;
  const GemmVariant* cand = gemm_variants(c->prm.precision, &nv);
  std::fill(std::begin(c->tune_ms), std::end(c->tune_ms), 0.0f);
  uint8_t* act = nullptr;
  if (c->visc && c->nact) {
    // the viscosity of the current state and its line activity (recomputed
    // by the next step)
    const ViscArgs v = visc_args(c);
    if (!c->ps_valid) HIPCHK(c, launch_proxy(v, c->stream));
    c->ps_valid = true;
    HIPCHK(c, launch_viscosity(v, c->stream));
    act = v.act;
  }
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float best = 1e30f;
  GemmVariant bestv = c->var[PH_EULER];
  for (int q = 0; q < nv; ++q) {
    c->var[PH_EULER] = cand[q];
    build_tiles(c, PH_EULER);
    if (c->phase_tiles[PH_EULER].size() > c->tile_cap[PH_EULER]) continue;
    fcs_status st = upload(c, "TILE0", c->phase_tiles[PH_EULER].data(),
                           c->phase_tiles[PH_EULER].size() * sizeof(GemmTile));
    if (st != FCS_OK) return st;
    if (act)
      HIPCHK(c, launch_tile_activity(c->d_tasks[PH_EULER][0], c->d_tiles[PH_EULER],
                                     static_cast<int>(c->phase_tiles[PH_EULER].size()), nullptr, nullptr, 0, act,
                                     c->stream));
    if ((st = run_gemm(c, PH_EULER, 0, c->prm.precision, false)) != FCS_OK) return st;
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < kTuneReps; ++r)
      if ((st = run_gemm(c, PH_EULER, 0, c->prm.precision, false)) != FCS_OK) return st;
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    c->tune_ms[q] = ms / kTuneReps;
  }
  // the earliest candidate within 2 % of the fastest: near-ties (within the
  // timing noise) resolve the same way from run to run
  for (int q = 0; q < nv; ++q)
    if (c->tune_ms[q] > 0 && c->tune_ms[q] < best) best = c->tune_ms[q];
  for (int q = 0; q < nv; ++q)
    if (c->tune_ms[q] > 0 && c->tune_ms[q] <= 1.02f * best) {
      bestv = cand[q];
      c->stage_variant = q;
      break;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  for (int ph : {PH_EULER, PH_CROSS, PH_EULER0}) {
    c->var[ph] = bestv;
    build_tiles(c, ph);
    if (c->phase_tiles[ph].empty()) continue;
    std::string name = "TILE" + std::to_string(ph);
    fcs_status st = upload(c, name.c_str(), c->phase_tiles[ph].data(), c->phase_tiles[ph].size() * sizeof(GemmTile));
    if (st != FCS_OK) return st;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FCS_OK;
}

}  // namespace

extern "C" fcs_status fcs_advance(fcs_ctx* c, int64_t n_stages, double* t_out) {
  if (!c) return FCS_EINVAL;
  if (!c->bound) return c->fail(FCS_ESTATE, "fcs_advance before fcs_bind");
  if (n_stages < 0) return c->fail(FCS_EINVAL, "negative stage count");
  fcs_status st;
  if (!c->tuned && (st = autotune(c)) != FCS_OK) return st;
  const bool graph = c->prm.use_graph && c->stream != nullptr;
  while (n_stages > 0) {
    if (c->stage_in_step == 0 && !c->past_t0 && !c->t0_prepared && (st = prepare_t0(c)) != FCS_OK) return st;
    if (c->stage_in_step == 0 && n_stages >= 5) {
      int wf = (c->prm.filter && c->past_t0) ? 1 : 0;
      // the step that smears the initial data runs once, eagerly
      if (graph && !(c->prm.smear && !c->past_t0)) {
        if ((st = capture_step(c, wf, c->prof)) != FCS_OK) return st;
        if (c->visc && !c->ps_valid) HIPCHK(c, launch_proxy(visc_args(c), c->stream));
        HIPCHK(c, hipGraphLaunch(c->prof ? c->pgexec[wf] : c->gexec[wf], c->stream));
        c->ps_valid = c->visc;
        c->cur = c->arr[A_U0];
        if (c->prof) {
          // the events of a profiled graph are re-recorded by every replay
          HIPCHK(c, hipStreamSynchronize(c->stream));
          for (int q = 1; q < 5; ++q) {  // stages 1..4 carry the timed launches
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, c->pev[wf][2 * q], c->pev[wf][2 * q + 1]));
            c->prof_ms += ms;
            c->prof_n++;
          }
          float ms = 0;
          HIPCHK(c, hipEventElapsedTime(&ms, c->pev[wf][10], c->pev[wf][11]));
          c->prof_ovh_ms += ms;
          c->prof_ovh_n++;
          if ((st = prof_account(c, 4)) != FCS_OK) return st;
        }
      } else {
        if ((st = full_step_eager(c)) != FCS_OK) return st;
        if (c->prof && (st = prof_account(c, 4)) != FCS_OK) return st;
      }
      c->steps++;
      c->past_t0 = true;
      c->stages += 5;
      n_stages -= 5;
      continue;
    }
    if (c->stage_in_step == 0)
      if ((st = per_step(c)) != FCS_OK) return st;
    if ((st = one_stage(c, c->stage_in_step)) != FCS_OK) return st;
    if (c->prof && c->stage_in_step > 0 && (st = prof_account(c, 1)) != FCS_OK) return st;
    c->stages++;
    n_stages--;
    if (++c->stage_in_step == 5) {
      c->stage_in_step = 0;
      c->steps++;
      c->past_t0 = true;
    }
  }
  if (t_out) {
    if ((st = check_bad(c)) != FCS_OK) return st;
    // time after the completed stages: end of the step at a step boundary
    const double* tp = c->dptr<double>("SCAL") + (c->stage_in_step == 0 ? 4 : 0);
    HIPCHK(c, hipMemcpyAsync(&c->t_host, tp, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *t_out = c->t_host;
  }
  return FCS_OK;
}

extern "C" fcs_status fcs_get_field(fcs_ctx* c, int32_t patch, int32_t field, double* dst, int32_t dst_on_device) {
  if (!c || !dst) return FCS_EINVAL;
  if (!c->bound) return c->fail(FCS_ESTATE, "fcs_get_field before fcs_bind");
  if (patch < 0 || patch >= static_cast<int32_t>(c->grids.size())) return c->fail(FCS_EINVAL, "bad patch index");
  if (field < 0 || field > FCS_FIELD_MUHAT) return c->fail(FCS_EINVAL, "bad field");
  if (!c->visc && field >= FCS_FIELD_MU) return c->fail(FCS_EINVAL, "viscosity fields need av_mode != OFF");
  const Grid& g = c->grids[patch];
  const size_t np = g.np();
  std::vector<double> h(np, 0.0);
  if (field <= FCS_FIELD_MACH) {
    std::vector<double> e(4 * np);
    for (int q = 0; q < 4; ++q)
      HIPCHK(c, hipMemcpyAsync(e.data() + q * np, c->cur + q * c->P + g.offset, np * 8, hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double gm = c->prm.gamma;
    for (size_t k = 0; k < np; ++k) {
      if (field <= FCS_FIELD_E) {
        h[k] = e[field * np + k];
      } else if (g.mask[k]) {
        double r = e[k], mx = e[np + k], my = e[2 * np + k], E = e[3 * np + k];
        double pr = (gm - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
        h[k] = field == FCS_FIELD_P ? pr : std::sqrt(mx * mx + my * my) / r * std::sqrt(r / (gm * pr));
      }
    }
  } else if (field == FCS_FIELD_TAU0 || field == FCS_FIELD_TAU1) {
    std::vector<uint8_t> t(np);
    HIPCHK(c, hipMemcpyAsync(t.data(), c->dptr<uint8_t>("TAU") + (field - FCS_FIELD_TAU0) * c->P + g.offset, np,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < np; ++k) h[k] = t[k];
  } else {
    const double* src = field == FCS_FIELD_MU ? c->arr[A_MU] : c->dptr<double>("MUHAT");
    HIPCHK(c, hipMemcpyAsync(h.data(), src + g.offset, np * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (dst_on_device) {
    HIPCHK(c, hipMemcpyAsync(dst, h.data(), np * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::copy(h.begin(), h.end(), dst);
  }
  return FCS_OK;
}

extern "C" fcs_status fcs_autotune_times(const fcs_ctx* c, int32_t n, double* ms) {
  if (!c || !ms || n < 0 || n > 16) return FCS_EINVAL;
  for (int32_t q = 0; q < n; ++q) ms[q] = c->tune_ms[q];
  return FCS_OK;
}

extern "C" fcs_status fcs_stats(fcs_ctx* c, fcs_stats_t* out) {
  if (!c || !out) return FCS_EINVAL;
  if (!c->bound) return c->fail(FCS_ESTATE, "fcs_stats before fcs_bind");
  double scal[5];
  std::vector<double> e(4 * c->P);
  HIPCHK(c, hipMemcpyAsync(scal, c->dptr<double>("SCAL"), 40, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(e.data(), c->cur, 4 * c->P * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->steps = c->steps;
  out->stages = c->stages;
  out->t = c->stage_in_step == 0 ? scal[4] : scal[0];
  out->dt = scal[2];
  out->mass = out->energy = 0;
  for (int64_t k = 0; k < c->P; ++k)
    if (c->flags[k] & kActive) {
      out->mass += e[k];
      out->energy += e[3 * c->P + k];
    }
  out->npoints = c->nactive;
  out->stage_variant = c->stage_variant;
  out->reserved = 0;
  return check_bad(c);
}

extern "C" fcs_status fcs_profile_stage(fcs_ctx* c, int32_t reps, double* avg_ms, double* flops, double* bytes) {
  if (!c || reps <= 0 || !avg_ms) return FCS_EINVAL;
  if (!c->bound || !c->tuned) return c->fail(FCS_ESTATE, "fcs_profile_stage before the first advance");
  fcs_status st;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  // one launch to warm up, then reps back to back between two events
  if ((st = run_gemm(c, PH_EULER, 0, c->prm.precision, false)) != FCS_OK) return st;
  HIPCHK(c, hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r)
    if ((st = run_gemm(c, PH_EULER, 0, c->prm.precision, false)) != FCS_OK) return st;
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_ms = ms / reps;
  double f = 0, b = 0;
  if ((st = stage_work(c, &f, &b)) != FCS_OK) return st;
  if (flops) *flops = f;
  if (bytes) *bytes = b;
  return FCS_OK;
}

extern "C" fcs_status fcs_set_stage_variant(fcs_ctx* c, int32_t index) {
  if (!c) return FCS_EINVAL;
  if (!c->bound) return c->fail(FCS_ESTATE, "fcs_set_stage_variant before fcs_bind");
  int nv = 0;
  const GemmVariant* cand = gemm_variants(c->prm.precision, &nv);
  if (index < 0 || index >= nv) return c->fail(FCS_EINVAL, "stage variant index out of range");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto* g : {c->gexec, c->pgexec})
    for (int k = 0; k < 2; ++k)
      if (g[k]) {
        HIPCHK(c, hipGraphExecDestroy(g[k]));
        g[k] = nullptr;
      }
  for (int ph : {PH_EULER, PH_CROSS, PH_EULER0}) {
    c->var[ph] = cand[index];
    build_tiles(c, ph);
    if (c->phase_tiles[ph].empty()) continue;
    if (c->phase_tiles[ph].size() > c->tile_cap[ph]) return c->fail(FCS_EINVAL, "tile list exceeds its capacity");
    std::string name = "TILE" + std::to_string(ph);
    fcs_status st = upload(c, name.c_str(), c->phase_tiles[ph].data(), c->phase_tiles[ph].size() * sizeof(GemmTile));
    if (st != FCS_OK) return st;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->stage_variant = index;
  c->tuned = true;
  return FCS_OK;
}

extern "C" fcs_status fcs_retune(fcs_ctx* c) {
  if (!c) return FCS_EINVAL;
  if (!c->bound) return c->fail(FCS_ESTATE, "fcs_retune before fcs_bind");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto* g : {c->gexec, c->pgexec})
    for (int k = 0; k < 2; ++k)
      if (g[k]) {
        HIPCHK(c, hipGraphExecDestroy(g[k]));
        g[k] = nullptr;
      }
  c->tuned = false;
  return FCS_OK;
}

extern "C" fcs_status fcs_profile_enable(fcs_ctx* c, int32_t on) {
  if (!c) return FCS_EINVAL;
  if (on && c->ev.empty()) {
    c->ev.resize(8192);
    for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
  }
  c->prof = on != 0;
  c->ev_used = 0;
  c->prof_ms = 0;
  c->prof_n = 0;
  c->prof_ovh_ms = 0;
  c->prof_ovh_n = 0;
  c->prof_flops = 0;
  c->prof_bytes = 0;
  c->prof_fn = 0;
  return FCS_OK;
}

extern "C" fcs_status fcs_profile_read(fcs_ctx* c, double* avg_ms, double* flops, double* bytes, int64_t* launches,
                                       double* event_latency_ms) {
  if (!c) return FCS_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t q = 0; q + 1 < c->ev_used; q += 2) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[q], c->ev[q + 1]));
    c->prof_ms += ms;
    c->prof_n++;
  }
  c->ev_used = 0;
  if (avg_ms) *avg_ms = c->prof_n ? c->prof_ms / c->prof_n : 0.0;
  // useful work per timed launch: the lines each step needed (all lines
  // before any profiled step)
  if (flops) *flops = c->prof_fn ? c->prof_flops / c->prof_fn : exact_flops(c->phase_tasks[PH_EULER]);
  if (bytes) {
    // algorithmic bytes: each operand line read once, each result written once
    double b = 0;
    for (const auto& t : c->phase_tasks[PH_EULER]) b += task_bytes(c, t) * static_cast<double>(t.nrow) * t.ncomp;
    *bytes = c->prof_fn ? c->prof_bytes / c->prof_fn : b;
  }
  if (launches) *launches = c->prof_n;
  if (event_latency_ms) *event_latency_ms = c->prof_ovh_n ? c->prof_ovh_ms / c->prof_ovh_n : 0.0;
  return FCS_OK;
}

extern "C" void fcs_destroy(fcs_ctx* c) {
  if (!c) return;
  for (auto& g : c->gexec)
    if (g) hipGraphExecDestroy(g);
  for (auto& g : c->pgexec)
    if (g) hipGraphExecDestroy(g);
  for (auto& row : c->pev)
    for (auto& e : row)
      if (e) hipEventDestroy(e);
  for (auto& e : c->ev) hipEventDestroy(e);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->ev_fork2) hipEventDestroy(c->ev_fork2);
  if (c->ev_join2) hipEventDestroy(c->ev_join2);
  if (c->stream2) hipStreamDestroy(c->stream2);
  delete c;
}
