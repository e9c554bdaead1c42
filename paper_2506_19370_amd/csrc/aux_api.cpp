// C ABI: FC operators on the host, the batched derivative sweep, standalone
// window classification and line-wise operator application.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/fcsdnn.h"
#include "fc_builder.h"
#include "gemm.h"
#include "kernels.h"
#include "sdnn_train.h"
#include "window_kernels.h"

using namespace fcs;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

extern "C" fcs_status fcs_fc_continuation(int32_t d, int32_t C, double* Q, double* A) {
  if (!Q || !A) return FCS_EINVAL;
  return fc_continuation(d, C, Q, A) ? FCS_OK : FCS_EINVAL;
}

extern "C" fcs_status fcs_fc_operator(int32_t n, int32_t d, int32_t C, int32_t kind, double* out) {
  if (!out || d < 1 || d > 12 || C < 4 || C > 64) return FCS_EINVAL;
  const std::vector<double>* op = fc_operator(n, d, C, kind);
  if (!op) return FCS_EINVAL;
  std::copy(op->begin(), op->end(), out);
  return FCS_OK;
}

// ------------------------------------------------------------------ sweep
struct fcs_sweep {
  int npatch = 0, ncomp = 0, precision = 0, d = 0, C = 0;
  std::vector<int32_t> n1, n2;
  std::vector<int64_t> poff;  // element offset of each patch (ncomp * n1 * n2 per patch)
  int64_t total = 0, npoints = 0;
  OpPack ops;
  std::vector<GemmTask> tasks;
  std::vector<GemmTile> tiles;
  char* ws = nullptr;
  size_t need = 0;
  size_t o_ctr = 0, o_off = 0, o_roff = 0, o_ld = 0, o_f64 = 0, o_f32 = 0, o_bhi = 0, o_blo = 0, o_bmid = 0, o_row = 0, o_task = 0, o_tile = 0;
  hipStream_t stream = nullptr;
  const double* last_in = nullptr;
  double *last_d1 = nullptr, *last_d2 = nullptr;
  OpTables tab{};
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double ms = 0;
  int64_t launches = 0;
  GemmVariant var;
  size_t tile_cap = 0;
};

namespace {
void sweep_tiles(fcs_sweep* s) {
  std::vector<int32_t> n(s->tasks.size()), nl(s->tasks.size());
  for (size_t q = 0; q < s->tasks.size(); ++q) {
    n[q] = s->tasks[q].n;
    nl[q] = s->tasks[q].nrow * s->tasks[q].ncomp;
  }
  gemm_build_tiles(s->var, n.data(), nl.data(), s->tasks.size(), s->tiles);
}
}  // namespace

extern "C" fcs_status fcs_sweep_create(int32_t npatch, const int32_t* n1n2, int32_t ncomp, int32_t precision,
                                       int32_t d, int32_t C, fcs_sweep** out) {
  if (!out || !n1n2 || npatch <= 0 || ncomp <= 0 || ncomp > 64 || precision < 0 || precision > 3) return FCS_EINVAL;
  if (d < 1 || d > 12 || C < 4 || C > 64) return FCS_EINVAL;
  std::unique_ptr<fcs_sweep> s(new (std::nothrow) fcs_sweep());
  if (!s) return FCS_ENOMEM;
  s->npatch = npatch;
  s->ncomp = ncomp;
  s->precision = precision;
  s->d = d;
  s->C = C;
  for (int p = 0; p < npatch; ++p) {
    int a = n1n2[2 * p], b = n1n2[2 * p + 1];
    if (a < 2 * d || b < 2 * d || a > 1024 || b > 1024) return FCS_EINVAL;
    s->n1.push_back(a);
    s->n2.push_back(b);
    s->poff.push_back(s->total);
    s->total += static_cast<int64_t>(ncomp) * a * b;
    s->npoints += static_cast<int64_t>(a) * b;
    s->ops.add(a, FCS_OP_D1);
    s->ops.add(b, FCS_OP_D1);
  }
  // tasks: per patch, q^1 (all rows of all components) and q^2; the
  // component stride is one (n2, n1) block
  for (int p = 0; p < npatch; ++p) {
    int a = s->n1[p], b = s->n2[p];
    GemmTask t{};
    t.comp_stride = static_cast<int64_t>(a) * b;
    t.ncomp = ncomp;
    // q^1 lines: row r of component c
    t.row_stride = a;
    t.s_stride = 1;
    t.nrow = b;
    t.n = a;
    t.op = s->ops.add(a, FCS_OP_D1);
    t.src = reinterpret_cast<const double*>(static_cast<intptr_t>(s->poff[p]));  // offsets; rebased at run
    t.dst = reinterpret_cast<double*>(static_cast<intptr_t>(s->poff[p]));
    s->tasks.push_back(t);
    t.row_stride = 1;
    t.s_stride = a;
    t.nrow = a;
    t.n = b;
    t.op = s->ops.add(b, FCS_OP_D1);
    s->tasks.push_back(t);
  }
  // room for the tile list of every candidate shape
  {
    int nv = 0;
    const GemmVariant* cand = gemm_variants(precision, &nv);
    for (int q = 0; q < nv; ++q) {
      s->var = cand[q];
      sweep_tiles(s.get());
      s->tile_cap = std::max(s->tile_cap, s->tiles.size());
    }
    s->var = GemmVariant{};
  }
  sweep_tiles(s.get());
  s->tile_cap = std::max(s->tile_cap, s->tiles.size());
  size_t u = 0;
  auto take = [&](size_t b) {
    size_t o = u;
    u = align_up(u + std::max<size_t>(b, 1));
    return o;
  };
  s->o_ctr = take(kGemmCounters * 4);
  s->o_off = take(s->ops.off.size() * 8);
  s->o_roff = take(s->ops.roff.size() * 8);
  s->o_ld = take(s->ops.ld.size() * 4);
  s->o_f64 = take(s->ops.elems * 8);
  s->o_row = take(s->ops.rows * 8);
  s->o_f32 = take(precision == 1 ? s->ops.elems * 4 : 0);
  s->o_bhi = take(precision >= 2 ? s->ops.elems * 2 : 0);
  s->o_blo = take(precision >= 2 ? s->ops.elems * 2 : 0);
  s->o_bmid = take(precision == 3 ? s->ops.elems * 2 : 0);
  s->o_task = take(s->tasks.size() * sizeof(GemmTask));
  s->o_tile = take(s->tiles.size() * sizeof(GemmTile));
  s->need = u;
  *out = s.release();
  return FCS_OK;
}

extern "C" fcs_status fcs_sweep_workspace_size(const fcs_sweep* s, size_t* bytes) {
  if (!s || !bytes) return FCS_EINVAL;
  *bytes = s->need;
  return FCS_OK;
}

extern "C" fcs_status fcs_sweep_points(const fcs_sweep* s, int64_t* npoints) {
  if (!s || !npoints) return FCS_EINVAL;
  *npoints = s->npoints;
  return FCS_OK;
}

extern "C" fcs_status fcs_sweep_bind(fcs_sweep* s, void* workspace, size_t bytes, void* stream) {
  if (!s || !workspace || bytes < s->need || reinterpret_cast<uintptr_t>(workspace) % kAlign) return FCS_EINVAL;
  s->ws = static_cast<char*>(workspace);
  s->stream = static_cast<hipStream_t>(stream);
  std::vector<double> f64, rows;
  if (!s->ops.fill(s->d, s->C, f64, rows)) return FCS_EINVAL;
  std::vector<float> f32;
  std::vector<uint16_t> bhi, blo, bmid;
  hipStream_t st = s->stream;
  // tile counters of the persistent variants start at zero
  if (hipMemsetAsync(s->ws + s->o_ctr, 0, kGemmCounters * 4, st)) return FCS_EHIP;
  if (hipMemcpyAsync(s->ws + s->o_off, s->ops.off.data(), s->ops.off.size() * 8, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s->ws + s->o_roff, s->ops.roff.data(), s->ops.roff.size() * 8, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s->ws + s->o_ld, s->ops.ld.data(), s->ops.ld.size() * 4, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s->ws + s->o_f64, f64.data(), f64.size() * 8, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(s->ws + s->o_row, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, st))
    return FCS_EHIP;
  if (s->precision == 1) {
    f32.assign(f64.begin(), f64.end());
    if (hipMemcpyAsync(s->ws + s->o_f32, f32.data(), f32.size() * 4, hipMemcpyHostToDevice, st)) return FCS_EHIP;
  }
  if (s->precision >= 2) {
    if (s->precision == 3)
      split_bf16x3(f64, bhi, bmid, blo);
    else
      split_bf16(f64, bhi, blo);
    if (hipMemcpyAsync(s->ws + s->o_bhi, bhi.data(), bhi.size() * 2, hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(s->ws + s->o_blo, blo.data(), blo.size() * 2, hipMemcpyHostToDevice, st))
      return FCS_EHIP;
    if (s->precision == 3 &&
        hipMemcpyAsync(s->ws + s->o_bmid, bmid.data(), bmid.size() * 2, hipMemcpyHostToDevice, st))
      return FCS_EHIP;
  }
  if (hipMemcpyAsync(s->ws + s->o_tile, s->tiles.data(), s->tiles.size() * sizeof(GemmTile), hipMemcpyHostToDevice,
                     st))
    return FCS_EHIP;
  if (hipStreamSynchronize(st)) return FCS_EHIP;
  s->tab.off = reinterpret_cast<const int64_t*>(s->ws + s->o_off);
  s->tab.roff = reinterpret_cast<const int64_t*>(s->ws + s->o_roff);
  s->tab.ld = reinterpret_cast<const int32_t*>(s->ws + s->o_ld);
  s->tab.f64 = reinterpret_cast<const double*>(s->ws + s->o_f64);
  s->tab.rowsum = reinterpret_cast<const double*>(s->ws + s->o_row);
  s->tab.f32 = reinterpret_cast<const float*>(s->ws + s->o_f32);
  s->tab.bhi = reinterpret_cast<const uint16_t*>(s->ws + s->o_bhi);
  s->tab.blo = reinterpret_cast<const uint16_t*>(s->ws + s->o_blo);
  s->tab.bmid = s->precision == 3 ? reinterpret_cast<const uint16_t*>(s->ws + s->o_bmid) : nullptr;
  s->last_in = nullptr;
  return FCS_OK;
}

extern "C" fcs_status fcs_sweep_run(fcs_sweep* s, const double* in, double* d1, double* d2) {
  if (!s || !in || !d1 || !d2 || !s->ws) return FCS_EINVAL;
  if (in != s->last_in || d1 != s->last_d1 || d2 != s->last_d2) {
    std::vector<GemmTask> t = s->tasks;
    for (size_t q = 0; q < t.size(); ++q) {
      int64_t o = static_cast<int64_t>(reinterpret_cast<intptr_t>(s->tasks[q].src));
      t[q].src = in + o;
      t[q].dst = (q % 2 == 0 ? d1 : d2) + o;
    }
    if (hipMemcpyAsync(s->ws + s->o_task, t.data(), t.size() * sizeof(GemmTask), hipMemcpyHostToDevice, s->stream) ||
        hipStreamSynchronize(s->stream))
      return FCS_EHIP;
    s->last_in = in;
    s->last_d1 = d1;
    s->last_d2 = d2;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s->prof && s->ev_used + 2 <= s->ev.size()) {
    e0 = s->ev[s->ev_used++];
    e1 = s->ev[s->ev_used++];
    if (hipEventRecord(e0, s->stream)) return FCS_EHIP;
  }
  if (launch_gemm(s->precision, s->var, reinterpret_cast<const GemmTask*>(s->ws + s->o_task),
                  reinterpret_cast<const GemmTile*>(s->ws + s->o_tile), static_cast<int>(s->tiles.size()), s->tab,
                  reinterpret_cast<int*>(s->ws + s->o_ctr), s->stream) != hipSuccess)
    return FCS_EHIP;
  if (e1 && hipEventRecord(e1, s->stream)) return FCS_EHIP;
  return FCS_OK;
}

extern "C" int32_t fcs_gemm_variant_count(int32_t precision) {
  if (precision < 0 || precision > 3) return 0;
  int nv = 0;
  gemm_variants(precision, &nv);
  return nv;
}

extern "C" fcs_status fcs_gemm_variant_name(int32_t precision, int32_t index, char* buf, int32_t len) {
  if (!buf || len <= 0 || precision < 0 || precision > 3) return FCS_EINVAL;
  int nv = 0;
  const GemmVariant* cand = gemm_variants(precision, &nv);
  if (index < 0 || index >= nv) return FCS_EINVAL;
  const GemmVariant& v = cand[index];
  std::string name;
  if (precision == 3) {
    name = "k_gemm_bf16x6";
  } else if (precision == 2 && v.line) {
    name = "k_gemm_bf16x3_line<" + std::to_string(v.lines) + ">";
  } else if (precision == 2 && v.xw) {
    name = "k_gemm_xw_bf16x3<128, " + std::to_string(v.tb) + ">";
  } else if (precision == 2) {
    name = std::string(v.persist ? "k_gemm_bf16x3_persist<" : "k_gemm_bf16x3<") + std::to_string(v.tb);
    if (!v.persist) name += ", " + std::to_string(v.kc) + ", " + std::to_string(v.pf);
    name += ">";
  } else if (v.xw) {
    name = std::string("k_gemm_xw<") + (precision == 0 ? "double, 64, " : "float, 128, ") + std::to_string(v.tb) +
           ">";
  } else {
    const char* kind = v.xs ? "k_gemm_xs<" : (v.persist ? "k_gemm_fp_persist<" : "k_gemm_fp<");
    name = std::string(kind) + (precision == 0 ? "double" : "float") + ", " + std::to_string(v.kc) + ", " +
           std::to_string(v.tb);
    // the staged kernel carries its workgroups per CU (launch bound)
    if (!v.xs && !v.persist) {
      name += ", " + std::to_string(v.minb) + ", " + std::to_string(v.pf);
    }
    name += ">";
  }
  if (static_cast<int32_t>(name.size()) >= len) return FCS_EINVAL;
  std::memcpy(buf, name.c_str(), name.size() + 1);
  return FCS_OK;
}

extern "C" fcs_status fcs_sweep_set_variant(fcs_sweep* s, int32_t index) {
  if (!s || !s->ws) return FCS_EINVAL;
  int nv = 0;
  const GemmVariant* cand = gemm_variants(s->precision, &nv);
  if (index < 0 || index >= nv) return FCS_EINVAL;
  const GemmVariant saved = s->var;
  s->var = cand[index];
  sweep_tiles(s);
  if (s->tiles.size() > s->tile_cap) {
    s->var = saved;
    sweep_tiles(s);
    return FCS_EINVAL;
  }
  if (hipMemcpyAsync(s->ws + s->o_tile, s->tiles.data(), s->tiles.size() * sizeof(GemmTile), hipMemcpyHostToDevice,
                     s->stream) ||
      hipStreamSynchronize(s->stream))
    return FCS_EHIP;
  return FCS_OK;
}

// Time every candidate tile shape on the given arrays and keep the fastest.
extern "C" fcs_status fcs_sweep_autotune(fcs_sweep* s, const double* in, double* d1, double* d2, double* ms_out) {
  if (!s || !s->ws) return FCS_EINVAL;
  int nv = 0;
  const GemmVariant* cand = gemm_variants(s->precision, &nv);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) || hipEventCreate(&e1)) return FCS_EHIP;
  float best = 1e30f;
  GemmVariant bestv = s->var;
  bool saved = s->prof;
  s->prof = false;
  fcs_status st = FCS_OK;
  for (int q = 0; q < nv && st == FCS_OK; ++q) {
    s->var = cand[q];
    sweep_tiles(s);
    if (s->tiles.size() > s->tile_cap) continue;
    if (hipMemcpyAsync(s->ws + s->o_tile, s->tiles.data(), s->tiles.size() * sizeof(GemmTile),
                       hipMemcpyHostToDevice, s->stream) ||
        hipStreamSynchronize(s->stream)) {
      st = FCS_EHIP;
      break;
    }
    if ((st = fcs_sweep_run(s, in, d1, d2)) != FCS_OK) break;
    hipEventRecord(e0, s->stream);
    for (int r = 0; r < 3 && st == FCS_OK; ++r) st = fcs_sweep_run(s, in, d1, d2);
    hipEventRecord(e1, s->stream);
    hipEventSynchronize(e1);
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    ms /= 3;
    if (ms_out) ms_out[q] = ms;
    if (ms < best) {
      best = ms;
      bestv = cand[q];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  s->prof = saved;
  if (st != FCS_OK) return st;
  s->var = bestv;
  sweep_tiles(s);
  if (hipMemcpyAsync(s->ws + s->o_tile, s->tiles.data(), s->tiles.size() * sizeof(GemmTile), hipMemcpyHostToDevice,
                     s->stream) ||
      hipStreamSynchronize(s->stream))
    return FCS_EHIP;
  return FCS_OK;
}

extern "C" fcs_status fcs_sweep_profile(fcs_sweep* s, int32_t on, double* avg_ms, double* flops, double* bytes,
                                        int64_t* launches) {
  if (!s) return FCS_EINVAL;
  if (hipStreamSynchronize(s->stream)) return FCS_EHIP;
  for (size_t q = 0; q + 1 < s->ev_used; q += 2) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, s->ev[q], s->ev[q + 1])) return FCS_EHIP;
    s->ms += ms;
    s->launches++;
  }
  s->ev_used = 0;
  if (avg_ms) *avg_ms = s->launches ? s->ms / s->launches : 0.0;
  if (launches) *launches = s->launches;
  double f = 0, b = 0;
  for (const auto& t : s->tasks) {
    f += 2.0 * t.n * t.n * static_cast<double>(t.nrow) * t.ncomp;
    b += 2.0 * 8.0 * t.n * static_cast<double>(t.nrow) * t.ncomp;
  }
  if (flops) *flops = f;
  if (bytes) *bytes = b;
  if (on >= 0) {
    if (on && s->ev.empty()) {
      s->ev.resize(4096);
      for (auto& e : s->ev)
        if (hipEventCreate(&e)) return FCS_EHIP;
    }
    if (on != static_cast<int>(s->prof) || on) {
      s->ms = 0;
      s->launches = 0;
    }
    s->prof = on != 0;
  }
  return FCS_OK;
}

extern "C" void fcs_sweep_destroy(fcs_sweep* s) {
  if (!s) return;
  for (auto& e : s->ev) hipEventDestroy(e);
  delete s;
}

// ------------------------------------------------------------------ classification
extern "C" fcs_status fcs_sdnn_infer(const float* params, const double* windows, int64_t nwin, uint8_t* tau,
                                     float* logits, void* stream) {
  if (!params || (!windows && nwin) || (!tau && nwin) || nwin < 0) return FCS_EINVAL;
  ModalBasis b{};
  return launch_classify_windows(2, params, b, windows, nwin, tau, logits, static_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? FCS_OK
             : FCS_EHIP;
}

extern "C" fcs_status fcs_modal_infer(const double* windows, int64_t nwin, uint8_t* tau, void* stream) {
  if ((!windows && nwin) || (!tau && nwin) || nwin < 0) return FCS_EINVAL;
  static ModalBasis b;
  static bool init = false;
  if (!init) {
    modal_basis16(b.v);
    init = true;
  }
  return launch_classify_windows(1, nullptr, b, windows, nwin, tau, nullptr, static_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? FCS_OK
             : FCS_EHIP;
}

// ------------------------------------------------------------------ training
extern "C" size_t fcs_sdnn_train_workspace(int32_t batch) {
  if (batch <= 0) return 0;
  return sdnn_train_floats(batch) * sizeof(float);
}

extern "C" fcs_status fcs_sdnn_train_step(float* params, float* m, float* v, int32_t t, float lr, const float* x,
                                          const int32_t* labels, const float* class_weight, int32_t batch,
                                          float* loss, float* grads, int32_t flags, void* workspace, size_t bytes,
                                          void* stream) {
  if (!params || !m || !v || !x || !labels || !class_weight || !loss || !workspace || batch <= 0 || t < 1 ||
      batch > (1 << 22))
    return FCS_EINVAL;
  if (bytes < fcs_sdnn_train_workspace(batch)) return FCS_ENOMEM;
  return launch_sdnn_train(params, m, v, t, lr, x, labels, class_weight, batch, loss, grads,
                           static_cast<float*>(workspace), flags & 1, static_cast<hipStream_t>(stream)) == hipSuccess
             ? FCS_OK
             : FCS_EHIP;
}

// ------------------------------------------------------------------ lines
extern "C" size_t fcs_lines_workspace(int32_t n, int64_t nlines) {
  if (n <= 0 || nlines <= 0) return 0;
  const int64_t ntiles = ((nlines + 63) / 64) * ((n + 63) / 64);
  return align_up(static_cast<size_t>(op_rows(n)) * op_ld(n) * 8) + align_up(64) + align_up(sizeof(GemmTask)) +
         align_up(static_cast<size_t>(ntiles) * sizeof(GemmTile));
}

extern "C" fcs_status fcs_lines_apply(int32_t n, int64_t nlines, int32_t kind, int32_t d, int32_t C,
                                      const double* in, double* out, void* workspace, size_t bytes, void* stream) {
  if (!in || !out || !workspace || nlines <= 0 || nlines > (1ll << 31) / 1024) return FCS_EINVAL;
  if (bytes < fcs_lines_workspace(n, nlines) || reinterpret_cast<uintptr_t>(workspace) % kAlign) return FCS_EINVAL;
  if (d < 1 || d > 12 || C < 4 || C > 64 || kind < FCS_OP_D1 || kind > FCS_OP_SMEAR) return FCS_EINVAL;
  OpPack pk;
  pk.add(n, kind);
  std::vector<double> f64, rows;
  if (!pk.fill(d, C, f64, rows)) return FCS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  // small tables: operator offset (8 B), row-sum offset (8 B), leading dimension (4 B)
  struct {
    int64_t off, roff;
    int32_t ld, pad;
  } small{0, 0, pk.ld[0], 0};
  const size_t o_op = 0, o_small = align_up(f64.size() * 8), o_task = o_small + align_up(64),
               o_tile = o_task + align_up(sizeof(GemmTask));
  GemmTask t{};
  t.src = in;
  t.dst = out;
  t.comp_stride = static_cast<int64_t>(nlines) * n;
  t.row_stride = n;
  t.s_stride = 1;
  t.nrow = static_cast<int32_t>(nlines);
  t.ncomp = 1;
  t.n = n;
  t.op = 0;
  std::vector<GemmTile> tiles;
  const GemmVariant v{};
  for (int t0 = 0; t0 < n; t0 += gemm_outputs_per_tile(v))
    for (int64_t l0 = 0; l0 < nlines; l0 += gemm_lines_per_tile()) tiles.push_back({0, static_cast<int32_t>(l0), t0, 0});
  if (hipMemcpyAsync(ws + o_op, f64.data(), f64.size() * 8, hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(ws + o_small, &small, sizeof(small), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(ws + o_task, &t, sizeof(t), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(ws + o_tile, tiles.data(), tiles.size() * sizeof(GemmTile), hipMemcpyHostToDevice, st))
    return FCS_EHIP;
  OpTables tab{};
  tab.off = reinterpret_cast<const int64_t*>(ws + o_small);
  tab.roff = reinterpret_cast<const int64_t*>(ws + o_small + 8);
  tab.ld = reinterpret_cast<const int32_t*>(ws + o_small + 16);
  tab.f64 = reinterpret_cast<const double*>(ws + o_op);
  if (launch_gemm(0, v, reinterpret_cast<const GemmTask*>(ws + o_task), reinterpret_cast<const GemmTile*>(ws + o_tile),
                  static_cast<int>(tiles.size()), tab, nullptr, st) != hipSuccess)
    return FCS_EHIP;
  // the host staging vectors must outlive the copies
  return hipStreamSynchronize(st) == hipSuccess ? FCS_OK : FCS_EHIP;
}
