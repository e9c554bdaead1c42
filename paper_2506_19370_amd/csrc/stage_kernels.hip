// Elementwise, stencil and gather kernels of one FC-SDNN step.
//
// Per stage (the stage algorithm of Sec. 5 and the stage loop of Alg. 1):
// fluxes of the Euler system (Sec. 2) as contraction operands, assembly of
// the spatial operator from the FC derivatives and the Jacobian of the
// inverse mapping (chain rule; viscous term mu Lap(w) + grad mu . grad w),
// the SSPRK(5,4) stage update in Shu-Osher form, boundary conditions, and the
// fringe exchange/interpolation (Sec. 3.3).  Per step: proxy variable, window
// classification, wave-speed bound and preliminary viscosity (Alg. 3), its
// smoothing and blend across subpatches (Sec. 4), the filter's variable
// change (Alg. 4; theta = p / ((gamma - 1) rho)) and the adaptive step.
#include "stage_kernels.h"

#include "classify.h"

#include <cmath>

namespace fcs {

namespace {

__device__ __forceinline__ double pressure(double r, double mx, double my, double E, double gm1) {
  return gm1 * (E - 0.5 * (mx * mx + my * my) / r);
}

// Euler fluxes of one state as the 8 operand components of the stage
// contraction: contravariant q^k_x f_x + q^k_y f_y on affine subpatches,
// f_x and f_y otherwise; zero at inactive points.
__device__ __forceinline__ void flux_of(const FluxOut& fo, int64_t k, uint8_t f, double r, double mx, double my,
                                        double E, double (&v)[8]) {
  for (int q = 0; q < 8; ++q) v[q] = 0.0;
  if (f & kActive) {
    const double p = pressure(r, mx, my, E, fo.gm1);
    const double u = mx / r, w = my / r;
    const double fx[4] = {mx, mx * u + p, mx * w, u * (E + p)};
    const double fy[4] = {my, my * u, my * w + p, w * (E + p)};
    if (f & kAffine) {
      const PatchDev& pd = fo.patches[fo.pid[k]];
      const double a = pd.t1x, b = pd.t1y, c = pd.t2x, d = pd.t2y;
      for (int q = 0; q < 4; ++q) {
        v[q] = a * fx[q] + b * fy[q];
        v[4 + q] = c * fx[q] + d * fy[q];
      }
    } else {
      for (int q = 0; q < 4; ++q) {
        v[q] = fx[q];
        v[4 + q] = fy[q];
      }
    }
  }
}
__device__ __forceinline__ void store_flux(const FluxOut& fo, int64_t P, int64_t k, uint8_t f, double r, double mx,
                                           double my, double E) {
  double v[8];
  flux_of(fo, k, f, r, mx, my, E, v);
  for (int q = 0; q < 8; ++q) fo.F[q * P + k] = v[q];
}

// Mach-number proxy and wave speed |u| + a of one state (the inputs of the
// smoothness classifier and of the preliminary viscosity, Alg. 3).
__device__ __forceinline__ double2 proxy_speed(double r, double mx, double my, double E, double gamma) {
  const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
  const double speed = sqrt(mx * mx + my * my) / r;
  return double2{speed * sqrt(r / (gamma * p)), speed + sqrt(gamma * p / r)};
}

__global__ void k_flux(const double* __restrict__ U, const uint8_t* __restrict__ flags, FluxOut fo, int64_t P) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  store_flux(fo, P, k, flags[k], U[k], U[P + k], U[2 * P + k], U[3 * P + k]);
}

// Boundary conditions of one point (Sec. 5 item 4): slip (normal momentum
// removed, pressure kept; zero momentum at a corner of two slip sides), then
// Dirichlet data (fixed state, or the isentropic vortex at t).
__device__ __forceinline__ void apply_bc(const BcEntry& b, double gamma, double t, const VortexArgs& v, double& r,
                                         double& mx, double& my, double& E) {
  const double gm1 = gamma - 1.0;
  if (b.slip) {
    const double p = gm1 * (E - 0.5 * (mx * mx + my * my) / r);
    if (b.slip == 2) {
      mx = 0.0;
      my = 0.0;
    } else {
      const double mn = mx * b.nx + my * b.ny;
      mx = mx - mn * b.nx;
      my = my - mn * b.ny;
    }
    E = p / gm1 + 0.5 * (mx * mx + my * my) / r;
  }
  if (b.dirichlet == 1) {
    r = b.e[0];
    mx = b.e[1];
    my = b.e[2];
    E = b.e[3];
  } else if (b.dirichlet == 2) {
    const double pi = 3.141592653589793;
    const double dx = b.x - v.x0 - v.u0 * t, dy = b.y - v.y0 - v.v0 * t;
    const double r2 = dx * dx + dy * dy;
    const double g = exp(0.5 * (1.0 - r2));
    const double du = -v.beta / (2 * pi) * g * dy, dv = v.beta / (2 * pi) * g * dx;
    const double T = 1.0 - (gamma - 1.0) * v.beta * v.beta / (8 * gamma * pi * pi) * exp(1.0 - r2);
    const double rho = pow(T, 1.0 / (gamma - 1.0));
    const double p = pow(rho, gamma);
    const double u = v.u0 + du, w = v.v0 + dv;
    r = rho;
    mx = rho * u;
    my = rho * w;
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + w * w);
  }
}

// Boundary conditions of every boundary point, in place (the initial data
// made to satisfy them before the first step; the stages apply them in
// k_stage).
__global__ void k_bc_state(double* __restrict__ U, const uint8_t* __restrict__ flags, BcArgs b, double t, int64_t P) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  if (!(flags[k] & kActive) || !(flags[k] & kBoundary)) return;
  double r = U[k], mx = U[P + k], my = U[2 * P + k], E = U[3 * P + k];
  apply_bc(b.bc[b.bcidx[k]], b.gamma, t, b.vortex, r, mx, my, E);
  U[k] = r;
  U[P + k] = mx;
  U[2 * P + k] = my;
  U[3 * P + k] = E;
}

// No-slip adiabatic walls, part 1: per line, the wall values of theta that
// make the FC first derivative along the line vanish at its wall nodes (one
// node: one equation; two: the 2 x 2 system), from the state before any
// wall correction.
__global__ void k_wall_theta(const double* __restrict__ U, const WallLine* __restrict__ lines, int nlines,
                             OpTables ops, double* __restrict__ wth, int64_t P, double gm1) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlines) return;
  const WallLine w = lines[l];
  const double* D = ops.f64 + ops.off[w.op];
  const int ld = ops.ld[w.op];
  const int p0 = w.pos[0], p1 = w.pos[1];
  double r0 = 0.0, r1 = 0.0;
  for (int s = 0; s < w.n; ++s) {
    if (s == p0 || s == p1) continue;
    const int64_t k = w.first + static_cast<int64_t>(s) * w.stride;
    const double r = U[k], mx = U[P + k], my = U[2 * P + k], E = U[3 * P + k];
    const double th = (E - 0.5 * (mx * mx + my * my) / r) / r;  // p / ((gamma - 1) rho)
    r0 -= D[static_cast<int64_t>(p0) * ld + s] * th;
    if (p1 >= 0) r1 -= D[static_cast<int64_t>(p1) * ld + s] * th;
  }
  if (p1 < 0) {
    wth[2 * l] = r0 / D[static_cast<int64_t>(p0) * ld + p0];
    wth[2 * l + 1] = 0.0;
  } else {
    const double a = D[static_cast<int64_t>(p0) * ld + p0], b = D[static_cast<int64_t>(p0) * ld + p1];
    const double c = D[static_cast<int64_t>(p1) * ld + p0], d = D[static_cast<int64_t>(p1) * ld + p1];
    const double det = a * d - b * c;
    wth[2 * l] = (d * r0 - b * r1) / det;
    wth[2 * l + 1] = (a * r1 - c * r0) / det;
  }
  (void)gm1;
}

// Part 2: zero momentum, rho kept, E = rho theta at every wall node; the
// fluxes and proxy values of the corrected points when requested.
__global__ void k_wall_apply(double* __restrict__ U, const WallLine* __restrict__ lines, int nlines,
                             const double* __restrict__ wth, const uint8_t* __restrict__ flags, int64_t P,
                             double gamma, FluxOut fo, double2* __restrict__ ps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * nlines) return;
  const WallLine w = lines[q >> 1];
  const int pos = w.pos[q & 1];
  if (pos < 0 || w.keep[q & 1]) return;
  const int64_t k = w.first + static_cast<int64_t>(pos) * w.stride;
  const double r = U[k], E = r * wth[q];
  U[P + k] = 0.0;
  U[2 * P + k] = 0.0;
  U[3 * P + k] = E;
  if (fo.F) store_flux(fo, P, k, flags[k], r, 0.0, 0.0, E);
  if (ps) ps[k] = proxy_speed(r, 0.0, 0.0, E, gamma);
}

// Fluxes of one point as store_flux, with the contravariant metric terms of
// its subpatch (used on affine subpatches) already loaded.
__device__ __forceinline__ void store_flux_m(const FluxOut& fo, int64_t P, int64_t k, uint8_t f, double r, double mx,
                                             double my, double E, const double (&m)[4]) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (f & kActive) {
    const double p = pressure(r, mx, my, E, fo.gm1);
    const double u = mx / r, w = my / r;
    const double fx[4] = {mx, mx * u + p, mx * w, u * (E + p)};
    const double fy[4] = {my, my * u, my * w + p, w * (E + p)};
    if (f & kAffine) {
      for (int q = 0; q < 4; ++q) {
        v[q] = m[0] * fx[q] + m[1] * fy[q];
        v[4 + q] = m[2] * fx[q] + m[3] * fy[q];
      }
    } else {
      for (int q = 0; q < 4; ++q) {
        v[q] = fx[q];
        v[4 + q] = fy[q];
      }
    }
  }
  for (int q = 0; q < 8; ++q) fo.F[q * P + k] = v[q];
}

// DT: element type of the stage derivatives (double, or float in the mixed
// forms, where the contractions themselves are FP32 or split BF16).
// S: the stage (0..4), so that each instantiation reads only the registers
// its combination uses.  W1T: element type of the viscous first derivative
// along q^1 (FP64 in the mixed forms when it feeds the mixed-derivative
// contraction).
//
// A stage update is a stream of independent per-point loads, so the kernel
// issues them in as few dependent rounds as the data allows: (1) the
// point's flag, copy donor and subpatch; (2) everything the update reads at
// the donor (the donor's own flag first where it is another point): stage
// derivatives, mu and its derivatives, the stage input, U0 and the
// accumulator, the subpatch's flux metrics; (3) only where mu or one of its
// derivatives is nonzero, the viscous derivatives and metric terms.  No
// loaded value is consumed inside a branch of its round, and inactive
// points take the same path, storing zeros at the end.
template <typename DT, int S, typename W1T>
__global__ __launch_bounds__(256) void k_stage(StageArgs a) {
  const DT* DF1 = static_cast<const DT*>(a.DF1);
  const DT* DF2 = static_cast<const DT*>(a.DF2);
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t P = a.P;
  if (k >= P) return;
  // round 1
  const uint8_t fk = a.flags[k];
  // A fringe point filled by a copy (its donor on a common lattice, never a
  // recipient itself) takes its donor's update here instead of in the fringe
  // kernel: the donor's inputs, this point's outputs and fluxes.  It keeps
  // its own accumulator slot, which holds the same values as the donor's
  // (both are formed from equal inputs), so the read-modify-write of the
  // fourth stage does not race with the donor's thread.
  // (without copy points the donor load re-reads the subpatch index: no
  // branch, so no wait before the next round)
  const int32_t ck = (a.csrc ? a.csrc : a.pid)[k];
  const int32_t pk = a.pid[k];
  const int64_t ks = a.csrc ? ck : k;
  const double dt = *a.dt;
  const bool act = fk & kActive;
  // the donor's flag and subpatch (copy points only: one more round there)
  uint8_t f = fk;
  int32_t pks = pk;
  if (ks != k) {
    f = a.flags[ks];
    pks = a.pid[ks];
  }
  const bool aff = f & kAffine;

  // round 2.  Stage derivatives: affine subpatches need d1 G^1 and d2 G^2
  // only; the other subpatches also d1 G^2, d2 G^1 and the metric terms,
  // whose loads read the affine entries' addresses (or entry 0) on affine
  // points, so that they fetch nothing more from memory there.
  DT d1a[4], d1b[4], d2a[4], d2b[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    d1a[q] = DF1[q * P + ks];
    d2b[q] = DF2[(4 + q) * P + ks];
    d1b[q] = DF1[(aff ? q : 4 + q) * P + ks];
    d2a[q] = DF2[(aff ? 4 + q : q) * P + ks];
  }
  const int64_t km = aff ? 0 : ks;
  const double t1x = a.t1x[km], t1y = a.t1y[km], t2x = a.t2x[km], t2y = a.t2y[km];
  double mu = 0.0, mu1 = 0.0, mu2 = 0.0;
  if (a.visc) {
    mu = a.mu[ks];
    mu1 = a.mu1[ks];
    mu2 = a.mu2[ks];
  }
  double in[4], u0[4], ac[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    in[q] = a.in[q * P + ks];
    if constexpr (S >= 1 && S <= 3) u0[q] = a.U0[q * P + ks];
    if constexpr (S >= 3) ac[q] = a.acc[q * P + k];
  }
  double fm[4] = {0.0, 0.0, 0.0, 0.0};
  if (a.flux.F) {
    const PatchDev* pd = a.patches + pk;
    fm[0] = pd->t1x;
    fm[1] = pd->t1y;
    fm[2] = pd->t2x;
    fm[3] = pd->t2y;
  }

  double L[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double e1 = -(static_cast<double>(d1a[q]) + static_cast<double>(d2b[q]));
    const double e2 = -(t1x * static_cast<double>(d1a[q]) + t1y * static_cast<double>(d1b[q]) +
                        t2x * static_cast<double>(d2a[q]) + t2y * static_cast<double>(d2b[q]));
    L[q] = aff ? e1 : e2;
  }
  // round 3.  Where mu and both of its derivatives vanish the viscous term
  // is an exact zero: the derivatives of w there are not read (on skipped
  // lines they may be those of an earlier step).
  if (mu != 0.0 || mu1 != 0.0 || mu2 != 0.0) {
    const PatchDev* pd = a.patches + pks;
    // constant metrics on affine subpatches, whose index coordinates are
    // harmonic (no Laplacian terms)
    const double pg11 = pd->g11, pg12 = pd->g12, pg22 = pd->g22;
    const double cg11 = a.g11[km], cg12 = a.g12[km], cg22 = a.g22[km], cl1 = a.lap1[km], cl2 = a.lap2[km];
    const W1T* W1 = static_cast<const W1T*>(a.W1);
    const DT *W2 = static_cast<const DT*>(a.W2), *W11 = static_cast<const DT*>(a.W11),
             *W22 = static_cast<const DT*>(a.W22);
    // without the mixed-derivative array the load re-reads W2's entry and
    // the term is zero
    const bool has12 = a.W12 != nullptr;
    const DT* W12 = has12 ? static_cast<const DT*>(a.W12) : W2;
    double w1[4], w2[4], w11[4], w22[4], w12[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      w1[q] = W1[q * P + ks];
      w2[q] = W2[q * P + ks];
      w11[q] = W11[q * P + ks];
      w22[q] = W22[q * P + ks];
      w12[q] = W12[q * P + ks];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) w12[q] = has12 ? w12[q] : 0.0;
    const double g11 = aff ? pg11 : cg11, g12 = aff ? pg12 : cg12, g22 = aff ? pg22 : cg22;
    const double l1 = aff ? 0.0 : cl1, l2 = aff ? 0.0 : cl2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double lap = g11 * w11[q] + 2.0 * g12 * w12[q] + g22 * w22[q] + l1 * w1[q] + l2 * w2[q];
      double grad = g11 * mu1 * w1[q] + g12 * (mu1 * w2[q] + mu2 * w1[q]) + g22 * mu2 * w2[q];
      L[q] = L[q] + mu * lap + grad;
    }
  }
  double o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (S == 0) {
      o[q] = in[q] + a.c[0] * dt * L[q];  // the input of the first stage is U0
    } else if constexpr (S == 1) {
      o[q] = a.c[1] * u0[q] + a.c[2] * in[q] + a.c[3] * dt * L[q];
    } else if constexpr (S == 2) {
      if (act) a.acc[q * P + k] = a.c[4] * in[q];
      o[q] = a.c[1] * u0[q] + a.c[2] * in[q] + a.c[3] * dt * L[q];
    } else if constexpr (S == 3) {
      if (act) a.acc[q * P + k] = ac[q] + a.c[4] * in[q] + a.c[5] * dt * L[q];
      o[q] = a.c[1] * u0[q] + a.c[2] * in[q] + a.c[3] * dt * L[q];
    } else {
      o[q] = ac[q] + a.c[4] * in[q] + a.c[5] * dt * L[q];
    }
  }
  if (act) {
    bool bad = false;
    for (int q = 0; q < 4; ++q)
      if (!isfinite(o[q])) bad = true;
    if (!bad) {
      const double p = pressure(o[0], o[1], o[2], o[3], a.gm1);
      bad = !(o[0] > 0.0) || !(p > 0.0);
    }
    if (bad) *a.bad_flag = 1;
    if (f & kBoundary) {
      const double t = *a.bcs.t + a.bcs.frac * dt;
      apply_bc(a.bcs.bc[a.bcs.bcidx[ks]], a.bcs.gamma, t, a.bcs.vortex, o[0], o[1], o[2], o[3]);
    }
  } else {
    for (int q = 0; q < 4; ++q) o[q] = 0.0;
  }
  for (int q = 0; q < 4; ++q) a.out[q * P + k] = o[q];
  if (a.flux.F) store_flux_m(a.flux, P, k, fk, o[0], o[1], o[2], o[3], fm);
  // the last stage also evaluates the next step's proxy (Alg. 3 input)
  if (a.ps) a.ps[k] = act ? proxy_speed(o[0], o[1], o[2], o[3], a.bcs.gamma) : double2{0.0, 0.0};
}

// Fringe fill (Sec. 3.3): rows 0 .. ncopy-1 copy one donor value (common
// lattice), the rest evaluate an interpolation row; donors are never
// recipients, so all rows are independent.  The fluxes of each filled point
// follow when fo.F is set.  Four lanes share a row: lane j of the four
// accumulates the row's entries j, j + 4, ... (consecutive lanes read
// consecutive entries), a butterfly over the four gives each of them the
// same sums, and lane j stores field j and flux components j and j + 4.
constexpr int kFringeLanes = 4;
__global__ void k_fringe(double* __restrict__ U, const uint8_t* __restrict__ flags, const int64_t* __restrict__ pairs,
                         int ncopy, const int64_t* __restrict__ dst, const int32_t* __restrict__ ptr,
                         const int64_t* __restrict__ col, const double* __restrict__ val, int ninterp, int64_t P,
                         FluxOut fo, double2* __restrict__ ps, double gamma) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int q = static_cast<int>(g / kFringeLanes);
  const int j = static_cast<int>(g % kFringeLanes);
  // rows are whole groups of four lanes, so a group is in or out together
  if (q >= ncopy + ninterp) return;
  double s[4] = {0, 0, 0, 0};
  int64_t k;
  if (q < ncopy) {
    k = pairs[2 * q];
    const int64_t src = pairs[2 * q + 1];
    if (j == 0)
      for (int m = 0; m < 4; ++m) s[m] = U[m * P + src];
  } else {
    q -= ncopy;
    k = dst[q];
    for (int e = ptr[q] + j; e < ptr[q + 1]; e += kFringeLanes) {
      const double w = val[e];
      const int64_t c = col[e];
      for (int m = 0; m < 4; ++m) s[m] += w * U[m * P + c];
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    s[m] += __shfl_xor(s[m], 1);
    s[m] += __shfl_xor(s[m], 2);
  }
  U[j * P + k] = s[j];
  if (fo.F) {
    double v[8];
    flux_of(fo, k, flags[k], s[0], s[1], s[2], s[3], v);
    fo.F[j * P + k] = v[j];
    fo.F[(4 + j) * P + k] = v[4 + j];
  }
  if (ps && j == 0) ps[k] = proxy_speed(s[0], s[1], s[2], s[3], gamma);
}

// Proxy (Mach number) and |u| + a at every point.
__global__ void k_proxy(const double* __restrict__ U, const uint8_t* __restrict__ flags, double2* __restrict__ ps,
                        int64_t P, double gamma) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  if (!(flags[k] & kActive)) {
    ps[k] = double2{0.0, 0.0};
    return;
  }
  ps[k] = proxy_speed(U[k], U[P + k], U[2 * P + k], U[3 * P + k], gamma);
}

// Window geometry of point k along direction dir: start index of the
// 16-point window (shifted to stay inside the run) as element base and
// stride; false when the point is inactive or its run is shorter than 16.
__device__ __forceinline__ bool window_at(const ClassifyArgs& a, int64_t k, uint8_t f, int dir, int64_t& base,
                                          int64_t& stride) {
  if (!(f & kActive)) return false;
  const PatchDev pd = a.patches[a.pid[k]];
  const int32_t ij = a.ij[k];
  const int j = ij >> 16, i = ij & 0xFFFF;
  const int2 run = dir == 0 ? a.rowrun[pd.row_run + j] : a.colrun[pd.col_run + i];
  if (run.y < 16) return false;
  const int pos = dir == 0 ? i : j;
  const int ws = min(max(pos - 8, run.x), run.x + run.y - 16);
  base = dir == 0 ? (pd.offset + static_cast<int64_t>(j) * pd.n1 + ws) : (pd.offset + static_cast<int64_t>(ws) * pd.n1 + i);
  stride = dir == 0 ? 1 : pd.n1;
  return true;
}

__device__ __forceinline__ double muhat_of(const ClassifyArgs& a, int64_t k, uint8_t f, int t0, int t1, double smax) {
  const double alpha[3] = {0.0, 0.5, 1.0};
  const double al = fmax(alpha[t0], alpha[t1]);
  const bool keep = (f & kActive) && !(f & (kFringe | kXFringe));
  return keep ? a.c_mu * a.hx[k] * smax * al : 0.0;
}

// Alg. 3 with the modal fallback (mode 1) or frozen classes (mode 3): one
// point per thread.
__global__ __launch_bounds__(256) void k_classify(ClassifyArgs a) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= a.P) return;
  const uint8_t f = a.flags[k];
  int tau[2] = {0, 0};
  double smax = 0.0;
  double v[16];
  for (int dir = 0; dir < 2; ++dir) {
    int64_t base, stride;
    if (!window_at(a, k, f, dir, base, stride)) continue;
    for (int m = 0; m < 16; ++m) smax = fmax(smax, a.ps[base + m * stride].y);
    if (a.mode == 3) {
      tau[dir] = a.tau[dir * a.P + k];
    } else {
      for (int m = 0; m < 16; ++m) v[m] = a.ps[base + m * stride].x;
      tau[dir] = classify_modal(v, a.basis);
    }
  }
  if (a.mode != 3) {
    a.tau[k] = static_cast<uint8_t>(tau[0]);
    a.tau[a.P + k] = static_cast<uint8_t>(tau[1]);
  }
  a.muhat[k] = muhat_of(a, k, f, tau[0], tau[1], smax);
}

// Window geometry of every point in both directions (window_at), stored
// as (start, stride) pairs with start -1 where the point has no window.
__global__ void k_window_geo(ClassifyArgs a, int4* __restrict__ out) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= a.P) return;
  const uint8_t f = a.flags[k];
  int4 g{-1, 0, -1, 0};
  int64_t base, stride;
  if (window_at(a, k, f, 0, base, stride)) {
    g.x = static_cast<int>(base);
    g.y = static_cast<int>(stride);
  }
  if (window_at(a, k, f, 1, base, stride)) {
    g.z = static_cast<int>(base);
    g.w = static_cast<int>(stride);
  }
  out[k] = g;
}

// Alg. 3 with the SDNN: each wave classifies the two windows of 64 points
// in 8 rounds of 16 windows on the matrix cores (see sdnn_mfma).  Per
// direction, lane l first gathers the whole window of point l of the chunk
// (16 independent loads in flight, coalesced across the lanes: neighbouring
// points' windows are neighbouring addresses) into its row of an LDS block,
// keeping the window's largest wave speed; round pg then hands window
// 16 pg + c to lanes c, c + 16, c + 32, c + 48, four values each, read from
// LDS.  Lane l writes the classes and the preliminary viscosity of its point.
//
// Persistent: the grid holds a fixed number of waves (a multiple of the 8
// XCDs), each loads its weight fragments once and walks chunks of 64
// points.  Workgroup b runs on XCD b % 8 and takes the chunks of the XCD's
// contiguous share, so the grid rows that the column windows of
// neighbouring chunks share stay in one XCD's L2.
constexpr int kClassifyBlocks = 768;  // 3 workgroups of 4 waves per CU (occupancy 3)
constexpr int kWinPitch = 18;         // doubles per LDS window row (16 + 2: bank spread)

__global__ __launch_bounds__(256) void k_classify_sdnn(ClassifyArgs a) {
  __shared__ __attribute__((aligned(16))) double win[4][64 * kWinPitch];
  SdnnFrag F;
  load_sdnn_frag(a.sdnn_table, F);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  double* W = win[threadIdx.x >> 6];
  const int64_t nchunk = (a.P + 63) / 64;
  const int xcd = static_cast<int>(blockIdx.x & 7);
  const int64_t per_xcd = static_cast<int64_t>(gridDim.x >> 3) * 4;  // waves per XCD
  const int64_t share = (nchunk + 7) / 8;
  const int64_t c_end = min(nchunk, share * (xcd + 1));
#pragma unroll 1
  for (int64_t ch = share * xcd + static_cast<int64_t>(blockIdx.x >> 3) * 4 + (threadIdx.x >> 6); ch < c_end;
       ch += per_xcd) {
    const int64_t kl = ch * 64 + lane;  // this lane's point
    const bool in = kl < a.P;
    const uint8_t fl = in ? a.flags[kl] : 0;
    const int4 geo = in ? a.wgeo[kl] : int4{-1, 0, -1, 0};
    int tau_own[2] = {0, 0};
    double smax = 0.0;
#pragma unroll 1
    for (int dir = 0; dir < 2; ++dir) {
      const int base = dir == 0 ? geo.x : geo.z, stride = dir == 0 ? geo.y : geo.w;
      const bool valid = base >= 0;
      // gather this lane's window: 16 loads in flight (a lane without a
      // window reads point 0 and stores zeros), proxy values to LDS, the
      // largest wave speed kept, and whether the window is flat (the test of
      // sdnn_features on the same values: a round of 16 flat windows gives
      // class 0 without the network)
      const double2* __restrict__ src = a.ps + (valid ? static_cast<int64_t>(base) : 0);
      const int64_t st = valid ? stride : 0;
      double sp = 0.0, lo = 0.0, hi = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double2 q[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) q[m] = src[(8 * h + m) * st];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          if (!valid) q[m] = double2{0.0, 0.0};
          lo = (h == 0 && m == 0) ? q[m].x : fmin(lo, q[m].x);
          hi = (h == 0 && m == 0) ? q[m].x : fmax(hi, q[m].x);
          sp = fmax(sp, q[m].y);
        }
#pragma unroll
        for (int m = 0; m < 8; m += 2)
          *reinterpret_cast<double2*>(&W[lane * kWinPitch + 8 * h + m]) = double2{q[m].x, q[m + 1].x};
      }
      if (valid) smax = fmax(smax, sp);
      const double am = fmax(fabs(lo), fabs(hi));
      const uint64_t livemask = __ballot(valid && !(hi - lo < 1e-3 * fmax(am, 1.0)));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      int tv = 0;  // class of window 16 pg + c along dir, kept by lane (pg, c) of the rounds
#pragma unroll 1
      for (int pg = 0; pg < 4; ++pg) {
        if (((livemask >> (16 * pg)) & 0xFFFFull) == 0) continue;  // 16 flat windows: class 0
        const double2 v01 = *reinterpret_cast<const double2*>(&W[(16 * pg + c) * kWinPitch + 4 * g]);
        const double2 v23 = *reinterpret_cast<const double2*>(&W[(16 * pg + c) * kWinPitch + 4 * g + 2]);
        const double v[4] = {v01.x, v01.y, v23.x, v23.y};
        float x[4], z[3] = {0.0f, 0.0f, 0.0f};
        const bool live = sdnn_features(v, x);
        // a flat window is smooth without the network: a round of 16 flat
        // windows skips it (the branch is uniform over the wave, and when
        // taken all 64 lanes run the matrix instructions)
        if (__ballot(live) != 0) sdnn_mfma(F, x, z);
        const int t = live ? sdnn_argmax(z) : 0;  // valid in lanes 0..15
        // lane 16 pg + c' takes the class of window c' from lane c'
        const int tt = __shfl(t, lane & 15);
        if ((lane >> 4) == pg) tv = tt;
      }
      tau_own[dir] = valid ? tv : 0;
      // the next direction overwrites this wave's LDS rows
      __builtin_amdgcn_wave_barrier();
    }
    if (in) {
      a.tau[kl] = static_cast<uint8_t>(tau_own[0]);
      a.tau[a.P + kl] = static_cast<uint8_t>(tau_own[1]);
      a.muhat[kl] = muhat_of(a, kl, fl, tau_own[0], tau_own[1], smax);
    }
  }
}

// Fragment table of the classifier (see classify.h), built once per
// context by one workgroup.
__global__ __launch_bounds__(256) void k_sdnn_pack(const float* __restrict__ W, uint32_t* __restrict__ table) {
  for (int q = threadIdx.x; q < 64 * kSdnnFragWords; q += blockDim.x)
    table[q] = sdnn_frag_word(W, q / kSdnnFragWords, q % kSdnnFragWords);
}

// One pass of the windowed max: out(k) = max_off in(k + off * stride) w(|off|)
// over the index box (dir 0 along q^1, 1 along q^2); the final pass zeroes
// inactive points.
__global__ void k_dilate(const double* __restrict__ in, double* __restrict__ out, const int32_t* __restrict__ pid,
                         const int32_t* __restrict__ ijs, const PatchDev* __restrict__ patches,
                         const uint8_t* __restrict__ flags, int64_t P, int dir, int nv, const double* __restrict__ w,
                         double* __restrict__ mu, uint8_t* __restrict__ act) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const PatchDev pd = patches[pid[k]];
  const int32_t ij = ijs[k];
  const int j = ij >> 16, i = ij & 0xFFFF;
  // line activity flags of lattice subpatches: cleared by the first pass (the
  // thread of each row's and column's first index), set by the final pass
  if (act && !mu && pd.act_row >= 0) {
    if (i == 0) act[pd.act_row + j] = 0;
    if (j == 0) act[pd.act_col + i] = 0;
  }
  const int pos = dir == 0 ? i : j, len = dir == 0 ? pd.n1 : pd.n2;
  const int64_t stride = dir == 0 ? 1 : pd.n1;
  double best = 0.0;
  if (nv == 9) {
    // the default radius: unrolled and branch-free, so all 19 loads are in
    // flight together (terms outside the line read the point itself with
    // weight 0, which cannot raise the max of non-negative values)
#pragma unroll
    for (int off = -9; off <= 9; ++off) {
      const bool ok = pos + off >= 0 && pos + off < len;
      const double val = in[k + (ok ? off : 0) * stride] * (ok ? w[off < 0 ? -off : off] : 0.0);
      best = fmax(best, val);
    }
  } else {
    for (int off = -nv; off <= nv; ++off) {
      int q = pos + off;
      if (q < 0 || q >= len) continue;
      double val = in[k + off * stride] * w[off < 0 ? -off : off];
      if (val > best) best = val;
    }
  }
  if (mu) {
    // final pass: inactive points carry no viscosity; the blend rows then
    // overwrite the points covered by several subpatches
    if (!(flags[k] & kActive)) best = 0.0;
    mu[k] = fmax(best, 0.0);
    if (act && pd.act_row >= 0 && best > 0.0) {
      act[pd.act_row + j] = 1;
      act[pd.act_col + i] = 1;
    }
  }
  out[k] = best;
}


// bact (or null): activity flags of the row and the column of each blended
// point (x < 0: not on a lattice subpatch with activity flags).
// A group of kBlendLanes lanes per row: lane j evaluates stencil row b = j of
// each of the row's terms (six contiguous values, gathers in flight
// together), then the group sums by shuffles.
constexpr int kBlendLanes = 8;
__global__ void k_blend_rows(const double* __restrict__ mut, double* __restrict__ mu,
                             const BlendRowDev* __restrict__ rows, const BlendTermDev* __restrict__ terms, int n,
                             const int2* __restrict__ bact, uint8_t* __restrict__ act) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int q = static_cast<int>(g / kBlendLanes), j = static_cast<int>(g % kBlendLanes);
  // every lane of a group exists (blockDim is a multiple of the group
  // size), so the shuffles below see whole groups; rows past n add nothing
  double s = 0.0;
  BlendRowDev r{};
  if (q < n) {
    r = rows[q];
    if (j == 0) s = r.wself * mut[r.dst];
    for (int t = r.t0; t < r.t1; ++t) {
      const BlendTermDev& T = terms[t];
      if (j < T.nj) {
        const double* u = mut + T.base + static_cast<int64_t>(j) * T.stride;
        double acc = 0.0;
        for (int a = 0; a < T.ni; ++a) acc += T.wi[a] * u[a];
        s += T.scale * T.wj[j] * acc;
      }
    }
  }
#pragma unroll
  for (int o = kBlendLanes / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kBlendLanes);
  if (q >= n || j != 0) return;
  mu[r.dst] = fmax(s, 0.0);
  if (act && s > 0.0) {
    const int2 a = bact[q];
    if (a.x >= 0) {
      act[a.x] = 1;
      act[a.y] = 1;
    }
  }
}

// Initial-data smearing (Alg. 4 at t = 0).  Indicator: 1 at the active
// non-fringe points whose class flags a discontinuity in either direction.
__global__ void k_smear_indicator(const uint8_t* __restrict__ tau, const uint8_t* __restrict__ flags, int64_t P,
                                  double* __restrict__ out) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint8_t f = flags[k];
  const bool on = (f & kActive) && !(f & (kFringe | kXFringe)) && (tau[k] >= 1 || tau[P + k] >= 1);
  out[k] = on ? 1.0 : 0.0;
}

// Blend of the strongly filtered (Qs) and the given (Q) rho, rho u, rho v,
// theta with the window w clipped to [0, 1]; E rebuilt.
__global__ void k_smear_post(const double* __restrict__ Qs, const double* __restrict__ Q,
                             const double* __restrict__ w, double* __restrict__ U, const uint8_t* __restrict__ flags,
                             int64_t P) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  if (!(flags[k] & kActive)) return;
  const double a = fmin(fmax(w[k], 0.0), 1.0), b = 1.0 - a;
  const double r = a * Qs[k] + b * Q[k];
  const double mx = a * Qs[P + k] + b * Q[P + k];
  const double my = a * Qs[2 * P + k] + b * Q[2 * P + k];
  const double th = a * Qs[3 * P + k] + b * Q[3 * P + k];
  U[k] = r;
  U[P + k] = mx;
  U[2 * P + k] = my;
  U[3 * P + k] = r * th + 0.5 * (mx * mx + my * my) / r;
}

__global__ void k_filter_pre(const double* __restrict__ U, double* __restrict__ Q, const uint8_t* __restrict__ flags,
                             int64_t P, double gamma) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  double r = U[k], mx = U[P + k], my = U[2 * P + k], E = U[3 * P + k];
  double th = 0.0;
  if (flags[k] & kActive) {
    double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
    th = p / ((gamma - 1.0) * r);
  }
  Q[k] = r;
  Q[P + k] = mx;
  Q[2 * P + k] = my;
  Q[3 * P + k] = th;
}

__global__ void k_filter_post(const double* __restrict__ Q, double* __restrict__ U, const uint8_t* __restrict__ flags,
                              int64_t P, FluxOut fo) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint8_t f = flags[k];
  if (!(f & kActive)) {
    for (int c = 0; c < 4; ++c) U[c * P + k] = 0.0;
    store_flux(fo, P, k, f, 0.0, 0.0, 0.0, 0.0);
    return;
  }
  const double r = Q[k], mx = Q[P + k], my = Q[2 * P + k], th = Q[3 * P + k];
  const double E = r * th + 0.5 * (mx * mx + my * my) / r;
  U[k] = r;
  U[P + k] = mx;
  U[2 * P + k] = my;
  U[3 * P + k] = E;
  store_flux(fo, P, k, f, r, mx, my, E);
}

__global__ __launch_bounds__(256) void k_dt_partial(const double* __restrict__ U, const uint8_t* __restrict__ flags,
                                                    const double* __restrict__ hx, const double* __restrict__ mu,
                                                    double* __restrict__ part, int64_t P, double gamma) {
  __shared__ double red[256];
  double best = INFINITY;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < P;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (!(flags[k] & kActive)) continue;
    double r = U[k], mx = U[P + k], my = U[2 * P + k], E = U[3 * P + k];
    double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
    double s = sqrt(mx * mx + my * my) / r + sqrt(gamma * p / r);
    double h = hx[k];
    best = fmin(best, h / s);
    if (mu) {
      double m = mu[k];
      if (m > 0.0) best = fmin(best, h * h / (4.0 * m));
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Minimum of the per-block partial minima; also commits the time reached by
// the previous step: scal[0] = t (start of this step), scal[1] = dt,
// scal[2] = dt of the previous step, scal[4] = t + dt (end of this step).
__global__ void k_dt_final(const double* __restrict__ part, int n, double cfl, double dt_fixed,
                           double* __restrict__ scal) {
  __shared__ double red[256];
  double best = INFINITY;
  for (int q = threadIdx.x; q < n; q += blockDim.x) best = fmin(best, part[q]);
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double t = scal[4];
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl * red[0];
    scal[2] = scal[1];
    scal[0] = t;
    scal[1] = dt;
    scal[4] = t + dt;
  }
}

}  // namespace

namespace {
inline dim3 grid_for(int64_t n, int b = 256) { return dim3(static_cast<unsigned>((n + b - 1) / b)); }

}  // namespace

hipError_t launch_flux(const double* U, const uint8_t* flags, const FluxOut& fo, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_flux, grid_for(P), dim3(256), 0, s, U, flags, fo, P);
  return hipGetLastError();
}

template <typename DT, typename W1T>
void launch_stage_dt(const StageArgs& a, hipStream_t s) {
  switch (a.stage) {
    case 0: hipLaunchKernelGGL((k_stage<DT, 0, W1T>), grid_for(a.P), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_stage<DT, 1, W1T>), grid_for(a.P), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_stage<DT, 2, W1T>), grid_for(a.P), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_stage<DT, 3, W1T>), grid_for(a.P), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_stage<DT, 4, W1T>), grid_for(a.P), dim3(256), 0, s, a); break;
  }
}

hipError_t launch_stage(const StageArgs& a, hipStream_t s) {
  if (a.stage < 0 || a.stage > 4) return hipErrorInvalidValue;
  if (a.deriv_f32 && a.w1_f64)
    launch_stage_dt<float, double>(a, s);
  else if (a.deriv_f32)
    launch_stage_dt<float, float>(a, s);
  else
    launch_stage_dt<double, double>(a, s);
  return hipGetLastError();
}

hipError_t launch_fringe(double* U, const uint8_t* flags, const int64_t* copy_pairs, int ncopy, const int64_t* idst,
                         const int32_t* iptr, const int64_t* icol, const double* ival, int ninterp, int64_t P,
                         const FluxOut& fo, double2* ps, double gamma, hipStream_t s) {
  if (ncopy + ninterp)
    hipLaunchKernelGGL(k_fringe, grid_for(static_cast<int64_t>(kFringeLanes) * (ncopy + ninterp)), dim3(256), 0, s, U,
                       flags, copy_pairs, ncopy, idst, iptr,
                       icol, ival, ninterp, P, fo, ps, gamma);
  return hipGetLastError();
}

hipError_t launch_bc_state(double* U, const uint8_t* flags, const BcArgs& b, double t, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_bc_state, grid_for(P), dim3(256), 0, s, U, flags, b, t, P);
  return hipGetLastError();
}

hipError_t launch_smear_window(const ViscArgs& v, double* ind, double* w, hipStream_t s) {
  hipLaunchKernelGGL(k_smear_indicator, grid_for(v.P), dim3(256), 0, s, v.tau, v.flags, v.P, ind);
  hipLaunchKernelGGL(k_dilate, grid_for(v.P), dim3(256), 0, s, ind, v.tmp, v.pid, v.ij, v.patches, v.flags, v.P,
                     0, v.nv, v.wdil, nullptr, nullptr);
  hipLaunchKernelGGL(k_dilate, grid_for(v.P), dim3(256), 0, s, v.tmp, v.mut, v.pid, v.ij, v.patches, v.flags, v.P,
                     1, v.nv, v.wdil, w, nullptr);
  if (v.nblend)
    hipLaunchKernelGGL(k_blend_rows, grid_for(static_cast<int64_t>(v.nblend) * kBlendLanes), dim3(256), 0, s, v.mut, w,
                       v.brow, v.bterm, v.nblend, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_smear_post(const double* Qs, const double* Q, const double* w, double* U, const uint8_t* flags,
                             int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_smear_post, grid_for(P), dim3(256), 0, s, Qs, Q, w, U, flags, P);
  return hipGetLastError();
}

hipError_t launch_walls(double* U, const WallLine* lines, int nlines, const OpTables& ops, double* wth,
                       const uint8_t* flags, int64_t P, double gamma, const FluxOut& fo, double2* ps, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wall_theta, grid_for(nlines), dim3(256), 0, s, U, lines, nlines, ops, wth, P, gamma - 1.0);
  hipLaunchKernelGGL(k_wall_apply, grid_for(2 * static_cast<int64_t>(nlines)), dim3(256), 0, s, U, lines, nlines, wth,
                     flags, P, gamma, fo, ps);
  return hipGetLastError();
}

hipError_t launch_sdnn_pack(const float* weights, uint32_t* table, hipStream_t s) {
  hipLaunchKernelGGL(k_sdnn_pack, dim3(1), dim3(256), 0, s, weights, table);
  return hipGetLastError();
}

hipError_t launch_proxy(const ViscArgs& v, hipStream_t s) {
  hipLaunchKernelGGL(k_proxy, grid_for(v.P), dim3(256), 0, s, v.U, v.flags, v.ps, v.P, v.gamma);
  return hipGetLastError();
}

// Classifier arguments of a viscosity evaluation.
static ClassifyArgs classify_args(const ViscArgs& v) {
  ClassifyArgs c;
  c.P = v.P;
  c.flags = v.flags;
  c.pid = v.pid;
  c.patches = v.patches;
  c.rowrun = v.rowrun;
  c.colrun = v.colrun;
  c.ps = v.ps;
  c.ij = v.ij;
  c.hx = v.hx;
  c.tau = v.tau;
  c.muhat = v.muhat;
  c.mode = v.mode;
  c.weights = v.weights;
  c.sdnn_table = v.sdnn_table;
  c.basis = v.basis;
  c.c_mu = v.c_mu;
  c.wgeo = v.wgeo;
  return c;
}

hipError_t launch_window_geo(const ViscArgs& v, hipStream_t s) {
  hipLaunchKernelGGL(k_window_geo, grid_for(v.P), dim3(256), 0, s, classify_args(v), v.wgeo);
  return hipGetLastError();
}

hipError_t launch_viscosity(const ViscArgs& v, hipStream_t s) {
  const ClassifyArgs c = classify_args(v);
  if (c.mode == 2)
    hipLaunchKernelGGL(k_classify_sdnn, dim3(kClassifyBlocks), dim3(256), 0, s, c);
  else
    hipLaunchKernelGGL(k_classify, grid_for(v.P), dim3(256), 0, s, c);
  hipLaunchKernelGGL(k_dilate, grid_for(v.P), dim3(256), 0, s, v.muhat, v.tmp, v.pid, v.ij, v.patches, v.flags, v.P,
                     0, v.nv, v.wdil, nullptr, v.act);
  hipLaunchKernelGGL(k_dilate, grid_for(v.P), dim3(256), 0, s, v.tmp, v.mut, v.pid, v.ij, v.patches, v.flags, v.P,
                     1, v.nv, v.wdil, v.mu, v.act);
  if (v.nblend)
    hipLaunchKernelGGL(k_blend_rows, grid_for(static_cast<int64_t>(v.nblend) * kBlendLanes), dim3(256), 0, s, v.mut,
                       v.mu, v.brow, v.bterm, v.nblend, v.bact, v.act);
  return hipGetLastError();
}

// Localized viscosity (Sec. 4): the viscous derivatives of a line are only
// needed where mu or its gradient is nonzero.  On a lattice subpatch
// (constant diagonal metric) the derivatives along a row enter the operator
// only through mu and d mu / dq^1 on that row, and both vanish identically
// when mu vanishes at every point of the row (the FC derivative of a zero
// line is an exact zero); columns likewise.  The dilation and blend kernels
// leave act[line] = 1 for the lines where mu is nonzero somewhere.  One wave
// per contraction tile: bit w of its skip flag is set when none of the
// tile's lines 16 w .. 16 w + 15 (line = component * nrow + row) lies on an
// active grid line (the contraction wave that owns them then neither
// multiplies nor stores); all four bits skip the tile.  Tiles of tasks
// without activity entries are always computed.  The two tile lists
// (n0 + n1 tiles) are marked in one launch.
__global__ __launch_bounds__(256) void k_tile_activity(const GemmTask* __restrict__ tasks0, GemmTile* tiles0, int n0,
                                                        const GemmTask* __restrict__ tasks1, GemmTile* tiles1, int n1,
                                                        const uint8_t* __restrict__ act) {
  int t = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n0 + n1) return;
  const GemmTask* tasks = tasks0;
  GemmTile* tiles = tiles0;
  if (t >= n0) {
    t -= n0;
    tasks = tasks1;
    tiles = tiles1;
  }
  const GemmTile tile = tiles[t];
  if (tile.task < 0) return;
  const GemmTask T = tasks[tile.task];
  bool need = true;
  if (T.act >= 0) {
    const int line = tile.line0 + lane;
    need = line < T.nrow * T.ncomp && act[T.act + line % T.nrow] != 0;
  }
  const uint64_t m = __ballot(need);
  int skip = 0;
  for (int w = 0; w < 4; ++w)
    if (!((m >> (16 * w)) & 0xFFFFull)) skip |= 1 << w;
  if (lane == 0) tiles[t].skip = skip;
}

hipError_t launch_tile_activity(const GemmTask* tasks0, GemmTile* tiles0, int n0, const GemmTask* tasks1,
                                GemmTile* tiles1, int n1, const uint8_t* act, hipStream_t s) {
  if (n0 + n1 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_activity, dim3((n0 + n1 + 3) / 4), dim3(256), 0, s, tasks0, tiles0, n0, tasks1, tiles1,
                     n1, act);
  return hipGetLastError();
}

hipError_t launch_filter_pre(const double* U, double* Q, const uint8_t* flags, int64_t P, double gamma,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_filter_pre, grid_for(P), dim3(256), 0, s, U, Q, flags, P, gamma);
  return hipGetLastError();
}

hipError_t launch_filter_post(const double* Q, double* U, const uint8_t* flags, int64_t P, const FluxOut& fo,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_filter_post, grid_for(P), dim3(256), 0, s, Q, U, flags, P, fo);
  return hipGetLastError();
}

hipError_t launch_dt(const double* U, const uint8_t* flags, const double* hx, const double* mu, double* part,
                     int nblocks, int64_t P, double gamma, double cfl, double dt_fixed, double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_partial, dim3(nblocks), dim3(256), 0, s, U, flags, hx, mu, part, P, gamma);
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, s, part, nblocks, cfl, dt_fixed, scal);
  return hipGetLastError();
}

}  // namespace fcs
