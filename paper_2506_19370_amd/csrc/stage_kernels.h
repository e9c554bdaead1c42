// Launch interface of the elementwise / stencil / gather kernels.
#pragma once
#include "kernels.h"

namespace fcs {


struct VortexArgs {
  double beta, x0, y0, u0, v0;
};

// Where a kernel that produces a state also stores the Euler fluxes of that
// state as the next stage's contraction operands (F == nullptr: not at all).
struct FluxOut {
  double* F;
  const double *t1x, *t1y, *t2x, *t2y;  // per-point metrics (non-affine subpatches)
  double gm1;
  const int32_t* pid;                   // subpatch of each point
  const PatchDev* patches;              // constant metrics of affine subpatches
};

// Boundary data applied by the stage kernel to the points flagged kBoundary.
struct BcArgs {
  const BcEntry* bc;
  const int32_t* bcidx;  // entry of each point (points without one: unused)
  double gamma;
  const double* t;       // device time of the step start
  double frac;           // stage time fraction of the step
  VortexArgs vortex;
};

struct StageArgs {
  int64_t P;
  int stage;
  double c[6];  // Shu-Osher coefficients of this stage (see ssprk table)
  double gm1;
  const uint8_t* flags;
  const double *in, *U0;
  double *out, *acc;
  const void *DF1, *DF2;  // stage derivatives: double, or float when deriv_f32
  const double *t1x, *t1y, *t2x, *t2y;
  int visc;
  const double *mu, *mu1, *mu2, *g11, *g12, *g22, *lap1, *lap2;
  const void *W1, *W2, *W11, *W22, *W12;
  int deriv_f32;
  int w1_f64;  // with deriv_f32: W1 is FP64 (operand of the cross contraction)
  const double* dt;
  int* bad_flag;
  BcArgs bcs;
  FluxOut flux;
  const int32_t* pid;
  const PatchDev* patches;
  const int32_t* csrc;  // per point: its copy donor (fringe points on a common lattice), else itself
  double2* ps;          // last stage of a step: proxy and wave speed of the new state (Alg. 3 input), or null
};

struct ClassifyArgs {
  int64_t P;
  const uint8_t* flags;
  const int32_t* pid;
  const PatchDev* patches;
  const int2 *rowrun, *colrun;
  const double2* ps;     // proxy and wave speed |u| + a of every point
  const int32_t* ij;     // (j << 16) | i of every point
  const int4* wgeo;      // window start and stride of every point along q^1, q^2 (start -1: none)
  const double* hx;
  uint8_t* tau;
  double* muhat;
  int mode;  // 1 modal, 2 sdnn, 3 frozen
  const float* weights;
  const uint32_t* sdnn_table;  // fragment table of the weights (mode 2)
  const double* basis;
  double c_mu;
};

struct ViscArgs {
  int64_t P;
  const double* U;
  const uint8_t* flags;
  const int32_t* pid;
  const PatchDev* patches;
  const int2 *rowrun, *colrun;
  double2* ps;
  const int32_t* ij;
  int4* wgeo;  // per-point window geometry, filled once by launch_window_geo
  const double* hx;
  uint8_t* tau;
  double *muhat, *tmp, *mut, *mu;
  int mode;
  const float* weights;
  const uint32_t* sdnn_table;
  const double* basis;
  double c_mu, gamma;
  int nv;
  const double* wdil;
  int nblend;
  const BlendRowDev* brow;
  const BlendTermDev* bterm;
  // (or null) line activity flags of lattice subpatches, one per row and
  // column: 1 where the final mu is nonzero somewhere on the line; bact:
  // the flags of the row and the column of each blend row's point
  uint8_t* act;
  const int2* bact;
};

// Skip flags of the tiles of two contraction task lists from the line
// activity flags that the viscosity kernels leave (see ViscArgs::act).
hipError_t launch_tile_activity(const GemmTask* tasks0, GemmTile* tiles0, int n0, const GemmTask* tasks1,
                                GemmTile* tiles1, int n1, const uint8_t* act, hipStream_t s);
hipError_t launch_flux(const double* U, const uint8_t* flags, const FluxOut& fo, int64_t P, hipStream_t s);
// Stage update, boundary conditions and (if a.flux.F) the fluxes of the new
// state at every active point.
hipError_t launch_stage(const StageArgs& a, hipStream_t s);
// Fringe fill (copy pairs and interpolation rows) and, if fo.F, the fluxes
// of the filled points.
// ps (or null): also store the proxy and wave speed of each filled point.
hipError_t launch_fringe(double* U, const uint8_t* flags, const int64_t* copy_pairs, int ncopy, const int64_t* idst,
                         const int32_t* iptr, const int64_t* icol, const double* ival, int ninterp, int64_t P,
                         const FluxOut& fo, double2* ps, double gamma, hipStream_t s);
// Boundary conditions of every boundary point of U, in place, at time t
// (b.t and b.frac are not used).
hipError_t launch_bc_state(double* U, const uint8_t* flags, const BcArgs& b, double t, int64_t P, hipStream_t s);
// Alg. 3 in two parts: the proxy variable and wave speeds (the only part
// that reads the state), then classification, preliminary viscosity,
// dilation and blend.
hipError_t launch_proxy(const ViscArgs& v, hipStream_t s);
// No-slip adiabatic walls of state U (see WallLine): wall theta per line into
// wth (2 doubles per line), then zero momentum and E = rho theta at the wall
// nodes, with their fluxes (fo.F) and proxy values (ps) when set.
hipError_t launch_walls(double* U, const WallLine* lines, int nlines, const OpTables& ops, double* wth,
                        const uint8_t* flags, int64_t P, double gamma, const FluxOut& fo, double2* ps, hipStream_t s);
// Window of the initial-data smearing into w (P doubles): the indicator of
// the classes in v.tau (a discontinuity flagged in either direction, off the
// fringe; into ind, P doubles) localized as the viscosity is (two dilation
// passes, blend rows); v.tmp and v.mut serve as scratch.
hipError_t launch_smear_window(const ViscArgs& v, double* ind, double* w, hipStream_t s);
// U <- w Qs + (1 - w) Q for rho, rho u, rho v, theta (w clipped to [0, 1]),
// E rebuilt; active points only.
hipError_t launch_smear_post(const double* Qs, const double* Q, const double* w, double* U, const uint8_t* flags,
                             int64_t P, hipStream_t s);
// Fragment table (64 x 84 words) of a classifier parameter blob.
hipError_t launch_sdnn_pack(const float* weights, uint32_t* table, hipStream_t s);
hipError_t launch_viscosity(const ViscArgs& v, hipStream_t s);
// Window start and stride of every point in both directions (static
// geometry; run once per bound context).
hipError_t launch_window_geo(const ViscArgs& v, hipStream_t s);
hipError_t launch_filter_pre(const double* U, double* Q, const uint8_t* flags, int64_t P, double gamma,
                             hipStream_t s);
// Rebuilds the state from the filtered variables and stores its fluxes (the
// operands of the step's first stage) through fo.
hipError_t launch_filter_post(const double* Q, double* U, const uint8_t* flags, int64_t P, const FluxOut& fo,
                              hipStream_t s);
// scal: device scalars [t, dt, last dt, bad flag, t + dt]
hipError_t launch_dt(const double* U, const uint8_t* flags, const double* hx, const double* mu, double* part,
                     int nblocks, int64_t P, double gamma, double cfl, double dt_fixed, double* scal, hipStream_t s);

}  // namespace fcs
