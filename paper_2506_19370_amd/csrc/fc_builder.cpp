// FC-Gram continuation and dense FC operators, built on the host in
// __float128 (quad) precision.
//
// Method: Sec. 2 of the paper (FC-Gram Fourier continuation of N equispaced
// values with d matching points and C continuation points; derivatives and
// the spectral filter applied in Fourier space on the periodic extension).
// The construction constants follow the reading documented with the
// library: each Gram polynomial (orthonormal for the discrete inner product
// on the d matching points) is continued by a trigonometric polynomial with
// 25 modes of period 76 h fitted, in the least-squares sense, to the
// polynomial on the matching interval and to zero on a 12-point interval
// that follows the C continuation points, both sampled 20 times per h.
// The least-squares problem is solved with Householder QR in quad precision.
//
// The dense operator for lines of n points composes extension, spectral
// multiplier and restriction: out[t] = sum_l K[(t - l) mod M] ext[l],
// M = n + C, with K the periodic kernel of the multiplier (first or second
// derivative in index units, Nyquist mode zeroed; or the filter
// exp(-alpha (2|m|/M)^36), alpha = 16 ln 10; kind 3: the same with order 8).
#include <quadmath.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "fc_builder.h"

namespace fcs {

namespace {

using q128 = __float128;

constexpr int kModes = 25;
constexpr int kPeriod = 76;
constexpr int kZero = 12;
constexpr int kOversample = 20;

// Householder QR of a (m x n, column-major) matrix in place; returns the
// Householder vectors below the diagonal, R on and above, and tau.
void householder_qr(std::vector<q128>& a, int m, int n, std::vector<q128>& tau) {
  tau.assign(n, 0);
  for (int k = 0; k < n; ++k) {
    q128 norm = 0;
    for (int i = k; i < m; ++i) norm += a[k * m + i] * a[k * m + i];
    norm = sqrtq(norm);
    if (norm == 0) continue;
    q128 alpha = a[k * m + k] > 0 ? -norm : norm;
    q128 v0 = a[k * m + k] - alpha;
    for (int i = k + 1; i < m; ++i) a[k * m + i] /= v0;
    a[k * m + k] = alpha;
    // tau = (alpha - a_kk_old) / alpha  with v = [1, a(k+1:m)/v0]
    tau[k] = -v0 / alpha;
    for (int j = k + 1; j < n; ++j) {
      q128 s = a[j * m + k];
      for (int i = k + 1; i < m; ++i) s += a[k * m + i] * a[j * m + i];
      s *= tau[k];
      a[j * m + k] -= s;
      for (int i = k + 1; i < m; ++i) a[j * m + i] -= s * a[k * m + i];
    }
  }
}

// Least-squares solution of min |A x - b| given the QR factors.
void qr_solve(const std::vector<q128>& qr, const std::vector<q128>& tau, int m, int n,
              std::vector<q128> b, std::vector<q128>& x) {
  for (int k = 0; k < n; ++k) {
    q128 s = b[k];
    for (int i = k + 1; i < m; ++i) s += qr[k * m + i] * b[i];
    s *= tau[k];
    b[k] -= s;
    for (int i = k + 1; i < m; ++i) b[i] -= s * qr[k * m + i];
  }
  x.assign(n, 0);
  for (int k = n - 1; k >= 0; --k) {
    q128 s = b[k];
    for (int j = k + 1; j < n; ++j) s -= qr[j * m + k] * x[j];
    x[k] = s / qr[k * m + k];
  }
}

void trig_row(q128 t, q128* row) {
  const q128 two_pi = 2 * M_PIq;
  row[0] = 1;
  for (int k = 1; k <= kModes; ++k) {
    q128 w = two_pi * k * t / kPeriod;
    row[2 * k - 1] = cosq(w);
    row[2 * k] = sinq(w);
  }
}

struct Continuation {
  std::vector<double> Q, A, B;  // d x d, C x d, C x d (row-major)
};

std::mutex g_mu;
std::map<std::pair<int, int>, Continuation> g_cont;
std::map<std::tuple<int, int, int, int>, std::vector<double>> g_ops;

const Continuation& continuation(int d, int C) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto key = std::make_pair(d, C);
  auto it = g_cont.find(key);
  if (it != g_cont.end()) return it->second;

  // Gram basis: modified Gram-Schmidt on the monomials 1, t, ..., t^(d-1)
  // sampled at t = 0..d-1; keep monomial coefficients of each q_k.
  std::vector<q128> vals(d * d), coef(d * d, 0);  // vals[k*d+i] = q_k(i); coef[k*d+j]
  for (int k = 0; k < d; ++k) {
    for (int i = 0; i < d; ++i) vals[k * d + i] = powq((q128)i, k);
    coef[k * d + k] = 1;
    for (int pass = 0; pass < 2; ++pass) {
      for (int l = 0; l < k; ++l) {
        q128 s = 0;
        for (int i = 0; i < d; ++i) s += vals[l * d + i] * vals[k * d + i];
        for (int i = 0; i < d; ++i) vals[k * d + i] -= s * vals[l * d + i];
        for (int j = 0; j < d; ++j) coef[k * d + j] -= s * coef[l * d + j];
      }
    }
    q128 nrm = 0;
    for (int i = 0; i < d; ++i) nrm += vals[k * d + i] * vals[k * d + i];
    nrm = sqrtq(nrm);
    for (int i = 0; i < d; ++i) vals[k * d + i] /= nrm;
    for (int j = 0; j < d; ++j) coef[k * d + j] /= nrm;
  }

  const int n_match = (d - 1) * kOversample + 1;
  const int n_zero = (kZero - 1) * kOversample + 1;
  const int m = n_match + n_zero;
  const int ncol = 2 * kModes + 1;
  std::vector<q128> a(static_cast<size_t>(m) * ncol);
  std::vector<q128> row(ncol);
  std::vector<q128> tm(n_match);
  for (int r = 0; r < m; ++r) {
    q128 t = r < n_match ? (q128)r / kOversample
                         : (q128)(d + C) + (q128)(r - n_match) / kOversample;
    if (r < n_match) tm[r] = t;
    trig_row(t, row.data());
    for (int c = 0; c < ncol; ++c) a[static_cast<size_t>(c) * m + r] = row[c];
  }
  std::vector<q128> tau;
  householder_qr(a, m, ncol, tau);

  std::vector<q128> Aq(static_cast<size_t>(C) * d);
  std::vector<q128> x;
  for (int k = 0; k < d; ++k) {
    std::vector<q128> b(m, 0);
    for (int r = 0; r < n_match; ++r) {
      q128 s = 0, p = 1;
      for (int j = 0; j < d; ++j) {
        s += coef[k * d + j] * p;
        p *= tm[r];
      }
      b[r] = s;
    }
    qr_solve(a, tau, m, ncol, b, x);
    for (int c = 0; c < C; ++c) {
      trig_row((q128)(d + c), row.data());
      q128 s = 0;
      for (int j = 0; j < ncol; ++j) s += row[j] * x[j];
      Aq[c * d + k] = s;
    }
  }
  Continuation out;
  out.Q.resize(d * d);
  out.A.resize(C * d);
  out.B.resize(C * d);
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) out.Q[i * d + k] = (double)vals[k * d + i];
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < d; ++k) out.A[c * d + k] = (double)Aq[c * d + k];
  // B = A Q^T: continuation of raw matching values
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < d; ++i) {
      q128 s = 0;
      for (int k = 0; k < d; ++k) s += Aq[c * d + k] * vals[k * d + i];
      out.B[c * d + i] = (double)s;
    }
  return g_cont.emplace(key, std::move(out)).first->second;
}

}  // namespace

bool fc_continuation(int d, int C, double* Q, double* A) {
  if (d < 1 || d > 12 || C < 4 || C > 64) return false;
  const Continuation& c = continuation(d, C);
  if (Q) std::memcpy(Q, c.Q.data(), sizeof(double) * d * d);
  if (A) std::memcpy(A, c.A.data(), sizeof(double) * C * d);
  return true;
}

const std::vector<double>* fc_operator(int n, int d, int C, int kind) {
  if (n < 2 * d || n > 1024 || kind < 0 || kind > 3) return nullptr;
  const Continuation& cont = continuation(d, C);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_ops.find(std::make_tuple(n, d, C, kind));
    if (it != g_ops.end()) return &it->second;
  }
  const int M = n + C;
  const int kmax = (M % 2 == 0) ? M / 2 - 1 : (M - 1) / 2;
  typedef long double ld;
  const ld two_pi = 2.0L * 3.14159265358979323846264338327950288L;
  std::vector<ld> sn(M), cs(M);
  for (int j = 0; j < M; ++j) {
    sn[j] = sinl(two_pi * j / M);
    cs[j] = cosl(two_pi * j / M);
  }
  const ld alpha = 16.0L * logl(10.0L);
  std::vector<ld> K(M);
  for (int mm = 0; mm < M; ++mm) {
    ld s = 0;
    for (int k = 1; k <= kmax; ++k) {
      int idx = static_cast<int>((static_cast<int64_t>(k) * mm) % M);
      ld w = two_pi * k / M;
      if (kind == 0) {
        s += w * sn[idx];
      } else if (kind == 1) {
        s += w * w * cs[idx];
      } else {
        // the filter of t > 0 (order 36) or the stronger one of the
        // initial-data smearing (order 8)
        ld eta = 2.0L * k / M;
        s += expl(-alpha * powl(eta, kind == 2 ? 36 : 8)) * cs[idx];
      }
    }
    if (kind == 0) K[mm] = -2.0L * s / M;
    else if (kind == 1) K[mm] = -2.0L * s / M;
    else K[mm] = (1.0L + 2.0L * s) / M;
  }
  std::vector<ld> op(static_cast<size_t>(n) * n, 0);
  for (int t = 0; t < n; ++t)
    for (int s = 0; s < n; ++s) op[static_cast<size_t>(t) * n + s] = K[((t - s) % M + M) % M];
  // continuation rows l = n + c: right part acts on s = n-d+i with B[c][i];
  // left part (mirrored) places B[c'][i] f[d-1-i] at l = n + C - 1 - c'.
  for (int t = 0; t < n; ++t) {
    for (int c = 0; c < C; ++c) {
      ld kr = K[((t - (n + c)) % M + M) % M];
      ld kl = K[((t - (n + C - 1 - c)) % M + M) % M];
      for (int i = 0; i < d; ++i) {
        op[static_cast<size_t>(t) * n + (n - d + i)] += kr * (ld)cont.B[c * d + i];
        op[static_cast<size_t>(t) * n + (d - 1 - i)] += kl * (ld)cont.B[c * d + i];
      }
    }
  }
  std::vector<double> out(op.size());
  for (size_t i = 0; i < op.size(); ++i) out[i] = (double)op[i];
  std::lock_guard<std::mutex> lock(g_mu);
  return &g_ops.emplace(std::make_tuple(n, d, C, kind), std::move(out)).first->second;
}

}  // namespace fcs

namespace fcs {
// Orthonormal discrete polynomials of degree 0..15 on 16 equispaced points
// of [-1, 1] (columns of a 16 x 16 row-major matrix), by modified
// Gram-Schmidt in quad precision: the modal basis of the fallback
// smoothness indicator.
void modal_basis16(double* out) {
  using q128 = __float128;
  const int n = 16;
  std::vector<q128> v(n * n);
  for (int k = 0; k < n; ++k) {
    for (int i = 0; i < n; ++i) v[k * n + i] = powq((q128)(2 * i) / (n - 1) - 1, k);
    for (int pass = 0; pass < 2; ++pass)
      for (int l = 0; l < k; ++l) {
        q128 s = 0;
        for (int i = 0; i < n; ++i) s += v[l * n + i] * v[k * n + i];
        for (int i = 0; i < n; ++i) v[k * n + i] -= s * v[l * n + i];
      }
    q128 nrm = 0;
    for (int i = 0; i < n; ++i) nrm += v[k * n + i] * v[k * n + i];
    nrm = sqrtq(nrm);
    for (int i = 0; i < n; ++i) v[k * n + i] /= nrm;
  }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) out[i * n + k] = (double)v[k * n + i];
}
}  // namespace fcs
