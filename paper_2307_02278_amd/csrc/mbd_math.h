// Scalar mathematics shared by the kernels (host+device so that it can be
// checked on the CPU): probe hashing, cardinal B-splines, the direct-space
// dipole kernel, and the tridiagonal eigensolver behind the Gauss quadrature.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace mbd {

#define MBD_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): output n of the stream seeded with x is
// mix(x + (n + 1) * golden). Used for the Rademacher probe signs (eq. dds).
// ---------------------------------------------------------------------------
MBD_HD uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
MBD_HD uint64_t splitmix_at(uint64_t seed, uint64_t n) {
  return splitmix_mix(seed + (n + 1ull) * 0x9E3779B97F4A7C15ull);
}

// ---------------------------------------------------------------------------
// Cardinal B-splines M_p (support [0, p], degree p - 1). For a fractional offset
// w in [0, 1) fill th[t] = M_p(w + t) and dth[t] = M_p'(w + t), t = 0..p-1,
// by the order recursion M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1),
// M_2(x) = 1 - |x - 1|, and M_n'(x) = M_{n-1}(x) - M_{n-1}(x - 1).
// ---------------------------------------------------------------------------
template <int P>
MBD_HD void bspline_weights(double w, double* th, double* dth) {
  double M[P];
#pragma unroll
  for (int t = 0; t < P; ++t) M[t] = 0.0;
  M[0] = w;          // M_2(w)
  M[1] = 1.0 - w;    // M_2(w + 1)
#pragma unroll
  for (int n = 3; n <= P; ++n) {
    if (n == P) {
      // derivative of order P from the order P-1 values
#pragma unroll
      for (int t = 0; t < P; ++t) dth[t] = M[t] - (t > 0 ? M[t - 1] : 0.0);
    }
    const double inv = 1.0 / (n - 1);
#pragma unroll
    for (int t = n - 1; t >= 0; --t) {
      const double x = w + t;
      const double lo = (t > 0) ? M[t - 1] : 0.0;
      M[t] = (x * M[t] + (n - x) * lo) * inv;
    }
  }
#pragma unroll
  for (int t = 0; t < P; ++t) th[t] = M[t];
}

// Same, plus the second derivatives ddth[t] = M_p''(w + t) = M_{p-2}(w + t)
// - 2 M_{p-2}(w + t - 1) + M_{p-2}(w + t - 2) (needed for forces; p >= 4).
template <int P>
MBD_HD void bspline_weights2(double w, double* th, double* dth, double* ddth) {
  double M[P];
#pragma unroll
  for (int t = 0; t < P; ++t) M[t] = 0.0;
  M[0] = w;
  M[1] = 1.0 - w;
#pragma unroll
  for (int n = 3; n <= P; ++n) {
    if (n == P - 1) {
#pragma unroll
      for (int t = 0; t < P; ++t)
        ddth[t] = M[t] - 2.0 * (t > 0 ? M[t - 1] : 0.0) + (t > 1 ? M[t - 2] : 0.0);
    }
    if (n == P) {
#pragma unroll
      for (int t = 0; t < P; ++t) dth[t] = M[t] - (t > 0 ? M[t - 1] : 0.0);
    }
    const double inv = 1.0 / (n - 1);
#pragma unroll
    for (int t = n - 1; t >= 0; --t) {
      const double x = w + t;
      const double lo = (t > 0) ? M[t - 1] : 0.0;
      M[t] = (x * M[t] + (n - x) * lo) * inv;
    }
  }
#pragma unroll
  for (int t = 0; t < P; ++t) th[t] = M[t];
}

// ---------------------------------------------------------------------------
// Direct-space Ewald dipole kernel with the damping correction (eq. fld_ewald):
//   T_dir(r) = T_erfc(r) - (1 - f(r)) T(r) = A(r) I - B(r) r r^T,
// with T = -grad grad 1/r and T_erfc = -grad grad erfc(tau r)/r.
// Equivalent form used where f is small (short range): T_dir = f T - T_erf with
// T_erf = -grad grad erf(tau r)/r, evaluated by its Taylor series for tau r < 0.5
// (single precision) to avoid cancelling two large terms.
// Series: r^3 A_erf = (2/sqrt(pi)) [2x^3/3 - 2x^5/5 + x^7/7 - x^9/27 + x^11/132 - x^13/780]
//         r^5 B_erf = (2/sqrt(pi)) [4x^5/5 - 4x^7/7 + 2x^9/9 - 2x^11/33 + x^13/78 - x^15/450]
// with x = tau r.
// ---------------------------------------------------------------------------
template <typename R> MBD_HD R m_exp(R x);
template <> MBD_HD double m_exp<double>(double x) { return exp(x); }
template <> MBD_HD float m_exp<float>(float x) { return expf(x); }
template <typename R> MBD_HD R m_erfc(R x);
template <> MBD_HD double m_erfc<double>(double x) { return erfc(x); }
template <> MBD_HD float m_erfc<float>(float x) { return erfcf(x); }
template <typename R> MBD_HD R m_sqrt(R x);
template <> MBD_HD double m_sqrt<double>(double x) { return sqrt(x); }
template <> MBD_HD float m_sqrt<float>(float x) { return sqrtf(x); }

template <typename R>
MBD_HD void direct_kernel(R r2, R tau, R inv_s, R damp_d, R& A, R& B) {
  const R r = m_sqrt<R>(r2);
  const R ir = R(1) / r;
  const R ir2 = ir * ir;
  const R ir3 = ir2 * ir;
  const R ir5 = ir3 * ir2;
  const R x = tau * r;
  const R x2 = x * x;
  const R two_over_sqrtpi = R(1.1283791670955126);
  const R z = damp_d * (r * inv_s - R(1));
  if (z >= R(0)) {
    // long range: 1 - f = 1 / (1 + e^z) is small
    const R omf = R(1) / (R(1) + m_exp<R>(z));
    const R ex = m_exp<R>(-x2);
    const R ec = m_erfc<R>(x);
    const R c = two_over_sqrtpi * x * ex;
    A = (ec + c) * ir3 - omf * ir3;
    B = (R(3) * ec + c * (R(3) + R(2) * x2)) * ir5 - omf * R(3) * ir5;
  } else {
    // short range: f = 1 / (1 + e^{-z}) is small
    const R f = R(1) / (R(1) + m_exp<R>(-z));
    R Ae, Be;
    if (sizeof(R) == 4 && x < R(0.5)) {
      const R t3 = tau * tau * tau;
      const R t5 = t3 * tau * tau;
      const R pa = R(2.0 / 3.0) + x2 * (R(-2.0 / 5.0) + x2 * (R(1.0 / 7.0) +
                   x2 * (R(-1.0 / 27.0) + x2 * (R(1.0 / 132.0) + x2 * R(-1.0 / 780.0)))));
      const R pb = R(4.0 / 5.0) + x2 * (R(-4.0 / 7.0) + x2 * (R(2.0 / 9.0) +
                   x2 * (R(-2.0 / 33.0) + x2 * (R(1.0 / 78.0) + x2 * R(-1.0 / 450.0)))));
      Ae = two_over_sqrtpi * t3 * pa;
      Be = two_over_sqrtpi * t5 * pb;
    } else {
      const R ex = m_exp<R>(-x2);
      const R er = R(1) - m_erfc<R>(x);
      const R c = two_over_sqrtpi * x * ex;
      Ae = (er - c) * ir3;
      Be = (R(3) * er - c * (R(3) + R(2) * x2)) * ir5;
    }
    A = f * ir3 - Ae;
    B = f * R(3) * ir5 - Be;
  }
}

// ---------------------------------------------------------------------------
// Gauss quadrature from a symmetric tridiagonal (eqs. sl3, tridiag2): nodes are
// the eigenvalues theta_k, weights the squared first components U_1k^2 of the
// eigenvectors (Golub-Welsch). Implicit symmetric QR with Wilkinson shifts and
// deflation; only the first row of the accumulated rotations is kept.
// d[0..n-1] diagonal, e[0..n-2] off-diagonal (both overwritten), q[0..n-1] work.
// Returns sum_k q_k^2 sqrt(theta_k); *theta_min gets min theta; *ok = 0 when
// the iteration did not converge.
// ---------------------------------------------------------------------------
// Radial derivatives of the direct-space kernel for forces, in double precision:
// with T_dir = A I - B r r^T, returns A, B, A'(r)/r and B'(r)/r. For the screened part
// (a -grad grad of a radial function) A_e' = -r B_e; with x = tau r,
// c = (2x/sqrt(pi)) e^{-x^2}, N = 3 erfc(x) + c (3 + 2x^2): B_e = N / r^5 and
// B_e' = -(4 x^4 c + 5 N) / r^6. The damping term (1 - f) T has f' = f (1 - f) d / S.
MBD_HD void direct_kernel_grad(double r2, double tau, double inv_s, double damp_d, double& A,
                               double& B, double& dA_r, double& dB_r) {
  direct_kernel<double>(r2, tau, inv_s, damp_d, A, B);
  const double r = sqrt(r2);
  const double ir = 1.0 / r, ir2 = ir * ir;
  const double ir5 = ir2 * ir2 * ir, ir7 = ir5 * ir2;
  const double x = tau * r, x2 = x * x;
  const double c = 1.1283791670955126 * x * exp(-x2);
  const double N = 3.0 * erfc(x) + c * (3.0 + 2.0 * x2);
  const double Be = N * ir5;
  const double dBe_r = -(4.0 * x2 * x2 * c + 5.0 * N) * ir7;
  const double z = damp_d * (r * inv_s - 1.0);
  double f, omf;
  if (z >= 0.0) {
    const double e = exp(-z);
    omf = e / (1.0 + e);
    f = 1.0 / (1.0 + e);
  } else {
    const double e = exp(z);
    f = e / (1.0 + e);
    omf = 1.0 / (1.0 + e);
  }
  const double fp = f * omf * damp_d * inv_s;  // df/dr
  dA_r = -Be + fp * ir2 * ir2 + 3.0 * omf * ir5;
  dB_r = dBe_r + 3.0 * fp * ir5 * ir + 15.0 * omf * ir7;
}

MBD_HD double tridiag_sqrt_quadrature(double* d, double* e, double* q, int n,
                                      double* theta_min, int* ok) {
  for (int k = 0; k < n; ++k) q[k] = (k == 0) ? 1.0 : 0.0;
  int hi = n - 1;
  int iter = 0;
  const double eps = 2.220446049250313e-16;
  *ok = 1;
  while (hi > 0) {
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
    if (++iter > 60 * n) { *ok = 0; break; }
    // Wilkinson shift from the trailing 2x2 block.
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * sqrt(delta * delta + eh * eh);
    const double mu = (den != 0.0) ? d[hi] - eh * eh / den : d[hi];
    double x = d[lo] - mu;
    double z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) { c = x / r; s = -z / r; }
      if (k > lo) e[k - 1] = r;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
      if (k + 1 < hi) {
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      const double qk = q[k], qk1 = q[k + 1];
      q[k] = c * qk - s * qk1;
      q[k + 1] = s * qk + c * qk1;
    }
  }
  double sum = 0.0;
  double tmin = d[0];
  for (int k = 0; k < n; ++k) {
    tmin = d[k] < tmin ? d[k] : tmin;
    sum += q[k] * q[k] * sqrt(d[k] > 0.0 ? d[k] : 0.0);
  }
  *theta_min = tmin;
  return sum;
}

// Same iteration, tracking the full eigenvector matrix U (row-major, u[i * ld + k] =
// U_ik, columns are eigenvectors) instead of its first row. On return d holds the
// eigenvalues. Returns 0 if the iteration did not converge.
MBD_HD int tridiag_eigen(double* d, double* e, double* u, int n, int ld) {
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) u[i * ld + k] = (i == k) ? 1.0 : 0.0;
  int hi = n - 1;
  int iter = 0;
  const double eps = 2.220446049250313e-16;
  while (hi > 0) {
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
    if (++iter > 60 * n) return 0;
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * sqrt(delta * delta + eh * eh);
    const double mu = (den != 0.0) ? d[hi] - eh * eh / den : d[hi];
    double x = d[lo] - mu;
    double z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) { c = x / r; s = -z / r; }
      if (k > lo) e[k - 1] = r;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
      if (k + 1 < hi) {
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      for (int i = 0; i < n; ++i) {
        const double a0 = u[i * ld + k], a1 = u[i * ld + k + 1];
        u[i * ld + k] = c * a0 - s * a1;
        u[i * ld + k + 1] = s * a0 + c * a1;
      }
    }
  }
  return 1;
}

// Same iteration, applying every rotation to the columns of a given nrows x n matrix P
// (row-major, leading dimension ld): on return d holds the eigenvalues and P has become
// P U, U the eigenvector matrix of the tridiagonal. Returns 0 if it did not converge.
MBD_HD int tridiag_eigen_rows(double* d, double* e, double* P, int n, int nrows, int ld) {
  int hi = n - 1;
  int iter = 0;
  const double eps = 2.220446049250313e-16;
  while (hi > 0) {
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
    if (++iter > 60 * n) return 0;
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * sqrt(delta * delta + eh * eh);
    const double mu = (den != 0.0) ? d[hi] - eh * eh / den : d[hi];
    double x = d[lo] - mu;
    double z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) { c = x / r; s = -z / r; }
      if (k > lo) e[k - 1] = r;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
      if (k + 1 < hi) {
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      for (int i = 0; i < nrows; ++i) {
        const double a0 = P[i * ld + k], a1 = P[i * ld + k + 1];
        P[i * ld + k] = c * a0 - s * a1;
        P[i * ld + k + 1] = s * a0 + c * a1;
      }
    }
  }
  return 1;
}

// Adjoint of the Gauss quadrature Q = e1^T sqrt(T) e1 with respect to the
// tridiagonal T = U diag(theta) U^T: dQ/dT = U (F o c c^T) U^T with c = U^T e1 and the
// divided differences F_ij = 1 / (sqrt(theta_i) + sqrt(theta_j)) of the square root
// (Daleckii-Krein). Returns abar[k] = dQ/dT_kk and bbar[k] = dQ/dT_{k-1,k} +
// dQ/dT_{k,k-1} for k >= 1 (bbar[0] = 0). u (ld >= n) and theta come from
// tridiag_eigen; work needs 2 n doubles.
MBD_HD void tridiag_sqrt_adjoint(const double* theta, const double* u, int n, int ld,
                                 double* work, double* abar, double* bbar) {
  double* sq = work;
  double* v = work + n;
  for (int i = 0; i < n; ++i) sq[i] = sqrt(theta[i] > 0.0 ? theta[i] : 0.0);
  for (int k = 0; k < n; ++k) {
    // v = (F o c c^T) U[k, :]^T, with c = U[0, :]
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) {
        const double den = sq[i] + sq[j];
        acc += (den > 0.0 ? 1.0 / den : 0.0) * u[j] * u[k * ld + j];
      }
      v[i] = acc * u[i];
    }
    double mkk = 0.0, mkm = 0.0;
    for (int i = 0; i < n; ++i) {
      mkk += u[k * ld + i] * v[i];
      if (k > 0) mkm += u[(k - 1) * ld + i] * v[i];
    }
    abar[k] = mkk;
    bbar[k] = (k > 0) ? 2.0 * mkm : 0.0;
  }
}

// Screening tensor of the range-separated SCS, T_SR = (1 - f) T_GG = A I - B r r^T, at
// squared distance r2 for a pair with sigma_ij^2 = sig2, damping radius S and steepness d:
//   1 - f = 1 / (1 + exp(d (r / S - 1))),
//   A = (1 - f) (erf z - c) / r^3,  B = (1 - f) (3 erf z - c (3 + 2 z^2)) / r^5,
//   z^2 = r2 / sig2,  c = (2 / sqrt pi) z exp(-z^2).
// Beyond r = 7 sigma_ij, erf z = 1 and c (3 + 2 z^2) < 1e-18, so the bare tensor is used
// (identical in float64).
MBD_HD void scs_kernel(double r2, double sig2, double S, double d, double& A, double& B) {
  const double r = sqrt(r2);
  const double omf = 1.0 / (1.0 + exp(d * (r / S - 1.0)));
  const double z2 = r2 / sig2;
  const double ir2 = 1.0 / r2;
  const double ir3 = ir2 / r;
  A = omf * ir3;
  B = 3.0 * omf * ir3 * ir2;
  if (z2 < 49.0) {
    const double z = sqrt(z2);
    const double c = 1.1283791670955126 * z * exp(-z2);
    const double er = erf(z);
    A = omf * (er - c) * ir3;
    B = omf * (3.0 * er - c * (3.0 + 2.0 * z2)) * ir3 * ir2;
  }
}

// Gauss-Legendre rule on [-1, 1]: the nodes are the roots of the Legendre polynomial
// P_n, found by Newton's method from the asymptotic guesses cos(pi (i + 3/4) / (n + 1/2));
// P_n and P_n' come from the three-term recurrence (j + 1) P_{j+1} = (2j + 1) x P_j - j P_{j-1}
// and P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1); the weights are 2 / ((1 - x^2) P_n'(x)^2).
// Nodes are returned in ascending order.
inline void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double pm = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * pm) / j;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      const double dz = p0 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    x[i] = -z;  // the guesses descend from 1; their negatives ascend (the rule is symmetric)
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace mbd
