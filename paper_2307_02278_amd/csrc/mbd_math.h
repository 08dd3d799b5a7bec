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

}  // namespace mbd
