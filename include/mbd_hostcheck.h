/*
 * mbd_hostcheck.h - the scalar mathematics of the GPU kernels, compiled for the CPU.
 *
 * For CPU-side checks only (libmbd_hostcheck.so): these functions run the exact
 * host+device source the kernels use, on the host, so that it can be compared
 * with an independent reference without a GPU. All pointers are host memory
 * owned by the caller. No function here touches a device.
 */
#ifndef MBD_HOSTCHECK_H
#define MBD_HOSTCHECK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Output number n of the SplitMix64 stream seeded with `seed` (probe signs, eq. dds). */
uint64_t mbdh_splitmix(uint64_t seed, uint64_t n);

/* B-spline weights th[t] = M_p(w + t), dth[t] = M_p'(w + t), t = 0..p-1, p in {4,6,8},
 * w in [0, 1) (interpolation of eq. scaledfractional / spme). Returns 0, or -1 for bad p. */
int32_t mbdh_bspline(int32_t p, double w, double* th, double* dth);

/* Direct-space kernel T_dir = A I - B r r^T at distance^2 r2 (eq. fld_ewald with the
 * damping correction), in double (prec 0) or single (prec 1) precision. */
void mbdh_direct_kernel(int32_t prec, double r2, double tau, double inv_s, double damp_d,
                        double* A, double* B);

/* Gauss quadrature sum_k U_1k^2 sqrt(theta_k) of the symmetric tridiagonal with diagonal
 * a[0..n-1] and off-diagonal b[0..n-2] (eqs. sl3, tridiag2). Inputs are not modified;
 * theta_min receives the smallest eigenvalue; returns 1 on convergence, else 0. */
int32_t mbdh_tridiag_quadrature(const double* a, const double* b, int32_t n, double* q,
                                double* theta_min);

/* As mbdh_bspline, plus ddth[t] = M_p''(w + t) (B-spline second derivatives, used for forces). */
int32_t mbdh_bspline2(int32_t p, double w, double* th, double* dth, double* ddth);

/* Direct-space kernel and its radial derivatives in double precision: A, B as in
 * mbdh_direct_kernel and dA_r = A'(r) / r, dB_r = B'(r) / r (pair forces). */
void mbdh_direct_kernel_grad(double r2, double tau, double inv_s, double damp_d, double* A,
                             double* B, double* dA_r, double* dB_r);

/* Adjoint of the Gauss quadrature of the tridiagonal (a, b) as above: abar[k] = dQ/da_k and
 * bbar[k] = dQ/db_{k-1} for k >= 1 (bbar[0] = 0), where b_{k-1} couples rows k-1 and k.
 * Returns 1 on convergence, else 0. */
int32_t mbdh_tridiag_adjoint(const double* a, const double* b, int32_t n, double* abar,
                             double* bbar);

/* Gauss-Legendre nodes x[0..n-1] (ascending) and weights w[0..n-1] on [-1, 1], n >= 1: the
 * rule behind the imaginary-frequency grid of mbd_scs. */
void mbdh_gauss_legendre(int32_t n, double* x, double* w);

/* Screening tensor of mbd_scs, T_SR = (1 - f) T_GG = A I - B r r^T, at squared distance r2,
 * sigma_ij^2 = sig2, damping radius S = beta (R_i + R_j) and steepness d. */
void mbdh_scs_kernel(double r2, double sig2, double S, double d, double* A, double* B);

#ifdef __cplusplus
}
#endif

#endif
