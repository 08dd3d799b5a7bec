// Host-side entry points that run the kernels' scalar math on the CPU.
#include "../../include/mbd_hostcheck.h"

#include <vector>

#include "mbd_math.h"

extern "C" {

uint64_t mbdh_splitmix(uint64_t seed, uint64_t n) { return mbd::splitmix_at(seed, n); }

int32_t mbdh_bspline(int32_t p, double w, double* th, double* dth) {
  switch (p) {
    case 4: mbd::bspline_weights<4>(w, th, dth); return 0;
    case 6: mbd::bspline_weights<6>(w, th, dth); return 0;
    case 8: mbd::bspline_weights<8>(w, th, dth); return 0;
    default: return -1;
  }
}

void mbdh_direct_kernel(int32_t prec, double r2, double tau, double inv_s, double damp_d,
                        double* A, double* B) {
  if (prec == 1) {
    float a, b;
    mbd::direct_kernel<float>((float)r2, (float)tau, (float)inv_s, (float)damp_d, a, b);
    *A = a;
    *B = b;
  } else {
    mbd::direct_kernel<double>(r2, tau, inv_s, damp_d, *A, *B);
  }
}

int32_t mbdh_tridiag_quadrature(const double* a, const double* b, int32_t n, double* q,
                                double* theta_min) {
  std::vector<double> d(a, a + n), e(n, 0.0), z(n);
  for (int k = 0; k + 1 < n; ++k) e[k] = b[k];
  int ok = 0;
  *q = mbd::tridiag_sqrt_quadrature(d.data(), e.data(), z.data(), n, theta_min, &ok);
  return ok;
}

int32_t mbdh_bspline2(int32_t p, double w, double* th, double* dth, double* ddth) {
  switch (p) {
    case 4: mbd::bspline_weights2<4>(w, th, dth, ddth); return 0;
    case 6: mbd::bspline_weights2<6>(w, th, dth, ddth); return 0;
    case 8: mbd::bspline_weights2<8>(w, th, dth, ddth); return 0;
    default: return -1;
  }
}

void mbdh_direct_kernel_grad(double r2, double tau, double inv_s, double damp_d, double* A,
                             double* B, double* dA_r, double* dB_r) {
  mbd::direct_kernel_grad(r2, tau, inv_s, damp_d, *A, *B, *dA_r, *dB_r);
}

int32_t mbdh_tridiag_adjoint(const double* a, const double* b, int32_t n, double* abar,
                             double* bbar) {
  std::vector<double> d(a, a + n), e(n, 0.0), u((size_t)n * n), work(2 * (size_t)n);
  for (int k = 0; k + 1 < n; ++k) e[k] = b[k];
  if (!mbd::tridiag_eigen(d.data(), e.data(), u.data(), n, n)) return 0;
  mbd::tridiag_sqrt_adjoint(d.data(), u.data(), n, n, work.data(), abar, bbar);
  return 1;
}

void mbdh_gauss_legendre(int32_t n, double* x, double* w) { mbd::gauss_legendre(n, x, w); }

void mbdh_scs_kernel(double r2, double sig2, double S, double d, double* A, double* B) {
  mbd::scs_kernel(r2, sig2, S, d, *A, *B);
}

}  // extern "C"
