// Lanczos recurrence, Gauss quadrature and energy in double precision
// (eqs. hutch, dds, recurs2, sl3, sl4, plasmonic2; Algorithms 1 and 2).
//
// The Krylov vectors are kept unnormalized: w_0 = v (||v|| = 1), and with
// nrm_k = ||w_k||, y_k = w_k / nrm_k, l~_k = C w_k,
//   a_k     = (w_k . l~_k) / nrm_k^2
//   w_{k+1} = l~_k / nrm_k - a_k w_k / nrm_k - nrm_k w_{k-1} / nrm_{k-1}
// which is the three-term recurrence b_{k+1} y_{k+1} = l_k - a_k y_k - b_k y_{k-1}
// with b_{k+1} = nrm_{k+1}; the generalized dipoles of the next step are
// d = g * w_{k+1} (stored in the SPME precision). Every reduction over atoms is
// done in a fixed order (per-block partial sums, then one block per RHS).
#include "common.h"
#include "mbd_math.h"

namespace mbd {

namespace {

// Block layout for [n][3][B] element-wise kernels: RB lanes over right-hand
// sides, 256 / RB rows over (atom, component); blockIdx.y selects the RHS group.
template <int RB>
struct RowLayout {
  static constexpr int ROWS = 256 / RB;
};

__device__ __forceinline__ void block_reduce_rows(double* red, int rb_lanes, int rows) {
  const int lane = threadIdx.x % rb_lanes;
  const int row = threadIdx.x / rb_lanes;
  for (int h = rows / 2; h > 0; h >>= 1) {
    if (row < h) red[threadIdx.x] += red[threadIdx.x + h * rb_lanes];
    __syncthreads();
  }
  (void)lane;
}

template <int RB>
__global__ void __launch_bounds__(256)
k_probes(int n, int B, int nb, int probe0, uint64_t zs, const int* __restrict__ perm,
         const double* __restrict__ g, double* __restrict__ w0, double* __restrict__ dtmp,
         float* __restrict__ df, int use_float) {
  constexpr int ROWS = 256 / RB;
  const int b = blockIdx.y * RB + threadIdx.x % RB;
  const int row0 = blockIdx.x * ROWS + threadIdx.x / RB;
  if (b >= B) return;
  const uint64_t D = 3ull * (uint64_t)n;
  const double inv = 1.0 / sqrt((double)D);
  for (int row = row0; row < 3 * n; row += gridDim.x * ROWS) {
    const int s = row / 3, a = row % 3;
    double v = 0.0;
    if (b < nb) {
      const uint64_t l = (uint64_t)(probe0 + b);
      const uint64_t idx = l * D + 3ull * (uint64_t)perm[s] + (uint64_t)a;
      const uint64_t h = splitmix_at(zs, idx);
      v = (h >> 63) ? -inv : inv;
    }
    const size_t o = (size_t)row * B + b;
    w0[o] = v;
    const double d = g[s] * v;
    if (use_float) df[o] = (float)d; else dtmp[o] = d;
  }
}

template <int RB>
__global__ void __launch_bounds__(256)
k_update(int n, int B, int nb, int k, int m, int probe0, const double* __restrict__ lt,
         const double* __restrict__ wk, const double* __restrict__ wkm1,
         const double* __restrict__ a, const double* __restrict__ nrm,
         const int* __restrict__ meff, const double* __restrict__ g, double* __restrict__ wn,
         double* __restrict__ dtmp, float* __restrict__ df, int use_float, int write_d,
         double* __restrict__ part) {
  constexpr int ROWS = 256 / RB;
  __shared__ double red[256];
  const int lane = threadIdx.x % RB;
  const int b = blockIdx.y * RB + lane;
  const int row0 = blockIdx.x * ROWS + threadIdx.x / RB;
  double ss = 0.0;
  if (b < B) {
    bool live = false;
    double c_l = 0.0, c_k = 0.0, c_km1 = 0.0;
    if (b < nb) {
      const int l = probe0 + b;
      live = meff[l] > k;  // w_{k+1} is needed only while the probe has not broken down
      const double nk = nrm[l * m + k];
      c_l = 1.0 / nk;
      c_k = a[l * m + k] / nk;
      c_km1 = (k > 0) ? nk / nrm[l * m + k - 1] : 0.0;
    }
    for (int row = row0; row < 3 * n; row += gridDim.x * ROWS) {
      const size_t o = (size_t)row * B + b;
      double v = 0.0;
      if (live) {
        v = c_l * lt[o] - c_k * wk[o];
        if (k > 0) v -= c_km1 * wkm1[o];
      }
      wn[o] = v;
      ss += v * v;
      if (write_d) {
        const double d = g[row / 3] * v;
        if (use_float) df[o] = (float)d; else dtmp[o] = d;
      }
    }
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  block_reduce_rows(red, RB, ROWS);
  if (threadIdx.x < RB && b < B) part[((size_t)blockIdx.x * kPartSlots + 1) * B + b] = red[threadIdx.x];
}

// Dot products of w with earlier Krylov vectors for re-orthogonalization:
// coef[b][j] partials of (w . w_j) for j in [j0, j1), written to part slot 2.. via a
// separate pass per j (the count is small: 2 for LOCAL).
template <int RB>
__global__ void __launch_bounds__(256)
k_dot(int n, int B, const double* __restrict__ x, const double* __restrict__ y,
      double* __restrict__ part, int slot) {
  constexpr int ROWS = 256 / RB;
  __shared__ double red[256];
  const int lane = threadIdx.x % RB;
  const int b = blockIdx.y * RB + lane;
  const int row0 = blockIdx.x * ROWS + threadIdx.x / RB;
  double ss = 0.0;
  if (b < B)
    for (int row = row0; row < 3 * n; row += gridDim.x * ROWS) {
      const size_t o = (size_t)row * B + b;
      ss += x[o] * y[o];
    }
  red[threadIdx.x] = ss;
  __syncthreads();
  block_reduce_rows(red, RB, ROWS);
  if (threadIdx.x < RB && b < B) part[((size_t)blockIdx.x * kPartSlots + slot) * B + b] = red[threadIdx.x];
}

// Sum the per-block partials of one slot for each RHS, in a fixed order.
__global__ void __launch_bounds__(256)
k_sum_slot(int B, int slot, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < kRedBlocks; k += 256) s += part[((size_t)k * kPartSlots + slot) * B + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

// w <- w - sum_j c_j w_j with c_j = (w . w_j) / nrm_j^2 for the listed j; then the
// norm partials and (optionally) the dipoles.
template <int RB>
__global__ void __launch_bounds__(256)
k_orth_apply(int n, int B, int nb, int m, int probe0, const double* __restrict__ W,
             size_t vstride, int j0, int j1, const double* __restrict__ dots,
             const double* __restrict__ nrm, const int* __restrict__ meff, int k,
             const double* __restrict__ g, double* __restrict__ w, double* __restrict__ dtmp,
             float* __restrict__ df, int use_float, double* __restrict__ part) {
  constexpr int ROWS = 256 / RB;
  __shared__ double red[256];
  const int lane = threadIdx.x % RB;
  const int b = blockIdx.y * RB + lane;
  const int row0 = blockIdx.x * ROWS + threadIdx.x / RB;
  double ss = 0.0;
  if (b < B) {
    double c[kMaxSteps < 64 ? kMaxSteps : 64];
    const int nj = j1 - j0;
    bool live = false;
    if (b < nb) {
      const int l = probe0 + b;
      live = meff[l] > k;
      for (int j = 0; j < nj; ++j) {
        const double nj2 = nrm[l * m + j0 + j];
        c[j] = dots[(size_t)j * B + b] / (nj2 * nj2);
      }
    }
    for (int row = row0; row < 3 * n; row += gridDim.x * ROWS) {
      const size_t o = (size_t)row * B + b;
      double v = w[o];
      if (live)
        for (int j = 0; j < nj; ++j) v -= c[j] * W[(size_t)(j0 + j) * vstride + o];
      else
        v = 0.0;
      w[o] = v;
      ss += v * v;
      const double d = g[row / 3] * v;
      if (use_float) df[o] = (float)d; else dtmp[o] = d;
    }
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  block_reduce_rows(red, RB, ROWS);
  if (threadIdx.x < RB && b < B) part[((size_t)blockIdx.x * kPartSlots + 1) * B + b] = red[threadIdx.x];
}

// a_k from the epilogue partials (slot 0).
__global__ void k_finish_a(int B, int nb, int k, int m, int probe0, const double* __restrict__ sums,
                           const double* __restrict__ nrm, double* __restrict__ a,
                           const int* __restrict__ meff, uint32_t* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int l = probe0 + b;
  if (meff[l] <= k) return;
  const double nk = nrm[l * m + k];
  const double v = sums[b] / (nk * nk);
  a[l * m + k] = v;
  if (!isfinite(v)) atomicOr(status, kErrNonfinite);
}

// nrm_{k+1} from the update partials (slot 1); breakdown truncates the tridiagonal.
__global__ void k_finish_norm(int B, int nb, int k, int m, int probe0,
                              const double* __restrict__ sums, double* __restrict__ nrm,
                              const double* __restrict__ a, int* __restrict__ meff,
                              uint32_t* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int l = probe0 + b;
  if (meff[l] <= k) return;
  const double v = sqrt(sums[b]);
  nrm[l * m + k + 1] = v;
  const double scale = fmax(fabs(a[l * m + k]), nrm[l * m + k]);
  if (!isfinite(v)) atomicOr(status, kErrNonfinite);
  if (!(v > 1e-12 * scale)) meff[l] = k + 1;
}

__global__ void k_init_probe_scalars(int nb, int m, int probe0, double* __restrict__ nrm,
                                     double* __restrict__ a, int* __restrict__ meff) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int l = probe0 + b;
  for (int k = 0; k < m; ++k) {
    nrm[l * m + k] = 0.0;
    a[l * m + k] = 0.0;
  }
  nrm[l * m] = 1.0;
  meff[l] = m;
}

// Gauss quadrature per probe from its tridiagonal (implicit QR, first-row tracking):
// one work-group per probe, its working arrays in LDS (the iteration is sequential and
// runs on lane 0; LDS instead of private arrays avoids scratch-memory latency).
__global__ void __launch_bounds__(64)
k_tridiag(int m, int probe0, const double* __restrict__ a, const double* __restrict__ nrm,
          const int* __restrict__ meff, double* __restrict__ q, uint32_t* __restrict__ status) {
  __shared__ double d[kMaxSteps], e[kMaxSteps], z[kMaxSteps];
  const int l = probe0 + blockIdx.x;
  const int n = meff[l];
  for (int k = threadIdx.x; k < n; k += 64) {
    d[k] = a[l * m + k];
    e[k] = (k + 1 < n) ? nrm[l * m + k + 1] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tmin;
  int ok;
  const double v = tridiag_sqrt_quadrature(d, e, z, n, &tmin, &ok);
  q[l] = v;
  if (!ok) atomicOr(status, kErrNoConverge);
  if (!(tmin > 0.0)) atomicOr(status, kErrNotPosdef);
  if (!isfinite(v)) atomicOr(status, kErrNonfinite);
}

// E = 1/2 (3N / R) sum_l Q_l - 3/2 sum_i omega_i, summed in probe order.
__global__ void k_energy(int n, int R, const double* __restrict__ q,
                         const double* __restrict__ g, const double* __restrict__ om2,
                         double* __restrict__ out, double* __restrict__ sd_out,
                         uint32_t* __restrict__ status) {
  __shared__ double red[256];
  double so = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) so += sqrt(om2[i]);
  red[threadIdx.x] = so;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sq = 0.0;
    for (int l = 0; l < R; ++l) sq += q[l];
    const double E = 0.5 * (3.0 * n / R) * sq - 1.5 * red[0];
    out[0] = E;
    if (!isfinite(E)) atomicOr(status, kErrNonfinite);
    if (sd_out) {
      // spread of the R samples of the trace estimator (two passes, fixed order)
      const double mean = sq / R;
      double ss = 0.0;
      for (int l = 0; l < R; ++l) ss += (q[l] - mean) * (q[l] - mean);
      sd_out[0] = R > 1 ? 0.5 * (3.0 * n) * sqrt(ss / (R - 1)) / sqrt((double)R)
                        : __builtin_nan("");
    }
  }
  (void)g;
}

// Caller layout [nrhs][N][3] (caller atom order) <-> internal [n][3][B] (sorted).
__global__ void k_pack(int n, int nrhs, int B, const int* __restrict__ perm,
                       const double* __restrict__ v, const double* __restrict__ g,
                       double* __restrict__ w, double* __restrict__ dtmp,
                       float* __restrict__ df, int use_float) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)3 * n * B) return;
  const int b = (int)(t % B);
  const long row = t / B;
  const int s = (int)(row / 3), a = (int)(row % 3);
  const double x = (b < nrhs) ? v[((size_t)b * n + perm[s]) * 3 + a] : 0.0;
  w[t] = x;
  const double d = g[s] * x;
  if (use_float) df[t] = (float)d; else dtmp[t] = d;
}

__global__ void k_unpack(int n, int nrhs, int B, const int* __restrict__ perm,
                         const double* __restrict__ lt, double* __restrict__ out) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)3 * n * B) return;
  const int b = (int)(t % B);
  if (b >= nrhs) return;
  const long row = t / B;
  const int s = (int)(row / 3), a = (int)(row % 3);
  out[((size_t)b * n + perm[s]) * 3 + a] = lt[t];
}


// ---------------------------------------------------------------------------
// Forces: reverse sweep through the recurrence (derivative of the fixed-probe
// estimator). In terms of y_k = w_k / nrm_k, l_k = C y_k, b_k = nrm_k:
//   w_{k+1} = l_k - a_k y_k - b_k y_{k-1},  y_{k+1} = w_{k+1} / b_{k+1},  a_k = y_k . l_k.
// Going back from k = m-1 with the adjoints abar_k = dQ/da_k, bbar_k = dQ/db_k of the
// quadrature and ybar (adjoint of y):
//   wbar  = (ybar_{k+1} - (ybar_{k+1} . y_{k+1}) y_{k+1}) / b_{k+1} + bbar_{k+1} y_{k+1}
//   abar_k -= wbar . y_k,  bbar_k -= wbar . y_{k-1}
//   lbar_k = wbar + abar_k y_k
//   ybar_k += -a_k wbar + abar_k l_k + C lbar_k,  ybar_{k-1} += -b_k wbar
// and dQ/dR = sum_k lbar_k^T (dC/dR) y_k. l_k is rebuilt from the recurrence
// (l_k = w_{k+1} + a_k y_k + b_k y_{k-1}); the last one is the stored C w_{m-1}.
// Re-orthogonalization corrections are not differentiated.
// ---------------------------------------------------------------------------

// Per probe (one 64-lane work-group each): eigenvectors of its tridiagonal by the
// implicit symmetric QR iteration with Wilkinson shift, then the quadrature adjoint
// dQ/dT = U (F o c c^T) U^T, c = U^T e1, F_ij = 1 / (sqrt(theta_i) + sqrt(theta_j)).
// Lane 0 deflates and computes the Givens rotations of one sweep into LDS; every lane
// then applies them to its own rows of U (rows never move between lanes, so no other
// synchronization is needed). The adjoint's O(m^3) sums are split over the lanes.
__global__ void __launch_bounds__(64)
k_tridiag_adjoint(int m, int probe0, const double* __restrict__ a,
                  const double* __restrict__ nrm, const int* __restrict__ meff,
                  double* __restrict__ tz, double* __restrict__ abar, double* __restrict__ bbar,
                  uint32_t* __restrict__ status) {
  __shared__ double d[kMaxSteps], e[kMaxSteps], cs[kMaxSteps], sn[kMaxSteps];
  __shared__ int ctl[3];  // lo, hi, state (0 sweep, 1 done, 2 no convergence)
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int l = probe0 + b;
  const int n = meff[l];
  double* u = tz + (size_t)b * m * m;
  double* ab = abar + (size_t)b * m;
  double* bb = bbar + (size_t)b * m;
  for (int k = lane; k < m; k += 64) {
    ab[k] = 0.0;
    bb[k] = 0.0;
    if (k < n) {
      d[k] = a[l * m + k];
      e[k] = (k + 1 < n) ? nrm[l * m + k + 1] : 0.0;
    }
  }
  for (int i = lane; i < n; i += 64)
    for (int k = 0; k < n; ++k) u[(size_t)i * m + k] = (i == k) ? 1.0 : 0.0;
  if (lane == 0) ctl[1] = n - 1;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  int iter = 0;
  while (true) {
    if (lane == 0) {
      int hi = ctl[1], st = 0;
      while (hi > 0 && fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
        e[hi - 1] = 0.0;
        --hi;
      }
      if (hi <= 0) {
        st = 1;
      } else if (++iter > 60 * n) {
        st = 2;
      } else {
        int lo = hi - 1;
        while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * sqrt(delta * delta + eh * eh);
        const double mu = (den != 0.0) ? d[hi] - eh * eh / den : d[hi];
        double x = d[lo] - mu;
        double z = e[lo];
        for (int k = lo; k < hi; ++k) {
          const double r = hypot(x, z);
          double c = 1.0, sg = 0.0;
          if (r != 0.0) { c = x / r; sg = -z / r; }
          if (k > lo) e[k - 1] = r;
          const double dk = d[k], dk1 = d[k + 1], ek = e[k];
          d[k] = c * c * dk - 2.0 * c * sg * ek + sg * sg * dk1;
          d[k + 1] = sg * sg * dk + 2.0 * c * sg * ek + c * c * dk1;
          e[k] = c * sg * (dk - dk1) + (c * c - sg * sg) * ek;
          if (k + 1 < hi) {
            z = -sg * e[k + 1];
            e[k + 1] = c * e[k + 1];
            x = e[k];
          }
          cs[k] = c;
          sn[k] = sg;
        }
        ctl[0] = lo;
      }
      ctl[1] = hi;
      ctl[2] = st;
    }
    __syncthreads();
    const int st = ctl[2];
    if (st != 0) break;
    const int lo = ctl[0], hi = ctl[1];
    for (int i = lane; i < n; i += 64) {
      double* ui = u + (size_t)i * m;
      for (int k = lo; k < hi; ++k) {
        const double a0 = ui[k], a1 = ui[k + 1];
        ui[k] = cs[k] * a0 - sn[k] * a1;
        ui[k + 1] = sn[k] * a0 + cs[k] * a1;
      }
    }
    __syncthreads();
  }
  if (ctl[2] == 2) {
    if (lane == 0) atomicOr(status, kErrNoConverge);
    return;
  }
  // eigenvalues d, eigenvectors in the columns of u; sqrt(theta) into cs
  for (int k = lane; k < n; k += 64) {
    if (!(d[k] > 0.0)) atomicOr(status, kErrNotPosdef);
    cs[k] = sqrt(d[k] > 0.0 ? d[k] : 0.0);
  }
  __syncthreads();
  const double* c0 = u;  // first row: c_j = U_0j
  for (int k = lane; k < n; k += 64) {
    const double* uk = u + (size_t)k * m;
    const double* ukm = k > 0 ? u + (size_t)(k - 1) * m : uk;
    double mkk = 0.0, mkm = 0.0;
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) {
        const double den = cs[i] + cs[j];
        acc += (den > 0.0 ? 1.0 / den : 0.0) * c0[j] * uk[j];
      }
      const double v = acc * c0[i];
      mkk += uk[i] * v;
      mkm += ukm[i] * v;
    }
    ab[k] = mkk;
    bb[k] = k > 0 ? 2.0 * mkm : 0.0;
  }
}

// Five dot products per right-hand side into partial slots 0..4:
//   ybar_{k+1}.w_{k+1}, ybar_{k+1}.w_k, ybar_{k+1}.w_{k-1}, w_{k+1}.w_k, w_{k+1}.w_{k-1}.
template <int RB>
__global__ void __launch_bounds__(256)
k_adj_dots(int n, int B, const double* __restrict__ yn, const double* __restrict__ wn,
           const double* __restrict__ wk, const double* __restrict__ wkm1, int has_km1,
           double* __restrict__ part) {
  constexpr int ROWS = 256 / RB;
  __shared__ double red[256];
  const int lane = threadIdx.x % RB;
  const int b = blockIdx.y * RB + lane;
  const int row0 = blockIdx.x * ROWS + threadIdx.x / RB;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (b < B)
    for (int row = row0; row < 3 * n; row += gridDim.x * ROWS) {
      const size_t o = (size_t)row * B + b;
      const double y = yn[o], w1 = wn[o], w0 = wk[o];
      const double wm = has_km1 ? wkm1[o] : 0.0;
      s[0] += y * w1;
      s[1] += y * w0;
      s[2] += y * wm;
      s[3] += w1 * w0;
      s[4] += w1 * wm;
    }
  for (int q = 0; q < 5; ++q) {
    red[threadIdx.x] = s[q];
    __syncthreads();
    block_reduce_rows(red, RB, ROWS);
    if (threadIdx.x < RB && b < B)
      part[((size_t)blockIdx.x * kPartSlots + q) * B + b] = red[threadIdx.x];
    __syncthreads();
  }
}

// Per-probe scalars of step k from the dot sums (sums[q * B + b]); updates abar_k and
// bbar_k in place and writes the coefficients of the element-wise update:
//   c[0] ybar_{k+1} + c[1] w_{k+1} = wbar;  lbar = wbar + c[2] w_k;
//   l_k = w_{k+1} + c[3] w_k + c[4] w_{k-1} (k < m-1) or c[5] Lt (k = m-1);
//   ybar_k += c[6] wbar + c[7] l_k;  ybar_{k-1} += c[8] wbar;  q = g c[9] w_k.
__global__ void k_adj_scalars(int B, int nb, int k, int m, int probe0,
                              const double* __restrict__ sums, const double* __restrict__ a,
                              const double* __restrict__ nrm, const int* __restrict__ meff,
                              double* __restrict__ abar, double* __restrict__ bbar,
                              double* __restrict__ coef) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double* c = coef + (size_t)b * 16;
  for (int q = 0; q < 16; ++q) c[q] = 0.0;
  if (b >= nb) return;
  const int l = probe0 + b;
  const int me = meff[l];
  if (k >= me) return;
  const double nk = nrm[l * m + k];
  const double nkm1 = k > 0 ? nrm[l * m + k - 1] : 1.0;
  double c0 = 0.0, c1 = 0.0, wy_k = 0.0, wy_km1 = 0.0;
  if (k + 1 < me) {
    const double beta = nrm[l * m + k + 1];
    const double sa = sums[0 * B + b] / beta;
    const double sb = sums[1 * B + b] / nk;
    const double sc = k > 0 ? sums[2 * B + b] / nkm1 : 0.0;
    const double sd = sums[3 * B + b] / (beta * nk);
    const double se = k > 0 ? sums[4 * B + b] / (beta * nkm1) : 0.0;
    const double al1 = 1.0 / beta;
    const double al2 = bbar[(size_t)b * m + k + 1] - sa / beta;
    c0 = al1;
    c1 = al2 / beta;
    wy_k = al1 * sb + al2 * sd;
    wy_km1 = al1 * sc + al2 * se;
  }
  const double ab = abar[(size_t)b * m + k] - wy_k;
  abar[(size_t)b * m + k] = ab;
  if (k > 0) bbar[(size_t)b * m + k] -= wy_km1;
  const double ak = a[l * m + k];
  c[0] = c0;
  c[1] = c1;
  c[2] = ab / nk;
  c[3] = ak / nk;
  c[4] = k > 0 ? nk / nkm1 : 0.0;
  c[5] = 1.0 / nk;
  c[6] = -ak;
  c[7] = ab;
  c[8] = -nk;
  c[9] = 1.0 / nk;
}

template <int RB>
__global__ void __launch_bounds__(256)
k_adj_update(int n, int B, int k, int m, const double* __restrict__ coef,
             const double* __restrict__ wn, const double* __restrict__ wk,
             const double* __restrict__ wkm1, const double* __restrict__ lt,
             const double* __restrict__ g, double* __restrict__ yn, double* __restrict__ yc,
             double* __restrict__ yp, double* __restrict__ lbar, double* __restrict__ pd,
             float* __restrict__ pf, double* __restrict__ qd, float* __restrict__ qf,
             int use_float) {
  constexpr int ROWS = 256 / RB;
  const int lane = threadIdx.x % RB;
  const int b = blockIdx.y * RB + lane;
  const int row0 = blockIdx.x * ROWS + threadIdx.x / RB;
  if (b >= B) return;
  const double* c = coef + (size_t)b * 16;
  const double c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5], c6 = c[6],
               c7 = c[7], c8 = c[8], c9 = c[9];
  const bool last = (k + 1 == m);
  for (int row = row0; row < 3 * n; row += gridDim.x * ROWS) {
    const size_t o = (size_t)row * B + b;
    const double w0 = wk[o];
    double wbar = 0.0, lk;
    if (!last) {
      const double w1 = wn[o];
      wbar = c0 * yn[o] + c1 * w1;
      lk = w1 + c3 * w0 + (k > 0 ? c4 * wkm1[o] : 0.0);
    } else {
      lk = c5 * lt[o];
    }
    const double lb = wbar + c2 * w0;
    yc[o] += c6 * wbar + c7 * lk;
    if (k > 0) yp[o] += c8 * wbar;
    lbar[o] = lb;
    const double gs = g[row / 3];
    if (use_float) {
      pf[o] = (float)(gs * lb);
      qf[o] = (float)(gs * c9 * w0);
    } else {
      pd[o] = gs * lb;
      qd[o] = gs * c9 * w0;
    }
  }
}

__global__ void k_axpy_vec(size_t count, const double* __restrict__ x, double* __restrict__ y) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) y[t] += x[t];
}

__global__ void k_fill_double(double* __restrict__ p, double v, size_t count) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

// F = -dE/dR = -1/2 (3N / R) dsum/dR, back to caller order; dsum/dR is the sum of
// the reciprocal half and the direct (pair) half of fsum.
__global__ void k_forces_finish(int n, int R, const int* __restrict__ perm,
                                const double* __restrict__ fsum, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double sc = -0.5 * (3.0 * n / R);
  const int i = perm[s];
  for (int a = 0; a < 3; ++a)
    out[3 * i + a] = sc * (fsum[3 * s + a] + fsum[3 * ((size_t)n + s) + a]);
}

inline int rb_for(int B) { return B >= 64 ? 64 : B; }

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
#define MBD_RB_SWITCH(RBV, CALL)         \
  switch (RBV) {                         \
    case 1: { constexpr int RB = 1; CALL; } break;   \
    case 2: { constexpr int RB = 2; CALL; } break;   \
    case 4: { constexpr int RB = 4; CALL; } break;   \
    case 8: { constexpr int RB = 8; CALL; } break;   \
    case 16: { constexpr int RB = 16; CALL; } break; \
    case 32: { constexpr int RB = 32; CALL; } break; \
    default: { constexpr int RB = 64; CALL; } break; \
  }

void launch_probes(const Geometry& geo, const SysBuffers& b, int B, int nb, int probe0,
                   uint64_t seed, int system, bool use_float, hipStream_t st) {
  const uint64_t zs = splitmix_at(seed, (uint64_t)system);
  const int rb = rb_for(B);
  dim3 grd(kRedBlocks, (B + rb - 1) / rb);
  MBD_RB_SWITCH(rb, (k_probes<RB><<<grd, 256, 0, st>>>(geo.n, B, nb, probe0, zs, b.perm, b.g,
                                                       b.W, (double*)b.dv, (float*)b.dv,
                                                       use_float ? 1 : 0)));
}

void launch_init_scalars(const SysBuffers& b, int nb, int m, int probe0, hipStream_t st) {
  k_init_probe_scalars<<<(nb + 63) / 64, 64, 0, st>>>(nb, m, probe0, b.b, b.a, b.meff);
}

void launch_update(const Geometry& geo, const SysBuffers& b, int B, int nb, int k, int m,
                   int probe0, bool use_float, bool write_d, hipStream_t st) {
  const size_t vs = (size_t)geo.n * 3 * B;
  const int rb = rb_for(B);
  dim3 grd(kRedBlocks, (B + rb - 1) / rb);
  const double* wk = b.W + (size_t)k * vs;
  const double* wkm1 = k > 0 ? b.W + (size_t)(k - 1) * vs : b.W;
  double* wn = b.W + (size_t)(k + 1) * vs;
  MBD_RB_SWITCH(rb, (k_update<RB><<<grd, 256, 0, st>>>(
                         geo.n, B, nb, k, m, probe0, b.Lt, wk, wkm1, b.a, b.b, b.meff, b.g, wn,
                         (double*)b.dv, (float*)b.dv, use_float ? 1 : 0, write_d ? 1 : 0,
                         b.part)));
}

// Re-orthogonalize w_{k+1} against w_j for j in [j0, k] (classical Gram-Schmidt,
// in chunks of at most 64 earlier vectors).
void launch_reorth(const Geometry& geo, const SysBuffers& b, int B, int nb, int k, int m,
                   int probe0, int j0, bool use_float, hipStream_t st) {
  const size_t vs = (size_t)geo.n * 3 * B;
  const int rb = rb_for(B);
  dim3 grd(kRedBlocks, (B + rb - 1) / rb);
  double* w = b.W + (size_t)(k + 1) * vs;
  for (int c0 = j0; c0 <= k; c0 += 64) {
    const int c1 = (k + 1 < c0 + 64) ? k + 1 : c0 + 64;
    for (int j = c0; j < c1; ++j) {
      MBD_RB_SWITCH(rb, (k_dot<RB><<<grd, 256, 0, st>>>(geo.n, B, w, b.W + (size_t)j * vs,
                                                        b.part, 2)));
      k_sum_slot<<<B, 256, 0, st>>>(B, 2, b.part, b.coef + (size_t)(j - c0) * B);
    }
    MBD_RB_SWITCH(rb, (k_orth_apply<RB><<<grd, 256, 0, st>>>(
                           geo.n, B, nb, m, probe0, b.W, vs, c0, c1, b.coef, b.b, b.meff, k,
                           b.g, w, (double*)b.dv, (float*)b.dv, use_float ? 1 : 0, b.part)));
  }
}

void launch_finish_a(const SysBuffers& b, int B, int nb, int k, int m, int probe0,
                     uint32_t* status, hipStream_t st) {
  k_sum_slot<<<B, 256, 0, st>>>(B, 0, b.part, b.coef);
  k_finish_a<<<(nb + 63) / 64, 64, 0, st>>>(B, nb, k, m, probe0, b.coef, b.b, b.a, b.meff,
                                            status);
}

void launch_finish_norm(const SysBuffers& b, int B, int nb, int k, int m, int probe0,
                        uint32_t* status, hipStream_t st) {
  k_sum_slot<<<B, 256, 0, st>>>(B, 1, b.part, b.coef);
  k_finish_norm<<<(nb + 63) / 64, 64, 0, st>>>(B, nb, k, m, probe0, b.coef, b.b, b.a, b.meff,
                                               status);
}

void launch_tridiag(const SysBuffers& b, int nb, int m, int probe0, uint32_t* status,
                    hipStream_t st) {
  k_tridiag<<<nb, 64, 0, st>>>(m, probe0, b.a, b.b, b.meff, b.q, status);
}

void launch_energy(const Geometry& geo, const SysBuffers& b, int R, double* energy_out,
                   double* sd_out, uint32_t* status, hipStream_t st) {
  k_energy<<<1, 256, 0, st>>>(geo.n, R, b.q, b.g, b.om2, energy_out, sd_out, status);
}


void fill_double(double* p, double v, size_t n, hipStream_t st) {
  if (n == 0) return;
  k_fill_double<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, v, n);
}

void launch_tridiag_adjoint(const SysBuffers& b, int nb, int m, int probe0, uint32_t* status,
                            hipStream_t st) {
  k_tridiag_adjoint<<<nb, 64, 0, st>>>(m, probe0, b.a, b.b, b.meff, b.tz, b.abar, b.bbar,
                                       status);
}

// One reverse step k: dots, scalars and the element-wise update, which leaves lbar_k in
// b.lbar, g * lbar_k in b.dv and g * y_k in b.dq for the adjoint matvec and force terms.
void launch_adjoint_step(const Geometry& geo, const SysBuffers& b, int B, int nb, int k, int m,
                         int probe0, bool use_float, hipStream_t st) {
  const size_t vs = (size_t)geo.n * 3 * B;
  const int rb = rb_for(B);
  dim3 grd(kRedBlocks, (B + rb - 1) / rb);
  double* Y0 = b.ybar;
  double* yn = Y0 + (size_t)((k + 1) % 3) * vs;
  double* yc = Y0 + (size_t)(k % 3) * vs;
  double* yp = Y0 + (size_t)((k + 2) % 3) * vs;
  // ybar_{k-1} starts from zero (its buffer last held ybar_{k+2})
  fill_double(yp, 0.0, vs, st);
  const double* wk = b.W + (size_t)k * vs;
  const double* wn = (k + 1 < m) ? b.W + (size_t)(k + 1) * vs : wk;
  const double* wkm1 = k > 0 ? b.W + (size_t)(k - 1) * vs : wk;
  if (k + 1 < m) {
    MBD_RB_SWITCH(rb, (k_adj_dots<RB><<<grd, 256, 0, st>>>(geo.n, B, yn, wn, wk, wkm1,
                                                           k > 0 ? 1 : 0, b.part)));
    for (int q = 0; q < 5; ++q)
      k_sum_slot<<<B, 256, 0, st>>>(B, q, b.part, b.coef + (size_t)q * B);
  } else {
    fill_double(b.coef, 0.0, (size_t)5 * B, st);
  }
  k_adj_scalars<<<(B + 63) / 64, 64, 0, st>>>(B, nb, k, m, probe0, b.coef, b.a, b.b, b.meff,
                                              b.abar, b.bbar, b.adj);
  MBD_RB_SWITCH(rb, (k_adj_update<RB><<<grd, 256, 0, st>>>(
                         geo.n, B, k, m, b.adj, wn, wk, wkm1, b.Lt, b.g, yn, yc, yp, b.lbar,
                         (double*)b.dv, (float*)b.dv, (double*)b.dq, (float*)b.dq,
                         use_float ? 1 : 0)));
}

// ybar_k += C lbar_k (the adjoint matvec's output in b.Lt).
void launch_adjoint_accumulate(const Geometry& geo, const SysBuffers& b, int B, int k,
                               hipStream_t st) {
  const size_t vs = (size_t)geo.n * 3 * B;
  k_axpy_vec<<<(unsigned)((vs + 255) / 256), 256, 0, st>>>(vs, b.Lt,
                                                          b.ybar + (size_t)(k % 3) * vs);
}

void launch_forces_finish(const Geometry& geo, const SysBuffers& b, int R, double* forces,
                          hipStream_t st) {
  k_forces_finish<<<(geo.n + 255) / 256, 256, 0, st>>>(geo.n, R, b.perm, b.fsum, forces);
}

void launch_pack(const Geometry& geo, const SysBuffers& b, const double* v, int nrhs, int B,
                 bool use_float, hipStream_t st) {
  const long tot = (long)3 * geo.n * B;
  k_pack<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(geo.n, nrhs, B, b.perm, v, b.g, b.W,
                                                         (double*)b.dv, (float*)b.dv,
                                                         use_float ? 1 : 0);
}

void launch_unpack(const Geometry& geo, const SysBuffers& b, double* out, int nrhs, int B,
                   hipStream_t st) {
  const long tot = (long)3 * geo.n * B;
  k_unpack<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(geo.n, nrhs, B, b.perm, b.Lt, out);
}

}  // namespace mbd
