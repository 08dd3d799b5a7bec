// Block Lanczos quadrature: the recurrence of Algorithm 2 run on blocks of KB probes.
//
// The B right-hand sides of a plan hold B / KB independent Krylov blocks (columns
// [q KB, q KB + KB) form block q). With Y_k the orthonormal basis block of step k:
//   A_k = Y_k^T C Y_k (symmetrized),  W = C Y_k - Y_k A_k - Y_{k-1} B_{k-1}^T,
//   W = Y_{k+1} B_k by Cholesky QR applied twice (B_k upper triangular),
// and the probe block V = Y_0 R_0 the same way. The block tridiagonal T (diagonal
// blocks A_k, sub-diagonal blocks B_k) gives the per-probe values
//   Q_l = [R_0^T E_1^T sqrt(T) E_1 R_0]_ll,
// reduced by Householder tridiagonalization (tracking the first KB rows of the
// orthogonal factor) and the implicit QR iteration of the single-probe path, with its
// rotations applied to those rows. A residual block whose Cholesky pivot falls below
// (1e-10 s)^2, s = max_i (A_k)_ii, ends that Krylov block: T keeps the steps done and
// the later basis blocks are zero.
//
// Vectors are [3n][B] float64 (row = 3 atom + component, sorted atoms).
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "mbd_math.h"

namespace mbd {
namespace {

constexpr double kBlockBreakdown = 1e-10;

// part[blk][e] = sum over the block's rows of X[row][q KB + r1] Y[row][q KB + r2],
// e = (q KB + r1) KB + r2.
template <int KB>
__global__ void __launch_bounds__(256)
k_bgram(const double* __restrict__ X, const double* __restrict__ Y, int rows, int B,
        int rows_per_blk, double* __restrict__ part) {
  const int E = B * KB;
  const int r0 = blockIdx.x * rows_per_blk;
  const int r1 = min(rows, r0 + rows_per_blk);
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int q = e / (KB * KB), i = (e / KB) % KB, j = e % KB;
    const int cx = q * KB + i, cy = q * KB + j;
    double acc = 0.0;
    for (int r = r0; r < r1; ++r) acc += X[(size_t)r * B + cx] * Y[(size_t)r * B + cy];
    part[(size_t)blockIdx.x * E + e] = acc;
  }
}

__global__ void k_bgram_sum(const double* __restrict__ part, int nblk, int E,
                            double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * E + e];
  G[e] = s;
}

// A_k of every Krylov block: the symmetric part of the Gram matrix Y_k^T L.
template <int KB>
__global__ void k_bstore_a(const double* __restrict__ G, int nkb, double* __restrict__ A) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nkb * KB * KB) return;
  const int q = e / (KB * KB), i = (e / KB) % KB, j = e % KB;
  const double* g = G + (size_t)q * KB * KB;
  A[e] = 0.5 * (g[i * KB + j] + g[j * KB + i]);
}

// Cholesky G = R^T R of every block's Gram matrix (thread per Krylov block). Pass 1 of
// a QR: a pivot below (1e-10 s)^2 ends the block (flag, meff = step), with s = max_i
// (A_k)_ii the scale of the step when A is given, else s^2 = max diag G (probe block and
// pass 2). Pass 2: R1 = R2, and Racc (B_k or R_0) = R2 R1.
template <int KB>
__global__ void k_bchol(const double* __restrict__ G, const double* __restrict__ A, int nkb,
                        int pass, int step, double* __restrict__ R1, double* __restrict__ Racc,
                        int* __restrict__ flag, int* __restrict__ meff) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nkb) return;
  const double* g = G + (size_t)q * KB * KB;
  double R[KB][KB];
  bool bad = flag[q] != 0;
  double dmax = 0.0;
  if (A && pass == 1) {
    const double* a = A + (size_t)q * KB * KB;
    double s = 0.0;
    for (int i = 0; i < KB; ++i) s = fmax(s, a[i * KB + i]);
    dmax = s * s;
  } else {
    for (int i = 0; i < KB; ++i) dmax = fmax(dmax, g[i * KB + i]);
  }
  for (int i = 0; i < KB; ++i)
    for (int j = 0; j < KB; ++j) R[i][j] = 0.0;
  for (int j = 0; j < KB && !bad; ++j) {
    double s = g[j * KB + j];
    for (int i = 0; i < j; ++i) s -= R[i][j] * R[i][j];
    if (!(s > kBlockBreakdown * kBlockBreakdown * dmax) || !isfinite(s)) {
      bad = true;
      break;
    }
    R[j][j] = sqrt(s);
    for (int c = j + 1; c < KB; ++c) {
      double t = g[j * KB + c];
      for (int i = 0; i < j; ++i) t -= R[i][j] * R[i][c];
      R[j][c] = t / R[j][j];
    }
  }
  if (bad) {
    if (!flag[q]) {
      flag[q] = 1;
      meff[q] = step;
    }
    for (int i = 0; i < KB; ++i)
      for (int j = 0; j < KB; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
  }
  double* r1 = R1 + (size_t)q * KB * KB;
  if (pass == 1) {
    for (int i = 0; i < KB; ++i)
      for (int j = 0; j < KB; ++j) r1[i * KB + j] = R[i][j];
  } else {
    double* ra = Racc + (size_t)q * KB * KB;
    for (int i = 0; i < KB; ++i)
      for (int j = 0; j < KB; ++j) {
        double t = 0.0;
        for (int c = i; c <= j; ++c) t += R[i][c] * r1[c * KB + j];
        ra[i * KB + j] = bad ? 0.0 : t;
      }
    for (int i = 0; i < KB; ++i)
      for (int j = 0; j < KB; ++j) r1[i * KB + j] = R[i][j];
  }
}

// Y = W R^-1 row by row within every Krylov block (in place allowed); zero for ended
// blocks; optionally d = g * Y in the matvec's precision.
template <int KB>
__global__ void k_btrsm(const double* __restrict__ W, double* Y, const double* __restrict__ R,
                        const int* __restrict__ flag, int rows, int B, const double* __restrict__ g,
                        double* __restrict__ dd, float* __restrict__ df, int use_float,
                        int write_d) {
  const int nkb = B / KB;
  const size_t total = (size_t)rows * nkb;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(t % nkb);
    const size_t row = t / nkb;
    const double* r = R + (size_t)q * KB * KB;
    const size_t o = row * B + (size_t)q * KB;
    double y[KB];
    const bool dead = flag[q] != 0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      double v = W[o + j];
#pragma unroll
      for (int i = 0; i < j; ++i) v -= y[i] * r[i * KB + j];
      y[j] = dead ? 0.0 : v / r[j * KB + j];
    }
    const double gs = g[row / 3];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      Y[o + j] = y[j];
      if (write_d) {
        if (use_float) df[o + j] = (float)(gs * y[j]);
        else dd[o + j] = gs * y[j];
      }
    }
  }
}

// W = L - Y_k A_k - Y_{k-1} B_{k-1}^T within every Krylov block.
template <int KB>
__global__ void k_bupdate(const double* __restrict__ L, const double* __restrict__ Yk,
                          const double* __restrict__ Ykm1, const double* __restrict__ A,
                          const double* __restrict__ Bm1, double* __restrict__ W, int rows,
                          int B) {
  const int nkb = B / KB;
  const size_t total = (size_t)rows * nkb;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(t % nkb);
    const size_t o = (t / nkb) * B + (size_t)q * KB;
    const double* a = A + (size_t)q * KB * KB;
    double yk[KB], ykm[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      yk[i] = Yk[o + i];
      ykm[i] = Ykm1 ? Ykm1[o + i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      double v = L[o + j];
#pragma unroll
      for (int i = 0; i < KB; ++i) v -= yk[i] * a[i * KB + j];
      if (Ykm1) {
        const double* bm = Bm1 + (size_t)q * KB * KB;
#pragma unroll
        for (int i = 0; i < KB; ++i) v -= ykm[i] * bm[j * KB + i];
      }
      W[o + j] = v;
    }
  }
}

// One work-group per Krylov block: assemble T, reduce it to tridiagonal form by
// Householder reflections H_k (applied from both sides; the first KB rows of
// H_0 H_1 ... kept in P), diagonalize the tridiagonal with P's columns rotated along,
// and form Q_l = sum_j sqrt(theta_j) (sum_i R0_il P_ij)^2.
template <int KB>
__global__ void __launch_bounds__(256)
k_bquad(const double* __restrict__ Ablk, const double* __restrict__ Bblk,
        const double* __restrict__ R0, const int* __restrict__ meff, int m, double* __restrict__ Tws,
        double* __restrict__ Pws, double* __restrict__ dws, double* __restrict__ ews,
        double* __restrict__ qout, uint32_t* __restrict__ status) {
  __shared__ double v[kBlockMaxDim];
  __shared__ double w[kBlockMaxDim];
  __shared__ double red[256];
  __shared__ double sc[4];
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int ld = m * KB;
  const int mk = meff[q];
  const int n = mk * KB;
  double* T = Tws + (size_t)q * ld * ld;
  double* P = Pws + (size_t)q * KB * ld;
  double* d = dws + (size_t)q * ld;
  double* e = ews + (size_t)q * ld;
  const size_t bs = (size_t)KB * KB;
  // assemble
  for (int idx = tid; idx < n * n; idx += 256) {
    const int i = idx / n, j = idx % n;
    const int bi = i / KB, bj = j / KB, ii = i % KB, jj = j % KB;
    double val = 0.0;
    if (bi == bj) val = Ablk[((size_t)q * m + bi) * bs + ii * KB + jj];
    else if (bi == bj + 1) val = Bblk[((size_t)q * m + bj) * bs + ii * KB + jj];
    else if (bj == bi + 1) val = Bblk[((size_t)q * m + bi) * bs + jj * KB + ii];
    T[(size_t)i * ld + j] = val;
  }
  for (int idx = tid; idx < KB * n; idx += 256) {
    const int r = idx / n, c = idx % n;
    P[(size_t)r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    // x = T[k+1..n-1][k]
    double s = 0.0;
    for (int i = k + 1 + tid; i < n; i += 256) {
      const double x = T[(size_t)i * ld + k];
      v[i] = x;
      s += x * x;
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) {
      const double nrm2 = red[0];
      const double x0 = v[k + 1];
      const double nrm = sqrt(nrm2);
      const double tail = nrm2 - x0 * x0;
      if (tail <= 1e-300) {
        sc[0] = 0.0;          // already tridiagonal in this column
        sc[1] = x0;
      } else {
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        v[k + 1] = x0 - alpha;
        const double vtv = tail + v[k + 1] * v[k + 1];
        sc[0] = 2.0 / vtv;
        sc[1] = alpha;
      }
    }
    __syncthreads();
    const double beta = sc[0];
    if (beta != 0.0) {
      // p = beta T_sub v
      for (int i = k + 1 + tid; i < n; i += 256) {
        double acc = 0.0;
        for (int j = k + 1; j < n; ++j) acc += T[(size_t)i * ld + j] * v[j];
        w[i] = beta * acc;
      }
      __syncthreads();
      double pv = 0.0;
      for (int i = k + 1 + tid; i < n; i += 256) pv += w[i] * v[i];
      red[tid] = pv;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
      }
      const double K = 0.5 * beta * red[0];
      __syncthreads();
      for (int i = k + 1 + tid; i < n; i += 256) w[i] -= K * v[i];
      __syncthreads();
      for (int idx = tid; idx < (n - k - 1) * (n - k - 1); idx += 256) {
        const int i = k + 1 + idx / (n - k - 1), j = k + 1 + idx % (n - k - 1);
        T[(size_t)i * ld + j] -= v[i] * w[j] + w[i] * v[j];
      }
      // P <- P H: P[r][k+1..] -= beta (P[r] . v) v
      if (tid < KB) {
        double dp = 0.0;
        for (int j = k + 1; j < n; ++j) dp += P[(size_t)tid * ld + j] * v[j];
        for (int j = k + 1; j < n; ++j) P[(size_t)tid * ld + j] -= beta * dp * v[j];
      }
    }
    if (tid == 0) {
      T[(size_t)(k + 1) * ld + k] = sc[1];
      T[(size_t)k * ld + k + 1] = sc[1];
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) {
    d[i] = T[(size_t)i * ld + i];
    e[i] = (i + 1 < n) ? T[(size_t)(i + 1) * ld + i] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    const int ok = n > 0 ? tridiag_eigen_rows(d, e, P, n, KB, ld) : 1;
    if (!ok) atomicOr(status, kErrNoConverge);
    for (int i = 0; i < n; ++i)
      if (!(d[i] > 0.0)) {
        atomicOr(status, kErrNotPosdef);
        break;
      }
  }
  __syncthreads();
  if (tid < KB) {
    const double* r0 = R0 + (size_t)q * KB * KB;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      double c = 0.0;
      for (int i = 0; i <= tid; ++i) c += r0[i * KB + tid] * P[(size_t)i * ld + j];
      acc += sqrt(d[j] > 0.0 ? d[j] : 0.0) * c * c;
    }
    qout[q * KB + tid] = acc;
  }
}

// dst[q][k] = src[q] for blocks of bsz values ([nkb][m][bsz] storage of A_k, B_k).
__global__ void k_bscatter(const double* __restrict__ src, int nkb, int bsz, int k, int m,
                           double* __restrict__ dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nkb * bsz) return;
  const int q = e / bsz, i = e % bsz;
  dst[((size_t)q * m + k) * bsz + i] = src[e];
}

__global__ void k_bfill(int nkb, int m, int* __restrict__ flag, int* __restrict__ meff) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nkb) return;
  flag[q] = 0;
  meff[q] = m;
}

int grid_rows(size_t total) { return (int)std::min<size_t>((total + 255) / 256, 8192); }

template <int KB>
void gram(const BlockWork& bw, const double* X, const double* Y, int rows, int B,
          hipStream_t st) {
  const int per = (rows + bw.nblk - 1) / bw.nblk;
  k_bgram<KB><<<bw.nblk, 256, 0, st>>>(X, Y, rows, B, per, bw.part);
  const int E = B * KB;
  k_bgram_sum<<<(E + 255) / 256, 256, 0, st>>>(bw.part, bw.nblk, E, bw.G);
}

// W -> Y (in place) with W = Y Racc; d = g * Y when write_d.
template <int KB>
void cholqr2(const BlockWork& bw, double* W, int rows, int B, int step, double* Racc,
             const double* Ascale, const double* g, void* dv, bool use_float, bool write_d,
             hipStream_t st) {
  const int nkb = B / KB;
  const size_t total = (size_t)rows * nkb;
  for (int pass = 1; pass <= 2; ++pass) {
    gram<KB>(bw, W, W, rows, B, st);
    k_bchol<KB><<<(nkb + 63) / 64, 64, 0, st>>>(bw.G, Ascale, nkb, pass, step, bw.R1, Racc,
                                                 bw.flag, bw.meff);
    const bool wd = write_d && pass == 2;
    k_btrsm<KB><<<grid_rows(total), 256, 0, st>>>(W, W, bw.R1, bw.flag, rows, B, g,
                                                  (double*)dv, (float*)dv, use_float ? 1 : 0,
                                                  wd ? 1 : 0);
  }
}

}  // namespace

template <int KB>
static void block_start_impl(const Geometry& geo, const SysBuffers& b, const BlockWork& bw,
                             int B, int m, bool use_float, hipStream_t st) {
  const int nkb = B / KB;
  k_bfill<<<(nkb + 63) / 64, 64, 0, st>>>(nkb, m, bw.flag, bw.meff);
  cholqr2<KB>(bw, b.W, 3 * geo.n, B, 0, bw.R0, nullptr, b.g, b.dv, use_float, true, st);
}

template <int KB>
static void block_step_impl(const Geometry& geo, const SysBuffers& b, const BlockWork& bw,
                            int B, int k, int m, bool use_float, hipStream_t st) {
  const int nkb = B / KB;
  const int rows = 3 * geo.n;
  const size_t vs = (size_t)rows * B;
  const size_t bs = (size_t)nkb * KB * KB;
  double* Yk = b.W + (size_t)k * vs;
  gram<KB>(bw, Yk, b.Lt, rows, B, st);
  // A_k and B_k are stored [q][k][KB][KB]: write through a strided view per block
  k_bstore_a<KB><<<(int)((bs + 255) / 256), 256, 0, st>>>(bw.G, nkb, bw.Atmp);
  k_bscatter<<<(int)((bs + 255) / 256), 256, 0, st>>>(bw.Atmp, nkb, KB * KB, k, m, bw.A);
  if (k + 1 < m) {
    double* Wn = b.W + (size_t)(k + 1) * vs;
    const double* Ykm1 = k > 0 ? b.W + (size_t)(k - 1) * vs : nullptr;
    k_bupdate<KB><<<grid_rows((size_t)rows * nkb), 256, 0, st>>>(
        b.Lt, Yk, Ykm1, bw.Atmp, k > 0 ? bw.Bprev : nullptr, Wn, rows, B);
    cholqr2<KB>(bw, Wn, rows, B, k + 1, bw.Bprev, bw.Atmp, b.g, b.dv, use_float, true, st);
    k_bscatter<<<(int)((bs + 255) / 256), 256, 0, st>>>(bw.Bprev, nkb, KB * KB, k, m, bw.B);
  }
}

template <int KB>
static void block_quad_impl(const BlockWork& bw, int nkb, int m, double* q_out,
                            uint32_t* status, hipStream_t st) {
  k_bquad<KB><<<nkb, 256, 0, st>>>(bw.A, bw.B, bw.R0, bw.meff, m, bw.T, bw.P, bw.d, bw.e,
                                   q_out, status);
}

void launch_block_start(const Geometry& geo, const SysBuffers& b, const BlockWork& bw, int B,
                        int m, bool use_float, hipStream_t st) {
  switch (bw.kb) {
    case 2: block_start_impl<2>(geo, b, bw, B, m, use_float, st); break;
    case 4: block_start_impl<4>(geo, b, bw, B, m, use_float, st); break;
    default: block_start_impl<8>(geo, b, bw, B, m, use_float, st); break;
  }
}

void launch_block_step(const Geometry& geo, const SysBuffers& b, const BlockWork& bw, int B,
                       int k, int m, bool use_float, hipStream_t st) {
  switch (bw.kb) {
    case 2: block_step_impl<2>(geo, b, bw, B, k, m, use_float, st); break;
    case 4: block_step_impl<4>(geo, b, bw, B, k, m, use_float, st); break;
    default: block_step_impl<8>(geo, b, bw, B, k, m, use_float, st); break;
  }
}

void launch_block_quadrature(const BlockWork& bw, int nkb, int m, double* q_out,
                             uint32_t* status, hipStream_t st) {
  switch (bw.kb) {
    case 2: block_quad_impl<2>(bw, nkb, m, q_out, status, st); break;
    case 4: block_quad_impl<4>(bw, nkb, m, q_out, status, st); break;
    default: block_quad_impl<8>(bw, nkb, m, q_out, status, st); break;
  }
}

}  // namespace mbd
