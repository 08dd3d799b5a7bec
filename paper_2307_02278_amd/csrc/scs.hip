// Range-separated self-consistent screening of the polarizabilities on the GPU.
//
// For every imaginary frequency u_q the Dyson-like screening equation (Review
// section; MBD@rsSCS) is solved matrix-free:
//   (A(iu)^-1 + T_SR(iu)) X = E,   E = three right-hand sides, E_k = unit vector k on every atom,
//   alpha_i(iu) = alpha_i / (1 + (u / omega_i)^2),
//   T_SR = (1 - f) T_GG,  T_GG = -grad grad (erf(r / sigma_ij) / r) = A I - B r r^T,
//   A = (erf z - c) / r^3,  B = (3 erf z - c (3 + 2 z^2)) / r^5,  z = r / sigma_ij,
//   c = (2 / sqrt pi) z exp(-z^2),  sigma_ij^2 = sigma_i^2 + sigma_j^2,
//   sigma_i = (sqrt(2 / pi) alpha_i(iu) / 3)^(1/3),
// with f the Fermi damping of the MBD step, summed over every periodic image within
// the plan's pair cutoff. Then alpha^SCS_i(iu) = (1/3) sum_k X_{i,k}(E_k).
//
// All right-hand sides (3 per frequency, "columns") run together through a
// Jacobi-preconditioned conjugate gradient in float64. Vectors are [n][3][ncol]
// over the plan's sorted atoms, column = 3 q + k.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "mbd_math.h"

namespace mbd {
namespace {

// 1 - f = 1 / (1 + e^z) is below 1e-16 for z > 36.8: such pairs add nothing in float64
constexpr double kDampSkip = 36.8;

// CG scalar rows of ScsWork::sc ([kScsRows][ncol])
enum { kRz = 0, kPq = 1, kAlpha = 2, kBeta = 3, kRr = 4, kActive = 5, kBb = 6, kScsRows = 8 };

// Sorted cell-local positions in float64 (the same frame as the pair kernels:
// position minus the corner of its cell), the damping radius beta R_vdW, and per
// (atom, frequency) 1 / alpha(iu) and sigma(u)^2.
__global__ void k_scs_prepare(const Geometry geo, const int* __restrict__ perm,
                              const int* __restrict__ scell, const double* __restrict__ wpos,
                              const double* __restrict__ alpha, const double* __restrict__ omega,
                              const double* __restrict__ rvdw, const double* __restrict__ u,
                              int nq, double* __restrict__ locd, double* __restrict__ ainv,
                              double* __restrict__ sig2) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  const int i = perm[s];
  int c[3];
  cell_coords(scell[s], c[0], c[1], c[2]);
  double lf[3];
  for (int a = 0; a < 3; ++a) lf[a] = wpos[3 * i + a] - (double)c[a] / geo.nc[a];
  for (int k = 0; k < 3; ++k)
    locd[4 * s + k] = lf[0] * geo.A[0][k] + lf[1] * geo.A[1][k] + lf[2] * geo.A[2][k];
  locd[4 * s + 3] = geo.beta * rvdw[i];
  const double al = alpha[i], om = omega[i];
  for (int q = 0; q < nq; ++q) {
    const double x = u[q] / om;
    const double au = al / (1.0 + x * x);
    ainv[(size_t)s * nq + q] = 1.0 / au;
    const double sg = cbrt(0.7978845608028654 * au / 3.0);  // sqrt(2 / pi) alpha / 3
    sig2[(size_t)s * nq + q] = sg * sg;
  }
}

// q = A^-1 p + T_SR p. One wavefront per sorted target; lane = f + NQP * sl handles
// frequency f for the sources j = j0 + sl, j0 + sl + SL, ... of every neighbour cell
// (SL = 64 / NQP lanes share a frequency), then the SL partial fields are summed
// with cross-lane exchanges. The pair geometry and the damping are evaluated by all
// lanes of a source alike, so branches split only between source lanes.
template <int NQP>
__global__ void __launch_bounds__(64)
k_scs_apply(const Geometry geo, const int* __restrict__ cell_start,
            const int* __restrict__ scell, const double* __restrict__ locd,
            const double* __restrict__ ainv, const double* __restrict__ sig2, int nq,
            const double* __restrict__ p, double* __restrict__ qv) {
  constexpr int SL = 64 / NQP;
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  const int f = lane % NQP, sl = lane / NQP;
  const bool fv = f < nq;
  const int fq = fv ? f : 0;
  const int ncol = 3 * nq;
  int cx, cy, cz;
  cell_coords(scell[s], cx, cy, cz);
  const double xi = locd[4 * s], yi = locd[4 * s + 1], zi = locd[4 * s + 2];
  const double Si = locd[4 * s + 3];
  const double s2i = sig2[(size_t)s * nq + fq];
  const double rp2 = geo.r_pair * geo.r_pair;
  const double dd = geo.damp_d;
  double acc[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) acc[a][0] = acc[a][1] = acc[a][2] = 0.0;
  for (int oz = -geo.nr[2]; oz <= geo.nr[2]; ++oz) {
    int wz = (cz + oz) % geo.nc[2];
    if (wz < 0) wz += geo.nc[2];
    for (int oy = -geo.nr[1]; oy <= geo.nr[1]; ++oy) {
      int wy = (cy + oy) % geo.nc[1];
      if (wy < 0) wy += geo.nc[1];
      for (int ox = -geo.nr[0]; ox <= geo.nr[0]; ++ox) {
        int wx = (cx + ox) % geo.nc[0];
        if (wx < 0) wx += geo.nc[0];
        const double sx = ox * geo.hv[0][0] + oy * geo.hv[1][0] + oz * geo.hv[2][0];
        const double sy = ox * geo.hv[0][1] + oy * geo.hv[1][1] + oz * geo.hv[2][1];
        const double sz = ox * geo.hv[0][2] + oy * geo.hv[1][2] + oz * geo.hv[2][2];
        const bool zero = (ox == 0 && oy == 0 && oz == 0);
        const int cc = cell_index(wx, wy, wz);
        const int j1 = cell_start[cc + 1];
        for (int j = cell_start[cc] + sl; j < j1; j += SL) {
          if (zero && j == s) continue;
          const double rx = locd[4 * j] - xi + sx;
          const double ry = locd[4 * j + 1] - yi + sy;
          const double rz = locd[4 * j + 2] - zi + sz;
          const double r2 = rx * rx + ry * ry + rz * rz;
          if (r2 >= rp2) continue;
          const double S = Si + locd[4 * j + 3];
          if (dd * (sqrt(r2) / S - 1.0) > kDampSkip || !fv) continue;
          double A, Bk;
          scs_kernel(r2, s2i + sig2[(size_t)j * nq + f], S, dd, A, Bk);
          const double* pj = p + (size_t)j * 3 * ncol + 3 * f;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double x0 = pj[k], x1 = pj[ncol + k], x2 = pj[2 * ncol + k];
            const double rd = Bk * (rx * x0 + ry * x1 + rz * x2);
            acc[0][k] += A * x0 - rx * rd;
            acc[1][k] += A * x1 - ry * rd;
            acc[2][k] += A * x2 - rz * rd;
          }
        }
      }
    }
  }
#pragma unroll
  for (int off = NQP; off < 64; off <<= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[a][k] += __shfl_xor(acc[a][k], off);
  if (sl == 0 && fv) {
    const double ai = ainv[(size_t)s * nq + f];
    const size_t o = (size_t)s * 3 * ncol + 3 * f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        qv[o + (size_t)a * ncol + k] = ai * p[o + (size_t)a * ncol + k] + acc[a][k];
  }
}

// Partial sums over blocks of rows: part[b][0][c] = sum_r X[r][c] Y[r][c] and, when X2
// is given, part[b][1][c] = sum_r X2[r][c] Y2[r][c]. Thread t takes column t % ncol and
// every (256 / ncol)-th row of the block's range; the lanes of a column are summed in
// a fixed order, so results do not depend on scheduling.
__global__ void __launch_bounds__(256)
k_col_dots(const double* __restrict__ X, const double* __restrict__ Y,
           const double* __restrict__ X2, const double* __restrict__ Y2, int rows, int ncol,
           int rows_per_block, double* __restrict__ part) {
  __shared__ double s1[256], s2[256];
  const int t = threadIdx.x;
  const int nrl = 256 / ncol;
  const int c = t % ncol, rl = t / ncol;
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = min(rows, r0 + rows_per_block);
  double a1 = 0.0, a2 = 0.0;
  if (rl < nrl) {
    for (int r = r0 + rl; r < r1; r += nrl) {
      const size_t o = (size_t)r * ncol + c;
      a1 += X[o] * Y[o];
      if (X2) a2 += X2[o] * Y2[o];
    }
  }
  s1[t] = a1;
  s2[t] = a2;
  __syncthreads();
  if (t < ncol) {
    double b1 = 0.0, b2 = 0.0;
    for (int i = 0; i < nrl; ++i) {
      b1 += s1[t + i * ncol];
      b2 += s2[t + i * ncol];
    }
    part[((size_t)blockIdx.x * 2) * ncol + t] = b1;
    part[((size_t)blockIdx.x * 2 + 1) * ncol + t] = b2;
  }
}

// x = 0, r = E, z = P r, p = z (P = diag alpha(iu), the Jacobi preconditioner).
__global__ void k_scs_init(int n, int nq, const double* __restrict__ ainv, double* __restrict__ x,
                           double* __restrict__ r, double* __restrict__ z,
                           double* __restrict__ p) {
  const int ncol = 3 * nq;
  const size_t total = (size_t)n * 3 * ncol;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % ncol);
    const int a = (int)((e / ncol) % 3);
    const size_t s = e / (3 * (size_t)ncol);
    const int f = col / 3, k = col % 3;
    const double rv = (a == k) ? 1.0 : 0.0;
    const double zv = rv / ainv[s * nq + f];
    x[e] = 0.0;
    r[e] = rv;
    z[e] = zv;
    p[e] = zv;
  }
}

// sums[k][c] = sum over the nblk row blocks of part[b][k][c] (k = 0, 1): one work-group
// per column, a fixed strided split and a fixed tree, so the order never changes.
__global__ void __launch_bounds__(256)
k_col_sums(const double* __restrict__ part, int nblk, int ncol, double* __restrict__ sums) {
  __shared__ double r1[256], r2[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double v1 = 0.0, v2 = 0.0;
  for (int b = t; b < nblk; b += 256) {
    v1 += part[((size_t)b * 2) * ncol + c];
    v2 += part[((size_t)b * 2 + 1) * ncol + c];
  }
  r1[t] = v1;
  r2[t] = v2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      r1[t] += r1[t + h];
      r2[t] += r2[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    sums[c] = r1[0];
    sums[ncol + c] = r2[0];
  }
}

__device__ inline void sum_parts(const double* sums, int ncol, int c, double& v1, double& v2) {
  v1 = sums[c];
  v2 = sums[ncol + c];
}

// After the initial dots (r.z, r.r): rz, bb = ||E_k||^2, every column active.
__global__ void k_scs_start(const double* __restrict__ part, int nblk, int ncol,
                            double* __restrict__ sc, int* __restrict__ nact) {
  const int c = threadIdx.x;
  if (c >= ncol) return;
  double rz, rr;
  sum_parts(part, ncol, c, rz, rr);
  sc[kRz * ncol + c] = rz;
  sc[kRr * ncol + c] = rr;
  sc[kBb * ncol + c] = rr;
  sc[kActive * ncol + c] = 1.0;
  sc[kAlpha * ncol + c] = 0.0;
  sc[kBeta * ncol + c] = 0.0;
  if (c == 0) nact[0] = ncol;
}

// alpha_c = rz_c / (p.q)_c for active columns; p.q <= 0 (or not finite) means the
// screening matrix is not positive definite: the column stops and the status is set.
__global__ void k_scs_alpha(const double* __restrict__ part, int nblk, int ncol,
                            double* __restrict__ sc, uint32_t* __restrict__ status) {
  const int c = threadIdx.x;
  if (c >= ncol) return;
  double pq, unused;
  sum_parts(part, ncol, c, pq, unused);
  double al = 0.0;
  if (sc[kActive * ncol + c] != 0.0) {
    if (!(pq > 0.0) || !isfinite(pq)) {
      sc[kActive * ncol + c] = 0.0;
      atomicOr(status, kErrNotPosdef);
    } else {
      al = sc[kRz * ncol + c] / pq;
    }
  }
  sc[kAlpha * ncol + c] = al;
}

// x += alpha p, r -= alpha q, z = P r.
__global__ void k_scs_update(int n, int nq, const double* __restrict__ ainv,
                             const double* __restrict__ sc, const double* __restrict__ p,
                             const double* __restrict__ qv, double* __restrict__ x,
                             double* __restrict__ r, double* __restrict__ z) {
  const int ncol = 3 * nq;
  const size_t total = (size_t)n * 3 * ncol;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % ncol);
    const size_t s = e / (3 * (size_t)ncol);
    const double al = sc[kAlpha * ncol + col];
    x[e] += al * p[e];
    const double rv = r[e] - al * qv[e];
    r[e] = rv;
    z[e] = rv / ainv[s * nq + col / 3];
  }
}

// beta_c = (r.z)_new / (r.z)_old; a column whose ||r|| <= tol ||E_k|| stops.
__global__ void k_scs_beta(const double* __restrict__ part, int nblk, int ncol, double tol2,
                           double* __restrict__ sc, int* __restrict__ nact) {
  __shared__ int cnt[128];
  const int c = threadIdx.x;
  int act = 0;
  if (c < ncol) {
    double rz, rr;
    sum_parts(part, ncol, c, rz, rr);
    double be = 0.0;
    if (sc[kActive * ncol + c] != 0.0) {
      sc[kRr * ncol + c] = rr;
      if (!isfinite(rr) || rr <= tol2 * sc[kBb * ncol + c]) {
        sc[kActive * ncol + c] = 0.0;
      } else {
        be = rz / sc[kRz * ncol + c];
        sc[kRz * ncol + c] = rz;
        act = 1;
      }
    }
    sc[kBeta * ncol + c] = be;
  }
  cnt[c] = act;
  __syncthreads();
  if (c == 0) {
    int t = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) t += cnt[i];
    nact[0] = t;
  }
}

// p = z + beta p.
__global__ void k_scs_direction(size_t total, int ncol, const double* __restrict__ sc,
                                const double* __restrict__ z, double* __restrict__ p) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = z[e] + sc[kBeta * ncol + (int)(e % ncol)] * p[e];
}

// alpha^SCS_i(iu_q) = (1/3) sum_k x[i][k][3q + k]; C6 by the quadrature weights w
// (node 0 is the static point u = 0 and carries no weight); omega^SCS, R^SCS.
// Outputs in the caller's atom order.
__global__ void k_scs_output(int n, int nq, const int* __restrict__ perm,
                             const double* __restrict__ x, const double* __restrict__ w,
                             const double* __restrict__ alpha, const double* __restrict__ rvdw,
                             double* __restrict__ a_out, double* __restrict__ om_out,
                             double* __restrict__ rv_out, double* __restrict__ af_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  const int ncol = 3 * nq;
  const double* xs = x + (size_t)s * 3 * ncol;
  double a0 = 0.0, c6 = 0.0;
  for (int f = 0; f < nq; ++f) {
    const double af = (xs[3 * f] + xs[ncol + 3 * f + 1] + xs[2 * ncol + 3 * f + 2]) / 3.0;
    if (f == 0) a0 = af;
    else {
      c6 += w[f] * af * af;
      if (af_out) af_out[(size_t)(f - 1) * n + i] = af;
    }
  }
  c6 *= 3.0 / M_PI;
  a_out[i] = a0;
  om_out[i] = 4.0 * c6 / (3.0 * a0 * a0);
  rv_out[i] = rvdw[i] * cbrt(a0 / alpha[i]);
}

int grid_for(size_t total) {
  return (int)std::min<size_t>((total + 255) / 256, 4096);
}

}  // namespace

void launch_scs_prepare(const Geometry& g, const SysBuffers& b, const double* alpha,
                        const double* omega, const double* rvdw, const double* u,
                        const ScsWork& w, hipStream_t st) {
  k_scs_prepare<<<(g.n + 127) / 128, 128, 0, st>>>(g, b.perm, b.scell, b.wpos, alpha, omega,
                                                   rvdw, u, w.nq, w.locd, w.ainv, w.sig2);
}

void launch_scs_apply(const Geometry& g, const SysBuffers& b, const ScsWork& w, const double* p,
                      double* q, hipStream_t st) {
#define MBD_SCS(NQP)                                                                           \
  k_scs_apply<NQP><<<g.n, 64, 0, st>>>(g, b.cell_start, b.scell, w.locd, w.ainv, w.sig2, w.nq, \
                                       p, q)
  if (w.nq <= 2) MBD_SCS(2);
  else if (w.nq <= 4) MBD_SCS(4);
  else if (w.nq <= 8) MBD_SCS(8);
  else if (w.nq <= 16) MBD_SCS(16);
  else MBD_SCS(32);
#undef MBD_SCS
}

void launch_scs_dots(const ScsWork& w, const double* X, const double* Y, const double* X2,
                     const double* Y2, hipStream_t st) {
  const int rows = 3 * w.n;
  const int per = (rows + w.nblk - 1) / w.nblk;
  k_col_dots<<<w.nblk, 256, 0, st>>>(X, Y, X2, Y2, rows, w.ncol, per, w.part);
  k_col_sums<<<w.ncol, 256, 0, st>>>(w.part, w.nblk, w.ncol, w.sums);
}

void launch_scs_init(const ScsWork& w, hipStream_t st) {
  const size_t total = (size_t)w.n * 3 * w.ncol;
  k_scs_init<<<grid_for(total), 256, 0, st>>>(w.n, w.nq, w.ainv, w.x, w.r, w.z, w.p);
  launch_scs_dots(w, w.r, w.z, w.r, w.r, st);
  k_scs_start<<<1, 128, 0, st>>>(w.sums, w.nblk, w.ncol, w.sc, w.nact);
}

void launch_scs_iteration(const Geometry& g, const SysBuffers& b, const ScsWork& w, double tol,
                          uint32_t* status, hipStream_t st) {
  const size_t total = (size_t)w.n * 3 * w.ncol;
  launch_scs_apply(g, b, w, w.p, w.q, st);
  launch_scs_dots(w, w.p, w.q, nullptr, nullptr, st);
  k_scs_alpha<<<1, 128, 0, st>>>(w.sums, w.nblk, w.ncol, w.sc, status);
  k_scs_update<<<grid_for(total), 256, 0, st>>>(w.n, w.nq, w.ainv, w.sc, w.p, w.q, w.x, w.r,
                                                w.z);
  launch_scs_dots(w, w.r, w.z, w.r, w.r, st);
  k_scs_beta<<<1, 128, 0, st>>>(w.sums, w.nblk, w.ncol, tol * tol, w.sc, w.nact);
  k_scs_direction<<<grid_for(total), 256, 0, st>>>(total, w.ncol, w.sc, w.z, w.p);
}

void launch_scs_output(const SysBuffers& b, const ScsWork& w, const double* wq,
                       const double* alpha, const double* rvdw, double* a_out, double* om_out,
                       double* rv_out, double* af_out, hipStream_t st) {
  k_scs_output<<<(w.n + 127) / 128, 128, 0, st>>>(w.n, w.nq, b.perm, w.x, wq, alpha, rvdw,
                                                  a_out, om_out, rv_out, af_out);
}

}  // namespace mbd
