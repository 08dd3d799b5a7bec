// SPME spreading and gather (eqs. dipolarr and spme).
//
// Spread: D(k) = sum_j sum_a d_ja dW_j(k)/dR_a with W_j(k) = prod_a M_p(u_ja - k_a),
// stencil k_a = base_a - t_a (t_a = 0..p-1, periodic wrap). With u = Mu R (Mu = rows
// K_a a*_a, any cell), d . grad_R W = sum_b (Mu d)_b dW/du_b: the kernels transform the
// dipole (spread), the gradient (gather) and the Hessian (force gather) with Mu and
// use the derivative tables in u.
// One wavefront owns a 4x4x4 tile of grid points for one chunk of BG right-hand
// sides, accumulates in registers every atom whose stencil reaches the tile, in a
// fixed order, and writes the tile once: no atomics, no clearing pass, and a
// deterministic sum. With one lane per right-hand side the atom's indices and
// spline weights are wave-uniform.
//
// Gather + epilogue: E_rec,i = sum_k grad_i W_i(k) phi(k) (eq. spme), then the
// generalized field E* = E_dir + E_rec + E_self and
//   l~ = Omega w + Diag(g) E*      (eq. lk3, in double precision)
// with per-block partial sums of w . l~ for a_k (eq. recurs2). Again one wavefront
// per atom and one lane per right-hand side.
#include "common.h"

namespace mbd {

namespace {

// Lanes of a wavefront: BG right-hand sides x NSUB sub-lanes that share the stencil.
template <int BG>
struct Lanes {
  static constexpr int NSUB = 64 / BG;
};

// Spread with register tiles: one wavefront owns a 4x4x4 tile of grid points for BG
// right-hand sides and keeps the 64 point values of its lane in registers
// (64 / NSUB per lane when fewer than 64 right-hand sides share the wavefront).
// It walks the tile's atom list in a fixed order, so the result is deterministic.
// For one atom the weights along each axis of the tile are uniform scalars:
//   w_a(q) = M_p(u_a - k_a) for the tile point k_a = tile origin + q,
// nonzero only when 0 <= t = (base_a - k_a) mod K_a < p, i.e. t = o_a - q with
// o_a = (base_a - origin_a) mod K_a.
template <typename R, int P, int BG>
__global__ void __launch_bounds__(256)
k_spread(const Geometry geo, const int* __restrict__ tile_start,
         const int* __restrict__ tile_atoms, const int* __restrict__ base,
         const R* __restrict__ th, const R* __restrict__ dth, const R* __restrict__ dv, int B,
         R* __restrict__ grid, size_t chunk_elems, int chunk0) {
  constexpr int T = kSpreadTile;
  constexpr int NSUB = Lanes<BG>::NSUB;
  constexpr int NP = T * T * T / NSUB;  // points per lane
  constexpr int NWT = 6 * T;            // staged weights per atom: w, dw along x, y, z
  __shared__ R wts_all[4][64][NWT];
  __shared__ int sat_all[4][64];        // atom index of each staged slot
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lane = threadIdx.x & 63;
  R(*wts)[NWT] = wts_all[wave];
  int* sat = sat_all[wave];
  const int ntiles = geo.tiles[0] * geo.tiles[1] * geo.tiles[2];
  // Blocks are dealt round-robin to the 8 XCDs (gridDim.x is a multiple of 8):
  // each XCD takes one contiguous range of tiles, a slab of the grid, so the
  // dipoles of the atoms it spreads stay in its L2.
  const int per = gridDim.x / 8;
  const int tile = ((blockIdx.x % 8) * per + blockIdx.x / 8) * 4 + wave;
  if (tile >= ntiles) return;
  const int chunk = blockIdx.y + chunk0;
  const int b = lane % BG;
  const int sub = lane / BG;
  const int bg = chunk * BG + b;
  const int tx = tile % geo.tiles[0];
  const int ty = (tile / geo.tiles[0]) % geo.tiles[1];
  const int tz = tile / (geo.tiles[0] * geo.tiles[1]);
  const int x0 = tx * T, y0 = ty * T, z0 = tz * T;
  const int K1 = geo.K[0], K2 = geo.K[1], K3 = geo.K[2];
  R acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = R(0);
  const int lo = tile_start[tile], hi = tile_start[tile + 1];
  for (int a0 = lo; a0 < hi; a0 += 64) {
    const int na = min(64, hi - a0);
    // Stage: lane i computes the tile-clipped weights of the batch's atom i.
    // For one atom the weights along each axis of the tile are
    //   w_a(q) = M_p(u_a - k_a) at the tile point k_a = origin_a + q,
    // nonzero only when t = o_a - q lies in [0, p), o_a = (base_a - origin_a) mod K_a.
    if (lane < na) {
      const int s = tile_atoms[a0 + lane];
      int o[3] = {base[3 * s] - x0, base[3 * s + 1] - y0, base[3 * s + 2] - z0};
      if (o[0] < 0) o[0] += K1;
      if (o[1] < 0) o[1] += K2;
      if (o[2] < 0) o[2] += K3;
      const R* thp = th + (size_t)s * 3 * P;
      const R* dthp = dth + (size_t)s * 3 * P;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
#pragma unroll
        for (int q = 0; q < T; ++q) {
          const int t = o[ax] - q;
          const bool v = t >= 0 && t < P;
          wts[lane][(2 * ax) * T + q] = v ? thp[ax * P + t] : R(0);
          wts[lane][(2 * ax + 1) * T + q] = v ? dthp[ax * P + t] : R(0);
        }
      sat[lane] = s;
    }
    // the batch's LDS writes are visible to the whole wavefront before it reads them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const R m00 = (R)geo.Mu[0][0], m01 = (R)geo.Mu[0][1], m02 = (R)geo.Mu[0][2];
    const R m10 = (R)geo.Mu[1][0], m11 = (R)geo.Mu[1][1], m12 = (R)geo.Mu[1][2];
    const R m20 = (R)geo.Mu[2][0], m21 = (R)geo.Mu[2][1], m22 = (R)geo.Mu[2][2];
    int s = __builtin_amdgcn_readfirstlane(sat[0]);
    R n0 = dv[((size_t)s * 3 + 0) * B + bg];
    R n1 = dv[((size_t)s * 3 + 1) * B + bg];
    R n2 = dv[((size_t)s * 3 + 2) * B + bg];
    for (int a = 0; a < na; ++a) {
      // dipole in u: (Mu d)_b
      const R d0 = m00 * n0 + m01 * n1 + m02 * n2;
      const R d1 = m10 * n0 + m11 * n1 + m12 * n2;
      const R d2 = m20 * n0 + m21 * n1 + m22 * n2;
      if (a + 1 < na) {  // next atom's dipoles while this one is spread
        s = __builtin_amdgcn_readfirstlane(sat[a + 1]);
        n0 = dv[((size_t)s * 3 + 0) * B + bg];
        n1 = dv[((size_t)s * 3 + 1) * B + bg];
        n2 = dv[((size_t)s * 3 + 2) * B + bg];
      }
      const R* wa = wts[a];
      R wx[T], dwx[T], wy[T], dwy[T], wz[T], dwz[T];
#pragma unroll
      for (int q = 0; q < T; ++q) {
        wx[q] = wa[q]; dwx[q] = wa[T + q];
        wy[q] = wa[2 * T + q]; dwy[q] = wa[3 * T + q];
        wz[q] = wa[4 * T + q]; dwz[q] = wa[5 * T + q];
      }
      if (NSUB == 1) {
        // every point of the tile: the staged weights are zero outside the stencil, and
        // a branch-free loop issues fewer instructions than uniform per-point tests
#pragma unroll
        for (int pz = 0; pz < T; ++pz) {
#pragma unroll
          for (int py = 0; py < T; ++py) {
            const R A = d0 * wy[py] * wz[pz];
            const R Bc = d1 * dwy[py] * wz[pz] + d2 * wy[py] * dwz[pz];
#pragma unroll
            for (int px = 0; px < T; ++px) {
              R& q = acc[(pz * T + py) * T + px];
              q = fma(dwx[px], A, q);
              q = fma(wx[px], Bc, q);
            }
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const int p = sub + i * NSUB;
          const int px = p % T, py = (p / T) % T, pz = p / (T * T);
          acc[i] += (dwx[px] * wy[py] * wz[pz]) * d0 + (wx[px] * dwy[py] * wz[pz]) * d1 +
                    (wx[px] * wy[py] * dwz[pz]) * d2;
        }
      }
    }
    // all reads of this batch are done before the next batch overwrites the stage
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  R* g = grid + (size_t)chunk * chunk_elems;
  const int XS = K1 + 2;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int p = sub + i * NSUB;
    const int x = x0 + p % T, y = y0 + (p / T) % T, z = z0 + p / (T * T);
    if (x < K1 && y < K2 && z < K3) g[(((size_t)z * K2 + y) * XS + x) * BG + b] = acc[i];
  }
}

template <typename R, int P, int BG>
__global__ void __launch_bounds__(512)
k_gather_epilogue(const Geometry geo, const int* __restrict__ base, const R* __restrict__ th,
                  const R* __restrict__ dth, const R* __restrict__ grid, size_t chunk_elems,
                  const R* __restrict__ Ed, const double* __restrict__ w,
                  const double* __restrict__ g, const double* __restrict__ om2, int B,
                  uint32_t comps, double self_coef, double* __restrict__ lt,
                  double* __restrict__ part, int chunk0) {
  constexpr int NSUB = Lanes<BG>::NSUB;
  __shared__ double red[512];
  const int nw = blockDim.x >> 6;  // wavefronts per work-group (4 or 8)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lane = threadIdx.x & 63;
  const int b = lane % BG;
  const int sub = lane / BG;
  const int chunk = blockIdx.y + chunk0;
  const int bg = chunk * BG + b;
  const R* gr = grid + (size_t)chunk * chunk_elems;
  const int K1 = geo.K[0], K2 = geo.K[1], K3 = geo.K[2];
  const int XS = K1 + 2;
  double dot = 0.0;
  // Blocks are dealt round-robin to the 8 XCDs. Each XCD takes one contiguous range
  // of sorted atoms and sweeps it with all of its wavefronts side by side (wave lw
  // takes atoms lo + lw, lo + lw + nwx, ...), so the atoms in flight on an XCD at
  // any time are consecutive, i.e. spatially compact, and their stencils share L2.
  const int nb8 = gridDim.x / 8;
  const int xcd = blockIdx.x % 8;
  const int nwx = nb8 * nw;
  const int lw = (blockIdx.x / 8) * nw + wave;
  const int x_lo = (int)(((long)geo.n * xcd) / 8);
  const int x_hi = (int)(((long)geo.n * (xcd + 1)) / 8);
  for (int s = x_lo + lw; s < x_hi; s += nwx) {
    R e0 = R(0), e1 = R(0), e2 = R(0);
    if (comps & MBD_C_REC) {
      const R* thp = th + s * 3 * P;
      const R* dthp = dth + s * 3 * P;
      R mx[P], dmx[P], my[P], dmy[P], mz[P], dmz[P];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        mx[t] = thp[t]; dmx[t] = dthp[t];
        my[t] = thp[P + t]; dmy[t] = dthp[P + t];
        mz[t] = thp[2 * P + t]; dmz[t] = dthp[2 * P + t];
      }
      const int bx = base[3 * s], by = base[3 * s + 1], bz = base[3 * s + 2];
      int kxs[P];
#pragma unroll
      for (int t1 = 0; t1 < P; ++t1) {
        int k1 = bx - t1;
        if (k1 < 0) k1 += K1;
        kxs[t1] = k1 * BG + b;
      }
#pragma unroll
      for (int t3 = 0; t3 < P; ++t3) {
        int k3 = bz - t3;
        if (k3 < 0) k3 += K3;
#pragma unroll
        for (int t2 = 0; t2 < P; ++t2) {
          if ((t3 * P + t2) % NSUB != sub) continue;
          int k2 = by - t2;
          if (k2 < 0) k2 += K2;
          const R* line = gr + ((size_t)k3 * K2 + k2) * XS * BG;
          R sx = R(0), sy = R(0);
#pragma unroll
          for (int t1 = 0; t1 < P; ++t1) {
            const R phi = line[kxs[t1]];
            sx += dmx[t1] * phi;
            sy += mx[t1] * phi;
          }
          e0 += sx * my[t2] * mz[t3];
          e1 += sy * dmy[t2] * mz[t3];
          e2 += sy * my[t2] * dmz[t3];
        }
      }
      // combine the sub-lanes that split the stencil rows
#pragma unroll
      for (int off = BG; off < 64; off <<= 1) {
        e0 += __shfl_xor(e0, off);
        e1 += __shfl_xor(e1, off);
        e2 += __shfl_xor(e2, off);
      }
      // gradient in u -> Cartesian: E_c = sum_b Mu[b][c] (dE/du_b)
      const R g0 = e0, g1 = e1, g2 = e2;
      e0 = (R)geo.Mu[0][0] * g0 + (R)geo.Mu[1][0] * g1 + (R)geo.Mu[2][0] * g2;
      e1 = (R)geo.Mu[0][1] * g0 + (R)geo.Mu[1][1] * g1 + (R)geo.Mu[2][1] * g2;
      e2 = (R)geo.Mu[0][2] * g0 + (R)geo.Mu[1][2] * g1 + (R)geo.Mu[2][2] * g2;
    }
    if (sub == 0) {
      const double gs = g[s];
      const double o2 = om2[s];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t idx = ((size_t)s * 3 + a) * B + bg;
        const double wv = w[idx];
        double E = (a == 0) ? (double)e0 : (a == 1) ? (double)e1 : (double)e2;
        if (comps & MBD_C_DIR) E += (double)Ed[idx];
        if (comps & MBD_C_SELF) E += self_coef * gs * wv;
        double l = gs * E;
        if (comps & MBD_C_DIAG) l += o2 * wv;
        lt[idx] = l;
        dot += wv * l;
      }
    }
  }
  // per-RHS sum over the work-group's wavefronts (sub-lanes hold zero)
  red[threadIdx.x] = dot;
  __syncthreads();
  if (threadIdx.x < BG) {
    double t = 0.0;
    for (int wv = 0; wv < nw; ++wv)
      for (int sb = 0; sb < NSUB; ++sb) t += red[wv * 64 + sb * BG + threadIdx.x];
    part[((size_t)blockIdx.x * kPartSlots + 0) * B + chunk * BG + threadIdx.x] = t;
  }
}

// Reciprocal-space part of the bilinear force term for one reverse step: with
// S = D_p^T phi_q (D_x the spread of dipoles x, phi_x = G~ * D_x, symmetric in p, q),
//   dS/dR_a = sum_k H_a(k) (p_a phi_q(k) + q_a phi_p(k)),  H_a(k) = grad_a grad_a W_a(k),
// the Hessian of the atom's weight product (d^2/du^2 along one axis: ddth; mixed
// axes: dth dth). One call adds sum_k H_a(k) h_a phi(k) for one grid (phi) and the
// other dipole set h, summed over the chunk's right-hand sides, to fsum (wavefront
// per atom, lanes over right-hand sides and stencil rows as in the gather).
template <typename R, int P, int BG>
__global__ void __launch_bounds__(512)
k_spme_force(const Geometry geo, const int* __restrict__ base, const R* __restrict__ th,
             const R* __restrict__ dth, const R* __restrict__ ddth, const R* __restrict__ grid,
             size_t chunk_elems, const R* __restrict__ hv, int B, int chunk0,
             double* __restrict__ fsum, const double* __restrict__ hscale) {
  constexpr int NSUB = Lanes<BG>::NSUB;
  const int nw = blockDim.x >> 6;  // wavefronts per work-group (4 or 8)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lane = threadIdx.x & 63;
  const int b = lane % BG;
  const int sub = lane / BG;
  const int chunk = blockIdx.y + chunk0;
  const int bg = chunk * BG + b;
  const R* gr = grid + (size_t)chunk * chunk_elems;
  const int K1 = geo.K[0], K2 = geo.K[1], K3 = geo.K[2];
  const int XS = K1 + 2;
  const int nb8 = gridDim.x / 8;
  const int xcd = blockIdx.x % 8;
  const int nwx = nb8 * nw;
  const int lw = (blockIdx.x / 8) * nw + wave;
  const int x_lo = (int)(((long)geo.n * xcd) / 8);
  const int x_hi = (int)(((long)geo.n * (xcd + 1)) / 8);
  for (int s = x_lo + lw; s < x_hi; s += nwx) {
    const R* tp = th + (size_t)s * 3 * P;
    const R* dp = dth + (size_t)s * 3 * P;
    const R* ddp = ddth + (size_t)s * 3 * P;
    R mx[P], dmx[P], ddmx[P], my[P], dmy[P], ddmy[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      mx[t] = tp[t]; dmx[t] = dp[t]; ddmx[t] = ddp[t];
      my[t] = tp[P + t]; dmy[t] = dp[P + t]; ddmy[t] = ddp[P + t];
    }
    const int bx = base[3 * s], by = base[3 * s + 1], bz = base[3 * s + 2];
    int kxs[P];
#pragma unroll
    for (int t1 = 0; t1 < P; ++t1) {
      int k1 = bx - t1;
      if (k1 < 0) k1 += K1;
      kxs[t1] = k1 * BG + b;
    }
    R hxx = R(0), hyy = R(0), hzz = R(0), hxy = R(0), hxz = R(0), hyz = R(0);
    // one z plane of the stencil at a time (not unrolled: unrolled, the compiler keeps
    // all p^3 grid values of an atom in flight and the kernel runs at 2 waves per SIMD)
#pragma unroll 1
    for (int t3 = 0; t3 < P; ++t3) {
      const R mz3 = tp[2 * P + t3], dmz3 = dp[2 * P + t3], ddmz3 = ddp[2 * P + t3];
      int k3 = bz - t3;
      if (k3 < 0) k3 += K3;
#pragma unroll
      for (int t2 = 0; t2 < P; ++t2) {
        if ((t3 * P + t2) % NSUB != sub) continue;
        int k2 = by - t2;
        if (k2 < 0) k2 += K2;
        const R* line = gr + ((size_t)k3 * K2 + k2) * XS * BG;
        R s0 = R(0), s1 = R(0), s2 = R(0);
#pragma unroll
        for (int t1 = 0; t1 < P; ++t1) {
          const R phi = line[kxs[t1]];
          s0 += mx[t1] * phi;
          s1 += dmx[t1] * phi;
          s2 += ddmx[t1] * phi;
        }
        hxx += s2 * my[t2] * mz3;
        hyy += s0 * ddmy[t2] * mz3;
        hzz += s0 * my[t2] * ddmz3;
        hxy += s1 * dmy[t2] * mz3;
        hxz += s1 * my[t2] * dmz3;
        hyz += s0 * dmy[t2] * dmz3;
      }
    }
    const size_t o = (size_t)s * 3 * B + bg;
    // h, times a per-right-hand-side factor when the grid belongs to a scaled dipole set
    const R hs = hscale ? (R)hscale[(size_t)bg * 16] : R(1);
    const R c0 = hs * hv[o], c1 = hs * hv[o + B], c2 = hs * hv[o + 2 * B];
    // Hessian in u: H_R = Mu^T H_u Mu, applied as Mu^T (H_u (Mu h))
    const R h0 = (R)geo.Mu[0][0] * c0 + (R)geo.Mu[0][1] * c1 + (R)geo.Mu[0][2] * c2;
    const R h1 = (R)geo.Mu[1][0] * c0 + (R)geo.Mu[1][1] * c1 + (R)geo.Mu[1][2] * c2;
    const R h2 = (R)geo.Mu[2][0] * c0 + (R)geo.Mu[2][1] * c1 + (R)geo.Mu[2][2] * c2;
    const R u0 = hxx * h0 + hxy * h1 + hxz * h2;
    const R u1 = hxy * h0 + hyy * h1 + hyz * h2;
    const R u2 = hxz * h0 + hyz * h1 + hzz * h2;
    double f0 = (double)((R)geo.Mu[0][0] * u0 + (R)geo.Mu[1][0] * u1 + (R)geo.Mu[2][0] * u2);
    double f1 = (double)((R)geo.Mu[0][1] * u0 + (R)geo.Mu[1][1] * u1 + (R)geo.Mu[2][1] * u2);
    double f2 = (double)((R)geo.Mu[0][2] * u0 + (R)geo.Mu[1][2] * u1 + (R)geo.Mu[2][2] * u2);
    for (int off = 1; off < 64; off <<= 1) {
      f0 += __shfl_xor(f0, off);
      f1 += __shfl_xor(f1, off);
      f2 += __shfl_xor(f2, off);
    }
    if (lane == 0) {
      fsum[3 * (size_t)s] += f0;
      fsum[3 * (size_t)s + 1] += f1;
      fsum[3 * (size_t)s + 2] += f2;
    }
  }
}

// Wavefronts per work-group of the gather-type kernels (one atom per wavefront at a
// time; kRedBlocks work-groups per chunk).
int gather_waves(const Geometry& geo) { return geo.gather_waves == 8 ? 8 : 4; }

}  // namespace

template <typename R>
void launch_spread(const Geometry& geo, const SysBuffers& b, int B, int BG, int chunk0,
                   int nchunks, hipStream_t st) {
  const size_t chunk = (size_t)geo.K[2] * geo.K[1] * (geo.K[0] + 2) * BG;
  const int ntiles = geo.tiles[0] * geo.tiles[1] * geo.tiles[2];
  dim3 grd(((ntiles + 3) / 4 + 7) / 8 * 8, nchunks);  // a multiple of 8 (XCD remap)
#define MBD_SPREAD(PP, BB)                                                                  \
  k_spread<R, PP, BB><<<grd, 256, 0, st>>>(geo, b.tile_start, b.tile_atoms, b.base,        \
                                           (const R*)b.th, (const R*)b.dth, (const R*)b.dv, \
                                           B, (R*)b.grid, chunk, chunk0)
#define MBD_SPREAD_P(BB)                    \
  switch (geo.p) {                          \
    case 4: MBD_SPREAD(4, BB); break;       \
    case 6: MBD_SPREAD(6, BB); break;       \
    case 8: MBD_SPREAD(8, BB); break;       \
  }
  switch (BG) {
    case 1: MBD_SPREAD_P(1); break;
    case 2: MBD_SPREAD_P(2); break;
    case 4: MBD_SPREAD_P(4); break;
    case 8: MBD_SPREAD_P(8); break;
    case 16: MBD_SPREAD_P(16); break;
    case 32: MBD_SPREAD_P(32); break;
    case 64: MBD_SPREAD_P(64); break;
  }
#undef MBD_SPREAD_P
#undef MBD_SPREAD
}

template <typename R>
void launch_epilogue(const Geometry& geo, const SysBuffers& b, const double* w, int B, int BG,
                     int chunk0, int nchunks, uint32_t comps, hipStream_t st) {
  const size_t chunk = (size_t)geo.K[2] * geo.K[1] * (geo.K[0] + 2) * BG;
  dim3 grd(kRedBlocks, nchunks);
  const double self_coef = -4.0 * geo.tau * geo.tau * geo.tau / (3.0 * sqrt(M_PI));
#define MBD_GATHER(PP, BB)                                                                  \
  k_gather_epilogue<R, PP, BB><<<grd, 64 * gather_waves(geo), 0, st>>>(                   \
      geo, b.base, (const R*)b.th, (const R*)b.dth, (const R*)b.grid, chunk,               \
      (const R*)b.Ed, w, b.g, b.om2, B, comps, self_coef, b.Lt, b.part, chunk0)
#define MBD_GATHER_P(BB)                    \
  switch (geo.p) {                          \
    case 4: MBD_GATHER(4, BB); break;       \
    case 6: MBD_GATHER(6, BB); break;       \
    case 8: MBD_GATHER(8, BB); break;       \
  }
  switch (BG) {
    case 1: MBD_GATHER_P(1); break;
    case 2: MBD_GATHER_P(2); break;
    case 4: MBD_GATHER_P(4); break;
    case 8: MBD_GATHER_P(8); break;
    case 16: MBD_GATHER_P(16); break;
    case 32: MBD_GATHER_P(32); break;
    case 64: MBD_GATHER_P(64); break;
  }
#undef MBD_GATHER_P
#undef MBD_GATHER
}

template <typename R>
void launch_spme_force(const Geometry& geo, const SysBuffers& b, const void* h, int B, int BG,
                       int chunk0, hipStream_t st, const double* hscale) {
  const size_t chunk = (size_t)geo.K[2] * geo.K[1] * (geo.K[0] + 2) * BG;
  dim3 grd(kRedBlocks, 1);
#define MBD_SF(PP, BB)                                                                      \
  k_spme_force<R, PP, BB><<<grd, 64 * gather_waves(geo), 0, st>>>(                       \
      geo, b.base, (const R*)b.th, (const R*)b.dth,                                         \
                                               (const R*)b.ddth, (const R*)b.grid, chunk,     \
                                               (const R*)h, B, chunk0, b.fsum, hscale)
#define MBD_SF_P(BB)                 \
  switch (geo.p) {                   \
    case 4: MBD_SF(4, BB); break;    \
    case 6: MBD_SF(6, BB); break;    \
    case 8: MBD_SF(8, BB); break;    \
  }
  switch (BG) {
    case 1: MBD_SF_P(1); break;
    case 2: MBD_SF_P(2); break;
    case 4: MBD_SF_P(4); break;
    case 8: MBD_SF_P(8); break;
    case 16: MBD_SF_P(16); break;
    case 32: MBD_SF_P(32); break;
    case 64: MBD_SF_P(64); break;
  }
#undef MBD_SF_P
#undef MBD_SF
}

template void launch_spme_force<float>(const Geometry&, const SysBuffers&, const void*, int, int,
                                       int, hipStream_t, const double*);
template void launch_spme_force<double>(const Geometry&, const SysBuffers&, const void*, int,
                                        int, int, hipStream_t, const double*);

template void launch_spread<float>(const Geometry&, const SysBuffers&, int, int, int, int,
                                   hipStream_t);
template void launch_spread<double>(const Geometry&, const SysBuffers&, int, int, int, int,
                                    hipStream_t);
template void launch_epilogue<float>(const Geometry&, const SysBuffers&, const double*, int, int,
                                     int, int, uint32_t, hipStream_t);
template void launch_epilogue<double>(const Geometry&, const SysBuffers&, const double*, int, int,
                                      int, int, uint32_t, hipStream_t);

}  // namespace mbd
