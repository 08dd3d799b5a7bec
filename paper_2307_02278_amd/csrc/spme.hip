// SPME spreading and gather (eqs. dipolarr and spme).
//
// Spread: D(k) = sum_j sum_a d_ja dW_j(k)/dR_a with W_j(k) = prod_a M_p(u_ja - k_a),
// stencil k_a = base_a - t_a (t_a = 0..p-1, periodic wrap). The derivative table
// dth already carries the K_a / L_a chain-rule factor (orthorhombic cells).
// One work-group owns an 8x8x8 tile of grid points for one chunk of BG right-hand
// sides, accumulates every atom whose stencil reaches the tile in LDS, then writes
// the tile once (no global atomics, no clearing pass).
//
// Gather + epilogue: E_rec,i = sum_k grad_i W_i(k) phi(k) (eq. spme), then the
// generalized field E* = E_dir + E_rec + E_self and
//   l~ = Omega w + Diag(g) E*      (eq. lk3, in double precision)
// together with per-block partial sums of w . l~ for a_k (eq. recurs2).
#include "common.h"

namespace mbd {

namespace {

template <typename R, int P, int BG>
__global__ void __launch_bounds__(256)
k_spread(const Geometry geo, const int* __restrict__ tile_start,
         const int* __restrict__ tile_atoms, const int* __restrict__ base,
         const R* __restrict__ th, const R* __restrict__ dth, const R* __restrict__ dv, int B,
         R* __restrict__ grid, size_t chunk_elems) {
  constexpr int T = kSpreadTile;
  __shared__ R acc[T * T * T * BG];
  const int tile = blockIdx.x;
  const int chunk = blockIdx.y;
  const int tx = tile % geo.tiles[0];
  const int ty = (tile / geo.tiles[0]) % geo.tiles[1];
  const int tz = tile / (geo.tiles[0] * geo.tiles[1]);
  const int x0 = tx * T, y0 = ty * T, z0 = tz * T;
  for (int i = threadIdx.x; i < T * T * T * BG; i += blockDim.x) acc[i] = R(0);
  __syncthreads();
  const int lo = tile_start[tile], hi = tile_start[tile + 1];
  const int items = (hi - lo) * P * P * BG;
  const int K1 = geo.K[0], K2 = geo.K[1], K3 = geo.K[2];
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int b = it % BG;
    const int rest = it / BG;
    const int row = rest % (P * P);
    const int a = rest / (P * P);
    const int t2 = row / P, t3 = row % P;
    const int s = tile_atoms[lo + a];
    int k2 = base[3 * s + 1] - t2;
    if (k2 < 0) k2 += K2;
    int k3 = base[3 * s + 2] - t3;
    if (k3 < 0) k3 += K3;
    const int ly = k2 - y0, lz = k3 - z0;
    if (ly < 0 || ly >= T || lz < 0 || lz >= T) continue;
    const int bg = chunk * BG + b;
    const R d0 = dv[(s * 3 + 0) * B + bg];
    const R d1 = dv[(s * 3 + 1) * B + bg];
    const R d2 = dv[(s * 3 + 2) * B + bg];
    const R* thp = th + s * 3 * P;
    const R* dthp = dth + s * 3 * P;
    const R m1 = thp[P + t2], dm1 = dthp[P + t2];
    const R m2 = thp[2 * P + t3], dm2 = dthp[2 * P + t3];
    const R A = d0 * m1 * m2;
    const R Bc = d1 * dm1 * m2 + d2 * m1 * dm2;
    const int bx = base[3 * s + 0];
#pragma unroll
    for (int t1 = 0; t1 < P; ++t1) {
      int k1 = bx - t1;
      if (k1 < 0) k1 += K1;
      const int lx = k1 - x0;
      if (lx < 0 || lx >= T) continue;
      const R v = dthp[t1] * A + thp[t1] * Bc;
      atomicAdd(&acc[((lz * T + ly) * T + lx) * BG + b], v);
    }
  }
  __syncthreads();
  R* g = grid + (size_t)chunk * chunk_elems;
  const int XS = K1 + 2;
  for (int i = threadIdx.x; i < T * T * T * BG; i += blockDim.x) {
    const int b = i % BG;
    const int pt = i / BG;
    const int lx = pt % T, ly = (pt / T) % T, lz = pt / (T * T);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    if (x < K1 && y < K2 && z < K3) g[(((size_t)z * K2 + y) * XS + x) * BG + b] = acc[i];
  }
}

template <typename R, int P, int BG>
__global__ void __launch_bounds__(256)
k_gather_epilogue(const Geometry geo, const int* __restrict__ base, const R* __restrict__ th,
                  const R* __restrict__ dth, const R* __restrict__ grid, size_t chunk_elems,
                  const R* __restrict__ Ed, const double* __restrict__ w,
                  const double* __restrict__ g, const double* __restrict__ om2, int B,
                  uint32_t comps, double self_coef, double* __restrict__ lt,
                  double* __restrict__ part) {
  constexpr int ROWS = 256 / BG;
  __shared__ double red[256];
  const int b = threadIdx.x % BG;
  const int row = threadIdx.x / BG;
  const int chunk = blockIdx.y;
  const int bg = chunk * BG + b;
  const R* gr = grid + (size_t)chunk * chunk_elems;
  const int K1 = geo.K[0], K2 = geo.K[1], K3 = geo.K[2];
  const int XS = K1 + 2;
  double dot = 0.0;
  for (int s = blockIdx.x * ROWS + row; s < geo.n; s += gridDim.x * ROWS) {
    R e0 = R(0), e1 = R(0), e2 = R(0);
    if (comps & MBD_C_REC) {
      const R* thp = th + s * 3 * P;
      const R* dthp = dth + s * 3 * P;
      const int bx = base[3 * s], by = base[3 * s + 1], bz = base[3 * s + 2];
#pragma unroll 1
      for (int t3 = 0; t3 < P; ++t3) {
        int k3 = bz - t3;
        if (k3 < 0) k3 += K3;
        const R m3 = thp[2 * P + t3], dm3 = dthp[2 * P + t3];
#pragma unroll 1
        for (int t2 = 0; t2 < P; ++t2) {
          int k2 = by - t2;
          if (k2 < 0) k2 += K2;
          const R m2 = thp[P + t2], dm2 = dthp[P + t2];
          const R* line = gr + ((size_t)k3 * K2 + k2) * XS * BG + b;
          R sx = R(0), sy = R(0);
#pragma unroll
          for (int t1 = 0; t1 < P; ++t1) {
            int k1 = bx - t1;
            if (k1 < 0) k1 += K1;
            const R phi = line[(size_t)k1 * BG];
            sx += dthp[t1] * phi;
            sy += thp[t1] * phi;
          }
          e0 += sx * m2 * m3;
          e1 += sy * dm2 * m3;
          e2 += sy * m2 * dm3;
        }
      }
    }
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
  red[threadIdx.x] = dot;
  __syncthreads();
  for (int h = ROWS / 2; h > 0; h >>= 1) {
    if (row < h) red[threadIdx.x] += red[threadIdx.x + h * BG];
    __syncthreads();
  }
  if (row == 0) part[((size_t)blockIdx.x * 4 + 0) * B + bg] = red[threadIdx.x];
}

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace

template <typename R>
void launch_spread(const Geometry& geo, const SysBuffers& b, int B, int BG, hipStream_t st) {
  const size_t chunk = (size_t)geo.K[2] * geo.K[1] * (geo.K[0] + 2) * BG;
  const int ntiles = geo.tiles[0] * geo.tiles[1] * geo.tiles[2];
  dim3 grd(ntiles, B / BG);
#define MBD_SPREAD(PP, BB)                                                                   \
  k_spread<R, PP, BB><<<grd, 256, 0, st>>>(geo, b.tile_start, b.tile_atoms, b.base,         \
                                           (const R*)b.th, (const R*)b.dth, (const R*)b.dv, \
                                           B, (R*)b.grid, chunk)
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
    case 32:
      if constexpr (sizeof(R) == 4) { MBD_SPREAD_P(32); }
      break;
  }
#undef MBD_SPREAD_P
#undef MBD_SPREAD
}

template <typename R>
void launch_epilogue(const Geometry& geo, const SysBuffers& b, const double* w, int B, int BG,
                     uint32_t comps, hipStream_t st) {
  const size_t chunk = (size_t)geo.K[2] * geo.K[1] * (geo.K[0] + 2) * BG;
  dim3 grd(kRedBlocks, B / BG);
  const double self_coef = -4.0 * geo.tau * geo.tau * geo.tau / (3.0 * sqrt(M_PI));
#define MBD_GATHER(PP, BB)                                                                  \
  k_gather_epilogue<R, PP, BB><<<grd, 256, 0, st>>>(                                       \
      geo, b.base, (const R*)b.th, (const R*)b.dth, (const R*)b.grid, chunk,               \
      (const R*)b.Ed, w, b.g, b.om2, B, comps, self_coef, b.Lt, b.part)
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
  }
#undef MBD_GATHER_P
#undef MBD_GATHER
}

template void launch_spread<float>(const Geometry&, const SysBuffers&, int, int, hipStream_t);
template void launch_spread<double>(const Geometry&, const SysBuffers&, int, int, hipStream_t);
template void launch_epilogue<float>(const Geometry&, const SysBuffers&, const double*, int, int,
                                     uint32_t, hipStream_t);
template void launch_epilogue<double>(const Geometry&, const SysBuffers&, const double*, int, int,
                                      uint32_t, hipStream_t);

}  // namespace mbd
