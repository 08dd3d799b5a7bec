// Direct-space Ewald field with the damping correction (eq. fld_ewald):
//   E_dir,i = sum over images n and atoms j with |R_j + n - R_i| < r_pair,
//             except (j = i, n = 0), of T_dir(R_j + n - R_i) d_j,
//   T_dir = T_erfc - (1 - f_ij) T = A(r) I - B(r) r r^T.
// Cell list: atoms sorted by cell (edge >= r_pair / 2); the neighbour cells of a
// cell are the offsets o in [-nr, nr]^3, wrapped periodically, and the
// displacement is r = loc_j - loc_i + o * h with cell-local coordinates, so it
// stays accurate in single precision and covers several images when r_pair
// exceeds half the box.
//
// Two variants:
//  - direct: one thread per target atom, all right-hand sides (B <= 8) in registers;
//  - tiled:  a work-group per (target cell, group of BP right-hand sides). Phase 1
//    evaluates the tensor for up to 256 (target, source) candidates, one per lane,
//    into LDS; phase 2 has one lane per right-hand side and applies the stored
//    3x3 tensors of the valid pairs to the source dipoles.
#include "common.h"
#include "mbd_math.h"

namespace mbd {

namespace {

template <typename R, int NB>
__global__ void __launch_bounds__(128)
k_pair_direct(const Geometry geo, const int* __restrict__ cell_start,
              const int* __restrict__ scell, const R* __restrict__ loc,
              const R* __restrict__ dv, R* __restrict__ Ed, int B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  const int c = scell[s];
  const int cx = c % geo.nc[0], cy = (c / geo.nc[0]) % geo.nc[1], cz = c / (geo.nc[0] * geo.nc[1]);
  const R xi = loc[4 * s], yi = loc[4 * s + 1], zi = loc[4 * s + 2], si = loc[4 * s + 3];
  const R tau = (R)geo.tau, dd = (R)geo.damp_d;
  const R rp2 = (R)(geo.r_pair * geo.r_pair);
  R acc[NB][3];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b][0] = acc[b][1] = acc[b][2] = R(0);
  for (int oz = -geo.nr[2]; oz <= geo.nr[2]; ++oz) {
    int wz = (cz + oz) % geo.nc[2];
    if (wz < 0) wz += geo.nc[2];
    const R sz = (R)(oz * geo.hc[2]);
    for (int oy = -geo.nr[1]; oy <= geo.nr[1]; ++oy) {
      int wy = (cy + oy) % geo.nc[1];
      if (wy < 0) wy += geo.nc[1];
      const R sy = (R)(oy * geo.hc[1]);
      for (int ox = -geo.nr[0]; ox <= geo.nr[0]; ++ox) {
        int wx = (cx + ox) % geo.nc[0];
        if (wx < 0) wx += geo.nc[0];
        const R sx = (R)(ox * geo.hc[0]);
        const bool zero = (ox == 0 && oy == 0 && oz == 0);
        const int cc = (wz * geo.nc[1] + wy) * geo.nc[0] + wx;
        const int j0 = cell_start[cc], j1 = cell_start[cc + 1];
        for (int j = j0; j < j1; ++j) {
          if (zero && j == s) continue;
          const R rx = loc[4 * j] - xi + sx;
          const R ry = loc[4 * j + 1] - yi + sy;
          const R rz = loc[4 * j + 2] - zi + sz;
          const R r2 = rx * rx + ry * ry + rz * rz;
          if (r2 >= rp2) continue;
          const R S = loc[4 * j + 3] + si;
          R A, Bk;
          direct_kernel<R>(r2, tau, R(1) / S, dd, A, Bk);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if (b >= B) break;
            const R d0 = dv[(j * 3 + 0) * B + b];
            const R d1 = dv[(j * 3 + 1) * B + b];
            const R d2 = dv[(j * 3 + 2) * B + b];
            const R rd = Bk * (rx * d0 + ry * d1 + rz * d2);
            acc[b][0] += A * d0 - rx * rd;
            acc[b][1] += A * d1 - ry * rd;
            acc[b][2] += A * d2 - rz * rd;
          }
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b >= B) break;
    Ed[(s * 3 + 0) * B + b] = acc[b][0];
    Ed[(s * 3 + 1) * B + b] = acc[b][1];
    Ed[(s * 3 + 2) * B + b] = acc[b][2];
  }
}

template <typename R, int BP>
__global__ void __launch_bounds__(256)
k_pair_tiled(const Geometry geo, const int* __restrict__ cell_start, const R* __restrict__ loc,
             const R* __restrict__ dv, R* __restrict__ Ed, int B) {
  constexpr int NT = 256 / BP;  // targets per pass
  constexpr int NS = BP;        // sources per batch
  __shared__ R Tt[NT][NS][6];
  __shared__ unsigned char ok[NT][NS];
  const int c = blockIdx.x;
  const int rhs = blockIdx.y * BP + (threadIdx.x % BP);
  const int ti = threadIdx.x / BP;  // phase-2 target slot
  const int pt = threadIdx.x / NS;  // phase-1 target slot
  const int ps = threadIdx.x % NS;  // phase-1 source slot
  const int cx = c % geo.nc[0], cy = (c / geo.nc[0]) % geo.nc[1], cz = c / (geo.nc[0] * geo.nc[1]);
  const int i0 = cell_start[c], i1 = cell_start[c + 1];
  const R tau = (R)geo.tau, dd = (R)geo.damp_d;
  const R rp2 = (R)(geo.r_pair * geo.r_pair);
  for (int tg = i0; tg < i1; tg += NT) {
    const int ia = tg + pt;  // phase-1 target atom
    R xi = R(0), yi = R(0), zi = R(0), si = R(0);
    if (ia < i1) {
      xi = loc[4 * ia]; yi = loc[4 * ia + 1]; zi = loc[4 * ia + 2]; si = loc[4 * ia + 3];
    }
    R e0 = R(0), e1 = R(0), e2 = R(0);
    for (int oz = -geo.nr[2]; oz <= geo.nr[2]; ++oz) {
      int wz = (cz + oz) % geo.nc[2];
      if (wz < 0) wz += geo.nc[2];
      const R sz = (R)(oz * geo.hc[2]);
      for (int oy = -geo.nr[1]; oy <= geo.nr[1]; ++oy) {
        int wy = (cy + oy) % geo.nc[1];
        if (wy < 0) wy += geo.nc[1];
        const R sy = (R)(oy * geo.hc[1]);
        for (int ox = -geo.nr[0]; ox <= geo.nr[0]; ++ox) {
          int wx = (cx + ox) % geo.nc[0];
          if (wx < 0) wx += geo.nc[0];
          const R sx = (R)(ox * geo.hc[0]);
          const bool zero = (ox == 0 && oy == 0 && oz == 0);
          const int cc = (wz * geo.nc[1] + wy) * geo.nc[0] + wx;
          const int j0 = cell_start[cc], j1 = cell_start[cc + 1];
          for (int sb = j0; sb < j1; sb += NS) {
            // phase 1: one candidate pair per lane
            {
              const int j = sb + ps;
              bool v = (ia < i1) && (j < j1) && !(zero && j == ia);
              R A = R(0), Bk = R(0), rx = R(0), ry = R(0), rz = R(0);
              if (v) {
                rx = loc[4 * j] - xi + sx;
                ry = loc[4 * j + 1] - yi + sy;
                rz = loc[4 * j + 2] - zi + sz;
                const R r2 = rx * rx + ry * ry + rz * rz;
                v = r2 < rp2;
                if (v) direct_kernel<R>(r2, tau, R(1) / (loc[4 * j + 3] + si), dd, A, Bk);
              }
              ok[pt][ps] = v ? 1 : 0;
              Tt[pt][ps][0] = A - Bk * rx * rx;
              Tt[pt][ps][1] = A - Bk * ry * ry;
              Tt[pt][ps][2] = A - Bk * rz * rz;
              Tt[pt][ps][3] = -Bk * rx * ry;
              Tt[pt][ps][4] = -Bk * rx * rz;
              Tt[pt][ps][5] = -Bk * ry * rz;
            }
            __syncthreads();
            // phase 2: one lane per right-hand side
            if (rhs < B) {
              const int ns = min(NS, j1 - sb);
              for (int q = 0; q < ns; ++q) {
                if (!ok[ti][q]) continue;
                const int j = sb + q;
                const R d0 = dv[(j * 3 + 0) * B + rhs];
                const R d1 = dv[(j * 3 + 1) * B + rhs];
                const R d2 = dv[(j * 3 + 2) * B + rhs];
                const R* T = Tt[ti][q];
                e0 += T[0] * d0 + T[3] * d1 + T[4] * d2;
                e1 += T[3] * d0 + T[1] * d1 + T[5] * d2;
                e2 += T[4] * d0 + T[5] * d1 + T[2] * d2;
              }
            }
            __syncthreads();
          }
        }
      }
    }
    const int it = tg + ti;
    if (it < i1 && rhs < B) {
      Ed[(it * 3 + 0) * B + rhs] = e0;
      Ed[(it * 3 + 1) * B + rhs] = e1;
      Ed[(it * 3 + 2) * B + rhs] = e2;
    }
  }
}

template <typename R>
__global__ void k_count_pairs(const Geometry geo, const int* __restrict__ cell_start,
                              const int* __restrict__ scell, const R* __restrict__ loc,
                              unsigned long long* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  const int c = scell[s];
  const int cx = c % geo.nc[0], cy = (c / geo.nc[0]) % geo.nc[1], cz = c / (geo.nc[0] * geo.nc[1]);
  const R xi = loc[4 * s], yi = loc[4 * s + 1], zi = loc[4 * s + 2];
  const R rp2 = (R)(geo.r_pair * geo.r_pair);
  unsigned long long cnt = 0;
  for (int oz = -geo.nr[2]; oz <= geo.nr[2]; ++oz) {
    int wz = ((cz + oz) % geo.nc[2] + geo.nc[2]) % geo.nc[2];
    for (int oy = -geo.nr[1]; oy <= geo.nr[1]; ++oy) {
      int wy = ((cy + oy) % geo.nc[1] + geo.nc[1]) % geo.nc[1];
      for (int ox = -geo.nr[0]; ox <= geo.nr[0]; ++ox) {
        int wx = ((cx + ox) % geo.nc[0] + geo.nc[0]) % geo.nc[0];
        const bool zero = (ox == 0 && oy == 0 && oz == 0);
        const int cc = (wz * geo.nc[1] + wy) * geo.nc[0] + wx;
        for (int j = cell_start[cc]; j < cell_start[cc + 1]; ++j) {
          if (zero && j == s) continue;
          const R rx = loc[4 * j] - xi + (R)(ox * geo.hc[0]);
          const R ry = loc[4 * j + 1] - yi + (R)(oy * geo.hc[1]);
          const R rz = loc[4 * j + 2] - zi + (R)(oz * geo.hc[2]);
          cnt += (rx * rx + ry * ry + rz * rz < rp2) ? 1 : 0;
        }
      }
    }
  }
  atomicAdd(count, cnt);
}

}  // namespace

template <typename R>
long long count_pairs(const Geometry& g, const SysBuffers& b, hipStream_t st) {
  unsigned long long* d = nullptr;
  unsigned long long h = 0;
  if (hipMalloc(&d, sizeof(h)) != hipSuccess) return -1;
  hipMemsetAsync(d, 0, sizeof(h), st);
  k_count_pairs<R><<<(g.n + 127) / 128, 128, 0, st>>>(g, b.cell_start, b.scell, (const R*)b.loc, d);
  hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  hipFree(d);
  return (long long)h;
}

template long long count_pairs<float>(const Geometry&, const SysBuffers&, hipStream_t);
template long long count_pairs<double>(const Geometry&, const SysBuffers&, hipStream_t);

template <typename R>
void launch_pair(const Geometry& g, const SysBuffers& b, int B, hipStream_t st) {
  const R* loc = (const R*)b.loc;
  const R* dv = (const R*)b.dv;
  R* Ed = (R*)b.Ed;
  if (B <= 8) {
    const int blocks = (g.n + 127) / 128;
    switch (B) {
      case 1: k_pair_direct<R, 1><<<blocks, 128, 0, st>>>(g, b.cell_start, b.scell, loc, dv, Ed, B); break;
      case 2: k_pair_direct<R, 2><<<blocks, 128, 0, st>>>(g, b.cell_start, b.scell, loc, dv, Ed, B); break;
      case 3:
      case 4: k_pair_direct<R, 4><<<blocks, 128, 0, st>>>(g, b.cell_start, b.scell, loc, dv, Ed, B); break;
      default: k_pair_direct<R, 8><<<blocks, 128, 0, st>>>(g, b.cell_start, b.scell, loc, dv, Ed, B); break;
    }
    return;
  }
  const int ncell = g.nc[0] * g.nc[1] * g.nc[2];
  if (B >= 64) {
    dim3 grd(ncell, (B + 63) / 64);
    k_pair_tiled<R, 64><<<grd, 256, 0, st>>>(g, b.cell_start, loc, dv, Ed, B);
  } else if (B >= 32) {
    dim3 grd(ncell, (B + 31) / 32);
    k_pair_tiled<R, 32><<<grd, 256, 0, st>>>(g, b.cell_start, loc, dv, Ed, B);
  } else {
    dim3 grd(ncell, (B + 15) / 16);
    k_pair_tiled<R, 16><<<grd, 256, 0, st>>>(g, b.cell_start, loc, dv, Ed, B);
  }
}

template void launch_pair<float>(const Geometry&, const SysBuffers&, int, hipStream_t);
template void launch_pair<double>(const Geometry&, const SysBuffers&, int, hipStream_t);

}  // namespace mbd
