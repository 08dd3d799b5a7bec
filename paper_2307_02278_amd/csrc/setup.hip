// Position-dependent setup (once per energy evaluation): fractional coordinates
// a*_a . R wrapped into the cell, sort atoms by cell-list cell (cells are slices of
// the fractional coordinates, so any right-handed cell works), cell-local Cartesian
// coordinates for the pair kernel, B-spline tables at the scaled fractional
// coordinates u_a = K_a a*_a . R (eq. scaledfractional, formed in double precision),
// and the per-tile atom lists of the spread kernel.
#include "common.h"
#include "mbd_math.h"

namespace mbd {

namespace {

__global__ void k_wrap_count(const Geometry geo, const double* __restrict__ pos,
                             double* __restrict__ wpos, int* __restrict__ cell_of,
                             uint32_t* __restrict__ subkey, int* __restrict__ count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= geo.n) return;
  const double R0 = pos[3 * i], R1 = pos[3 * i + 1], R2 = pos[3 * i + 2];
  int c[3], f[3];
  for (int a = 0; a < 3; ++a) {
    // fractional coordinate a*_a . R, wrapped into [0, 1)
    double x = geo.Ar[a][0] * R0 + geo.Ar[a][1] * R1 + geo.Ar[a][2] * R2;
    x -= floor(x);
    if (x >= 1.0) x -= 1.0;
    if (x < 0.0) x = 0.0;
    wpos[3 * i + a] = x;
    const double xc = x * geo.nc[a];
    int ci = (int)xc;
    c[a] = ci >= geo.nc[a] ? geo.nc[a] - 1 : ci;
    // 4 sub-cells per axis order the atoms inside the cell
    int fi = (int)((xc - c[a]) * 4.0);
    f[a] = fi < 0 ? 0 : (fi > 3 ? 3 : fi);
  }
  int cell = cell_index(c[0], c[1], c[2]);
  cell_of[i] = cell;
  subkey[i] = (uint32_t)cell_index(f[0], f[1], f[2]);
  atomicAdd(&count[cell], 1);
}

// Exclusive scan of count[0..m) into start[0..m]; one block.
__global__ void k_scan(int m, const int* __restrict__ count, int* __restrict__ start) {
  __shared__ int chunk_sums[1024];
  const int T = blockDim.x;
  const int per = (m + T - 1) / T;
  const int lo = threadIdx.x * per;
  const int hi = min(m, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += count[i];
  chunk_sums[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < T; ++t) {
      int v = chunk_sums[t];
      chunk_sums[t] = acc;
      acc += v;
    }
    start[m] = acc;
  }
  __syncthreads();
  int acc = chunk_sums[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    start[i] = acc;
    acc += count[i];
  }
}

__global__ void k_scatter(int n, const int* __restrict__ cell_of, const int* __restrict__ start,
                          int* __restrict__ cursor, int* __restrict__ perm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_of[i];
  int slot = atomicAdd(&cursor[c], 1);
  perm[start[c] + slot] = i;
}

// Deterministic order inside each cell: by sub-cell (Morton), then caller index.
__global__ void k_sort_cells(int ncell, const int* __restrict__ start,
                             const uint32_t* __restrict__ subkey, int* __restrict__ perm) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  int lo = start[c], hi = start[c + 1];
  for (int i = lo + 1; i < hi; ++i) {
    const int v = perm[i];
    const unsigned long long kv = ((unsigned long long)subkey[v] << 32) | (unsigned)v;
    int j = i - 1;
    while (j >= lo && (((unsigned long long)subkey[perm[j]] << 32) | (unsigned)perm[j]) > kv) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

template <typename R, int P>
__global__ void k_sorted_tables(Geometry geo, const int* __restrict__ perm,
                                const double* __restrict__ wpos,
                                const double* __restrict__ alpha, const double* __restrict__ omega,
                                const double* __restrict__ rvdw, R* __restrict__ loc,
                                double* __restrict__ g, double* __restrict__ om2,
                                int* __restrict__ base, R* __restrict__ th, R* __restrict__ dth,
                                R* __restrict__ ddth, int* __restrict__ tile_count,
                                int* __restrict__ scell) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  const int i = perm[s];
  double x[3];
  int c[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = wpos[3 * i + a];  // fractional
    int ci = (int)(x[a] * geo.nc[a]);
    c[a] = ci >= geo.nc[a] ? geo.nc[a] - 1 : ci;
  }
  // cell-local Cartesian position: sum_a (x_a - c_a / nc_a) a_a
  double rel[3];
  for (int a = 0; a < 3; ++a) rel[a] = x[a] - (double)c[a] / geo.nc[a];
  for (int q = 0; q < 3; ++q)
    loc[4 * s + q] = (R)(rel[0] * geo.A[0][q] + rel[1] * geo.A[1][q] + rel[2] * geo.A[2][q]);
  scell[s] = cell_index(c[0], c[1], c[2]);
  loc[4 * s + 3] = (R)(geo.beta * rvdw[i]);
  g[s] = omega[i] * sqrt(alpha[i]);
  om2[s] = omega[i] * omega[i];
  for (int a = 0; a < 3; ++a) {
    const double u = geo.K[a] * x[a];
    double fl = floor(u);
    double w = u - fl;
    int b0 = (int)fl;
    if (w >= 1.0) { w = 0.0; b0 += 1; }
    b0 %= geo.K[a];
    if (b0 < 0) b0 += geo.K[a];
    base[3 * s + a] = b0;
    // derivatives with respect to u_a; the kernels apply d u / d R = Mu
    double t[P], dt[P], ddt[P];
    if (ddth) {
      bspline_weights2<P>(w, t, dt, ddt);
      for (int k = 0; k < P; ++k) ddth[(s * 3 + a) * P + k] = (R)ddt[k];
    } else {
      bspline_weights<P>(w, t, dt);
    }
    for (int k = 0; k < P; ++k) {
      th[(s * 3 + a) * P + k] = (R)t[k];
      dth[(s * 3 + a) * P + k] = (R)dt[k];
    }
  }
  // tiles touched by the stencil k = base - t, t = 0..P-1 (mod K), per axis
  int tl[3][4], nt[3];
  for (int a = 0; a < 3; ++a) {
    nt[a] = 0;
    for (int k = 0; k < P; ++k) {
      int kk = base[3 * s + a] - k;
      if (kk < 0) kk += geo.K[a];
      int tt = kk / geo.tile[a];
      bool seen = false;
      for (int q = 0; q < nt[a]; ++q) seen |= (tl[a][q] == tt);
      if (!seen) tl[a][nt[a]++] = tt;
    }
  }
  for (int z = 0; z < nt[2]; ++z)
    for (int y = 0; y < nt[1]; ++y)
      for (int xx = 0; xx < nt[0]; ++xx) {
        int tile = (tl[2][z] * geo.tiles[1] + tl[1][y]) * geo.tiles[0] + tl[0][xx];
        atomicAdd(&tile_count[tile], 1);
      }
}

template <int P>
__global__ void k_tile_fill(Geometry geo, const int* __restrict__ base,
                            const int* __restrict__ tile_start, int* __restrict__ cursor,
                            int* __restrict__ tile_atoms) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  int tl[3][4], nt[3];
  for (int a = 0; a < 3; ++a) {
    nt[a] = 0;
    for (int k = 0; k < P; ++k) {
      int kk = base[3 * s + a] - k;
      if (kk < 0) kk += geo.K[a];
      int tt = kk / geo.tile[a];
      bool seen = false;
      for (int q = 0; q < nt[a]; ++q) seen |= (tl[a][q] == tt);
      if (!seen) tl[a][nt[a]++] = tt;
    }
  }
  for (int z = 0; z < nt[2]; ++z)
    for (int y = 0; y < nt[1]; ++y)
      for (int xx = 0; xx < nt[0]; ++xx) {
        int tile = (tl[2][z] * geo.tiles[1] + tl[1][y]) * geo.tiles[0] + tl[0][xx];
        int slot = atomicAdd(&cursor[tile], 1);
        tile_atoms[tile_start[tile] + slot] = s;
      }
}

// x-lines (y, z) covered by the y-z stencil of each atom: y = base_y - t_y, z = base_z - t_z
// (mod K), t = 0..P-1 (P distinct lines per axis, since K >= 2P). First a count per
// line, then, after a scan, the fill of entries (s << 8) | (t_y << 4) | t_z, whose order
// is the atom order.
template <int P>
__global__ void k_line_lists(Geometry geo, const int* __restrict__ base, int* __restrict__ count,
                             const int* __restrict__ start, int* __restrict__ list) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  for (int tz = 0; tz < P; ++tz) {
    int z = base[3 * s + 2] - tz;
    if (z < 0) z += geo.K[2];
    for (int ty = 0; ty < P; ++ty) {
      int y = base[3 * s + 1] - ty;
      if (y < 0) y += geo.K[1];
      const int line = z * geo.K[1] + y;
      const int slot = atomicAdd(&count[line], 1);
      if (start) list[start[line] + slot] = (s << 8) | (ty << 4) | tz;
    }
  }
}

// Deterministic order inside each tile's list.
__global__ void k_sort_tiles(int ntiles, const int* __restrict__ start, int* __restrict__ list) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ntiles) return;
  int lo = start[c], hi = start[c + 1];
  for (int i = lo + 1; i < hi; ++i) {
    int v = list[i];
    int j = i - 1;
    while (j >= lo && list[j] > v) {
      list[j + 1] = list[j];
      --j;
    }
    list[j + 1] = v;
  }
}

inline int blocks_for(int n, int t) { return (n + t - 1) / t; }

__global__ void k_fill_int(int* __restrict__ p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// Kernel-based clear (kept out of hipMemsetAsync so that the sequence can be captured).
void fill_int(int* p, int v, int n, hipStream_t st) {
  k_fill_int<<<blocks_for(n, 256), 256, 0, st>>>(p, v, n);
}

template <typename R>
void launch_setup(const Geometry& g, SysBuffers& b, const double* pos, const double* alpha,
                  const double* omega, const double* rvdw, hipStream_t st) {
  const int ncell = cell_slots(g);
  const int ntiles = g.tiles[0] * g.tiles[1] * g.tiles[2];
  fill_int(b.cell_cursor, 0, ncell, st);
  k_wrap_count<<<blocks_for(g.n, 256), 256, 0, st>>>(g, pos, b.wpos, b.cell_of, b.subkey,
                                                      b.cell_cursor);
  k_scan<<<1, 1024, 0, st>>>(ncell, b.cell_cursor, b.cell_start);
  fill_int(b.cell_cursor, 0, ncell, st);
  k_scatter<<<blocks_for(g.n, 256), 256, 0, st>>>(g.n, b.cell_of, b.cell_start, b.cell_cursor,
                                                   b.perm);
  k_sort_cells<<<blocks_for(ncell, 128), 128, 0, st>>>(ncell, b.cell_start, b.subkey, b.perm);
  fill_int(b.tile_count, 0, ntiles + 1, st);
#define MBD_TABLES(PP)                                                                        \
  k_sorted_tables<R, PP><<<blocks_for(g.n, 128), 128, 0, st>>>(                               \
      g, b.perm, b.wpos, alpha, omega, rvdw, (R*)b.loc, b.g, b.om2, b.base, (R*)b.th,        \
      (R*)b.dth, (R*)b.ddth, b.tile_count, b.scell)
  switch (g.p) {
    case 4: MBD_TABLES(4); break;
    case 6: MBD_TABLES(6); break;
    case 8: MBD_TABLES(8); break;
  }
#undef MBD_TABLES
  k_scan<<<1, 1024, 0, st>>>(ntiles, b.tile_count, b.tile_start);
  fill_int(b.tile_count, 0, ntiles + 1, st);
  switch (g.p) {
    case 4: k_tile_fill<4><<<blocks_for(g.n, 256), 256, 0, st>>>(g, b.base, b.tile_start,
                                                                  b.tile_count, b.tile_atoms);
      break;
    case 6: k_tile_fill<6><<<blocks_for(g.n, 256), 256, 0, st>>>(g, b.base, b.tile_start,
                                                                  b.tile_count, b.tile_atoms);
      break;
    case 8: k_tile_fill<8><<<blocks_for(g.n, 256), 256, 0, st>>>(g, b.base, b.tile_start,
                                                                  b.tile_count, b.tile_atoms);
      break;
  }
  k_sort_tiles<<<blocks_for(ntiles, 128), 128, 0, st>>>(ntiles, b.tile_start, b.tile_atoms);
  if (g.line_lists) launch_line_lists(g, b, st);
}

// Atoms of every (y, z) grid line for the fused x-line spread (p = 6), in atom order.
void launch_line_lists(const Geometry& g, SysBuffers& b, hipStream_t st) {
  if (b.line_start && g.p == 6) {
    const int nlines = g.K[1] * g.K[2];
    fill_int(b.line_count, 0, nlines + 1, st);
    k_line_lists<6><<<blocks_for(g.n, 256), 256, 0, st>>>(g, b.base, b.line_count, nullptr,
                                                          nullptr);
    k_scan<<<1, 1024, 0, st>>>(nlines, b.line_count, b.line_start);
    fill_int(b.line_count, 0, nlines + 1, st);
    k_line_lists<6><<<blocks_for(g.n, 256), 256, 0, st>>>(g, b.base, b.line_count,
                                                          b.line_start, b.line_atoms);
    k_sort_tiles<<<blocks_for(nlines, 128), 128, 0, st>>>(nlines, b.line_start, b.line_atoms);
  }
}

template void launch_setup<float>(const Geometry&, SysBuffers&, const double*, const double*,
                                  const double*, const double*, hipStream_t);
template void launch_setup<double>(const Geometry&, SysBuffers&, const double*, const double*,
                                   const double*, const double*, hipStream_t);

}  // namespace mbd
