// Direct-space Ewald field with the damping correction (eq. fld_ewald):
//   E_dir,i = sum over images n and atoms j with |R_j + n - R_i| < r_pair,
//             except (j = i, n = 0), of T_dir(R_j + n - R_i) d_j,
//   T_dir = T_erfc - (1 - f_ij) T = A(r) I - B(r) r r^T.
// Cell list: atoms sorted by cell (slices of the fractional coordinates, width
// >= r_pair / 2 perpendicular to the faces); the neighbour cells of a cell are the
// offsets o in [-nr, nr]^3, wrapped periodically, and the displacement is
// r = loc_j - loc_i + sum_a o_a h_a with cell-local Cartesian coordinates and the
// cell shift vectors h_a = a_a / nc_a, so it stays accurate in single precision,
// works for any cell shape and covers several images when r_pair exceeds half the box.
//
// Two variants:
//  - direct: one thread per target atom, all right-hand sides (B <= 8) in
//    registers, tensors evaluated on the fly;
//  - list:   for B >= 16. The positions do not change during a Lanczos run, so
//    the tensors are evaluated once per device setup (k_pair_build) and kept in
//    device memory, grouped by 16 consecutive sorted target atoms: for every
//    source image within r_pair of at least one target of the group, a header
//    (source, 16-bit target mask) and the 6 independent components of T_dir for
//    each of the 16 targets (zero where the pair is out of range). Each matvec
//    (k_pair_list) streams a group's tensors through LDS once and applies them to
//    all right-hand sides, one lane per right-hand side, so every source dipole
//    load serves all of the group's targets within range.
#include <algorithm>

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
  int cx, cy, cz;
  cell_coords(c, cx, cy, cz);
  const R xi = loc[4 * s], yi = loc[4 * s + 1], zi = loc[4 * s + 2], si = loc[4 * s + 3];
  const R tau = (R)geo.tau, dd = (R)geo.damp_d;
  const R rp2 = (R)(geo.r_pair * geo.r_pair);
  R acc[NB][3];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b][0] = acc[b][1] = acc[b][2] = R(0);
  for (int oz = -geo.nr[2]; oz <= geo.nr[2]; ++oz) {
    int wz = (cz + oz) % geo.nc[2];
    if (wz < 0) wz += geo.nc[2];
    for (int oy = -geo.nr[1]; oy <= geo.nr[1]; ++oy) {
      int wy = (cy + oy) % geo.nc[1];
      if (wy < 0) wy += geo.nc[1];
      for (int ox = -geo.nr[0]; ox <= geo.nr[0]; ++ox) {
        int wx = (cx + ox) % geo.nc[0];
        if (wx < 0) wx += geo.nc[0];
        const R sx = (R)(ox * geo.hv[0][0] + oy * geo.hv[1][0] + oz * geo.hv[2][0]);
        const R sy = (R)(ox * geo.hv[0][1] + oy * geo.hv[1][1] + oz * geo.hv[2][1]);
        const R sz = (R)(ox * geo.hv[0][2] + oy * geo.hv[1][2] + oz * geo.hv[2][2]);
        const bool zero = (ox == 0 && oy == 0 && oz == 0);
        const int cc = cell_index(wx, wy, wz);
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


// ---------------------------------------------------------------------------
// Tensor list: build (once per device setup) and apply (every matvec).
// ---------------------------------------------------------------------------

// One work-group (256 threads) per group of kGroup consecutive sorted targets.
// Candidate sources are the atoms of the cells around the group whose distance to
// the group's bounding box is below r_pair; those within r_pair of at least one
// target are appended with their tensors, in the order of the cell scan (z, y, x,
// then atom index). The cells are taken in chunks: their atom counts are prefix-summed
// in LDS, every thread tests one candidate of a 256-candidate round, the hits are
// compacted in order (wavefront ballots plus a prefix over the four wavefronts), and
// the tensors of a round are then written with one thread per (candidate, target)
// pair, so that consecutive threads store consecutive tensor words. With cap == 0
// only the counts are produced (plan sizing).
constexpr int kBuildCells = 256;  // cells per chunk of the scan
template <typename R>
__global__ void __launch_bounds__(256)
k_pair_build(const Geometry geo, const int* __restrict__ cell_start,
             const int* __restrict__ scell, const R* __restrict__ loc, int cap,
             int2* __restrict__ hdr, R* __restrict__ Tg, R* __restrict__ Fg,
             int* __restrict__ gcount, int* __restrict__ maxcount) {
  __shared__ R tgt[kGroup][4];
  __shared__ int tcell[kGroup][3];
  __shared__ int red_i[6];
  __shared__ R red_r[6];
  __shared__ int c_pre[kBuildCells + 1];   // prefix of the chunk's cell atom counts
  __shared__ int c_first[kBuildCells];     // first atom of each cell
  __shared__ int c_off[kBuildCells];       // packed (dx, dy, dz) cell offsets
  __shared__ int wcnt[4];
  __shared__ R s_p[256][4];                // compacted hits of a round: position, radius
  __shared__ int s_m[256];                 // their target masks
  __shared__ int s_o[256];                 // their packed cell offsets
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int group = blockIdx.x;
  const int g0 = group * kGroup;
  const int n = geo.n;
  const int nc0 = geo.nc[0], nc1 = geo.nc[1], nc2 = geo.nc[2];
  int c0x, c0y, c0z;
  cell_coords(scell[g0], c0x, c0y, c0z);
  const int ntg = min(kGroup, n - g0);
  // targets relative to the corner of the group's first cell
  if (tid < kGroup) {
    const int ti = g0 + (tid < ntg ? tid : 0);
    int tcx, tcy, tcz;
    cell_coords(scell[ti], tcx, tcy, tcz);
    const int dcx = tcx - c0x, dcy = tcy - c0y, dcz = tcz - c0z;
    const R* tl = loc + 4 * (size_t)ti;
    tgt[tid][0] = tl[0] + (R)(dcx * geo.hv[0][0] + dcy * geo.hv[1][0] + dcz * geo.hv[2][0]);
    tgt[tid][1] = tl[1] + (R)(dcx * geo.hv[0][1] + dcy * geo.hv[1][1] + dcz * geo.hv[2][1]);
    tgt[tid][2] = tl[2] + (R)(dcx * geo.hv[0][2] + dcy * geo.hv[1][2] + dcz * geo.hv[2][2]);
    tgt[tid][3] = tl[3];
    tcell[tid][0] = dcx; tcell[tid][1] = dcy; tcell[tid][2] = dcz;
  }
  __syncthreads();
  // bounding box of the targets and their cell-offset range (wavefront 0 reduces)
  if (wave == 0) {
    const int t = lane < ntg ? lane : 0;
    R b0 = tgt[t][0], b1 = tgt[t][0], b2 = tgt[t][1], b3 = tgt[t][1], b4 = tgt[t][2],
      b5 = tgt[t][2];
    int m0 = tcell[t][0], m1 = tcell[t][0], m2 = tcell[t][1], m3 = tcell[t][1],
        m4 = tcell[t][2], m5 = tcell[t][2];
    for (int off = 1; off < 16; off <<= 1) {
      b0 = min(b0, __shfl_xor(b0, off)); b1 = max(b1, __shfl_xor(b1, off));
      b2 = min(b2, __shfl_xor(b2, off)); b3 = max(b3, __shfl_xor(b3, off));
      b4 = min(b4, __shfl_xor(b4, off)); b5 = max(b5, __shfl_xor(b5, off));
      m0 = min(m0, __shfl_xor(m0, off)); m1 = max(m1, __shfl_xor(m1, off));
      m2 = min(m2, __shfl_xor(m2, off)); m3 = max(m3, __shfl_xor(m3, off));
      m4 = min(m4, __shfl_xor(m4, off)); m5 = max(m5, __shfl_xor(m5, off));
    }
    if (lane == 0) {
      red_r[0] = b0; red_r[1] = b1; red_r[2] = b2;
      red_r[3] = b3; red_r[4] = b4; red_r[5] = b5;
      red_i[0] = m0; red_i[1] = m1; red_i[2] = m2;
      red_i[3] = m3; red_i[4] = m4; red_i[5] = m5;
    }
  }
  __syncthreads();
  const R bx0 = red_r[0], bx1 = red_r[1], by0 = red_r[2], by1 = red_r[3];
  const R bz0 = red_r[4], bz1 = red_r[5];
  const int dx0 = red_i[0] - geo.nr[0], dx1 = red_i[1] + geo.nr[0];
  const int dy0 = red_i[2] - geo.nr[1], dy1 = red_i[3] + geo.nr[1];
  const int dz0 = red_i[4] - geo.nr[2], dz1 = red_i[5] + geo.nr[2];
  const int nx = dx1 - dx0 + 1, ny = dy1 - dy0 + 1, nz = dz1 - dz0 + 1;
  const int ncells = nx * ny * nz;
  const R tau = (R)geo.tau, dd = (R)geo.damp_d;
  const R rp2 = (R)(geo.r_pair * geo.r_pair);
  int count = 0;
  for (int cc0 = 0; cc0 < ncells; cc0 += kBuildCells) {
    const int ncc = min(kBuildCells, ncells - cc0);
    __syncthreads();  // the previous chunk's tables are no longer read
    int cnt_cell = 0;
    if (tid < ncc) {
      const int ci = cc0 + tid;  // scan order: z outermost, then y, then x
      const int dx = dx0 + ci % nx, dy = dy0 + (ci / nx) % ny, dz = dz0 + ci / (nx * ny);
      int wx = (c0x + dx) % nc0; if (wx < 0) wx += nc0;
      int wy = (c0y + dy) % nc1; if (wy < 0) wy += nc1;
      int wz = (c0z + dz) % nc2; if (wz < 0) wz += nc2;
      const int cc = cell_index(wx, wy, wz);
      c_first[tid] = cell_start[cc];
      cnt_cell = cell_start[cc + 1] - cell_start[cc];
      c_off[tid] = ((dx + 512) << 20) | ((dy + 512) << 10) | (dz + 512);
    }
    // prefix of the counts: scan within each wavefront, then the wavefront offsets
    int v = cnt_cell;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    if (lane == 63) wcnt[wave] = v;
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wave; ++w) woff += wcnt[w];
    if (tid < ncc) c_pre[tid + 1] = v + woff;
    if (tid == 0) c_pre[0] = 0;
    __syncthreads();
    const int total = c_pre[ncc];
    for (int r0 = 0; r0 < total; r0 += 256) {
      const int c = r0 + tid;
      uint32_t mask = 0;
      R px = R(0), py = R(0), pz = R(0), ps = R(0);
      int off = 0, j = 0;
      if (c < total) {
        // the cell holding candidate c: largest k with c_pre[k] <= c
        int lo = 0, hi = ncc - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (c_pre[mid] <= c) lo = mid; else hi = mid - 1;
        }
        j = c_first[lo] + (c - c_pre[lo]);
        off = c_off[lo];
        const int dx = (off >> 20) - 512, dy = ((off >> 10) & 1023) - 512,
                  dz = (off & 1023) - 512;
        const R sx = (R)(dx * geo.hv[0][0] + dy * geo.hv[1][0] + dz * geo.hv[2][0]);
        const R sy = (R)(dx * geo.hv[0][1] + dy * geo.hv[1][1] + dz * geo.hv[2][1]);
        const R sz = (R)(dx * geo.hv[0][2] + dy * geo.hv[1][2] + dz * geo.hv[2][2]);
        px = loc[4 * (size_t)j] + sx;
        py = loc[4 * (size_t)j + 1] + sy;
        pz = loc[4 * (size_t)j + 2] + sz;
        ps = loc[4 * (size_t)j + 3];
        const R ex = max(max(bx0 - px, px - bx1), R(0));
        const R ey = max(max(by0 - py, py - by1), R(0));
        const R ez = max(max(bz0 - pz, pz - bz1), R(0));
        if (ex * ex + ey * ey + ez * ez < rp2) {
          for (int t = 0; t < ntg; ++t) {
            const R rx = px - tgt[t][0], ry = py - tgt[t][1], rz = pz - tgt[t][2];
            const bool self = (j == g0 + t) && dx == tcell[t][0] && dy == tcell[t][1] &&
                              dz == tcell[t][2];
            if (!self && rx * rx + ry * ry + rz * rz < rp2) mask |= 1u << t;
          }
        }
      }
      // in-order compaction of the hits
      const unsigned long long bal = __ballot(mask != 0u);
      const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
      if (lane == 0) wcnt[wave] = __popcll(bal);
      __syncthreads();
      int wpre = 0;
      for (int w = 0; w < wave; ++w) wpre += wcnt[w];
      const int nloc = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
      if (mask != 0u) {
        const int li = wpre + below;
        s_p[li][0] = px; s_p[li][1] = py; s_p[li][2] = pz; s_p[li][3] = ps;
        s_m[li] = (int)mask;
        s_o[li] = off;
        const int slot = count + li;
        if (slot < cap) hdr[(size_t)group * cap + slot] = make_int2(j, (int)mask);
      }
      __syncthreads();
      if (cap > 0) {
        // tensors of the round's hits: thread <-> (hit, target)
        for (int p = tid; p < nloc * kGroup; p += 256) {
          const int li = p / kGroup, t = p % kGroup;
          const int slot = count + li;
          if (slot >= cap) continue;
          const uint32_t mk = (uint32_t)s_m[li];
          R A = R(0), Bk = R(0), rx = R(0), ry = R(0), rz = R(0);
          const R qx = s_p[li][0], qy = s_p[li][1], qz = s_p[li][2], qs = s_p[li][3];
          if ((mk >> t) & 1u) {
            rx = qx - tgt[t][0]; ry = qy - tgt[t][1]; rz = qz - tgt[t][2];
            direct_kernel<R>(rx * rx + ry * ry + rz * rz, tau, R(1) / (qs + tgt[t][3]), dd,
                             A, Bk);
          }
          const size_t e = (size_t)group * cap + slot;
          R* o = Tg + e * kCandStride + t * kTensorWords;
          o[0] = A - Bk * rx * rx;
          o[1] = A - Bk * ry * ry;
          o[2] = A - Bk * rz * rz;
          o[3] = -Bk * rx * ry;
          o[4] = -Bk * rx * rz;
          o[5] = -Bk * ry * rz;
          if (Fg) {
            // radial data for forces, evaluated in double precision
            double Ad = 0.0, Bd = 0.0, dA = 0.0, dB = 0.0;
            if ((mk >> t) & 1u) {
              const double r2 = (double)rx * rx + (double)ry * ry + (double)rz * rz;
              direct_kernel_grad(r2, geo.tau, 1.0 / ((double)qs + (double)tgt[t][3]),
                                 geo.damp_d, Ad, Bd, dA, dB);
            }
            R* f = Fg + e * kCandStride + t * kTensorWords;
            f[0] = rx; f[1] = ry; f[2] = rz;
            f[3] = (R)Bd; f[4] = (R)dA; f[5] = (R)dB;
          }
        }
      }
      count += nloc;
      __syncthreads();  // the round's staging is free again
    }
  }
  if (tid == 0) {
    gcount[group] = count;
    atomicMax(maxcount, count);
  }
}

// E_dir of one group at a time per work-group: WPB wavefronts, each with 64 / NSUB
// right-hand sides x NSUB target subsets (lane = rhs + BW * subset), so
// B = 64 WPB / NSUB. More subsets give more wavefronts per group (small systems) and
// fewer target slots per lane. Tensors of CH candidates at a time are staged in LDS;
// the wave-uniform target mask skips out-of-range (target, source) pairs.
// The launch may hold fewer work-groups than groups: each then walks its XCD's range
// of groups with a stride, which leaves compute units and LDS free for the grid
// stages running beside it on another stream.
template <typename R, int NSUB, int WPB>
__global__ void __launch_bounds__(64 * WPB)
k_pair_list(const Geometry geo, const int2* __restrict__ hdr, const R* __restrict__ Tg,
            const int* __restrict__ gcount, int cap, const R* __restrict__ dv,
            R* __restrict__ Ed, int B) {
  constexpr int NT = 64 * WPB;
  constexpr int CH = 16 * WPB < 64 ? 16 * WPB : 64;  // candidates per LDS chunk
  constexpr int KT = kGroup / NSUB;   // target slots per lane
  constexpr int BW = 64 / NSUB;       // right-hand sides per wavefront
  constexpr int W16 = (int)(kCandStride * sizeof(R) / 16);  // 16-byte words per candidate
  __shared__ uint4 Tl4[CH * W16];
  __shared__ int2 hl[CH];
  const R* Tl = reinterpret_cast<const R*>(Tl4);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int rhs = (tid >> 6) * BW + lane % BW;
  const int sub = lane / BW;
  // XCD-aware: each XCD owns a contiguous range of groups (work-groups are dealt to
  // the 8 XCDs round-robin; gridDim.x is a multiple of 8)
  const int ngroups = (geo.n + kGroup - 1) / kGroup;
  const int per = (ngroups + 7) / 8;
  const int nbx = gridDim.x / 8;
  for (int gi = blockIdx.x / 8; gi < per; gi += nbx) {
  const int group = (blockIdx.x % 8) * per + gi;
  if (group >= ngroups) return;  // uniform over the work-group
  const int cnt = min(gcount[group], cap);
  const int2* H = hdr + (size_t)group * cap;
  const uint4* T4 = reinterpret_cast<const uint4*>(Tg + (size_t)group * cap * kCandStride);

  R acc[KT][3];
#pragma unroll
  for (int k = 0; k < KT; ++k) acc[k][0] = acc[k][1] = acc[k][2] = R(0);

  for (int c0 = 0; c0 < cnt; c0 += CH) {
    const int nc = min(CH, cnt - c0);
    __syncthreads();
    for (int w = tid; w < nc * W16; w += NT) Tl4[w] = T4[(size_t)c0 * W16 + w];
    if (tid < nc) hl[tid] = H[c0 + tid];
    __syncthreads();
    int2 h = hl[0];
    int j = __builtin_amdgcn_readfirstlane(h.x);
    const R* dj = dv + (size_t)j * 3 * B + rhs;
    R n0 = dj[0], n1 = dj[B], n2 = dj[2 * B];
    for (int c = 0; c < nc; ++c) {
      const uint32_t msk = (uint32_t)__builtin_amdgcn_readfirstlane(h.y);
      const R d0 = n0, d1 = n1, d2 = n2;
      if (c + 1 < nc) {  // next candidate's dipoles while this one is applied
        h = hl[c + 1];
        j = __builtin_amdgcn_readfirstlane(h.x);
        dj = dv + (size_t)j * 3 * B + rhs;
        n0 = dj[0]; n1 = dj[B]; n2 = dj[2 * B];
      }
      const R* Tc = Tl + c * kCandStride + sub * kTensorWords;
      // masked slots only (the kernel is close to the LDS read bandwidth); the sums
      // go into the accumulators as fused multiply-add chains
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        if ((msk >> (k * NSUB)) & ((1u << NSUB) - 1u)) {
          const R* t = Tc + k * NSUB * kTensorWords;
          const R txx = t[0], tyy = t[1], tzz = t[2], txy = t[3], txz = t[4], tyz = t[5];
          R* a = acc[k];
          a[0] = fma(txx, d0, a[0]);
          a[0] = fma(txy, d1, a[0]);
          a[0] = fma(txz, d2, a[0]);
          a[1] = fma(txy, d0, a[1]);
          a[1] = fma(tyy, d1, a[1]);
          a[1] = fma(tyz, d2, a[1]);
          a[2] = fma(txz, d0, a[2]);
          a[2] = fma(tyz, d1, a[2]);
          a[2] = fma(tzz, d2, a[2]);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = group * kGroup + k * NSUB + sub;
    if (i < geo.n) {
      Ed[((size_t)i * 3 + 0) * B + rhs] = acc[k][0];
      Ed[((size_t)i * 3 + 1) * B + rhs] = acc[k][1];
      Ed[((size_t)i * 3 + 2) * B + rhs] = acc[k][2];
    }
  }
  }  // groups of this work-group
}

// E_dir of a group on the matrix cores (float, B a multiple of 64). For the group's 16
// targets t the field is one dense product over k = 3 c + b (candidate c, component b):
//   E[t][a][rhs] = sum_k T_(c,t)[a][b] d_(j(c))[b][rhs],
// the list's zero tensors standing for out-of-range (target, candidate) pairs. It is
// computed as three 16-row tiles (a = x, y, z) times NT column tiles of 16 right-hand
// sides with v_mfma_f32_16x16x4_f32, four rows of k per instruction: the instruction
// takes A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k and leaves D[i][j] in
// register i % 4 of lane j + 16 (i / 4). A wavefront owns 16 NT right-hand sides and
// every NK-th block of four candidates (three steps of four k rows); the NK partial
// products of a group are added in LDS
// in wavefront order, so the result does not depend on timing. The source atoms of up
// to kMfmaChunk candidates at a time are staged in LDS; each lane then reads its tensor
// row and dipole component straight from global memory, one block of three steps ahead
// of the matrix instructions that use them. With NK = 1 the k order is the vector
// kernel's, and so far the two have given the same bits.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaChunk = 1024;  // candidates per LDS chunk (a multiple of 4)

template <int NT>
struct MfmaOperands {
  float a[3];
  float b[NT];
};

template <int NK, int NT, int NN>
__global__ void __launch_bounds__(256)
k_pair_mfma(const Geometry geo, const int2* __restrict__ hdr, const float* __restrict__ Tg,
            const float* __restrict__ Tz, const int* __restrict__ gcount, int cap,
            const float* __restrict__ dv, float* __restrict__ Ed, int B) {
  // partial tiles of one component for the NK-way reduction: [wavefront][tile][lane]
  // for the work-group's NN x NK wavefronts (NN column wavefronts)
  __shared__ f32x4 red[NK > 1 ? NN * NK * NT * 64 : 1];
  __shared__ int jl[kMfmaChunk];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wk = wave % NK, wn = wave / NK;
  const int col = lane & 15, row = lane >> 4;
  // column col of column tile t is right-hand side rhs + t: a lane's NT right-hand
  // sides are contiguous, so its dipoles and results move as 16-byte vectors
  const int rhs = wn * 16 * NT + NT * col;
  const size_t Bs = (size_t)B;
  // XCD-aware walk over groups, as in the vector list kernel
  const int ngroups = (geo.n + kGroup - 1) / kGroup;
  const int per = (ngroups + 7) / 8;
  const int nbx = gridDim.x / 8;
  for (int gi = blockIdx.x / 8; gi < per; gi += nbx) {
    const int group = (blockIdx.x % 8) * per + gi;
    if (group >= ngroups) return;  // uniform over the work-group
    const int cnt = min(gcount[group], cap);
    const int2* H = hdr + (size_t)group * cap;
    const float* T = Tg + (size_t)group * cap * kCandStride;
    f32x4 acc[3][NT];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[a][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < cnt; c0 += kMfmaChunk) {
      const int nc = min(kMfmaChunk, cnt - c0);
      __syncthreads();  // the previous chunk's source atoms have been read
      for (int c = threadIdx.x; c < nc; c += blockDim.x) jl[c] = H[c0 + c].x;
      __syncthreads();
      const float* Tc = T + (size_t)c0 * kCandStride;
      // operands of one step: row b of the symmetric tensor (xx, yy, zz, xy, xz, yz) of
      // candidate c and target col (b = 0: xx xy xz, b = 1: xy yy yz, b = 2: xz yz zz)
      // and component b of the candidate's dipoles. Every load is issued: candidates
      // past the chunk read the zero tensor Tz and the chunk's first dipoles, so no
      // branch hides a load from the compiler's count of loads in flight.
      auto load = [&](int c, int b, const int (&w)[3], MfmaOperands<NT>& o) {
        const bool ok = c < nc;
        const float* tt = ok ? Tc + ((size_t)c * kGroup + col) * kTensorWords : Tz;
        const float4* dj =
            reinterpret_cast<const float4*>(dv + ((size_t)jl[ok ? c : 0] * 3 + b) * Bs + rhs);
        o.a[0] = tt[w[0]]; o.a[1] = tt[w[1]]; o.a[2] = tt[w[2]];
#pragma unroll
        for (int q = 0; q < NT / 4; ++q) {
          const float4 v = dj[q];
          o.b[4 * q] = v.x; o.b[4 * q + 1] = v.y; o.b[4 * q + 2] = v.z; o.b[4 * q + 3] = v.w;
        }
      };
      auto apply = [&](const MfmaOperands<NT>& o) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[a][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[a], o.b[t], acc[a][t], 0, 0, 0);
      };
      // The work comes in blocks of 4 candidates = 12 rows of k = 3 steps, and the
      // wavefront takes blocks p = wk, wk + NK, ...: lane row r of step u of block p has
      // k = 12 p + 4 u + r, so its candidate 4 p + (4 u + r) / 3 and component
      // (4 u + r) % 3 are fixed per lane and step. The operands of the next block are in
      // flight while the matrix instructions of this one run.
      int cu[3], bu[3], wu[3][3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int kq = 4 * u + row;
        cu[u] = kq / 3;
        bu[u] = kq % 3;
        wu[u][0] = bu[u] == 0 ? 0 : bu[u] == 1 ? 3 : 4;
        wu[u][1] = bu[u] == 0 ? 3 : bu[u] == 1 ? 1 : 5;
        wu[u][2] = bu[u] == 0 ? 4 : bu[u] == 1 ? 5 : 2;
      }
      const int nb = (nc + 3) / 4;
      const int m = wk < nb ? (nb - wk + NK - 1) / NK : 0;  // this wavefront's blocks
      MfmaOperands<NT> buf[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) load(4 * wk + cu[u], bu[u], wu[u], buf[u]);
      for (int i = 0; i < m; ++i) {
        const int cn = 4 * (wk + NK * (i + 1));  // first candidate of the next block
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          apply(buf[u]);
          load(cn + cu[u], bu[u], wu[u], buf[u]);
          // keep each step's instructions together: interleaving the accumulator chains
          // of neighbouring steps makes the register allocator double the accumulators
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // D[i][j] in register i % 4 of lane j + 16 (i / 4): target 4 row + r, column col;
    // the lane's four right-hand sides rhs + 4 q .. rhs + 4 q + 3 of component a
    auto store = [&](int a, int q, const f32x4 (&v)[4]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = group * kGroup + 4 * row + r;
        if (i < geo.n)
          *reinterpret_cast<float4*>(Ed + ((size_t)i * 3 + a) * Bs + rhs + 4 * q) =
              make_float4(v[0][r], v[1][r], v[2][r], v[3][r]);
      }
    };
    if constexpr (NK == 1) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < NT / 4; ++q) {
          const f32x4 v[4] = {acc[a][4 * q], acc[a][4 * q + 1], acc[a][4 * q + 2],
                              acc[a][4 * q + 3]};
          store(a, q, v);
        }
    } else {
      // one component at a time: every wavefront leaves its partial tiles in LDS, then
      // wavefront wk adds the NK partials of the quads q = wk, wk + NK, ... in wavefront
      // order and stores them
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        __syncthreads();  // the previous round's partials have been read
#pragma unroll
        for (int t = 0; t < NT; ++t) red[((wn * NK + wk) * NT + t) * 64 + lane] = acc[a][t];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NT / 4; ++q) {
          if (q % NK != wk) continue;
          f32x4 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            v[u] = red[((wn * NK) * NT + 4 * q + u) * 64 + lane];
#pragma unroll
            for (int w = 1; w < NK; ++w) v[u] += red[((wn * NK + w) * NT + 4 * q + u) * 64 + lane];
          }
          store(a, q, v);
        }
      }
    }
  }  // groups of this work-group
}


// Direct-space part of the bilinear force term for one reverse step: with
// p = g * lbar_k and q = g * y_k, dS/dR_t for S = sum_(t,j,n) p_t^T T_dir(r) q_j is
//   dS/dR_t = -sum_(j,n) grad_r u,  u = p_t^T T_dir(r) q_j + q_t^T T_dir(r) p_j,
// r = R_j + n - R_t; with T_dir = A I - B r r^T, X = p_t.q_j + q_t.p_j and
// Y = (p_t.r)(q_j.r) + (q_t.r)(p_j.r):
//   grad_r u = r (A'/r X - B'/r Y) - B [p_t (q_j.r) + q_j (p_t.r) + q_t (p_j.r) + p_j (q_t.r)].
// Work-group per group: TW x RS wavefronts; wavefront (tw, rs) owns the targets
// [tw 16/TW, (tw+1) 16/TW) and the right-hand sides [rs BW, (rs+1) BW) (BW = 64/NSUB,
// NSUB > 1 only when B < 64), so the mask branch is uniform and no lane idles on an
// out-of-range pair. TP target slots per pass keep p_t and q_t in registers. The sum
// over right-hand sides is reduced per target and added to fsum (each group owns its
// targets: no atomics, fixed order).
template <typename R, int NSUB, int TW, int RS, int TP>
__global__ void __launch_bounds__(64 * TW * RS)
k_pair_force(const Geometry geo, const int2* __restrict__ hdr, const R* __restrict__ Fg,
             const int* __restrict__ gcount, int cap, const R* __restrict__ pv,
             const R* __restrict__ qv, double* __restrict__ fsum, int B) {
  constexpr int NT = 64 * TW * RS;
  constexpr int CH = 16 * TW * RS < 64 ? 16 * TW * RS : 64;
  constexpr int TPW = kGroup / TW;
  constexpr int KT = TPW / NSUB;
  constexpr int NPASS = KT / TP;
  constexpr int BW = 64 / NSUB;
  constexpr int W16 = (int)(kCandStride * sizeof(R) / 16);
  static_assert(KT >= 1 && KT * NSUB * TW == kGroup && NPASS * TP == KT, "bad split");
  __shared__ uint4 Fl4[CH * W16];
  __shared__ int2 hl[CH];
  __shared__ double red[RS][kGroup][3];
  const R* Fl = reinterpret_cast<const R*>(Fl4);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int tw = wave % TW, rs = wave / TW;
  const int t0 = tw * TPW;
  const int rhs = rs * BW + lane % BW;
  const int sub = lane / BW;
  const int per = (gridDim.x + 7) / 8;
  const int group = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int ngroups = (geo.n + kGroup - 1) / kGroup;
  if (group >= ngroups) return;  // uniform over the work-group
  const int cnt = min(gcount[group], cap);
  const int2* H = hdr + (size_t)group * cap;
  const uint4* F4 = reinterpret_cast<const uint4*>(Fg + (size_t)group * cap * kCandStride);
  for (int pass = 0; pass < NPASS; ++pass) {
    R pt[TP][3], qt[TP][3], G[TP][3];
#pragma unroll
    for (int k = 0; k < TP; ++k) {
      const int i = group * kGroup + t0 + (pass * TP + k) * NSUB + sub;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        pt[k][a] = i < geo.n ? pv[((size_t)i * 3 + a) * B + rhs] : R(0);
        qt[k][a] = i < geo.n ? qv[((size_t)i * 3 + a) * B + rhs] : R(0);
        G[k][a] = R(0);
      }
    }
    for (int c0 = 0; c0 < cnt; c0 += CH) {
      const int nc = min(CH, cnt - c0);
      __syncthreads();
      for (int w = tid; w < nc * W16; w += NT) Fl4[w] = F4[(size_t)c0 * W16 + w];
      if (tid < nc) hl[tid] = H[c0 + tid];
      __syncthreads();
      for (int c = 0; c < nc; ++c) {
        const int2 h = hl[c];
        const int j = __builtin_amdgcn_readfirstlane(h.x);
        const uint32_t msk = (uint32_t)__builtin_amdgcn_readfirstlane(h.y) >> t0;
        const R* pj = pv + (size_t)j * 3 * B + rhs;
        const R* qj = qv + (size_t)j * 3 * B + rhs;
        const R p0 = pj[0], p1 = pj[B], p2 = pj[2 * B];
        const R q0 = qj[0], q1 = qj[B], q2 = qj[2 * B];
        const R* Fc = Fl + c * kCandStride + (t0 + sub) * kTensorWords;
#pragma unroll
        for (int k = 0; k < TP; ++k) {
          const int slot = pass * TP + k;
          if ((msk >> (slot * NSUB)) & ((1u << NSUB) - 1u)) {
            const R* f = Fc + slot * NSUB * kTensorWords;
            const R rx = f[0], ry = f[1], rz = f[2], Bk = f[3], c1 = f[4], c2 = f[5];
            const R prt = pt[k][0] * rx + pt[k][1] * ry + pt[k][2] * rz;
            const R qrt = qt[k][0] * rx + qt[k][1] * ry + qt[k][2] * rz;
            const R prj = p0 * rx + p1 * ry + p2 * rz;
            const R qrj = q0 * rx + q1 * ry + q2 * rz;
            const R X = pt[k][0] * q0 + pt[k][1] * q1 + pt[k][2] * q2 + qt[k][0] * p0 +
                        qt[k][1] * p1 + qt[k][2] * p2;
            const R Y = prt * qrj + qrt * prj;
            const R sc = c1 * X - c2 * Y;
            G[k][0] -= sc * rx - Bk * (pt[k][0] * qrj + q0 * prt + qt[k][0] * prj + p0 * qrt);
            G[k][1] -= sc * ry - Bk * (pt[k][1] * qrj + q1 * prt + qt[k][1] * prj + p1 * qrt);
            G[k][2] -= sc * rz - Bk * (pt[k][2] * qrj + q2 * prt + qt[k][2] * prj + p2 * qrt);
          }
        }
      }
    }
    // sum over the right-hand sides: the BW lanes of a target subset, then the slices
#pragma unroll
    for (int k = 0; k < TP; ++k) {
      double g0 = G[k][0], g1 = G[k][1], g2 = G[k][2];
      for (int off = 1; off < BW; off <<= 1) {
        g0 += __shfl_xor(g0, off);
        g1 += __shfl_xor(g1, off);
        g2 += __shfl_xor(g2, off);
      }
      const int t = t0 + (pass * TP + k) * NSUB + sub;
      if (lane % BW == 0) {
        red[rs][t][0] = g0;
        red[rs][t][1] = g1;
        red[rs][t][2] = g2;
      }
    }
    __syncthreads();
    if (tid < kGroup * 3) {
      const int t = tid / 3, a = tid % 3;
      if (((t % TPW) / NSUB) / TP == pass) {  // target t was handled in this pass
        double v = 0.0;
        for (int r = 0; r < RS; ++r) v += red[r][t][a];
        const int i = group * kGroup + t;
        if (i < geo.n) fsum[3 * (size_t)i + a] += v;
      }
    }
  }
}


// The same direct force term on the matrix cores (float, B a multiple of 16, at most
// 128). Summed over the right-hand sides, a pair's term needs only two 3x3 matrices,
//   M1 = sum_rhs p_t q_j^T,  M2 = sum_rhs q_t p_j^T:
//   X = tr M1 + tr M2,  (M1 + M1^T + M2 + M2^T) r = sum_rhs [p_t (q_j.r) + q_j (p_t.r)
//   + q_t (p_j.r) + p_j (q_t.r)] =: m,  Y = r.m / 2,
//   grad_r u = r (A'/r X - B'/r Y) - B m.
// For a group's 16 targets and a block of 16 candidates, M1 and M2 are dense products
// over the right-hand sides: 9 + 9 tiles of 16 x 16 (component pairs (a, b), rows =
// targets, columns = candidates) with v_mfma_f32_16x16x4_f32 over k = right-hand side.
// The order of k is free: in the u-th of four consecutive steps lane row kk takes right-
// hand side 16 s + 4 kk + u, so that each lane reads its four values as one 16-byte
// vector. The group's p_t and q_t sit in LDS for the whole group; the candidates' p_j and
// q_j come from global memory one group of four steps ahead. After a block's last step
// each lane holds M1 and M2 of the pairs (targets 4 kk .. 4 kk + 3, candidate lane % 16)
// and adds their terms (in-range pairs only) to its float64 partial forces; the 16
// candidate lanes, then the NK wavefronts of the group are summed in a fixed order and
// the group's forces added to fsum (each group owns its targets: no atomics).
template <int NK>
__global__ void __launch_bounds__(64 * NK)
k_pair_force_mfma(const Geometry geo, const int2* __restrict__ hdr, const float* __restrict__ Fg,
                  const int* __restrict__ gcount, int cap, const float* __restrict__ pv,
                  const float* __restrict__ qv, double* __restrict__ fsum, int B) {
  constexpr int kMaxB = 128;
  constexpr int RP = kMaxB + 4;  // padded row of one (vector, component, target) in LDS
  __shared__ float4 tl4[2 * 3 * kGroup * RP / 4];  // [p|q][a][t][rhs]
  __shared__ int jl[kMfmaChunk];
  __shared__ int ml[kMfmaChunk];
  __shared__ double red[NK][kGroup][3];
  float* tl = reinterpret_cast<float*>(tl4);
  const int lane = threadIdx.x & 63;
  const int wk = threadIdx.x >> 6;
  const int col = lane & 15, row = lane >> 4;
  const size_t Bs = (size_t)B;
  const int ngroups = (geo.n + kGroup - 1) / kGroup;
  const int per = (ngroups + 7) / 8;
  const int nbx = gridDim.x / 8;
  for (int gi = blockIdx.x / 8; gi < per; gi += nbx) {
    const int group = (blockIdx.x % 8) * per + gi;
    if (group >= ngroups) return;  // uniform over the work-group
    const int cnt = min(gcount[group], cap);
    const int2* H = hdr + (size_t)group * cap;
    const float* F = Fg + (size_t)group * cap * kCandStride;
    __syncthreads();  // the previous group's LDS contents have been read
    // the group's p_t and q_t: [x][a][t][rhs], zero for targets past the end
    for (int e = threadIdx.x; e < 2 * 3 * kGroup * B; e += 64 * NK) {
      const int r = e % B, t = (e / B) % kGroup, a = (e / (B * kGroup)) % 3, x = e / (B * kGroup * 3);
      const int i = group * kGroup + t;
      const float* src = x == 0 ? pv : qv;
      tl[((x * 3 + a) * kGroup + t) * RP + r] = i < geo.n ? src[((size_t)i * 3 + a) * Bs + r] : 0.f;
    }
    double G[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) G[r][0] = G[r][1] = G[r][2] = 0.0;
    for (int c0 = 0; c0 < cnt; c0 += kMfmaChunk) {
      const int nc = min(kMfmaChunk, cnt - c0);
      __syncthreads();  // the previous chunk's lists have been read
      for (int c = threadIdx.x; c < nc; c += 64 * NK) {
        const int2 h = H[c0 + c];
        jl[c] = h.x;
        ml[c] = h.y;
      }
      __syncthreads();
      const int nb = (nc + 15) / 16;  // blocks of 16 candidates
      for (int blk = wk; blk < nb; blk += NK) {
        const int c = blk * 16 + col;  // this lane's candidate column
        const bool ok = c < nc;
        const int j = jl[ok ? c : 0];
        const float4* pj4 = reinterpret_cast<const float4*>(pv + (size_t)j * 3 * Bs);
        const float4* qj4 = reinterpret_cast<const float4*>(qv + (size_t)j * 3 * Bs);
        f32x4 m1[9], m2[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) m1[q] = m2[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        // candidate operands of the four steps of group s: components b of p_j and q_j at
        // right-hand sides 16 s + 4 row .. + 3
        float4 bp[3], bq[3];
        auto load_b = [&](int s, float4 (&xp)[3], float4 (&xq)[3]) {
          const int o = (s < B / 16 ? 4 * s + row : row);  // float4 index within a row
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            xp[b] = pj4[b * (Bs / 4) + o];
            xq[b] = qj4[b * (Bs / 4) + o];
          }
        };
        load_b(0, bp, bq);
        for (int s = 0; s < B / 16; ++s) {
          float4 np[3], nq[3];
          load_b(s + 1, np, nq);
          // target operands from LDS: components a of p_t and q_t, target col
          float4 ap[3], aq[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            ap[a] = *reinterpret_cast<const float4*>(&tl[((0 * 3 + a) * kGroup + col) * RP + 16 * s + 4 * row]);
            aq[a] = *reinterpret_cast<const float4*>(&tl[((1 * 3 + a) * kGroup + col) * RP + 16 * s + 4 * row]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int b = 0; b < 3; ++b) {
                m1[3 * a + b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[a][u], bq[b][u], m1[3 * a + b], 0, 0, 0);
                m2[3 * a + b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[a][u], bp[b][u], m2[3 * a + b], 0, 0, 0);
              }
          }
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            bp[b] = np[b];
            bq[b] = nq[b];
          }
        }
        // the block's pairs (target 4 row + r, candidate c): D[i][j] sits in register
        // i % 4 of lane j + 16 (i / 4)
        const uint32_t msk = ok ? (uint32_t)ml[c] : 0u;
        const float* f = F + ((size_t)(c0 + (ok ? c : 0)) * kGroup + 4 * row) * kTensorWords;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!((msk >> (4 * row + r)) & 1u)) continue;
          const float rx = f[6 * r], ry = f[6 * r + 1], rz = f[6 * r + 2];
          const float Bk = f[6 * r + 3], c1 = f[6 * r + 4], c2 = f[6 * r + 5];
          float M[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) M[a][b] = m1[3 * a + b][r] + m2[3 * a + b][r];
          const float X = M[0][0] + M[1][1] + M[2][2];
          const float mx = (M[0][0] + M[0][0]) * rx + (M[0][1] + M[1][0]) * ry + (M[0][2] + M[2][0]) * rz;
          const float my = (M[1][0] + M[0][1]) * rx + (M[1][1] + M[1][1]) * ry + (M[1][2] + M[2][1]) * rz;
          const float mz = (M[2][0] + M[0][2]) * rx + (M[2][1] + M[1][2]) * ry + (M[2][2] + M[2][2]) * rz;
          const float Y = 0.5f * (rx * mx + ry * my + rz * mz);
          const float sc = c1 * X - c2 * Y;
          G[r][0] -= (double)(sc * rx - Bk * mx);
          G[r][1] -= (double)(sc * ry - Bk * my);
          G[r][2] -= (double)(sc * rz - Bk * mz);
        }
      }
    }
    // sum over the 16 candidate lanes of each row, then over the wavefronts in order
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double v = G[r][a];
        for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off);
        G[r][a] = v;
      }
    if (col == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) red[wk][4 * row + r][a] = G[r][a];
    }
    __syncthreads();
    if (threadIdx.x < kGroup * 3) {
      const int t = threadIdx.x / 3, a = threadIdx.x % 3;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < NK; ++w) v += red[w][t][a];
      const int i = group * kGroup + t;
      if (i < geo.n) fsum[3 * (size_t)i + a] += v;
    }
  }  // groups of this work-group
}


// Replica method (eq. replica): E_i = sum over images n and atoms j with
// |R_j + n - R_i| < R_cut, except (j = i, n = 0), of f T(r) d_j, the damped bare tensor
// (A = f / r^3, B = 3 f / r^5). Float64, any B <= 8 right-hand sides. One work-group
// per target; its threads stride over the (image, source) pairs, and the partial
// fields are reduced in LDS. Displacements are formed from fractional coordinates.
template <int NB>
__global__ void __launch_bounds__(256)
k_replica(const Geometry geo, const int* __restrict__ perm, const double* __restrict__ frac,
          const int* __restrict__ images, const double* __restrict__ loc,
          const double* __restrict__ dv, double* __restrict__ Ed, int B) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int n = geo.n;
  const int is = perm[s];
  const double fi0 = frac[3 * is], fi1 = frac[3 * is + 1], fi2 = frac[3 * is + 2];
  const double Si = loc[4 * s + 3];
  const double rc2 = geo.replica_cut * geo.replica_cut;
  double acc[NB][3];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b][0] = acc[b][1] = acc[b][2] = 0.0;
  const long total = (long)geo.n_images * n;
  for (long q = threadIdx.x; q < total; q += 256) {
    const int im = (int)(q / n), j = (int)(q % n);
    const int jo = perm[j];
    const double u0 = frac[3 * jo] - fi0 + images[3 * im];
    const double u1 = frac[3 * jo + 1] - fi1 + images[3 * im + 1];
    const double u2 = frac[3 * jo + 2] - fi2 + images[3 * im + 2];
    const double rx = u0 * geo.A[0][0] + u1 * geo.A[1][0] + u2 * geo.A[2][0];
    const double ry = u0 * geo.A[0][1] + u1 * geo.A[1][1] + u2 * geo.A[2][1];
    const double rz = u0 * geo.A[0][2] + u1 * geo.A[1][2] + u2 * geo.A[2][2];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 >= rc2 || (j == s && r2 < 1e-12)) continue;
    const double r = sqrt(r2);
    const double ir2 = 1.0 / r2, ir3 = ir2 / r;
    const double z = geo.damp_d * (r / (Si + loc[4 * j + 3]) - 1.0);
    const double f = 1.0 / (1.0 + exp(-z));
    const double A = f * ir3, Bk = 3.0 * f * ir3 * ir2;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b >= B) break;
      const double d0 = dv[(j * 3 + 0) * B + b];
      const double d1 = dv[(j * 3 + 1) * B + b];
      const double d2 = dv[(j * 3 + 2) * B + b];
      const double rd = Bk * (rx * d0 + ry * d1 + rz * d2);
      acc[b][0] += A * d0 - rx * rd;
      acc[b][1] += A * d1 - ry * rd;
      acc[b][2] += A * d2 - rz * rd;
    }
  }
  for (int b = 0; b < NB && b < B; ++b)
    for (int a = 0; a < 3; ++a) {
      red[threadIdx.x] = acc[b][a];
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
      }
      if (threadIdx.x == 0) Ed[((size_t)s * 3 + a) * B + b] = red[0];
      __syncthreads();
    }
}

template <typename R>
__global__ void k_count_pairs(const Geometry geo, const int* __restrict__ cell_start,
                              const int* __restrict__ scell, const R* __restrict__ loc,
                              unsigned long long* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= geo.n) return;
  const int c = scell[s];
  int cx, cy, cz;
  cell_coords(c, cx, cy, cz);
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
        const int cc = cell_index(wx, wy, wz);
        for (int j = cell_start[cc]; j < cell_start[cc + 1]; ++j) {
          if (zero && j == s) continue;
          const R rx = loc[4 * j] - xi +
                       (R)(ox * geo.hv[0][0] + oy * geo.hv[1][0] + oz * geo.hv[2][0]);
          const R ry = loc[4 * j + 1] - yi +
                       (R)(ox * geo.hv[0][1] + oy * geo.hv[1][1] + oz * geo.hv[2][1]);
          const R rz = loc[4 * j + 2] - zi +
                       (R)(ox * geo.hv[0][2] + oy * geo.hv[1][2] + oz * geo.hv[2][2]);
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

// Target subsets per wavefront for the list kernels: at least 64 / B (every lane
// busy); g.pair_ns when set and valid (a power of two, at least 64 / B, at most 4);
// otherwise doubled (up to 4) while the launch would have fewer than 4096 wavefronts
// (4 per SIMD), so that small systems still fill the GPU.
int pair_subsets(const Geometry& g, int ngroups, int B) {
  int ns = B >= 64 ? 1 : 64 / B;
  if (g.pair_ns > 0) return std::max(ns, std::min(4, g.pair_ns));
  while (ns < 4 && (long)ngroups * B * ns / 64 < 4096) ns *= 2;
  return ns;
}

// Work-groups of a list-kernel launch: one per group (rounded up to a multiple of 8),
// or g.pair_blocks when that is set and smaller (multiple of 8: each XCD gets the same
// number of work-groups).
int pair_blocks(const Geometry& g, int ngroups) {
  const int all = (ngroups + 7) / 8 * 8;
  return g.pair_blocks > 0 ? std::min(all, std::max(8, g.pair_blocks / 8 * 8)) : all;
}

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
  // a multiple of 8 work-groups, so that the XCD remap covers every group
  const int ngroups = (g.n + kGroup - 1) / kGroup;
  const int nblk = pair_blocks(g, ngroups);
  const int2* H = b.pg_hdr;
  const R* T = (const R*)b.pg_T;
  if constexpr (sizeof(R) == 4) {
    // matrix cores: 128 right-hand sides per wavefront (64 when B = 64 or 192, or with
    // pair_mode 2), B / wide column wavefronts x NK candidate shares per group (NK from
    // pair_ns, at most 4 wavefronts per work-group)
    if ((g.pair_mode == 1 || g.pair_mode == 2) && B % 64 == 0 && B <= 256) {
      const int wide = (g.pair_mode == 1 && B % 128 == 0) ? 128 : 64;
      const int nn = B / wide;
      int nk = g.pair_ns > 0 ? g.pair_ns : 1;
      while (nk > 1 && nn * nk > 4) nk /= 2;
      const dim3 blk(64 * nn * nk);
      const float* Tf = (const float*)T;
      const float* df = (const float*)dv;
      float* Ef = (float*)Ed;
#define MBD_PM(NK, NT, NN) \
      k_pair_mfma<NK, NT, NN><<<nblk, blk, 0, st>>>(g, H, Tf, (const float*)b.pg_zero, b.pg_count, \
                                            b.pg_cap, df, Ef, B)
      // (nk > 1 only with nn <= 2, and nn = 2 only with nk <= 2)
      if (nk == 1) {
        if (wide == 128) MBD_PM(1, 8, 1); else MBD_PM(1, 4, 1);
      } else if (wide == 128) {
        if (nk == 4) MBD_PM(4, 8, 1); else if (nn == 1) MBD_PM(2, 8, 1); else MBD_PM(2, 8, 2);
      } else {
        if (nk == 4) MBD_PM(4, 4, 1); else if (nn == 1) MBD_PM(2, 4, 1); else MBD_PM(2, 4, 2);
      }
#undef MBD_PM
      return;
    }
  }
  const int ns = pair_subsets(g, ngroups, B);
#define MBD_PL(NS, WP) \
  k_pair_list<R, NS, WP><<<nblk, 64 * WP, 0, st>>>(g, H, T, b.pg_count, b.pg_cap, dv, Ed, B)
  switch (B * 16 + ns) {
    case 16 * 16 + 4: MBD_PL(4, 1); break;
    case 32 * 16 + 2: MBD_PL(2, 1); break;
    case 32 * 16 + 4: MBD_PL(4, 2); break;
    case 64 * 16 + 1: MBD_PL(1, 1); break;
    case 64 * 16 + 2: MBD_PL(2, 2); break;
    case 64 * 16 + 4: MBD_PL(4, 4); break;
    case 128 * 16 + 1: MBD_PL(1, 2); break;
    case 128 * 16 + 2: MBD_PL(2, 4); break;
    case 128 * 16 + 4: MBD_PL(4, 8); break;
    case 256 * 16 + 1: MBD_PL(1, 4); break;
    case 256 * 16 + 2: MBD_PL(2, 8); break;
    default: MBD_PL(4, 16); break;
  }
#undef MBD_PL
}

template <typename R>
void launch_pair_build(const Geometry& g, const SysBuffers& b, bool count_only, hipStream_t st) {
  const int ngroups = (g.n + kGroup - 1) / kGroup;
  fill_int(b.pg_max, 0, 1, st);
  k_pair_build<R><<<ngroups, 256, 0, st>>>(
      g, b.cell_start, b.scell, (const R*)b.loc, count_only ? 0 : b.pg_cap, b.pg_hdr,
      (R*)b.pg_T, count_only ? nullptr : (R*)b.pg_F, b.pg_count, b.pg_max);
}

template <typename R>
void launch_pair_force(const Geometry& g, const SysBuffers& b, int B, hipStream_t st) {
  const int ngroups = (g.n + kGroup - 1) / kGroup;
  const int nblk = (ngroups + 7) / 8 * 8;
  const int2* H = b.pg_hdr;
  const R* F = (const R*)b.pg_F;
  const R* p = (const R*)b.dv;
  const R* q = (const R*)b.dq;
  if constexpr (sizeof(R) == 4) {
    // matrix cores, with the matrix-core direct sum: four wavefronts per group
    if ((g.pair_mode == 1 || g.pair_mode == 2) && B % 16 == 0 && B <= 128) {
      // one work-group per group, whatever residency cap the direct sum runs with
      k_pair_force_mfma<4><<<(ngroups + 7) / 8 * 8, 256, 0, st>>>(
          g, H, (const float*)F, b.pg_count, b.pg_cap, (const float*)p, (const float*)q,
          b.fsum + 3 * (size_t)g.n, B);
      return;
    }
  }
  // right-hand-side slices of 64 (or target subsets when B < 64), then target splits
  // over 1-4 wavefronts until the launch has 4096 wavefronts
  const int rs = B >= 64 ? B / 64 : 1;
  const int nsub = B >= 64 ? 1 : 64 / B;  // lane subsets: at most 16 / nsub wavefronts
  int tw = 1;
  while (tw < 4 && tw * nsub < 16 && tw * rs < 16 && (long)ngroups * tw * rs < 4096) tw *= 2;
#define MBD_PF(NS, TWV, RSV, TPV)                                                        \
  k_pair_force<R, NS, TWV, RSV, TPV><<<nblk, 64 * TWV * RSV, 0, st>>>(                   \
      g, H, F, b.pg_count, b.pg_cap, p, q, b.fsum + 3 * (size_t)g.n, B)
  switch (B * 16 + tw) {
    case 4 * 16 + 1: MBD_PF(16, 1, 1, 1); break;
    case 8 * 16 + 1: MBD_PF(8, 1, 1, 2); break;
    case 8 * 16 + 2: MBD_PF(8, 2, 1, 1); break;
    case 16 * 16 + 1: MBD_PF(4, 1, 1, 4); break;
    case 16 * 16 + 2: MBD_PF(4, 2, 1, 2); break;
    case 16 * 16 + 4: MBD_PF(4, 4, 1, 1); break;
    case 32 * 16 + 1: MBD_PF(2, 1, 1, 8); break;
    case 32 * 16 + 2: MBD_PF(2, 2, 1, 4); break;
    case 32 * 16 + 4: MBD_PF(2, 4, 1, 2); break;
    case 64 * 16 + 1: MBD_PF(1, 1, 1, 8); break;
    case 64 * 16 + 2: MBD_PF(1, 2, 1, 8); break;
    case 64 * 16 + 4: MBD_PF(1, 4, 1, 4); break;
    case 128 * 16 + 1: MBD_PF(1, 1, 2, 8); break;
    case 128 * 16 + 2: MBD_PF(1, 2, 2, 8); break;
    case 128 * 16 + 4: MBD_PF(1, 4, 2, 4); break;
    case 256 * 16 + 1: MBD_PF(1, 1, 4, 8); break;
    case 256 * 16 + 2: MBD_PF(1, 2, 4, 8); break;
    default: MBD_PF(1, 4, 4, 4); break;
  }
#undef MBD_PF
}

template void launch_pair_force<float>(const Geometry&, const SysBuffers&, int, hipStream_t);
template void launch_pair_force<double>(const Geometry&, const SysBuffers&, int, hipStream_t);


void launch_replica(const Geometry& g, const SysBuffers& b, int B, hipStream_t st) {
  const double* loc = (const double*)b.loc;
  const double* dv = (const double*)b.dv;
  double* Ed = (double*)b.Ed;
  switch (B) {
    case 1: k_replica<1><<<g.n, 256, 0, st>>>(g, b.perm, b.wpos, b.images, loc, dv, Ed, B); break;
    case 2: k_replica<2><<<g.n, 256, 0, st>>>(g, b.perm, b.wpos, b.images, loc, dv, Ed, B); break;
    case 4: k_replica<4><<<g.n, 256, 0, st>>>(g, b.perm, b.wpos, b.images, loc, dv, Ed, B); break;
    default: k_replica<8><<<g.n, 256, 0, st>>>(g, b.perm, b.wpos, b.images, loc, dv, Ed, B); break;
  }
}

template void launch_pair<float>(const Geometry&, const SysBuffers&, int, hipStream_t);
template void launch_pair<double>(const Geometry&, const SysBuffers&, int, hipStream_t);
template void launch_pair_build<float>(const Geometry&, const SysBuffers&, bool, hipStream_t);
template void launch_pair_build<double>(const Geometry&, const SysBuffers&, bool, hipStream_t);

}  // namespace mbd
