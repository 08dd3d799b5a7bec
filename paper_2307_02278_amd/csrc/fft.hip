// 3D FFT of the SPME dipole grid, batched over right-hand sides, with the
// influence-function convolution fused into the last axis (the convolution
// G * D of eq. spme done in Fourier space: forward transform, multiply by
// G(m) = exp(-pi^2 |m|^2 / tau^2) B(m) / (pi V |m|^2), inverse transform).
//
// Layout of one grid chunk (BG right-hand sides, innermost):
//   real value (x, y, z, b)      at ((z K2 + y) XS + x) BG + b,  XS = K1 + 2
//   spectrum (kx, ky, kz, b): re at ((kz K2 + ky) XS + 2 kx) BG + b, im at +BG
// Each pass transforms whole lines of one axis in place. A work-group loads NC
// "columns" (line, b) into LDS, runs a mixed-radix Stockham FFT (radices 4, 2, 3,
// 5) with one lane per column, and writes the columns back. Forward transforms
// use e^{-2 pi i jk/K}, inverse ones e^{+2 pi i jk/K}; neither is normalized.
#include "common.h"

namespace mbd {

namespace {

struct Radices {
  int r[12];
  int n;
};

constexpr Radices factorize(int K) {
  Radices f{};
  f.n = 0;
  int k = K;
  while (k % 4 == 0) { f.r[f.n++] = 4; k /= 4; }
  while (k % 2 == 0) { f.r[f.n++] = 2; k /= 2; }
  while (k % 3 == 0) { f.r[f.n++] = 3; k /= 3; }
  while (k % 5 == 0) { f.r[f.n++] = 5; k /= 5; }
  return f;
}

constexpr int prefix_product(int K, int S) {
  int p = 1;
  for (int i = 0; i < S; ++i) p *= factorize(K).r[i];
  return p;
}

// Length-r DFT in registers; sign -1 forward, +1 inverse.
template <typename R, int r, bool FWD>
__device__ __forceinline__ void small_dft(R* xr, R* xi) {
  constexpr R sg = FWD ? R(-1) : R(1);
  if constexpr (r == 2) {
    R ar = xr[0] + xr[1], ai = xi[0] + xi[1];
    R br = xr[0] - xr[1], bi = xi[0] - xi[1];
    xr[0] = ar; xi[0] = ai; xr[1] = br; xi[1] = bi;
  } else if constexpr (r == 4) {
    R s0r = xr[0] + xr[2], s0i = xi[0] + xi[2];
    R d0r = xr[0] - xr[2], d0i = xi[0] - xi[2];
    R s1r = xr[1] + xr[3], s1i = xi[1] + xi[3];
    R d1r = xr[1] - xr[3], d1i = xi[1] - xi[3];
    // multiply d1 by sg * i
    R jr = -sg * d1i, ji = sg * d1r;
    xr[0] = s0r + s1r; xi[0] = s0i + s1i;
    xr[2] = s0r - s1r; xi[2] = s0i - s1i;
    xr[1] = d0r + jr;  xi[1] = d0i + ji;
    xr[3] = d0r - jr;  xi[3] = d0i - ji;
  } else if constexpr (r == 3) {
    constexpr R h = R(0.86602540378443864676);
    R sr = xr[1] + xr[2], si = xi[1] + xi[2];
    R dr = xr[1] - xr[2], di = xi[1] - xi[2];
    R tr = xr[0] - R(0.5) * sr, ti = xi[0] - R(0.5) * si;
    // (sg * i * h) * d
    R ur = -sg * h * di, ui = sg * h * dr;
    xr[0] = xr[0] + sr; xi[0] = xi[0] + si;
    xr[1] = tr + ur; xi[1] = ti + ui;
    xr[2] = tr - ur; xi[2] = ti - ui;
  } else if constexpr (r == 5) {
    constexpr R c1 = R(0.30901699437494742410);   // cos(2 pi / 5)
    constexpr R c2 = R(-0.80901699437494742410);  // cos(4 pi / 5)
    constexpr R s1 = R(0.95105651629515357212);   // sin(2 pi / 5)
    constexpr R s2 = R(0.58778525229247312917);   // sin(4 pi / 5)
    R ar = xr[1] + xr[4], ai = xi[1] + xi[4];
    R br = xr[1] - xr[4], bi = xi[1] - xi[4];
    R cr = xr[2] + xr[3], ci = xi[2] + xi[3];
    R dr = xr[2] - xr[3], di = xi[2] - xi[3];
    R y0r = xr[0] + ar + cr, y0i = xi[0] + ai + ci;
    R p1r = xr[0] + c1 * ar + c2 * cr, p1i = xi[0] + c1 * ai + c2 * ci;
    R p2r = xr[0] + c2 * ar + c1 * cr, p2i = xi[0] + c2 * ai + c1 * ci;
    // q1 = sg * i * (s1 b + s2 d), q2 = sg * i * (s2 b - s1 d)
    R q1r = -sg * (s1 * bi + s2 * di), q1i = sg * (s1 * br + s2 * dr);
    R q2r = -sg * (s2 * bi - s1 * di), q2i = sg * (s2 * br - s1 * dr);
    xr[0] = y0r; xi[0] = y0i;
    xr[1] = p1r + q1r; xi[1] = p1i + q1i;
    xr[4] = p1r - q1r; xi[4] = p1i - q1i;
    xr[2] = p2r + q2r; xi[2] = p2i + q2i;
    xr[3] = p2r - q2r; xi[3] = p2i - q2i;
  }
}

// One Stockham stage (Govindaraju et al., SC'08 formulation): butterfly j reads
// x[j + t K/r], applies twiddles W_{Ns r}^{(j mod Ns) t}, does a radix-r DFT and
// writes y[(j / Ns) Ns r + (j mod Ns) + t Ns]. In-place in LDS with a barrier
// between the read and the write phase.
template <typename R, int K, int NC, int P, int S, bool FWD>
__device__ __forceinline__ void stockham(R* re, R* im, const R* __restrict__ twc,
                                         const R* __restrict__ tws, int c, int q) {
  constexpr Radices F = factorize(K);
  if constexpr (S < F.n) {
    constexpr int r = F.r[S];
    constexpr int NB = K / r;
    constexpr int PER = (NB + P - 1) / P;
    constexpr int Ns = prefix_product(K, S);
    constexpr int TWS = K / (Ns * r);
    R vr[PER][r], vi[PER][r];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = q + u * P;
      if (j < NB) {
        const int k = j % Ns;
#pragma unroll
        for (int t = 0; t < r; ++t) {
          R xr = re[(j + t * NB) * NC + c];
          R xi = im[(j + t * NB) * NC + c];
          if (t > 0 && Ns > 1) {
            const int idx = k * t * TWS;
            const R wc = twc[idx];
            const R ws = FWD ? -tws[idx] : tws[idx];
            const R yr = xr * wc - xi * ws;
            xi = xr * ws + xi * wc;
            xr = yr;
          }
          vr[u][t] = xr;
          vi[u][t] = xi;
        }
        small_dft<R, r, FWD>(vr[u], vi[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = q + u * P;
      if (j < NB) {
        const int k = j % Ns;
        const int base = (j / Ns) * Ns * r + k;
#pragma unroll
        for (int t = 0; t < r; ++t) {
          re[(base + t * Ns) * NC + c] = vr[u][t];
          im[(base + t * Ns) * NC + c] = vi[u][t];
        }
      }
    }
    __syncthreads();
    stockham<R, K, NC, P, S + 1, FWD>(re, im, twc, tws, c, q);
  }
}

enum Pass { kXFwd = 0, kYFwd = 1, kZConv = 2, kYInv = 3, kXInv = 4 };

struct GridDims {
  int K1, K2, K3, XS, KX, BG;
  size_t chunk_elems;
  int chunk0;
};

template <typename R, int K, int NC, int P, int MODE>
__global__ void __launch_bounds__(NC * P)
k_fft(R* __restrict__ grid, GridDims gd, const R* __restrict__ twc,
      const R* __restrict__ tws, const R* __restrict__ G) {
  extern __shared__ unsigned char smem_raw[];
  R* re = reinterpret_cast<R*>(smem_raw);
  R* im = re + K * NC;
  const int c = threadIdx.x % NC;
  const int q = threadIdx.x / NC;
  R* g = grid + (size_t)(blockIdx.y + gd.chunk0) * gd.chunk_elems;
  const long col = (long)blockIdx.x * NC + c;
  const int BG = gd.BG;
  const int b = (int)(col % BG);
  const long line = col / BG;
  long nlines;
  size_t base, stride;
  if (MODE == kXFwd || MODE == kXInv) {
    nlines = (long)gd.K2 * gd.K3;
    base = (size_t)line * gd.XS * BG + b;
    stride = BG;
  } else if (MODE == kYFwd || MODE == kYInv) {
    nlines = (long)gd.K3 * gd.KX;
    const long z = line / gd.KX, kx = line % gd.KX;
    base = ((size_t)z * gd.K2 * gd.XS + 2 * kx) * BG + b;
    stride = (size_t)gd.XS * BG;
  } else {
    nlines = (long)gd.K2 * gd.KX;
    const long y = line / gd.KX, kx = line % gd.KX;
    base = ((size_t)y * gd.XS + 2 * kx) * BG + b;
    stride = (size_t)gd.K2 * gd.XS * BG;
  }
  const bool active = line < nlines;

  // ---- load ----
  if (MODE == kXFwd) {
    for (int n = q; n < K; n += P) {
      re[n * NC + c] = active ? g[base + (size_t)n * stride] : R(0);
      im[n * NC + c] = R(0);
    }
  } else if (MODE == kXInv) {
    // half spectrum kx = 0..K/2, the rest from Hermitian symmetry X[K-k] = conj(X[k])
    for (int n = q; n < K; n += P) {
      const int kk = n <= K / 2 ? n : K - n;
      R xr = R(0), xi = R(0);
      if (active) {
        xr = g[base + (size_t)(2 * kk) * stride];
        xi = g[base + (size_t)(2 * kk + 1) * stride];
      }
      re[n * NC + c] = xr;
      im[n * NC + c] = n <= K / 2 ? xi : -xi;
    }
  } else {
    for (int n = q; n < K; n += P) {
      R xr = R(0), xi = R(0);
      if (active) {
        xr = g[base + (size_t)n * stride];
        xi = g[base + (size_t)n * stride + BG];
      }
      re[n * NC + c] = xr;
      im[n * NC + c] = xi;
    }
  }
  __syncthreads();

  constexpr bool FWD = (MODE == kXFwd || MODE == kYFwd || MODE == kZConv);
  stockham<R, K, NC, P, 0, FWD>(re, im, twc, tws, c, q);

  if (MODE == kZConv) {
    if (active) {
      const long y = line / gd.KX, kx = line % gd.KX;
      for (int n = q; n < K; n += P) {
        const R w = G[((size_t)n * gd.K2 + y) * gd.KX + kx];
        re[n * NC + c] *= w;
        im[n * NC + c] *= w;
      }
    }
    __syncthreads();
    stockham<R, K, NC, P, 0, false>(re, im, twc, tws, c, q);
  }

  // ---- store ----
  if (!active) return;
  if (MODE == kXFwd) {
    for (int n = q; n <= K / 2; n += P) {
      g[base + (size_t)(2 * n) * stride] = re[n * NC + c];
      g[base + (size_t)(2 * n + 1) * stride] = im[n * NC + c];
    }
  } else if (MODE == kXInv) {
    for (int n = q; n < K; n += P) g[base + (size_t)n * stride] = re[n * NC + c];
  } else {
    for (int n = q; n < K; n += P) {
      g[base + (size_t)n * stride] = re[n * NC + c];
      g[base + (size_t)n * stride + BG] = im[n * NC + c];
    }
  }
}

// ---------------------------------------------------------------------------
// Register-resident variant (float32): a lane pair owns one column (a line of K
// points for one right-hand side) and runs the Stockham stages on registers, with
// twiddles folded to compile-time constants. Consecutive lane pairs are
// consecutive right-hand sides, so every load and store of a wavefront touches
// two contiguous rows; there is no LDS traffic and no barrier.
// ---------------------------------------------------------------------------
constexpr double cx_sin_core(double x) {
  // x in [-pi, pi]; Taylor series to well below double rounding
  double term = x, sum = x;
  for (int n = 1; n < 40; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double cx_sin(double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  return cx_sin_core(x);
}
constexpr double cx_cos(double x) { return cx_sin(x + kPi / 2); }

template <int K>
struct TwTable {
  float c[K];
  float s[K];
  constexpr TwTable() : c(), s() {
    for (int j = 0; j < K; ++j) {
      c[j] = (float)cx_cos(2.0 * kPi * j / K);
      s[j] = (float)cx_sin(2.0 * kPi * j / K);
    }
  }
};

template <int K, int S, bool FWD>
__device__ __forceinline__ void reg_stages(float (&xr)[K], float (&xi)[K]) {
  constexpr Radices F = factorize(K);
  if constexpr (S < F.n) {
    constexpr int r = F.r[S];
    constexpr int NB = K / r;
    constexpr int Ns = prefix_product(K, S);
    constexpr int TWS = K / (Ns * r);
    constexpr TwTable<K> T{};
    float yr[K], yi[K];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = j % Ns;
      float vr[r], vi[r];
#pragma unroll
      for (int t = 0; t < r; ++t) {
        float ar = xr[j + t * NB], ai = xi[j + t * NB];
        if (t > 0 && k > 0) {
          const int idx = k * t * TWS;
          const float wc = T.c[idx];
          const float ws = FWD ? -T.s[idx] : T.s[idx];
          const float br = ar * wc - ai * ws;
          ai = ar * ws + ai * wc;
          ar = br;
        }
        vr[t] = ar;
        vi[t] = ai;
      }
      small_dft<float, r, FWD>(vr, vi);
      const int base = (j / Ns) * Ns * r + k;
#pragma unroll
      for (int t = 0; t < r; ++t) {
        yr[base + t * Ns] = vr[t];
        yi[base + t * Ns] = vi[t];
      }
    }
#pragma unroll
    for (int n = 0; n < K; ++n) {
      xr[n] = yr[n];
      xi[n] = yi[n];
    }
    reg_stages<K, S + 1, FWD>(xr, xi);
  }
}

// Value of the lane whose index differs in bit 0, by a DPP quad permutation (quad_perm
// 1,0,3,2): a register move inside each group of four lanes, without the LDS crossbar
// that a general shuffle goes through.
__device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

// One column is split over a lane pair (h = lane & 1): lane h holds the decimated
// samples x[2m + h], m < H = K/2, runs an H-point FFT in registers, and the pair
// finishes with one radix-2 step exchanged through a lane shuffle:
//   decimation in time:  X[k] = F0[k] + W^k F1[k],  X[k + H] = F0[k] - W^k F1[k]
//   (lane 0 ends with X[0..H), lane 1 with X[H..K));
//   decimation in frequency (used after the convolution, from natural halves):
//   y0[k] = x[k] + x[k + H], y1[k] = (x[k] - x[k + H]) W^k, then H-point FFTs give
//   X[2k] (lane 0) and X[2k + 1] (lane 1).
template <int K, bool FWD>
__device__ __forceinline__ void pair_dit(float (&xr)[K / 2], float (&xi)[K / 2], int h) {
  constexpr int H = K / 2;
  constexpr TwTable<K> T{};
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float pr = lane_xor1(xr[k]), pi = lane_xor1(xi[k]);
    const float er = h ? pr : xr[k], ei = h ? pi : xi[k];
    const float orr = h ? xr[k] : pr, oi = h ? xi[k] : pi;
    const float wc = T.c[k], ws = FWD ? -T.s[k] : T.s[k];
    const float tr = orr * wc - oi * ws, ti = orr * ws + oi * wc;
    xr[k] = h ? er - tr : er + tr;
    xi[k] = h ? ei - ti : ei + ti;
  }
}

template <int K, bool FWD>
__device__ __forceinline__ void pair_dif(float (&xr)[K / 2], float (&xi)[K / 2], int h) {
  constexpr int H = K / 2;
  constexpr TwTable<K> T{};
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float pr = lane_xor1(xr[k]), pi = lane_xor1(xi[k]);
    // lane 0 holds x[k], lane 1 holds x[k + H]
    const float ar = h ? pr : xr[k], ai = h ? pi : xi[k];
    const float br = h ? xr[k] : pr, bi = h ? xi[k] : pi;
    // both halves computed, one selected: no divergent branch per element
    const float dr = ar - br, di = ai - bi;
    const float wc = T.c[k], ws = FWD ? -T.s[k] : T.s[k];
    const float tr = dr * wc - di * ws, ti = dr * ws + di * wc;
    xr[k] = h ? tr : ar + br;
    xi[k] = h ? ti : ai + bi;
  }
}

// Element e of a grid line, addressed from a wave-uniform base by a 32-bit byte offset,
// so that every load and store is one scalar base plus a 32-bit per-lane offset (no
// per-element 64-bit address kept live). Offsets stay below 2^32 bytes: one grid chunk
// is at most 128 x 128 x 130 x 64 floats.
__device__ __forceinline__ float& at(float* base, uint32_t e) {
  return *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (e << 2));
}

// The same grid addressed through a buffer resource built from the wave-uniform base:
// a load or store takes a per-lane byte offset (one vector register shared by a whole
// line) plus a wave-uniform byte offset in a scalar register, so that a line of K
// elements holds one vector register of addresses instead of one per element. The
// range is left unbounded (4 GiB), since the offsets are those of at() above.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(float* base) {
  // word 3: 32-bit data format, the untyped-load setting for this architecture family
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, -1, 0x00020000);
}
__device__ __forceinline__ float ld_line(__amdgpu_buffer_rsrc_t r, uint32_t vbyte,
                                         uint32_t sbyte) {
  // the builtin moves 32-bit integers: reinterpret the bits, never convert the value
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vbyte, sbyte, 0));
}
__device__ __forceinline__ void st_line(__amdgpu_buffer_rsrc_t r, float v, uint32_t vbyte,
                                        uint32_t sbyte) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vbyte, sbyte, 0);
}

// Gz (the z pass with the convolution only): the influence function with kz innermost,
// [K2][K1/2 + 1][K3].
template <int K, int MODE>
__global__ void __launch_bounds__(64)
k_fft_reg(float* __restrict__ grid, GridDims gd, const float* __restrict__ Gz) {
  constexpr int H = K / 2;
  float* g = grid + (size_t)(blockIdx.y + gd.chunk0) * gd.chunk_elems;
  const int h = threadIdx.x & 1;
  const long col = (long)blockIdx.x * 32 + (threadIdx.x >> 1);
  const int BG = gd.BG;
  const int b = (int)(col % BG);
  const long line = col / BG;
  long nlines;
  size_t base;
  uint32_t stride;
  if (MODE == kXFwd || MODE == kXInv) {
    nlines = (long)gd.K2 * gd.K3;
    base = (size_t)line * gd.XS * BG + b;
    stride = BG;
  } else if (MODE == kYFwd || MODE == kYInv) {
    nlines = (long)gd.K3 * gd.KX;
    const long z = line / gd.KX, kx = line % gd.KX;
    base = ((size_t)z * gd.K2 * gd.XS + 2 * kx) * BG + b;
    stride = (uint32_t)gd.XS * BG;
  } else {
    nlines = (long)gd.K2 * gd.KX;
    const long y = line / gd.KX, kx = line % gd.KX;
    base = ((size_t)y * gd.XS + 2 * kx) * BG + b;
    stride = (uint32_t)(gd.K2 * gd.XS) * BG;
  }
  // Both lanes of a pair see the same column, so they leave together (the
  // shuffles below stay within active pairs).
  if (line >= nlines) return;
  // Wave-uniform base pointer plus a small per-lane 32-bit offset, so that the
  // per-element addresses are one scalar product plus one vector add.
  const size_t wbase = (size_t)__builtin_amdgcn_readfirstlane((unsigned)(base >> 32)) << 32 |
                       (size_t)(unsigned)__builtin_amdgcn_readfirstlane((unsigned)base);
  float* gw = g + wbase;
  const uint32_t lo = (uint32_t)(base - wbase);
  float xr[H], xi[H];
  if (MODE == kXFwd) {
#pragma unroll
    for (int m = 0; m < H; ++m) {
      xr[m] = at(gw, lo + (uint32_t)(2 * m + h) * stride);
      xi[m] = 0.f;
    }
  } else if (MODE == kXInv) {
#pragma unroll
    for (int m = 0; m < H; ++m) {
      const int n = 2 * m + h;
      const int kk = n <= H ? n : K - n;
      const float vr = at(gw, lo + (uint32_t)(2 * kk) * stride);
      const float vi = at(gw, lo + (uint32_t)(2 * kk + 1) * stride);
      xr[m] = vr;
      xi[m] = n <= H ? vi : -vi;
    }
  } else {
    // lane h reads x[2m + h]: lane part h stride (imaginary rows BG further), uniform
    // part 2m stride
    const __amdgpu_buffer_rsrc_t rs = wave_rsrc(gw);
    const uint32_t vb = (lo + (uint32_t)h * stride) << 2;
    const uint32_t vbi = vb + ((uint32_t)BG << 2);
#pragma unroll
    for (int m = 0; m < H; ++m) {
      const uint32_t sb = ((uint32_t)(2 * m) * stride) << 2;
      xr[m] = ld_line(rs, vb, sb);
      xi[m] = ld_line(rs, vbi, sb);
    }
  }
  constexpr bool FWD = (MODE == kXFwd || MODE == kYFwd || MODE == kZConv);
  reg_stages<H, 0, FWD>(xr, xi);
  pair_dit<K, FWD>(xr, xi, h);
  if (MODE == kZConv) {
    // natural halves: lane h holds X[h H + k]. With kz innermost the lane's H factors
    // are one run: one address and immediate offsets for all H loads.
    const float* gl = Gz + (size_t)line * K + h * H;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const float w = gl[k];
      xr[k] *= w;
      xi[k] *= w;
      // the product is formed here: folded into the exchange step below, it kept the
      // factor, the plain value and the product live together
      asm("" : "+v"(xr[k]), "+v"(xi[k]));
    }
    pair_dif<K, false>(xr, xi, h);
    reg_stages<H, 0, false>(xr, xi);
    // decimated output: lane h holds x[2k + h]
    const __amdgpu_buffer_rsrc_t rs = wave_rsrc(gw);
    const uint32_t vb = (lo + (uint32_t)h * stride) << 2;
    const uint32_t vbi = vb + ((uint32_t)BG << 2);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const uint32_t sb = ((uint32_t)(2 * k) * stride) << 2;
      st_line(rs, xr[k], vb, sb);
      st_line(rs, xi[k], vbi, sb);
    }
    return;
  }
  if (MODE == kXFwd) {
    if (h == 0) {
#pragma unroll
      for (int k = 0; k < H; ++k) {
        at(gw, lo + (uint32_t)(2 * k) * stride) = xr[k];
        at(gw, lo + (uint32_t)(2 * k + 1) * stride) = xi[k];
      }
    } else {
      at(gw, lo + (uint32_t)(2 * H) * stride) = xr[0];
      at(gw, lo + (uint32_t)(2 * H + 1) * stride) = xi[0];
    }
  } else if (MODE == kXInv) {
#pragma unroll
    for (int k = 0; k < H; ++k) at(gw, lo + (uint32_t)(h * H + k) * stride) = xr[k];
  } else {
    // lane h writes X[h H + k]: lane part h H stride, uniform part k stride
    const __amdgpu_buffer_rsrc_t rs = wave_rsrc(gw);
    const uint32_t vb = (lo + (uint32_t)(h * H) * stride) << 2;
    const uint32_t vbi = vb + ((uint32_t)BG << 2);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const uint32_t sb = ((uint32_t)k * stride) << 2;
      st_line(rs, xr[k], vb, sb);
      st_line(rs, xi[k], vbi, sb);
    }
  }
}

// x passes with one lane per column (K even, M = K/2). A real line of K points is packed
// as M complex points z[n] = x[2n] + i x[2n+1] and transformed with one M-point FFT:
//   forward:  X[k] = (Z[k] + conj Z[M-k]) / 2 + W_K^k (Z[k] - conj Z[M-k]) / 2i,
//             k = 0..M, with Z[M] = Z[0];
//   inverse:  Z'[k] = A[k] + i B[k],  A[k] = X[k] + conj X[M-k],
//             B[k] = (X[k] - conj X[M-k]) W_K^{-k},  then z = inverse M-point FFT of Z',
//             x[2n] = Re z[n], x[2n+1] = Im z[n].
// The imaginary parts of X[0] and X[M] are taken as zero, as in the real part of a full
// inverse transform. A wavefront covers 64 consecutive columns, so every load and store
// is one contiguous 256-byte row; no lane exchange is needed.
template <int K, bool FWD>
__global__ void __launch_bounds__(64)
k_fft_x_real(float* __restrict__ grid, GridDims gd) {
  constexpr int M = K / 2;
  constexpr TwTable<K> T{};
  float* g = grid + (size_t)(blockIdx.y + gd.chunk0) * gd.chunk_elems;
  const long col = (long)blockIdx.x * 64 + threadIdx.x;
  const int BG = gd.BG;
  const int b = (int)(col % BG);
  const long line = col / BG;
  if (line >= (long)gd.K2 * gd.K3) return;
  const size_t base = (size_t)line * gd.XS * BG + b;
  const size_t wbase = (size_t)__builtin_amdgcn_readfirstlane((unsigned)(base >> 32)) << 32 |
                       (size_t)(unsigned)__builtin_amdgcn_readfirstlane((unsigned)base);
  float* gw = g + wbase;
  const uint32_t lo = (uint32_t)(base - wbase);
  const uint32_t stride = (uint32_t)BG;
  float zr[M], zi[M];
#pragma unroll
  for (int n = 0; n < M; ++n) {
    zr[n] = at(gw, lo + (uint32_t)(2 * n) * stride);
    zi[n] = at(gw, lo + (uint32_t)(2 * n + 1) * stride);
  }
  // an opaque copy of the lane offset for the stores: otherwise the compiler keeps the
  // load addresses live through the transform to reuse them
  uint32_t lo_st = lo;
  if constexpr (FWD) {
    reg_stages<M, 0, true>(zr, zi);
    asm volatile("" : "+v"(lo_st));
    at(gw, lo_st) = zr[0] + zi[0];
    at(gw, lo_st + stride) = 0.f;
    at(gw, lo_st + (uint32_t)(2 * M) * stride) = zr[0] - zi[0];
    at(gw, lo_st + (uint32_t)(2 * M + 1) * stride) = 0.f;
    // bins k and M - k read the same two points, so they are formed together and both
    // points die at once (in plain k order every point stayed live until its mirror bin)
#pragma unroll
    for (int k = 1; k <= M / 2; ++k) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int j = e ? M - k : k;
        if (e && j == k) break;
        const float fer = 0.5f * (zr[j] + zr[M - j]), fei = 0.5f * (zi[j] - zi[M - j]);
        const float forr = 0.5f * (zi[j] + zi[M - j]), foi = -0.5f * (zr[j] - zr[M - j]);
        // W_K^j = cos - i sin
        const float wr = T.c[j] * forr + T.s[j] * foi, wi = T.c[j] * foi - T.s[j] * forr;
        at(gw, lo_st + (uint32_t)(2 * j) * stride) = fer + wr;
        at(gw, lo_st + (uint32_t)(2 * j + 1) * stride) = fei + wi;
      }
    }
  } else {
    // zr, zi hold X[0..M); X[M] is the last complex pair of the half spectrum
    const float xmr = at(gw, lo + (uint32_t)(2 * M) * stride);
    const float x0r = zr[0];
    zr[0] = x0r + xmr;
    zi[0] = x0r - xmr;
#pragma unroll
    for (int k = 1; k <= M / 2; ++k) {
      const int m = M - k;
      const float ar = zr[k], ai = zi[k], br = zr[m], bi = zi[m];
      {
        // index k: a = X[k], b = X[M-k]; twiddle W_K^{-k} = cos + i sin
        const float Ar = ar + br, Ai = ai - bi, Dr = ar - br, Di = ai + bi;
        const float Br = Dr * T.c[k] - Di * T.s[k], Bi = Dr * T.s[k] + Di * T.c[k];
        zr[k] = Ar - Bi;
        zi[k] = Ai + Br;
      }
      if (m != k) {
        const float Ar = br + ar, Ai = bi - ai, Dr = br - ar, Di = bi + ai;
        const float Br = Dr * T.c[m] - Di * T.s[m], Bi = Dr * T.s[m] + Di * T.c[m];
        zr[m] = Ar - Bi;
        zi[m] = Ai + Br;
      }
    }
    reg_stages<M, 0, false>(zr, zi);
    asm volatile("" : "+v"(lo_st));
#pragma unroll
    for (int n = 0; n < M; ++n) {
      at(gw, lo_st + (uint32_t)(2 * n) * stride) = zr[n];
      at(gw, lo_st + (uint32_t)(2 * n + 1) * stride) = zi[n];
    }
  }
}

// Spread along whole x-lines fused with the forward real x transform (float, 64
// right-hand sides per chunk, order P): one wavefront per (y, z) line of one chunk, lane
// = right-hand side. Each lane keeps its right-hand side's K line points in registers and
// adds, from every atom whose y-z stencil covers the line (the setup's line lists, in atom
// order), the atom's P x-points with the arithmetic of k_spread:
//   A = d_x w_y w_z,  B = d_y w'_y w_z + d_z w_y w'_z,  q = fma(w'_x, A, q), fma(w_x, B, q)
// (d = Mu d in u, w = M_P, w' = M_P'), in the same per-point order, so the real line
// equals k_spread's. The lane then packs the line as K/2 complex points, runs the
// transform of k_fft_x_real<K, true> in registers and stores the half spectrum: the real
// grid is never written and the separate x pass is not needed. A line-list entry packs the
// atom and its stencil offsets along y and z: (s << 8) | (t_y << 4) | t_z.
template <int K, int P>
__global__ void __launch_bounds__(64)
k_spread_xline(float* __restrict__ grid, GridDims gd, const Geometry geo,
               const int* __restrict__ line_start, const int* __restrict__ line_atoms,
               const int* __restrict__ base, const float* __restrict__ th,
               const float* __restrict__ dth, const float* __restrict__ dv, int B) {
  constexpr int BG = 64;
  constexpr int M = K / 2;
  const int lane = threadIdx.x;
  const int nlines = gd.K2 * gd.K3;
  // XCD-aware: each XCD takes a contiguous range of lines (work-groups are dealt to the
  // 8 XCDs round-robin; gridDim.x is a multiple of 8), so the atoms of neighbouring
  // lines, which share most of their dipoles, stay in one L2
  const int per = gridDim.x / 8;
  const int line = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (line >= nlines) return;  // uniform over the wavefront
  const int chunk = blockIdx.y + gd.chunk0;
  const int bg = chunk * BG + lane;
  const float m00 = (float)geo.Mu[0][0], m01 = (float)geo.Mu[0][1], m02 = (float)geo.Mu[0][2];
  const float m10 = (float)geo.Mu[1][0], m11 = (float)geo.Mu[1][1], m12 = (float)geo.Mu[1][2];
  const float m20 = (float)geo.Mu[2][0], m21 = (float)geo.Mu[2][1], m22 = (float)geo.Mu[2][2];
  // the lane's K line points in four register arrays of 32 (plain local arrays: a
  // wave-uniform index then selects a register by indexed moves, not scratch memory)
  float r0[32], r1[32], r2[32], r3[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) r0[i] = r1[i] = r2[i] = r3[i] = 0.f;
  const int lo = line_start[line], hi = line_start[line + 1];
  // atoms are taken NB at a time: their entries, dipoles, stencil bases and weights are
  // all requested before the first of them is added, so the loads of a batch overlap.
  // Entries, atoms and bases are the same for every lane; reading them through
  // readfirstlane makes the register index below wave-uniform, so the compiler selects
  // the line register by an indexed move instead of spilling the arrays to scratch
  constexpr int NB = 4;
  for (int a0 = lo; a0 < hi; a0 += NB) {
    int sc[NB], ty[NB], tz[NB], bx[NB];
    float e0[NB], e1[NB], e2[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int a = min(a0 + j, hi - 1);  // a batch's tail repeats the last atom, unused
      const int e = __builtin_amdgcn_readfirstlane(line_atoms[a]);
      sc[j] = e >> 8;
      ty[j] = (e >> 4) & 15;
      tz[j] = e & 15;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float* d = dv + (size_t)sc[j] * 3 * B + bg;
      e0[j] = d[0]; e1[j] = d[B]; e2[j] = d[2 * B];
      bx[j] = __builtin_amdgcn_readfirstlane(base[3 * sc[j]]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (a0 + j >= hi) break;  // uniform over the wavefront
      const float* tp = th + (size_t)sc[j] * 3 * P;
      const float* dp = dth + (size_t)sc[j] * 3 * P;
      const float wy = tp[P + ty[j]], dwy = dp[P + ty[j]];
      const float wz = tp[2 * P + tz[j]], dwz = dp[2 * P + tz[j]];
      // dipole in u: (Mu d)_b
      const float d0 = m00 * e0[j] + m01 * e1[j] + m02 * e2[j];
      const float d1 = m10 * e0[j] + m11 * e1[j] + m12 * e2[j];
      const float d2 = m20 * e0[j] + m21 * e1[j] + m22 * e2[j];
      const float A = d0 * wy * wz;
      const float Bc = d1 * dwy * wz + d2 * wy * dwz;
#pragma unroll
      for (int t = 0; t < P; ++t) {
        int x = bx[j] - t;
        if (x < 0) x += K;
        const float wa = dp[t], wb = tp[t];
        const int g = x >> 5, o = x & 31;
        // the empty asm statements differ per branch, so the compiler does not merge the
        // four updates into one through a pointer that selects the array, which would
        // put the arrays in scratch memory
        if (g == 0) {
          r0[o] = fma(wb, Bc, fma(wa, A, r0[o]));
          asm volatile("; line segment 0");
        } else if (g == 1) {
          r1[o] = fma(wb, Bc, fma(wa, A, r1[o]));
          asm volatile("; line segment 1");
        } else if (K > 64 && g == 2) {
          r2[o] = fma(wb, Bc, fma(wa, A, r2[o]));
          asm volatile("; line segment 2");
        } else if (K > 96) {
          r3[o] = fma(wb, Bc, fma(wa, A, r3[o]));
          asm volatile("; line segment 3");
        }
      }
    }
  }
  // the lane's real line, packed as K/2 complex points, and the transform of
  // k_fft_x_real<K, true>
  float zr[M], zi[M];
#pragma unroll
  for (int n = 0; n < M; ++n) {
    const int xa = 2 * n, xb = 2 * n + 1;
    zr[n] = xa < 32 ? r0[xa & 31] : xa < 64 ? r1[xa & 31] : xa < 96 ? r2[xa & 31] : r3[xa & 31];
    zi[n] = xb < 32 ? r0[xb & 31] : xb < 64 ? r1[xb & 31] : xb < 96 ? r2[xb & 31] : r3[xb & 31];
  }
  constexpr TwTable<K> T{};
  reg_stages<M, 0, true>(zr, zi);
  float* g = grid + (size_t)chunk * gd.chunk_elems;
  const size_t lbase = (size_t)line * gd.XS * BG;
  float* gw = g + lbase;
  const uint32_t lo_st = (uint32_t)lane;
  const uint32_t stride = (uint32_t)BG;
  at(gw, lo_st) = zr[0] + zi[0];
  at(gw, lo_st + stride) = 0.f;
  at(gw, lo_st + (uint32_t)(2 * M) * stride) = zr[0] - zi[0];
  at(gw, lo_st + (uint32_t)(2 * M + 1) * stride) = 0.f;
#pragma unroll
  for (int k = 1; k < M; ++k) {
    const float fer = 0.5f * (zr[k] + zr[M - k]), fei = 0.5f * (zi[k] - zi[M - k]);
    const float forr = 0.5f * (zi[k] + zi[M - k]), foi = -0.5f * (zr[k] - zr[M - k]);
    // W_K^k = cos - i sin
    const float wr = T.c[k] * forr + T.s[k] * foi, wi = T.c[k] * foi - T.s[k] * forr;
    at(gw, lo_st + (uint32_t)(2 * k) * stride) = fer + wr;
    at(gw, lo_st + (uint32_t)(2 * k + 1) * stride) = fei + wi;
  }
}

#define MBD_REG_SIZES(X) \
  X(8) X(10) X(12) X(16) X(18) X(20) X(24) X(30) X(32) X(36) X(40) X(48) X(50) X(54) \
  X(60) X(64) X(72) X(80) X(90) X(96) X(100) X(108) X(120) X(128)

#define MBD_FFT_SIZES(X) \
  X(8) X(10) X(12) X(16) X(18) X(20) X(24) X(30) X(32) X(36) X(40) X(48) X(50) X(54) \
  X(60) X(64) X(72) X(80) X(90) X(96) X(100) X(108) X(120) X(128)

template <typename R> struct FftShape;
template <> struct FftShape<float> { static constexpr int NC = 64, P = 4; };
template <> struct FftShape<double> { static constexpr int NC = 32, P = 8; };

template <typename R, int MODE>
void launch_pass(int K, R* grid, const GridDims& gd, int nchunks, const R* twc, const R* tws,
                 const R* G, const R* Gt, hipStream_t st) {
  constexpr int NC = FftShape<R>::NC, P = FftShape<R>::P;
  long nlines;
  if (MODE == kXFwd || MODE == kXInv) nlines = (long)gd.K2 * gd.K3;
  else if (MODE == kYFwd || MODE == kYInv) nlines = (long)gd.K3 * gd.KX;
  else nlines = (long)gd.K2 * gd.KX;
  const long cols = nlines * gd.BG;
  if constexpr (sizeof(R) == 4) {
    if (gd.BG >= 16) {
      if constexpr (MODE == kXFwd || MODE == kXInv) {
        dim3 g1((unsigned)((cols + 63) / 64), nchunks);
        switch (K) {
#define MBD_REGX(KK)                                                                    \
          case KK:                                                                      \
            k_fft_x_real<KK, MODE == kXFwd><<<g1, 64, 0, st>>>((float*)grid, gd);       \
            return;
          MBD_REG_SIZES(MBD_REGX)
#undef MBD_REGX
          default:
            break;
        }
      }
      dim3 g2((unsigned)((cols + 31) / 32), nchunks);
      switch (K) {
#define MBD_REG(KK)                                                                    \
        case KK:                                                                       \
          k_fft_reg<KK, MODE><<<g2, 64, 0, st>>>((float*)grid, gd, (const float*)Gt);   \
          return;
        MBD_REG_SIZES(MBD_REG)
#undef MBD_REG
        default:
          break;
      }
    }
  }
  dim3 grd((unsigned)((cols + NC - 1) / NC), nchunks);
  const size_t shm = 2 * (size_t)K * NC * sizeof(R);
  switch (K) {
#define MBD_CASE(KK)                                                                     \
    case KK:                                                                             \
      k_fft<R, KK, NC, P, MODE><<<grd, NC * P, shm, st>>>(grid, gd, twc, tws, G);       \
      break;
    MBD_FFT_SIZES(MBD_CASE)
#undef MBD_CASE
    default:
      break;
  }
}

}  // namespace

bool fft_supported(int k) {
  switch (k) {
#define MBD_CASE(KK) case KK: return true;
    MBD_FFT_SIZES(MBD_CASE)
#undef MBD_CASE
    default:
      return false;
  }
}

// One pass (0 forward x, 1 forward y, 2 z with convolution, 3 inverse y, 4 inverse x)
// over every grid chunk.
template <typename R>
void launch_fft_pass(const Geometry& geo, const SysBuffers& b, int B, int BG, int chunk0,
                     int nchunks, int pass, hipStream_t st) {
  GridDims gd;
  gd.K1 = geo.K[0];
  gd.K2 = geo.K[1];
  gd.K3 = geo.K[2];
  gd.XS = geo.K[0] + 2;
  gd.KX = geo.K[0] / 2 + 1;
  gd.BG = BG;
  gd.chunk_elems = (size_t)gd.K3 * gd.K2 * gd.XS * BG;
  gd.chunk0 = chunk0;
  (void)B;
  R* grid = (R*)b.grid;
  const R* tw = (const R*)b.tw;
  const int Ksum = geo.K[0] + geo.K[1] + geo.K[2];
  const R* c0 = tw;
  const R* c1 = tw + geo.K[0];
  const R* c2 = tw + geo.K[0] + geo.K[1];
  const R* G = (const R*)b.G;
  const R* Gt = (const R*)b.Gt;
  switch (pass) {
    case 0: launch_pass<R, kXFwd>(geo.K[0], grid, gd, nchunks, c0, c0 + Ksum, G, Gt, st); break;
    case 1: launch_pass<R, kYFwd>(geo.K[1], grid, gd, nchunks, c1, c1 + Ksum, G, Gt, st); break;
    case 2: launch_pass<R, kZConv>(geo.K[2], grid, gd, nchunks, c2, c2 + Ksum, G, Gt, st); break;
    case 3: launch_pass<R, kYInv>(geo.K[1], grid, gd, nchunks, c1, c1 + Ksum, G, Gt, st); break;
    default: launch_pass<R, kXInv>(geo.K[0], grid, gd, nchunks, c0, c0 + Ksum, G, Gt, st); break;
  }
}

// The spread of chunks [chunk0, chunk0 + nchunks) fused with their forward x pass, when
// compiled for this case (float, 64 right-hand sides per chunk, p = 6, a register-FFT
// length): returns false otherwise, and the caller runs k_spread and pass 0 instead.
bool launch_spread_xline(const Geometry& geo, const SysBuffers& b, int B, int BG, int chunk0,
                         int nchunks, hipStream_t st) {
  if (BG != 64 || geo.p != 6 || !b.line_start) return false;
  GridDims gd;
  gd.K1 = geo.K[0];
  gd.K2 = geo.K[1];
  gd.K3 = geo.K[2];
  gd.XS = geo.K[0] + 2;
  gd.KX = geo.K[0] / 2 + 1;
  gd.BG = BG;
  gd.chunk_elems = (size_t)gd.K3 * gd.K2 * gd.XS * BG;
  gd.chunk0 = chunk0;
  const int nlines = gd.K2 * gd.K3;
  dim3 grd((unsigned)((nlines + 7) / 8 * 8), nchunks);
  switch (geo.K[0]) {
#define MBD_SXL(KK)                                                                      \
    case KK:                                                                             \
      k_spread_xline<KK, 6><<<grd, 64, 0, st>>>((float*)b.grid, gd, geo, b.line_start,   \
                                               b.line_atoms, b.base, (const float*)b.th, \
                                               (const float*)b.dth, (const float*)b.dv, B); \
      return true;
    MBD_REG_SIZES(MBD_SXL)
#undef MBD_SXL
    default:
      return false;
  }
}

template void launch_fft_pass<float>(const Geometry&, const SysBuffers&, int, int, int, int, int,
                                     hipStream_t);
template void launch_fft_pass<double>(const Geometry&, const SysBuffers&, int, int, int, int, int,
                                      hipStream_t);

}  // namespace mbd
