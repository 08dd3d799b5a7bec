// Host runtime behind the C ABI: validation, parameter derivation, workspace,
// device setup and the Algorithm 1 driver (probe blocks x Lanczos steps).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "mbd_math.h"

namespace mbd {

namespace {
thread_local std::string g_last_error;

constexpr double kBohrAngstrom = 0.529177210903;

struct HipError {
  hipError_t e;
  const char* what;
};

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

// erfc(tau rc) / rc = eps with rc in Angstrom, bisection (tau in 1/Angstrom).
double tau_from_cutoff_angstrom(double rc, double eps = 1e-8) {
  double lo = 0.0, hi = 1.0;
  while (std::erfc(hi * rc) / rc > eps) hi *= 2.0;
  for (int i = 0; i < 200; ++i) {
    double mid = 0.5 * (lo + hi);
    if (std::erfc(mid * rc) / rc > eps) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Smallest even 2^a 3^b >= 1.4 points per Angstrom.
int grid_rule(double L_bohr) {
  const double target = 1.4 * L_bohr * kBohrAngstrom;
  int best = 0;
  for (int p2 = 2; p2 <= 4096; p2 *= 2)
    for (int k = p2; k <= 4096; k *= 3)
      if (k >= target && (best == 0 || k < best)) best = k;
  return best;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

double cell_volume(const double (&A)[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// Reciprocal vectors a*_a = (a_b x a_c) / V, (a, b, c) cyclic, so a*_a . a_b = delta_ab.
void reciprocal(const double (&A)[3][3], double (&Ar)[3][3]) {
  const double V = cell_volume(A);
  for (int a = 0; a < 3; ++a) {
    const double* u = A[(a + 1) % 3];
    const double* v = A[(a + 2) % 3];
    Ar[a][0] = (u[1] * v[2] - u[2] * v[1]) / V;
    Ar[a][1] = (u[2] * v[0] - u[0] * v[2]) / V;
    Ar[a][2] = (u[0] * v[1] - u[1] * v[0]) / V;
  }
}

template <typename T>
T* dalloc(Plan& plan, size_t count, size_t& bytes) {
  void* p = nullptr;
  const size_t nb = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) throw std::bad_alloc();
  plan.allocations.push_back(p);
  bytes += nb;
  return static_cast<T*>(p);
}

// Influence function on the half spectrum [K3][K2][K1/2+1] and twiddle tables.
template <typename R>
void host_tables(const Geometry& g, std::vector<R>& G, std::vector<R>& tw) {
  const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2], KX = K1 / 2 + 1;
  const double V = cell_volume(g.A);
  double th[kMaxOrder], dth[kMaxOrder];
  std::vector<double> Mk(g.p);
  switch (g.p) {
    case 4: bspline_weights<4>(0.0, th, dth); break;
    case 6: bspline_weights<6>(0.0, th, dth); break;
    default: bspline_weights<8>(0.0, th, dth); break;
  }
  // |b(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k+1) e^{2 pi i m k / K}|^2
  auto bmod = [&](int K) {
    std::vector<double> out(K);
    for (int m = 0; m < K; ++m) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k <= g.p - 2; ++k) {
        const double ph = 2.0 * M_PI * m * k / K;
        re += th[k + 1] * std::cos(ph);
        im += th[k + 1] * std::sin(ph);
      }
      out[m] = 1.0 / (re * re + im * im);
    }
    return out;
  };
  const auto b1 = bmod(K1), b2 = bmod(K2), b3 = bmod(K3);
  G.assign((size_t)K3 * K2 * KX, R(0));
  for (int kz = 0; kz < K3; ++kz) {
    const double fz = (kz <= K3 / 2 ? kz : kz - K3);
    for (int ky = 0; ky < K2; ++ky) {
      const double fy = (ky <= K2 / 2 ? ky : ky - K2);
      for (int kx = 0; kx < KX; ++kx) {
        // m = sum_a m_a a*_a (reciprocal lattice vector of the DFT index)
        double m2 = 0.0;
        for (int c = 0; c < 3; ++c) {
          const double mc = kx * g.Ar[0][c] + fy * g.Ar[1][c] + fz * g.Ar[2][c];
          m2 += mc * mc;
        }
        double v = 0.0;
        if (m2 > 0.0)
          v = std::exp(-M_PI * M_PI * m2 / (g.tau * g.tau)) * b1[kx] * b2[ky] * b3[kz] /
              (M_PI * V * m2);
        G[((size_t)kz * K2 + ky) * KX + kx] = (R)v;
      }
    }
  }
  const int Ks = K1 + K2 + K3;
  tw.assign(2 * (size_t)Ks, R(0));
  int off = 0;
  for (int a = 0; a < 3; ++a) {
    for (int j = 0; j < g.K[a]; ++j) {
      tw[off + j] = (R)std::cos(2.0 * M_PI * j / g.K[a]);
      tw[Ks + off + j] = (R)std::sin(2.0 * M_PI * j / g.K[a]);
    }
    off += g.K[a];
  }
}

template <typename R>
void allocate_system(Plan& plan, System& S, int R_probes, int m) {
  Geometry& g = S.geo;
  SysBuffers& b = S.buf;
  size_t& by = S.bytes;
  const int n = g.n, B = plan.B;
  const int ncell = cell_slots(g);
  const int ntiles = g.tiles[0] * g.tiles[1] * g.tiles[2];
  b.perm = dalloc<int>(plan, n, by);
  b.subkey = dalloc<uint32_t>(plan, n, by);
  b.cell_of = dalloc<int>(plan, n, by);
  b.cell_start = dalloc<int>(plan, ncell + 1, by);
  b.cell_cursor = dalloc<int>(plan, ncell, by);
  b.wpos = dalloc<double>(plan, 3 * (size_t)n, by);
  b.loc = dalloc<R>(plan, 4 * (size_t)n, by);
  b.g = dalloc<double>(plan, n, by);
  b.om2 = dalloc<double>(plan, n, by);
  b.base = dalloc<int>(plan, 3 * (size_t)n, by);
  b.scell = dalloc<int>(plan, n, by);
  b.th = dalloc<R>(plan, 3 * (size_t)n * g.p, by);
  b.dth = dalloc<R>(plan, 3 * (size_t)n * g.p, by);
  b.tile_count = dalloc<int>(plan, ntiles + 1, by);
  b.tile_start = dalloc<int>(plan, ntiles + 1, by);
  // at most ceil((p - 1) / tile) + 2 tiles per axis touched by one stencil
  size_t per_atom = 1;
  for (int a = 0; a < 3; ++a) per_atom *= (size_t)((g.p - 1 + g.tile[a] - 1) / g.tile[a] + 2);
  b.tile_atoms = dalloc<int>(plan, per_atom * (size_t)n, by);
  if (sizeof(R) == 4 && g.p == 6 && n < (1 << 23)) {  // line entries pack s << 8
    const size_t nlines = (size_t)g.K[1] * g.K[2];
    b.line_count = dalloc<int>(plan, nlines + 1, by);
    b.line_start = dalloc<int>(plan, nlines + 1, by);
    b.line_atoms = dalloc<int>(plan, (size_t)g.p * g.p * n, by);
  }
  b.G = dalloc<R>(plan, (size_t)g.K[2] * g.K[1] * (g.K[0] / 2 + 1), by);
  b.Gt = dalloc<R>(plan, (size_t)g.K[2] * g.K[1] * (g.K[0] / 2 + 1), by);
  b.tw = dalloc<R>(plan, 2 * (size_t)(g.K[0] + g.K[1] + g.K[2]), by);
  const size_t vec = 3 * (size_t)n * B;
  b.W = dalloc<double>(plan, vec * m, by);
  b.Lt = dalloc<double>(plan, vec, by);
  b.dv = dalloc<R>(plan, vec, by);
  b.Ed = dalloc<R>(plan, vec, by);
  b.grid = dalloc<R>(plan, (size_t)g.K[2] * g.K[1] * (g.K[0] + 2) * B, by);
  b.part = dalloc<double>(plan, (size_t)kRedBlocks * kPartSlots * B, by);
  b.coef = dalloc<double>(plan, (size_t)kMaxSteps * B, by);
  b.a = dalloc<double>(plan, (size_t)R_probes * m, by);
  b.b = dalloc<double>(plan, (size_t)R_probes * m, by);
  b.meff = dalloc<int>(plan, R_probes, by);
  b.q = dalloc<double>(plan, R_probes, by);
  b.sum_omega = dalloc<double>(plan, 1, by);
  if (plan.forces) {
    b.ddth = dalloc<R>(plan, 3 * (size_t)n * g.p, by);
    b.ybar = dalloc<double>(plan, 3 * vec, by);
    b.lbar = dalloc<double>(plan, vec, by);
    b.dq = dalloc<R>(plan, vec, by);
    b.tz = dalloc<double>(plan, (size_t)B * m * m, by);
    b.abar = dalloc<double>(plan, (size_t)B * m, by);
    b.bbar = dalloc<double>(plan, (size_t)B * m, by);
    b.adj = dalloc<double>(plan, (size_t)B * 16, by);
    if (plan.prm.store_grids)
      b.phi = dalloc<R>(plan, (size_t)m * g.K[2] * g.K[1] * (g.K[0] + 2) * B, by);
    b.fsum = dalloc<double>(plan, 6 * (size_t)n, by);
  }
  if (plan.prm.krylov_block > 1) {
    BlockWork& bw = b.blk;
    bw.kb = plan.prm.krylov_block;
    const size_t nkb = (size_t)B / bw.kb, kk = (size_t)bw.kb * bw.kb;
    const size_t nt = (size_t)m * bw.kb;
    bw.nblk = std::max(1, std::min(512, (3 * n + 255) / 256));
    bw.part = dalloc<double>(plan, (size_t)bw.nblk * B * bw.kb, by);
    bw.G = dalloc<double>(plan, nkb * kk, by);
    bw.R1 = dalloc<double>(plan, nkb * kk, by);
    bw.R0 = dalloc<double>(plan, nkb * kk, by);
    bw.Atmp = dalloc<double>(plan, nkb * kk, by);
    bw.Bprev = dalloc<double>(plan, nkb * kk, by);
    bw.A = dalloc<double>(plan, nkb * m * kk, by);
    bw.B = dalloc<double>(plan, nkb * m * kk, by);
    bw.T = dalloc<double>(plan, nkb * nt * nt, by);
    bw.P = dalloc<double>(plan, nkb * bw.kb * nt, by);
    bw.d = dalloc<double>(plan, nkb * nt, by);
    bw.e = dalloc<double>(plan, nkb * nt, by);
    bw.flag = dalloc<int>(plan, nkb, by);
    bw.meff = dalloc<int>(plan, nkb, by);
  }
  std::vector<R> G, tw;
  host_tables<R>(g, G, tw);
  check(hipMemcpy(b.G, G.data(), G.size() * sizeof(R), hipMemcpyHostToDevice), "copy G");
  {
    // the same values with kz innermost: one z line of G per (ky, kx), contiguous
    const size_t K2 = g.K[1], K3 = g.K[2], KX = g.K[0] / 2 + 1;
    std::vector<R> Gt(G.size());
    for (size_t z = 0; z < K3; ++z)
      for (size_t yx = 0; yx < K2 * KX; ++yx) Gt[yx * K3 + z] = G[z * K2 * KX + yx];
    check(hipMemcpy(b.Gt, Gt.data(), Gt.size() * sizeof(R), hipMemcpyHostToDevice),
          "copy Gt");
  }
  check(hipMemcpy(b.tw, tw.data(), tw.size() * sizeof(R), hipMemcpyHostToDevice), "copy tw");
}

// Bracket the launches that f makes on stream st with events when stage timing is on.
template <typename F>
void staged_on(Plan& plan, int stage, hipStream_t st, F&& f) {
  if (!plan.timer.on) {
    f();
    return;
  }
  hipEvent_t a = plan.timer.next(), b = plan.timer.next();
  check(hipEventRecord(a, st), "event record");
  f();
  check(hipEventRecord(b, st), "event record");
  plan.timer.recs.push_back({stage, a, b});
}

template <typename F>
void staged(Plan& plan, int stage, F&& f) {
  staged_on(plan, stage, plan.stream, std::forward<F>(f));
}

// Start work on the side stream of st, if st has one: it waits for everything enqueued
// on st so far. Returns nullptr (run on st itself) for streams without a side stream:
// the internal per-system streams of a batch plan, which overlap whole systems instead.
SideStream* fork_side(Plan& plan, hipStream_t st) {
  SideStream* sd = plan.side_of(st);
  if (!sd) return nullptr;
  check(hipEventRecord(sd->fork, st), "side fork");
  check(hipStreamWaitEvent(sd->side, sd->fork, 0), "side fork");
  return sd;
}

// Make st wait for the side-stream work enqueued before `done` was recorded.
void join_side(hipStream_t st, hipStream_t side, hipEvent_t done) {
  check(hipEventRecord(done, side), "side join");
  check(hipStreamWaitEvent(st, done, 0), "side join");
}

template <typename R>
void run_setup(Plan& plan, System& S, const double* pos) {
  staged(plan, MBD_STAGE_SETUP, [&] {
    launch_setup<R>(S.geo, S.buf, pos, S.src.alpha, S.src.omega, S.src.r_vdw, plan.stream);
    if (S.buf.pg_T) launch_pair_build<R>(S.geo, S.buf, false, plan.stream);
  });
}

// Size and build the direct-space tensor list (B >= 16) for the positions set up
// last: one counting pass, then a capacity of 1.25 x the largest group plus 32
// (room for later set_positions calls), then the build.
template <typename R>
void create_pair_list(Plan& plan, System& S) {
  SysBuffers& b = S.buf;
  const int ngroups = (S.geo.n + kGroup - 1) / kGroup;
  b.pg_count = dalloc<int>(plan, ngroups, S.bytes);
  b.pg_max = dalloc<int>(plan, 1, S.bytes);
  launch_pair_build<R>(S.geo, b, true, plan.stream);
  check(hipGetLastError(), "pair list count");
  int mx = 0;
  check(hipStreamSynchronize(plan.stream), "pair list count");
  check(hipMemcpy(&mx, b.pg_max, sizeof(int), hipMemcpyDeviceToHost), "pair list count");
  b.pg_cap = ((mx + mx / 4 + 32) + 15) / 16 * 16;
  b.pg_hdr = dalloc<int2>(plan, (size_t)ngroups * b.pg_cap, S.bytes);
  b.pg_T = dalloc<R>(plan, (size_t)ngroups * b.pg_cap * kCandStride, S.bytes);
  b.pg_zero = dalloc<R>(plan, kTensorWords, S.bytes);
  check(hipMemset(b.pg_zero, 0, kTensorWords * sizeof(R)), "zero tensor");
  if (plan.forces) b.pg_F = dalloc<R>(plan, (size_t)ngroups * b.pg_cap * kCandStride, S.bytes);
  launch_pair_build<R>(S.geo, b, false, plan.stream);
}

// Spread of grid chunk c of the dipoles in b.dv, fused with the forward x pass when the
// system's shape selects the line spread; returns the first transform pass still to run
// (1 after the fused spread, else 0).
template <typename R>
int spread_chunk(Plan& plan, System& S, const SysBuffers& b, int c, hipStream_t st) {
  int first = 0;
  staged(plan, MBD_STAGE_SPREAD, [&] {
    if (S.shape.spread_mode == 1 && launch_spread_xline(S.geo, b, plan.B, S.BG, c, 1, st))
      first = 1;
    else
      launch_spread<R>(S.geo, b, plan.B, S.BG, c, 1, st);
  });
  return first;
}

// The adjoint matvec C lbar_k (into Lt) together with the bilinear force terms
// lbar_k^T dC/dR y_k of one reverse step: the pair part, then per grid chunk the
// reciprocal part with phi of p = g lbar_k (left by the matvec) and with phi of
// q = g y_k. q is c9 g y_k with a per-right-hand-side factor c9 (b.adj[16 rhs + 9]), so
// when the forward sweep kept its grids phi of q is c9 times the kept phi of step k,
// and the factor moves onto p; otherwise q is spread and transformed once more. The
// pair kernel and the pair force (into the direct half of fsum) run on the side stream
// beside the grid stages, forked as in matvec_block.
template <typename R>
void adjoint_matvec_forces(Plan& plan, System& S, int k) {
  const hipStream_t st = plan.stream;
  const int BG = S.BG;
  const int nch = plan.B / BG;
  SysBuffers& b = S.buf;
  SysBuffers bq = b;
  bq.dv = b.dq;
  SideStream* sd = nullptr;
  auto pair_work = [&] {
    sd = S.overlap ? fork_side(plan, st) : nullptr;
    const hipStream_t ss = sd ? sd->side : st;
    staged_on(plan, MBD_STAGE_PAIR, ss, [&] { launch_pair<R>(S.geo, b, plan.B, ss); });
    if (sd) check(hipEventRecord(sd->pair_done, ss), "side join");
    staged_on(plan, MBD_STAGE_FORCE, ss, [&] { launch_pair_force<R>(S.geo, b, plan.B, ss); });
  };
  if (S.overlap != 2) pair_work();
  int first = 0;
  for (int c = 0; c < nch; ++c) first = spread_chunk<R>(plan, S, b, c, st);
  if (S.overlap == 2) pair_work();
  for (int c = 0; c < nch; ++c)
    for (int pass = first; pass < 5; ++pass)
      staged(plan, MBD_STAGE_FFT_X + pass,
             [&] { launch_fft_pass<R>(S.geo, b, plan.B, BG, c, 1, pass, st); });
  if (sd) check(hipStreamWaitEvent(st, sd->pair_done, 0), "side join");
  for (int c = 0; c < nch; ++c) {
    staged(plan, MBD_STAGE_GATHER, [&] {
      launch_epilogue<R>(S.geo, b, b.lbar, plan.B, BG, c, 1, MBD_C_ALL, st);
    });
    staged(plan, MBD_STAGE_FORCE,
           [&] { launch_spme_force<R>(S.geo, b, b.dq, plan.B, BG, c, st); });
    if (b.phi) {
      SysBuffers bk = b;
      bk.grid = (R*)b.phi +
                (size_t)k * S.geo.K[2] * S.geo.K[1] * (S.geo.K[0] + 2) * plan.B;
      staged(plan, MBD_STAGE_FORCE, [&] {
        launch_spme_force<R>(S.geo, bk, b.dv, plan.B, BG, c, st, b.adj + 9);
      });
      continue;
    }
    const int fq = spread_chunk<R>(plan, S, bq, c, st);
    for (int pass = fq; pass < 5; ++pass)
      staged(plan, MBD_STAGE_FFT_X + pass,
             [&] { launch_fft_pass<R>(S.geo, bq, plan.B, BG, c, 1, pass, st); });
    staged(plan, MBD_STAGE_FORCE,
           [&] { launch_spme_force<R>(S.geo, b, b.dv, plan.B, BG, c, st); });
  }
  if (sd) join_side(st, sd->side, sd->force_done);
}

// Reverse sweep for one block of probes (their Krylov vectors are still in W).
template <typename R>
void run_backward(Plan& plan, System& S, int l0, int nb) {
  const hipStream_t st = plan.stream;
  const int B = plan.B, m = plan.prm.n_steps;
  const bool fl = sizeof(R) == 4;
  const size_t vs = 3 * (size_t)S.geo.n * B;
  staged(plan, MBD_STAGE_ADJOINT, [&] {
    launch_tridiag_adjoint(S.buf, nb, m, l0, plan.status, st);
    fill_double(S.buf.ybar, 0.0, 3 * vs, st);
  });
  for (int k = m - 1; k >= 0; --k) {
    staged(plan, MBD_STAGE_ADJOINT,
           [&] { launch_adjoint_step(S.geo, S.buf, B, nb, k, m, l0, fl, st); });
    adjoint_matvec_forces<R>(plan, S, k);
    staged(plan, MBD_STAGE_ADJOINT, [&] { launch_adjoint_accumulate(S.geo, S.buf, B, k, st); });
  }
}

// One application of C to the block stored at w (internal layout), into Lt.
// The grid stages run on st, stage by stage over the grid chunks (BG right-hand sides
// each): the spreads, then the five transform passes of each chunk, then the gathers,
// which are the first readers of the direct-space field. With a side stream
// (S.overlap 1 or 2) the ALU-bound pair kernel runs there concurrently with the
// HBM-bound grid stages, forked before the spreads (1) or after them, beside the
// transforms only (2), and joined before the gathers.
template <typename R>
void matvec_block(Plan& plan, System& S, const double* w, uint32_t comps,
                  void* phi_out = nullptr) {
  const hipStream_t st = plan.stream;
  const int BG = S.BG;
  const int nch = plan.B / BG;
  // replica method: Omega w + g (sum over images of f T) g w; no Ewald split
  if (S.geo.replica_cut > 0.0) comps &= (MBD_C_DIAG | MBD_C_DIR);
  SideStream* sd = nullptr;
  auto pair_work = [&] {
    sd = S.overlap ? fork_side(plan, st) : nullptr;
    const hipStream_t ss = sd ? sd->side : st;
    staged_on(plan, MBD_STAGE_PAIR, ss, [&] {
      if (S.geo.replica_cut > 0.0) launch_replica(S.geo, S.buf, plan.B, ss);
      else launch_pair<R>(S.geo, S.buf, plan.B, ss);
    });
  };
  const bool rec = (comps & MBD_C_REC) != 0;
  // with phi_out the step's grids live in phi_out (kept for the reverse force terms)
  SysBuffers bb = S.buf;
  if (phi_out) bb.grid = phi_out;
  if ((comps & MBD_C_DIR) && (S.overlap != 2 || !rec)) pair_work();
  int first = 0;
  if (rec)
    for (int c = 0; c < nch; ++c) first = spread_chunk<R>(plan, S, bb, c, st);
  if ((comps & MBD_C_DIR) && S.overlap == 2 && rec) pair_work();
  if (rec)
    for (int c = 0; c < nch; ++c)
      for (int pass = first; pass < 5; ++pass)
        staged(plan, MBD_STAGE_FFT_X + pass,
               [&] { launch_fft_pass<R>(S.geo, bb, plan.B, BG, c, 1, pass, st); });
  if (sd) join_side(st, sd->side, sd->pair_done);
  for (int c = 0; c < nch; ++c)
    staged(plan, MBD_STAGE_GATHER,
           [&] { launch_epilogue<R>(S.geo, bb, w, plan.B, BG, c, 1, comps, st); });
}

template <typename R>
void run_backward(Plan& plan, System& S, int l0, int nb);

// Block Lanczos (krylov_block > 1): per batch of B probes, B / kb Krylov blocks run
// side by side through the same matvecs; each block step replaces the scalar update.
template <typename R>
void run_energy_block(Plan& plan, System& S, int sys_index, double* energy, double* sd) {
  const hipStream_t st = plan.stream;
  const int B = plan.B, m = plan.prm.n_steps, R_probes = plan.prm.n_probes;
  const bool fl = sizeof(R) == 4;
  const size_t vs = 3 * (size_t)S.geo.n * B;
  const BlockWork& bw = S.buf.blk;
  for (int l0 = 0; l0 < R_probes; l0 += B) {
    const int nb = std::min(B, R_probes - l0);
    staged(plan, MBD_STAGE_LANCZOS, [&] {
      launch_init_scalars(S.buf, nb, m, l0, st);
      launch_probes(S.geo, S.buf, B, nb, l0, plan.prm.seed, sys_index, fl, st);
      launch_block_start(S.geo, S.buf, bw, B, m, fl, st);
    });
    for (int k = 0; k < m; ++k) {
      matvec_block<R>(plan, S, S.buf.W + (size_t)k * vs, MBD_C_ALL);
      staged(plan, MBD_STAGE_LANCZOS,
             [&] { launch_block_step(S.geo, S.buf, bw, B, k, m, fl, st); });
    }
    staged(plan, MBD_STAGE_LANCZOS, [&] {
      launch_block_quadrature(bw, nb / bw.kb, m, S.buf.q + l0, plan.status, st);
    });
  }
  staged(plan, MBD_STAGE_LANCZOS,
         [&] { launch_energy(S.geo, S.buf, R_probes, energy, sd, plan.status, st); });
}

template <typename R>
void run_energy(Plan& plan, System& S, int sys_index, double* energy, double* sd, bool forces) {
  if (plan.prm.krylov_block > 1) {
    run_energy_block<R>(plan, S, sys_index, energy, sd);
    return;
  }
  const hipStream_t st = plan.stream;
  const int B = plan.B, m = plan.prm.n_steps, R_probes = plan.prm.n_probes;
  const bool fl = sizeof(R) == 4;
  const size_t vs = 3 * (size_t)S.geo.n * B;
  for (int l0 = 0; l0 < R_probes; l0 += B) {
    const int nb = std::min(B, R_probes - l0);
    staged(plan, MBD_STAGE_LANCZOS, [&] {
      launch_init_scalars(S.buf, nb, m, l0, st);
      launch_probes(S.geo, S.buf, B, nb, l0, plan.prm.seed, sys_index, fl, st);
    });
    const size_t gsz = (size_t)S.geo.K[2] * S.geo.K[1] * (S.geo.K[0] + 2) * B;
    for (int k = 0; k < m; ++k) {
      void* slot = (forces && S.buf.phi) ? (void*)((R*)S.buf.phi + (size_t)k * gsz) : nullptr;
      matvec_block<R>(plan, S, S.buf.W + (size_t)k * vs, MBD_C_ALL, slot);
      staged(plan, MBD_STAGE_LANCZOS, [&] {
        launch_finish_a(S.buf, B, nb, k, m, l0, plan.status, st);
        if (k + 1 < m) {
          const int ro = plan.prm.reorth;
          launch_update(S.geo, S.buf, B, nb, k, m, l0, fl, ro == MBD_REORTH_NONE, st);
          if (ro == MBD_REORTH_LOCAL) {
            launch_reorth(S.geo, S.buf, B, nb, k, m, l0, std::max(0, k - 1), fl, st);
          } else if (ro == MBD_REORTH_FULL) {
            launch_reorth(S.geo, S.buf, B, nb, k, m, l0, 0, fl, st);
            launch_reorth(S.geo, S.buf, B, nb, k, m, l0, 0, fl, st);
          }
          launch_finish_norm(S.buf, B, nb, k, m, l0, plan.status, st);
        }
      });
    }
    staged(plan, MBD_STAGE_LANCZOS,
           [&] { launch_tridiag(S.buf, nb, m, l0, plan.status, st); });
    if (forces) run_backward<R>(plan, S, l0, nb);
  }
  staged(plan, MBD_STAGE_LANCZOS,
         [&] { launch_energy(S.geo, S.buf, R_probes, energy, sd, plan.status, st); });
}

mbd_status fail(mbd_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Allocation-free screening workspace: one array per device, 64 MiB, kept until the
// process ends. Host code reaches it only through the address hipGetSymbolAddress
// returns for the device (resolved once per device when a plan is created there).
constexpr size_t kScsScratchDoubles = (size_t)64 << 17;  // 64 MiB of doubles
static __device__ __align__(256) double scratch[kScsScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {nullptr};

// Address of this device's scratch array (the current device must be `device`).
mbd_status resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(MBD_E_NODEVICE, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return MBD_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MBD_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return MBD_OK;
}

double* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return g_scratch_ptr[device];
}

// ---- launch shapes and their tuner ---------------------------------------------------
// A shape only changes how a system's matvec is laid out on the GPU: work-groups of the
// list kernel, lanes per target and a side stream for the pair kernel leave every result
// bit unchanged; the grid chunk width changes the summation order of the spread and the
// gather (sub-lanes share a stencil below 64 right-hand sides per chunk), and the
// matrix-core pair kernel the order of the direct-space sums.

constexpr mbd_shape kBuiltinShape = {0, 0, 0, 1, 0, 0, 0};

bool valid_shape(const mbd_shape& sh, int B) {
  const bool pow2chunk = sh.grid_chunk == 0 || (sh.grid_chunk > 0 && sh.grid_chunk <= 64 &&
                                                is_pow2(sh.grid_chunk) && B % sh.grid_chunk == 0);
  return sh.pair_wg_per_cu >= 0 && sh.pair_wg_per_cu <= 64 &&
         (sh.pair_subsets == 0 || sh.pair_subsets == 1 || sh.pair_subsets == 2 ||
          sh.pair_subsets == 4) &&
         pow2chunk && sh.overlap >= 0 && sh.overlap <= 2 &&
         (sh.gather_waves == 0 || sh.gather_waves == 4 || sh.gather_waves == 8) &&
         (sh.spread_mode == 0 || sh.spread_mode == 1) &&
         (sh.pair_mode >= 0 && sh.pair_mode <= 2);
}

void apply_shape(const Plan& plan, System& S, const mbd_shape& sh) {
  S.shape = sh;
  S.geo.pair_blocks = sh.pair_wg_per_cu * plan.cus;
  S.geo.pair_ns = sh.pair_subsets;
  S.geo.gather_waves = sh.gather_waves;
  S.BG = sh.grid_chunk > 0 ? sh.grid_chunk : plan.BG;
  // the per-system streams of a batch plan have no side stream
  S.overlap = plan.batch ? 0 : sh.overlap;
  S.shape.overlap = S.overlap;
  // the fused line spread exists for float grids, p = 6 and 64-wide chunks
  if (!(plan.prec == MBD_PREC_MIXED && S.geo.p == 6 && S.BG == 64 && S.buf.line_start))
    S.shape.spread_mode = 0;
  // its atom lists are built from here on (and by every later setup) only when used
  const int lines = S.shape.spread_mode == 1 ? 1 : 0;
  if (lines && !S.geo.line_lists) {
    S.geo.line_lists = 1;
    launch_line_lists(S.geo, S.buf, plan.stream);
  }
  S.geo.line_lists = lines;
  // the matrix-core list kernel exists for float tensors and block = 64, 128, 192, 256
  if (!(plan.prec == MBD_PREC_MIXED && plan.B % 64 == 0 && plan.B <= 256 && S.buf.pg_T &&
        S.geo.replica_cut <= 0.0))
    S.shape.pair_mode = 0;
  S.geo.pair_mode = S.shape.pair_mode;
}

std::string shape_key(const Plan& plan, const System& S) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|N=%d|K=%dx%dx%d|p=%d|B=%d|prec=%d|forces=%d|batch=%d",
                plan.arch.c_str(), S.geo.n, S.geo.K[0], S.geo.K[1], S.geo.K[2], S.geo.p, plan.B,
                plan.prec, plan.forces ? 1 : 0, plan.batch ? 1 : 0);
  return buf;
}

// Value of an integer or real field `"name": v` in one JSON line (false if absent).
bool json_number(const std::string& line, const char* name, double& v) {
  const std::string tag = std::string("\"") + name + "\":";
  const size_t at = line.find(tag);
  if (at == std::string::npos) return false;
  const char* p = line.c_str() + at + tag.size();
  char* end = nullptr;
  v = std::strtod(p, &end);
  return end != p;
}

// The last cached shape for key in a JSON-lines file, if any.
bool cache_lookup(const char* path, const std::string& key, mbd_shape& sh, double& ms) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[1024];
  const std::string tag = "\"key\": \"" + key + "\"";
  while (std::fgets(line, sizeof line, f)) {
    const std::string l(line);
    if (l.find(tag) == std::string::npos) continue;
    double a, b, c, d, e, f, g = 0.0, t = 0.0;
    if (json_number(l, "pair_wg_per_cu", a) && json_number(l, "pair_subsets", b) &&
        json_number(l, "grid_chunk", c) && json_number(l, "overlap", d) &&
        json_number(l, "gather_waves", e) && json_number(l, "spread_mode", f)) {
      json_number(l, "pair_mode", g);
      json_number(l, "matvec_ms", t);
      sh = mbd_shape{(int32_t)a, (int32_t)b, (int32_t)c, (int32_t)d, (int32_t)e, (int32_t)f,
                     (int32_t)g};
      ms = t;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const mbd_shape& sh, double ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\": \"%s\", \"pair_wg_per_cu\": %d, \"pair_subsets\": %d, "
               "\"grid_chunk\": %d, \"overlap\": %d, \"gather_waves\": %d, "
               "\"spread_mode\": %d, \"pair_mode\": %d, \"matvec_ms\": %.5f}\n",
               key.c_str(), sh.pair_wg_per_cu, sh.pair_subsets, sh.grid_chunk, sh.overlap,
               sh.gather_waves, sh.spread_mode, sh.pair_mode, ms);
  std::fclose(f);
}

// Fastest of `reps` timed applications of C to the probe block in W[0] (after one
// untimed application), in milliseconds, with the system's current shape.
template <typename R>
double time_matvec(Plan& plan, System& S, int reps) {
  hipEvent_t a = nullptr, b = nullptr;
  check(hipEventCreate(&a), "event create");
  check(hipEventCreate(&b), "event create");
  float best = 1e30f;
  try {
    matvec_block<R>(plan, S, S.buf.W, MBD_C_ALL);
    for (int r = 0; r < reps; ++r) {
      check(hipEventRecord(a, plan.stream), "event record");
      matvec_block<R>(plan, S, S.buf.W, MBD_C_ALL);
      check(hipEventRecord(b, plan.stream), "event record");
      check(hipEventSynchronize(b), "event sync");
      float t = 0.f;
      check(hipEventElapsedTime(&t, a, b), "event time");
      best = std::min(best, t);
    }
  } catch (...) {
    hipEventDestroy(a);
    hipEventDestroy(b);
    throw;
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return best;
}

// Coordinate search over the shape knobs on the system's real data: the pair kernel's
// residency together with the side stream, then its lanes per target or the matrix-core
// kernel with its candidate split, then the gather's work-group size, then the grid
// chunk width, then the residency once more under the chosen chunk. Where the
// matrix-core kernel applies it is the starting point, with its widest candidate split:
// alone it is the faster pair kernel by about a fifth, while beside the side stream's
// grid chain the two kernels often time within the 2 % margin, and a start from the
// vector kernel would then keep the slower one. The fused x-line
// spread is left out: it runs about four times slower than the tile spread plus the x
// pass on a 96^3 grid with 24,000 atoms (each atom's loads and weights are repeated on
// all 36 lines it touches).
template <typename R>
void tune_system(Plan& plan, System& S, int sys_index) {
  const int B = plan.B;
  launch_probes(S.geo, S.buf, B, B, 0, plan.prm.seed, sys_index, sizeof(R) == 4, plan.stream);
  const bool list = S.buf.pg_T != nullptr && S.geo.replica_cut <= 0.0;
  // the matrix-core launcher's rule: B / (128 or 64) column wavefronts times NK candidate
  // shares, at most 4 wavefronts per work-group
  const bool mfma = list && plan.prec == MBD_PREC_MIXED && B % 64 == 0 && B <= 256;
  const int mfma_nn = B / (B % 128 == 0 ? 128 : 64);
  mbd_shape best = kBuiltinShape;
  if (mfma) {
    best.pair_mode = 1;
    best.pair_subsets = mfma_nn * 4 <= 4 ? 4 : (mfma_nn * 2 <= 4 ? 2 : 1);
  }
  apply_shape(plan, S, best);
  best = S.shape;
  double tbest = time_matvec<R>(plan, S, 5);
  // a candidate replaces the best shape only when it is at least 2 % faster (fastest of
  // five timings each), so that timing noise does not pick residency caps or other
  // knobs that do not pay once the matvecs are replayed from a graph
  auto trial = [&](const mbd_shape& sh) {
    apply_shape(plan, S, sh);
    const double t = time_matvec<R>(plan, S, 5);
    if (t < 0.98 * tbest) {
      tbest = t;
      best = S.shape;
    }
  };
  auto residency = [&] {
    const mbd_shape base = best;
    for (int ov = plan.batch ? 0 : 2; ov >= 0; --ov)
      for (int wg : {0, 1, 2, 3, 4}) {
        if (!list && wg > 0) continue;
        mbd_shape sh = base;
        sh.overlap = ov;
        sh.pair_wg_per_cu = wg;
        if (sh.overlap != base.overlap || sh.pair_wg_per_cu != base.pair_wg_per_cu) trial(sh);
      }
  };
  residency();
  if (list) {
    const mbd_shape base = best;
    for (int ns : {1, 2, 4}) {
      if (ns * B < 64) continue;
      mbd_shape sh = base;
      sh.pair_mode = 0;
      sh.pair_subsets = ns;
      if (base.pair_mode != 0 || base.pair_subsets != ns) trial(sh);
    }
    // the matrix-core kernel with 4, 2 or 1 wavefronts per group's candidates, and, where
    // B is a multiple of 128, with 64-column wavefronts (fewer accumulator registers per
    // wavefront, which leaves room for the transforms beside it)
    if (mfma) {
      for (int nk : {4, 2, 1}) {
        if (mfma_nn * nk > 4) continue;
        mbd_shape sh = base;
        sh.pair_mode = 1;
        sh.pair_subsets = nk;
        if (base.pair_mode != 1 || base.pair_subsets != nk) trial(sh);
      }
      if (B % 128 == 0)
        for (int nk : {2, 1}) {
          if ((B / 64) * nk > 4) continue;
          mbd_shape sh = base;
          sh.pair_mode = 2;
          sh.pair_subsets = nk;
          trial(sh);
        }
    }
  }
  {
    mbd_shape sh = best;
    sh.gather_waves = 8;
    trial(sh);
  }
  {
    const mbd_shape base = best;
    const int dflt = plan.BG;
    for (int bg : {8, 16, 32, 64}) {
      if (bg > B || B % bg != 0 || bg == (base.grid_chunk ? base.grid_chunk : dflt)) continue;
      if (bg < dflt / 4) continue;
      mbd_shape sh = base;
      sh.grid_chunk = bg;
      trial(sh);
    }
  }
  residency();
  apply_shape(plan, S, best);
  S.shape_source = MBD_SHAPE_MEASURED;
  S.tune_ms = tbest;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

SideStream* Plan::side_of(hipStream_t origin) {
  for (SideStream& s : sides)
    if (s.origin == origin) return &s;
  return nullptr;
}

// Side stream and events for one origin stream (created right after the origin so that
// the two map to different hardware queues).
void add_side(Plan& plan, hipStream_t origin) {
  for (const SideStream& s : plan.sides)
    if (s.origin == origin) return;
  SideStream s;
  s.origin = origin;
  check(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking), "stream create");
  plan.sides.push_back(s);
  SideStream& t = plan.sides.back();
  check(hipEventCreateWithFlags(&t.fork, hipEventDisableTiming), "event create");
  check(hipEventCreateWithFlags(&t.pair_done, hipEventDisableTiming), "event create");
  check(hipEventCreateWithFlags(&t.force_done, hipEventDisableTiming), "event create");
}

hipEvent_t StageTimer::next() {
  if (used == pool.size()) {
    hipEvent_t e;
    check(hipEventCreate(&e), "event create");
    pool.push_back(e);
  }
  return pool[used++];
}

}  // namespace mbd

struct mbd_plan_s {
  mbd::Plan plan;
};

using mbd::fail;

extern "C" {

const char* mbd_last_error(void) { return mbd::g_last_error.c_str(); }

const char* mbd_status_string(mbd_status s) {
  switch (s) {
    case MBD_OK: return "ok";
    case MBD_E_ARG: return "invalid argument";
    case MBD_E_CELL: return "invalid cell";
    case MBD_E_GRID: return "unsupported grid";
    case MBD_E_NOT_POSDEF: return "coupling matrix not positive definite";
    case MBD_E_NONFINITE: return "non-finite value";
    case MBD_E_NODEVICE: return "no GPU device";
    case MBD_E_HIP: return "HIP runtime error";
    case MBD_E_OOM: return "out of device memory";
    case MBD_E_STATE: return "call out of order";
    case MBD_E_NOCONV: return "iterative solve did not converge";
    default: return "unknown status";
  }
}

int32_t mbd_grid_supported(int32_t k) { return mbd::fft_supported(k) ? 1 : 0; }

mbd_status mbd_plan_create(mbd_plan* out, const mbd_system* systems, int32_t n_sys,
                           const mbd_params* prm_in, void* stream) {
  using namespace mbd;
  if (!out) return fail(MBD_E_ARG, "out is NULL");
  *out = nullptr;
  if (!systems || n_sys < 1) return fail(MBD_E_ARG, "need at least one system");
  if (!prm_in) return fail(MBD_E_ARG, "params is NULL");
  mbd_params prm = *prm_in;
  if (!(prm.damp_beta > 0.0) || !std::isfinite(prm.damp_beta))
    return fail(MBD_E_ARG, "damp_beta must be > 0");
  if (!(prm.damp_d > 0.0) || !std::isfinite(prm.damp_d))
    return fail(MBD_E_ARG, "damp_d must be > 0");
  if (!(prm.real_cutoff > 0.0) || !std::isfinite(prm.real_cutoff))
    return fail(MBD_E_ARG, "real_cutoff must be > 0");
  if (!std::isfinite(prm.ewald_tau)) return fail(MBD_E_ARG, "ewald_tau is not finite");
  if (!std::isfinite(prm.damp_tol) || prm.damp_tol >= 0.5)
    return fail(MBD_E_ARG, "damp_tol must be < 0.5");
  if (prm.spline_order == 0) prm.spline_order = 6;
  if (prm.spline_order != 4 && prm.spline_order != 6 && prm.spline_order != 8)
    return fail(MBD_E_ARG, "spline_order must be 4, 6 or 8");
  if (prm.n_probes < 1) return fail(MBD_E_ARG, "n_probes must be >= 1");
  if (prm.n_steps < 1 || prm.n_steps > kMaxSteps)
    return fail(MBD_E_ARG, "n_steps must be in [1, 512]");
  if (prm.block == 0) {
    int b = 1;
    while (b < prm.n_probes && b < 128) b *= 2;
    prm.block = b;
  }
  if (!is_pow2(prm.block) || prm.block > 256)
    return fail(MBD_E_ARG, "block must be a power of two <= 256");
  if (prm.precision != MBD_PREC_FP64 && prm.precision != MBD_PREC_MIXED)
    return fail(MBD_E_ARG, "precision must be MBD_PREC_FP64 or MBD_PREC_MIXED");
  if (prm.reorth < MBD_REORTH_NONE || prm.reorth > MBD_REORTH_FULL)
    return fail(MBD_E_ARG, "reorth must be NONE, LOCAL or FULL");
  if (prm.want_forces != 0 && prm.want_forces != 1)
    return fail(MBD_E_ARG, "want_forces must be 0 or 1");
  if (prm.want_forces && prm.block < 4)
    return fail(MBD_E_ARG, "forces need block >= 4");
  if (prm.graph != 0 && prm.graph != 1) return fail(MBD_E_ARG, "graph must be 0 or 1");
  if (!std::isfinite(prm.replica_cutoff) || prm.replica_cutoff < 0.0)
    return fail(MBD_E_ARG, "replica_cutoff must be finite and >= 0");
  if (prm.replica_cutoff > 0.0) {
    if (prm.precision != MBD_PREC_FP64)
      return fail(MBD_E_ARG, "the replica method runs in float64 only");
    if (prm.want_forces) return fail(MBD_E_ARG, "the replica method has no forces");
    if (prm.block > 8) return fail(MBD_E_ARG, "the replica method needs block <= 8");
  }
  if (prm.krylov_block == 0) prm.krylov_block = 1;
  if (prm.krylov_block != 1 && prm.krylov_block != 2 && prm.krylov_block != 4 &&
      prm.krylov_block != 8)
    return fail(MBD_E_ARG, "krylov_block must be 0, 1, 2, 4 or 8");
  if (prm.krylov_block > 1) {
    const int kb = prm.krylov_block;
    if (prm.block % kb != 0) return fail(MBD_E_ARG, "block must be a multiple of krylov_block");
    if (prm.n_probes % kb != 0)
      return fail(MBD_E_ARG, "n_probes must be a multiple of krylov_block");
    if (prm.want_forces) return fail(MBD_E_ARG, "block Lanczos plans have no forces");
    if (prm.reorth != MBD_REORTH_NONE)
      return fail(MBD_E_ARG, "block Lanczos runs without re-orthogonalization");
    if (prm.n_steps * kb > kBlockMaxDim)
      return fail(MBD_E_ARG, "n_steps * krylov_block must be <= 512");
  }
  for (int a = 0; a < 3; ++a)
    if (prm.grid[a] < 0) return fail(MBD_E_ARG, "grid sizes must be >= 0");
  if (prm.tune != MBD_TUNE_OFF && prm.tune != MBD_TUNE_MEASURE && prm.tune != MBD_TUNE_GIVEN)
    return fail(MBD_E_ARG, "tune must be MBD_TUNE_OFF, MBD_TUNE_MEASURE or MBD_TUNE_GIVEN");
  if (prm.tune == MBD_TUNE_GIVEN && !valid_shape(prm.shape, prm.block))
    return fail(MBD_E_ARG, "shape: pair_wg_per_cu in [0, 64], pair_subsets 0/1/2/4, grid_chunk "
                           "0 or a power of two <= 64 dividing block, overlap 0/1/2, "
                           "gather_waves 0/4/8, spread_mode 0/1, pair_mode 0/1/2");

  const int BG_plan = std::min(prm.block, prm.precision == MBD_PREC_FP64 ? 16 : 64);
  std::vector<Geometry> geos(n_sys);
  for (int s = 0; s < n_sys; ++s) {
    const mbd_system& sy = systems[s];
    if (sy.n_atoms < 1) return fail(MBD_E_ARG, "n_atoms must be >= 1");
    if (3 * sy.n_atoms < prm.krylov_block)
      return fail(MBD_E_ARG, "krylov_block exceeds the dimension 3N of a system");
    if (!sy.pos || !sy.alpha || !sy.omega || !sy.r_vdw)
      return fail(MBD_E_ARG, "system arrays must be non-NULL device pointers");
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(sy.cell[i])) return fail(MBD_E_ARG, "cell is not finite");
    Geometry& g = geos[s];
    g.n = sy.n_atoms;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) g.A[r][c] = sy.cell[3 * r + c];
    const double vol = cell_volume(g.A);
    for (int a = 0; a < 3; ++a)
      g.L[a] = std::sqrt(g.A[a][0] * g.A[a][0] + g.A[a][1] * g.A[a][1] + g.A[a][2] * g.A[a][2]);
    if (!(vol > 1e-6 * g.L[0] * g.L[1] * g.L[2]))
      return fail(MBD_E_CELL, "cell vectors must be right-handed with a non-degenerate volume");
    reciprocal(g.A, g.Ar);
    g.p = prm.spline_order;
    for (int a = 0; a < 3; ++a) {
      int K = prm.grid[a] > 0 ? prm.grid[a] : grid_rule(g.L[a]);
      if (!fft_supported(K))
        return fail(MBD_E_GRID, "grid size " + std::to_string(K) +
                                     " unsupported (even 2^a 3^b 5^c in [8, 128])");
      if (K < 2 * g.p) return fail(MBD_E_GRID, "grid must be >= 2 p");
      g.K[a] = K;
    }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) g.Mu[a][c] = g.K[a] * g.Ar[a][c];
    // Spread tiles: 4x4x4 grid points, one wavefront each.
    g.tile[0] = g.tile[1] = g.tile[2] = kSpreadTile;
    for (int a = 0; a < 3; ++a) g.tiles[a] = (g.K[a] + g.tile[a] - 1) / g.tile[a];
    g.tau = prm.ewald_tau > 0.0
                ? prm.ewald_tau
                : tau_from_cutoff_angstrom(prm.real_cutoff * kBohrAngstrom) * kBohrAngstrom;
    g.beta = prm.damp_beta;
    g.damp_d = prm.damp_d;
    g.replica_cut = prm.replica_cutoff;
    g.n_images = 0;
  }

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(MBD_E_NODEVICE, "no HIP device available");
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MBD_E_HIP, "no current device");
    const mbd_status sr = resolve_scratch(dev);
    if (sr != MBD_OK) return sr;
  }

  auto* handle = new (std::nothrow) mbd_plan_s();
  if (!handle) return fail(MBD_E_OOM, "host allocation failed");
  Plan& plan = handle->plan;
  plan.prm = prm;
  plan.prec = prm.precision;
  plan.B = prm.block;
  plan.BG = BG_plan;
  plan.forces = prm.want_forces != 0;
  plan.use_graph = prm.graph != 0;
  plan.stream = static_cast<hipStream_t>(stream);
  plan.batch = n_sys > 1;
  hipGetDevice(&plan.device);
  {
    hipDeviceProp_t dp;
    if (hipGetDeviceProperties(&dp, plan.device) == hipSuccess) {
      plan.cus = std::max(1, dp.multiProcessorCount);
      plan.arch = dp.gcnArchName;
      const size_t colon = plan.arch.find(':');
      if (colon != std::string::npos) plan.arch.resize(colon);
    }
  }
  try {
    size_t sb = 0;
    add_side(plan, plan.stream);
    plan.status = dalloc<uint32_t>(plan, 1, sb);
    check(hipMemset(plan.status, 0, sizeof(uint32_t)), "clear status");
    plan.sys.resize(n_sys);
    for (int s = 0; s < n_sys; ++s) {
      const mbd_system& sy = systems[s];
      System& S = plan.sys[s];
      S.geo = geos[s];
      std::memcpy(S.host_cell, sy.cell, sizeof(S.host_cell));
      // host copies of the per-atom parameters: validation and the damping range
      std::vector<double> al(sy.n_atoms), om(sy.n_atoms), rv(sy.n_atoms);
      check(hipMemcpy(al.data(), sy.alpha, sizeof(double) * sy.n_atoms, hipMemcpyDeviceToHost),
            "read alpha");
      check(hipMemcpy(om.data(), sy.omega, sizeof(double) * sy.n_atoms, hipMemcpyDeviceToHost),
            "read omega");
      check(hipMemcpy(rv.data(), sy.r_vdw, sizeof(double) * sy.n_atoms, hipMemcpyDeviceToHost),
            "read r_vdw");
      double rmax = 0.0;
      for (int i = 0; i < sy.n_atoms; ++i) {
        if (!(al[i] > 0.0) || !std::isfinite(al[i]) || !(om[i] > 0.0) ||
            !std::isfinite(om[i]) || !(rv[i] > 0.0) || !std::isfinite(rv[i])) {
          mbd_plan_destroy(handle);
          return fail(MBD_E_ARG, "alpha, omega and r_vdw must be finite and > 0");
        }
        rmax = std::max(rmax, rv[i]);
      }
      S.src = sy;
      Geometry& g = S.geo;
      double rp = prm.real_cutoff;
      if (prm.damp_tol >= 0.0) {
        const double tol = prm.damp_tol > 0.0 ? prm.damp_tol : 1e-4;
        const double smax = prm.damp_beta * 2.0 * rmax;
        rp = std::max(rp, smax * (1.0 + std::log(1.0 / tol - 1.0) / prm.damp_d));
      }
      g.r_pair = rp;
      g.mbits = 0;
      for (int a = 0; a < 3; ++a) {
        // cells are slices of the fractional coordinates; their width perpendicular to
        // the faces is w_a / nc_a with w_a = 1 / |a*_a|, and a source within r_pair is
        // at most ceil(r_pair / width) cells away along each axis
        const double w = 1.0 / std::sqrt(g.Ar[a][0] * g.Ar[a][0] + g.Ar[a][1] * g.Ar[a][1] +
                                         g.Ar[a][2] * g.Ar[a][2]);
        g.nc[a] = std::max(1, (int)std::floor(w / (0.5 * rp)));
        g.nc[a] = std::min(g.nc[a], 64);
        g.hc[a] = w / g.nc[a];
        g.nr[a] = (int)std::ceil(rp / g.hc[a] - 1e-12);
        for (int c = 0; c < 3; ++c) g.hv[a][c] = g.A[a][c] / g.nc[a];
        while ((1 << g.mbits) < g.nc[a]) ++g.mbits;
      }
      if (g.replica_cut > 0.0) {
        // every lattice vector n with |n A| < R_cut + |a1| + |a2| + |a3| (any pair of
        // atoms of the cell is closer than the sum of the cell vector lengths)
        const double reach = g.replica_cut + g.L[0] + g.L[1] + g.L[2];
        int nmax[3];
        for (int a = 0; a < 3; ++a)
          nmax[a] = 1 + (int)std::ceil(reach * std::sqrt(g.Ar[a][0] * g.Ar[a][0] +
                                                         g.Ar[a][1] * g.Ar[a][1] +
                                                         g.Ar[a][2] * g.Ar[a][2]));
        std::vector<int> img;
        for (int i = -nmax[0]; i <= nmax[0]; ++i)
          for (int j = -nmax[1]; j <= nmax[1]; ++j)
            for (int k = -nmax[2]; k <= nmax[2]; ++k) {
              double v2 = 0.0;
              for (int c = 0; c < 3; ++c) {
                const double x = i * g.A[0][c] + j * g.A[1][c] + k * g.A[2][c];
                v2 += x * x;
              }
              if (v2 < reach * reach) {
                img.push_back(i);
                img.push_back(j);
                img.push_back(k);
              }
            }
        g.n_images = (int)(img.size() / 3);
        S.buf.images = dalloc<int>(plan, img.size(), S.bytes);
        check(hipMemcpy(S.buf.images, img.data(), img.size() * sizeof(int),
                        hipMemcpyHostToDevice), "copy images");
      }
      if (plan.prec == MBD_PREC_FP64) {
        allocate_system<double>(plan, S, prm.n_probes, prm.n_steps);
        run_setup<double>(plan, S, sy.pos);
        if (plan.B >= 16 || plan.forces) create_pair_list<double>(plan, S);
      } else {
        allocate_system<float>(plan, S, prm.n_probes, prm.n_steps);
        run_setup<float>(plan, S, sy.pos);
        if (plan.B >= 16 || plan.forces) create_pair_list<float>(plan, S);
      }
      check(hipGetLastError(), "setup launch");
      // launch shape: built in, given, cached or measured on this system
      if (prm.tune == MBD_TUNE_GIVEN) {
        apply_shape(plan, S, prm.shape);
        S.shape_source = MBD_SHAPE_GIVEN;
      } else if (prm.tune == MBD_TUNE_MEASURE && g.replica_cut <= 0.0) {
        const std::string key = shape_key(plan, S);
        mbd_shape sh;
        double ms = 0.0;
        if (cache_lookup(prm.tune_cache, key, sh, ms) && valid_shape(sh, plan.B)) {
          apply_shape(plan, S, sh);
          S.shape_source = MBD_SHAPE_CACHED;
          S.tune_ms = ms;
        } else {
          if (plan.prec == MBD_PREC_FP64) tune_system<double>(plan, S, s);
          else tune_system<float>(plan, S, s);
          cache_store(prm.tune_cache, key, S.shape, S.tune_ms);
        }
      } else {
        apply_shape(plan, S, kBuiltinShape);
        S.shape_source = MBD_SHAPE_BUILTIN;
      }
    }
    if (plan.use_graph) {
      check(hipStreamCreateWithFlags(&plan.gstream, hipStreamNonBlocking), "stream create");
      add_side(plan, plan.gstream);
      check(hipEventCreateWithFlags(&plan.g_in, hipEventDisableTiming), "event create");
      check(hipEventCreateWithFlags(&plan.g_out, hipEventDisableTiming), "event create");
      size_t nat = 0, gb = 0;
      for (const auto& S : plan.sys) nat += (size_t)S.geo.n;
      plan.e_out = dalloc<double>(plan, n_sys, gb);
      plan.sd_out = dalloc<double>(plan, n_sys, gb);
      if (plan.forces) plan.f_out = dalloc<double>(plan, 3 * nat, gb);
    }
    if (n_sys > 1) {
      // Longest-processing-time assignment of systems to up to 4 streams; the cost of
      // one system is taken as N + K1 K2 K3 (pair work and grid work per right-hand side).
      const int ns = std::min(n_sys, 4);
      plan.pool.resize(ns, nullptr);
      plan.pool_done.resize(ns, nullptr);
      for (int i = 0; i < ns; ++i) {
        check(hipStreamCreateWithFlags(&plan.pool[i], hipStreamNonBlocking), "stream create");
        check(hipEventCreateWithFlags(&plan.pool_done[i], hipEventDisableTiming), "event create");
      }
      check(hipEventCreateWithFlags(&plan.fork, hipEventDisableTiming), "event create");
      std::vector<int> order(n_sys);
      std::vector<double> cost(n_sys), load(ns, 0.0);
      for (int i = 0; i < n_sys; ++i) {
        const Geometry& g = plan.sys[i].geo;
        order[i] = i;
        cost[i] = (double)g.n + (double)g.K[0] * g.K[1] * g.K[2];
      }
      std::sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
      plan.sys_stream.assign(n_sys, 0);
      for (int i : order) {
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        plan.sys_stream[i] = j;
        load[j] += cost[i];
      }
    }
  } catch (const std::bad_alloc&) {
    mbd_plan_destroy(handle);
    return fail(MBD_E_OOM, "device allocation failed");
  } catch (const HipError& e) {
    std::string msg = std::string(e.what) + ": " + hipGetErrorString(e.e);
    mbd_plan_destroy(handle);
    return fail(MBD_E_HIP, msg);
  }
  // keep the caller's parameter pointers for set_positions
  *out = handle;
  return MBD_OK;
}

mbd_status mbd_plan_info(mbd_plan plan, int32_t sys, mbd_info* info) {
  if (!plan || !info) return fail(MBD_E_ARG, "NULL argument");
  mbd::Plan& P = plan->plan;
  if (sys < 0 || sys >= (int)P.sys.size()) return fail(MBD_E_ARG, "system index out of range");
  const mbd::Geometry& g = P.sys[sys].geo;
  info->tau = g.tau;
  info->r_pair = g.r_pair;
  for (int a = 0; a < 3; ++a) {
    info->grid[a] = g.K[a];
    info->cells[a] = g.nc[a];
  }
  info->spline_order = g.p;
  info->block = P.B;
  info->workspace_bytes = P.sys[sys].bytes;
  info->n_pairs = P.prec == MBD_PREC_FP64
                      ? mbd::count_pairs<double>(g, P.sys[sys].buf, P.stream)
                      : mbd::count_pairs<float>(g, P.sys[sys].buf, P.stream);
  info->shape = P.sys[sys].shape;
  info->shape_source = P.sys[sys].shape_source;
  info->tune_ms = P.sys[sys].tune_ms;
  if (info->n_pairs < 0) return fail(MBD_E_HIP, "pair count failed");
  return MBD_OK;
}

mbd_status mbd_set_positions(mbd_plan plan, int32_t sys, const double* pos) {
  using namespace mbd;
  if (!plan || !pos) return fail(MBD_E_ARG, "NULL argument");
  Plan& P = plan->plan;
  if (sys < 0 || sys >= (int)P.sys.size()) return fail(MBD_E_ARG, "system index out of range");
  try {
    if (P.prec == MBD_PREC_FP64) run_setup<double>(P, P.sys[sys], pos);
    else run_setup<float>(P, P.sys[sys], pos);
    check(hipGetLastError(), "setup launch");
  } catch (const HipError& e) {
    return fail(MBD_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  return MBD_OK;
}

mbd_status mbd_set_timing(mbd_plan plan, int32_t enable) {
  if (!plan) return fail(MBD_E_ARG, "NULL plan");
  plan->plan.timer.on = enable != 0;
  return MBD_OK;
}

mbd_status mbd_get_stage_times(mbd_plan plan, double* ms, int64_t* launches) {
  if (!plan || !ms || !launches) return fail(MBD_E_ARG, "NULL argument");
  mbd::Plan& P = plan->plan;
  if (hipStreamSynchronize(P.stream) != hipSuccess) return fail(MBD_E_HIP, "synchronize failed");
  for (int i = 0; i < MBD_N_STAGES; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (const auto& r : P.timer.recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(MBD_E_HIP, "event time");
    ms[r.stage] += t;
    launches[r.stage] += 1;
  }
  P.timer.recs.clear();
  P.timer.used = 0;
  return MBD_OK;
}

namespace mbd {
namespace {

// Enqueue the whole evaluation of system s on P.stream: its energy (and sd) into
// energy[s] (sd[s]) and its forces, if requested, into forces at its atom offset.
void enqueue_system(Plan& P, int s, double* energy, double* sd, double* forces) {
  System& S = P.sys[s];
  size_t off = 0;
  for (int k = 0; k < s; ++k) off += (size_t)P.sys[k].geo.n;
  if (forces) fill_double(S.buf.fsum, 0.0, 6 * (size_t)S.geo.n, P.stream);
  double* sds = sd ? sd + s : nullptr;
  if (P.prec == MBD_PREC_FP64) run_energy<double>(P, S, s, energy + s, sds, forces != nullptr);
  else run_energy<float>(P, S, s, energy + s, sds, forces != nullptr);
  if (forces)
    staged(P, MBD_STAGE_ADJOINT, [&] {
      launch_forces_finish(S.geo, S.buf, P.prm.n_probes, forces + 3 * off, P.stream);
    });
}

// Enqueue, on P.stream, every system assigned to per-system stream j (all when j < 0).
void enqueue_systems(Plan& P, int j, double* energy, double* sd, double* forces) {
  for (int s = 0; s < (int)P.sys.size(); ++s)
    if (j < 0 || P.sys_stream[s] == j) enqueue_system(P, s, energy, sd, forces);
}

// Enqueue one full evaluation (all systems) on plan.stream: clear the status word,
// fork to the per-system streams, run every system, join back.
void enqueue_execute(Plan& P, double* energy, double* sd, double* forces) {
  const hipStream_t caller = P.stream;
  fill_int(reinterpret_cast<int*>(P.status), 0, 1, caller);
  if (P.pool.empty()) {
    enqueue_systems(P, -1, energy, sd, forces);
    return;
  }
  check(hipEventRecord(P.fork, caller), "fork");
  for (hipStream_t q : P.pool) check(hipStreamWaitEvent(q, P.fork, 0), "fork");
  try {
    for (size_t j = 0; j < P.pool.size(); ++j) {
      P.stream = P.pool[j];  // this stream's systems, one after another
      enqueue_systems(P, (int)j, energy, sd, forces);
    }
  } catch (...) {
    P.stream = caller;
    throw;
  }
  P.stream = caller;
  for (size_t i = 0; i < P.pool.size(); ++i) {
    check(hipEventRecord(P.pool_done[i], P.pool[i]), "join");
    check(hipStreamWaitEvent(caller, P.pool_done[i], 0), "join");
  }
}

// Record the work of one stream into a graph: the whole evaluation on the capture stream
// (single-system plans, with the side stream as a parallel branch), or the systems of
// per-system stream j on that stream (batch plans).
hipGraphExec_t record_graph(Plan& P, hipStream_t on, int j, double* forces) {
  const hipStream_t caller = P.stream;
  hipGraph_t g = nullptr;
  P.stream = on;
  check(hipStreamBeginCapture(on, hipStreamCaptureModeRelaxed), "begin capture");
  try {
    if (j < 0) enqueue_execute(P, P.e_out, P.sd_out, forces);
    else enqueue_systems(P, j, P.e_out, P.sd_out, forces);
  } catch (...) {
    P.stream = caller;
    hipStreamEndCapture(on, &g);
    if (g) hipGraphDestroy(g);
    throw;
  }
  P.stream = caller;
  check(hipStreamEndCapture(on, &g), "end capture");
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  check(e, "graph instantiate");
  return ex;
}

}  // namespace
}  // namespace mbd

mbd_status mbd_execute(mbd_plan plan, double* energy, double* forces, double* energy_sd) {
  using namespace mbd;
  if (!plan || !energy) return fail(MBD_E_ARG, "NULL argument");
  Plan& P = plan->plan;
  if (forces && !P.forces)
    return fail(MBD_E_STATE, "forces requested from a plan created with want_forces = 0");
  try {
    if (!P.use_graph || P.timer.on) {
      enqueue_execute(P, energy, energy_sd, forces);
    } else {
      const int gi = forces ? 1 : 0;
      const hipStream_t caller = P.stream;
      double* fo = forces ? P.f_out : nullptr;
      if (P.pool.empty()) {
        // single system: one graph recorded from the plan's own stream (the caller's
        // may be the null stream, which cannot be captured)
        if (!P.gexec[gi]) P.gexec[gi] = record_graph(P, P.gstream, -1, fo);
        // replay after the caller's earlier work; the caller's later work waits for it
        check(hipEventRecord(P.g_in, caller), "graph fork");
        check(hipStreamWaitEvent(P.gstream, P.g_in, 0), "graph fork");
        check(hipGraphLaunch(P.gexec[gi], P.gstream), "graph launch");
        check(hipEventRecord(P.g_out, P.gstream), "graph join");
        check(hipStreamWaitEvent(caller, P.g_out, 0), "graph join");
      } else {
        // batch: one graph per per-system stream, replayed on that stream, so that the
        // streams still run side by side
        if (P.gpool[gi].empty())
          for (size_t j = 0; j < P.pool.size(); ++j)
            P.gpool[gi].push_back(record_graph(P, P.pool[j], (int)j, fo));
        fill_int(reinterpret_cast<int*>(P.status), 0, 1, caller);
        check(hipEventRecord(P.fork, caller), "graph fork");
        for (size_t j = 0; j < P.pool.size(); ++j) {
          check(hipStreamWaitEvent(P.pool[j], P.fork, 0), "graph fork");
          check(hipGraphLaunch(P.gpool[gi][j], P.pool[j]), "graph launch");
          check(hipEventRecord(P.pool_done[j], P.pool[j]), "graph join");
          check(hipStreamWaitEvent(caller, P.pool_done[j], 0), "graph join");
        }
      }
      size_t nat = 0;
      for (const auto& S : P.sys) nat += (size_t)S.geo.n;
      check(hipMemcpyAsync(energy, P.e_out, sizeof(double) * P.sys.size(),
                           hipMemcpyDeviceToDevice, P.stream), "copy energy");
      if (energy_sd)
        check(hipMemcpyAsync(energy_sd, P.sd_out, sizeof(double) * P.sys.size(),
                             hipMemcpyDeviceToDevice, P.stream), "copy energy s.d.");
      if (forces)
        check(hipMemcpyAsync(forces, P.f_out, sizeof(double) * 3 * nat, hipMemcpyDeviceToDevice,
                             P.stream), "copy forces");
    }
    check(hipGetLastError(), "execute launch");
  } catch (const HipError& e) {
    return fail(MBD_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  P.executed = true;
  return MBD_OK;
}

mbd_status mbd_check(mbd_plan plan) {
  if (!plan) return fail(MBD_E_ARG, "NULL plan");
  mbd::Plan& P = plan->plan;
  uint32_t st = 0;
  if (hipStreamSynchronize(P.stream) != hipSuccess)
    return fail(MBD_E_HIP, "stream synchronize failed");
  if (hipMemcpy(&st, P.status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MBD_E_HIP, "status read failed");
  for (const auto& S : P.sys) {
    if (!S.buf.pg_max) continue;
    int mx = 0;
    if (hipMemcpy(&mx, S.buf.pg_max, sizeof(mx), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(MBD_E_HIP, "status read failed");
    if (mx > S.buf.pg_cap)
      return fail(MBD_E_STATE, "direct-space tensor list overflow: the positions moved too far "
                               "from those the plan was created with; create a new plan");
  }
  if (st & mbd::kErrNotPosdef) return fail(MBD_E_NOT_POSDEF, "a Ritz value is <= 0");
  if (st & (mbd::kErrNonfinite | mbd::kErrNoConverge))
    return fail(MBD_E_NONFINITE, "non-finite value or non-converged tridiagonal");
  return MBD_OK;
}

mbd_status mbd_matvec(mbd_plan plan, int32_t sys, const double* v, double* out, int32_t nrhs,
                      uint32_t components) {
  using namespace mbd;
  if (!plan || !v || !out) return fail(MBD_E_ARG, "NULL argument");
  Plan& P = plan->plan;
  if (sys < 0 || sys >= (int)P.sys.size()) return fail(MBD_E_ARG, "system index out of range");
  if (nrhs < 1 || nrhs > P.B) return fail(MBD_E_ARG, "nrhs must be in [1, block]");
  if (components == 0 || components > MBD_C_ALL) return fail(MBD_E_ARG, "bad component mask");
  System& S = P.sys[sys];
  const bool fl = P.prec == MBD_PREC_MIXED;
  launch_pack(S.geo, S.buf, v, nrhs, P.B, fl, P.stream);
  if (fl) matvec_block<float>(P, S, S.buf.W, components);
  else matvec_block<double>(P, S, S.buf.W, components);
  launch_unpack(S.geo, S.buf, out, nrhs, P.B, P.stream);
  if (hipGetLastError() != hipSuccess) return fail(MBD_E_HIP, "matvec launch failed");
  return MBD_OK;
}

mbd_status mbd_get_tridiagonal(mbd_plan plan, int32_t sys, double* a, double* b,
                               int32_t* m_eff) {
  if (!plan || !a || !b || !m_eff) return fail(MBD_E_ARG, "NULL argument");
  mbd::Plan& P = plan->plan;
  if (sys < 0 || sys >= (int)P.sys.size()) return fail(MBD_E_ARG, "system index out of range");
  if (!P.executed) return fail(MBD_E_STATE, "no execute has run");
  if (P.prm.krylov_block > 1)
    return fail(MBD_E_STATE, "a block Lanczos plan has a block tridiagonal");
  const int R = P.prm.n_probes, m = P.prm.n_steps;
  const mbd::SysBuffers& B = P.sys[sys].buf;
  std::vector<double> nrm((size_t)R * m);
  if (hipStreamSynchronize(P.stream) != hipSuccess ||
      hipMemcpy(a, B.a, sizeof(double) * R * m, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(nrm.data(), B.b, sizeof(double) * R * m, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(m_eff, B.meff, sizeof(int32_t) * R, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MBD_E_HIP, "copy failed");
  for (int l = 0; l < R; ++l)
    for (int k = 0; k < m; ++k) b[(size_t)l * m + k] = (k + 1 < m) ? nrm[(size_t)l * m + k + 1] : 0.0;
  return MBD_OK;
}

mbd_status mbd_get_quadrature(mbd_plan plan, int32_t sys, double* q) {
  if (!plan || !q) return fail(MBD_E_ARG, "NULL argument");
  mbd::Plan& P = plan->plan;
  if (sys < 0 || sys >= (int)P.sys.size()) return fail(MBD_E_ARG, "system index out of range");
  if (!P.executed) return fail(MBD_E_STATE, "no execute has run");
  if (hipStreamSynchronize(P.stream) != hipSuccess ||
      hipMemcpy(q, P.sys[sys].buf.q, sizeof(double) * P.prm.n_probes, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return fail(MBD_E_HIP, "copy failed");
  return MBD_OK;
}

}  // extern "C"

namespace mbd {
namespace {

// Doubles of one screening workspace (n atoms, nq frequencies, nblk row blocks), every
// piece starting on a 256-byte boundary; carve_scs lays it out in this order.
constexpr size_t kScsAlign = 32;
size_t scs_piece(size_t count) { return (count + kScsAlign - 1) / kScsAlign * kScsAlign; }

size_t scs_doubles(int n, int nq, int nblk) {
  const size_t ncol = 3 * (size_t)nq, vec = (size_t)n * 3 * ncol;
  return scs_piece(4 * (size_t)n) + 2 * scs_piece((size_t)n * nq) + 5 * scs_piece(vec) +
         scs_piece((size_t)nblk * 2 * ncol) + scs_piece(2 * ncol) + scs_piece(8 * ncol) +
         scs_piece(1) + 2 * scs_piece((size_t)nq);
}

void carve_scs(double* base, ScsWork& w, double*& u_d, double*& w_d) {
  const size_t ncol = (size_t)w.ncol, vec = (size_t)w.n * 3 * ncol;
  double* p = base;
  auto take = [&](size_t count) {
    double* q = p;
    p += scs_piece(count);
    return q;
  };
  w.locd = take(4 * (size_t)w.n);
  w.ainv = take((size_t)w.n * w.nq);
  w.sig2 = take((size_t)w.n * w.nq);
  w.x = take(vec);
  w.r = take(vec);
  w.z = take(vec);
  w.p = take(vec);
  w.q = take(vec);
  w.part = take((size_t)w.nblk * 2 * ncol);
  w.sums = take(2 * ncol);
  w.sc = take(8 * ncol);
  w.nact = reinterpret_cast<int*>(take(1));
  u_d = take((size_t)w.nq);
  w_d = take((size_t)w.nq);
}

// Validated screening parameters and the workspace shape of one system.
mbd_status scs_prepare(Plan& P, int32_t sys, const mbd_scs_params* prm_in, mbd_scs_params& prm,
                       ScsWork& w) {
  if (sys < 0 || sys >= (int)P.sys.size()) return fail(MBD_E_ARG, "system index out of range");
  prm = *prm_in;
  if (prm.n_freq == 0) prm.n_freq = 15;
  if (prm.n_freq < 1 || prm.n_freq > 31) return fail(MBD_E_ARG, "n_freq must be in [1, 31]");
  if (!std::isfinite(prm.freq_scale) || !std::isfinite(prm.tol))
    return fail(MBD_E_ARG, "freq_scale and tol must be finite");
  if (prm.freq_scale <= 0.0) prm.freq_scale = 0.6;
  if (prm.tol <= 0.0) prm.tol = 1e-10;
  if (prm.max_iter <= 0) prm.max_iter = 1000;
  w.n = P.sys[sys].geo.n;
  w.nq = prm.n_freq + 1;  // the static point u = 0, then the quadrature nodes
  w.ncol = 3 * w.nq;
  w.nblk = std::max(1, std::min(512, (3 * w.n + 127) / 128));
  return MBD_OK;
}

// The screening solve of one system with its workspace at `ws` (device, scs_doubles
// long). Host arrays are fixed-size (n_freq <= 31): nothing is allocated here.
mbd_status scs_run(Plan& P, int32_t sys, const mbd_scs_params& prm, ScsWork& w, double* ws,
                   double* alpha_scs, double* omega_scs, double* rvdw_scs, double* alpha_freq,
                   mbd_scs_info* info) {
  System& S = P.sys[sys];
  const hipStream_t st = P.stream;
  // node 0: u = 0 (no weight); nodes 1..n: u = L (1 + x) / (1 - x), w = 2 L w_x / (1 - x)^2
  double x[32], wx[32], u[32] = {0.0}, wq[32] = {0.0}, sc[8 * 96];
  gauss_legendre(prm.n_freq, x, wx);
  for (int q = 0; q < prm.n_freq; ++q) {
    u[q + 1] = prm.freq_scale * (1.0 + x[q]) / (1.0 - x[q]);
    wq[q + 1] = wx[q] * 2.0 * prm.freq_scale / ((1.0 - x[q]) * (1.0 - x[q]));
  }
  double *u_d = nullptr, *w_d = nullptr;
  carve_scs(ws, w, u_d, w_d);
  int iters = 0, nact = 0;
  uint32_t stat = 0;
  try {
    check(hipStreamSynchronize(st), "scs");
    check(hipMemcpy(u_d, u, sizeof(double) * w.nq, hipMemcpyHostToDevice), "scs nodes");
    check(hipMemcpy(w_d, wq, sizeof(double) * w.nq, hipMemcpyHostToDevice), "scs nodes");
    fill_int(reinterpret_cast<int*>(P.status), 0, 1, st);
    launch_scs_prepare(S.geo, S.buf, S.src.alpha, S.src.omega, S.src.r_vdw, u_d, w, st);
    launch_scs_init(w, st);
    nact = w.ncol;
    while (nact > 0 && iters < prm.max_iter) {
      launch_scs_iteration(S.geo, S.buf, w, prm.tol, P.status, st);
      ++iters;
      check(hipGetLastError(), "scs iteration");
      check(hipMemcpyAsync(&nact, w.nact, sizeof(int), hipMemcpyDeviceToHost, st), "scs");
      check(hipStreamSynchronize(st), "scs");
    }
    launch_scs_output(S.buf, w, w_d, S.src.alpha, S.src.r_vdw, alpha_scs, omega_scs, rvdw_scs,
                      alpha_freq, st);
    check(hipGetLastError(), "scs output");
    check(hipMemcpyAsync(sc, w.sc, sizeof(double) * 8 * w.ncol, hipMemcpyDeviceToHost, st),
          "scs");
    check(hipMemcpyAsync(&stat, P.status, sizeof(stat), hipMemcpyDeviceToHost, st), "scs");
    check(hipStreamSynchronize(st), "scs");
  } catch (const HipError& e) {
    hipStreamSynchronize(st);
    return fail(MBD_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  if (info) {
    // sc rows 4 (||r||^2) and 6 (||E_k||^2)
    double worst = 0.0;
    for (int c = 0; c < w.ncol; ++c)
      worst = std::max(worst, std::sqrt(sc[4 * w.ncol + c] / sc[6 * w.ncol + c]));
    info->iterations = iters;
    info->max_rel_residual = worst;
  }
  if (stat & kErrNotPosdef)
    return fail(MBD_E_NOT_POSDEF, "screening matrix not positive definite (p^T M p <= 0)");
  if (nact > 0)
    return fail(MBD_E_NOCONV, "screening solve reached max_iter = " +
                                  std::to_string(prm.max_iter));
  return MBD_OK;
}


}  // namespace
}  // namespace mbd

extern "C" {

mbd_status mbd_scs(mbd_plan plan, int32_t sys, const mbd_scs_params* prm_in, double* alpha_scs,
                   double* omega_scs, double* rvdw_scs, double* alpha_freq, mbd_scs_info* info) {
  using namespace mbd;
  if (!plan || !prm_in || !alpha_scs || !omega_scs || !rvdw_scs)
    return fail(MBD_E_ARG, "NULL argument");
  Plan& P = plan->plan;
  mbd_scs_params prm;
  ScsWork w;
  const mbd_status v = scs_prepare(P, sys, prm_in, prm, w);
  if (v != MBD_OK) return v;
  void* ws = nullptr;
  if (hipStreamSynchronize(P.stream) != hipSuccess)
    return fail(MBD_E_HIP, "stream synchronize failed");
  if (hipMalloc(&ws, sizeof(double) * scs_doubles(w.n, w.nq, w.nblk)) != hipSuccess)
    return fail(MBD_E_OOM, "device allocation failed (scs workspace)");
  const mbd_status r = scs_run(P, sys, prm, w, static_cast<double*>(ws), alpha_scs, omega_scs,
                               rvdw_scs, alpha_freq, info);
  hipStreamSynchronize(P.stream);
  hipFree(ws);
  return r;
}

mbd_status mbd_scs_noalloc(mbd_plan plan, int32_t sys, const mbd_scs_params* prm_in,
                           double* alpha_scs, double* omega_scs, double* rvdw_scs,
                           double* alpha_freq, mbd_scs_info* info) {
  using namespace mbd;
  if (!plan || !prm_in || !alpha_scs || !omega_scs || !rvdw_scs)
    return fail(MBD_E_ARG, "NULL argument");
  Plan& P = plan->plan;
  mbd_scs_params prm;
  ScsWork w;
  const mbd_status v = scs_prepare(P, sys, prm_in, prm, w);
  if (v != MBD_OK) return v;
  const size_t need = scs_doubles(w.n, w.nq, w.nblk);
  if (need > kScsScratchDoubles)
    return fail(MBD_E_ARG, "screening workspace of " + std::to_string(need * sizeof(double)) +
                               " bytes exceeds the fixed " +
                               std::to_string(kScsScratchDoubles * sizeof(double)) +
                               "-byte scratch of mbd_scs_noalloc (fewer atoms or frequencies, "
                               "or mbd_scs)");
  double* ws = scratch_of(P.device);
  if (!ws) return fail(MBD_E_STATE, "no scratch address for the plan's device");
  return scs_run(P, sys, prm, w, ws, alpha_scs, omega_scs, rvdw_scs, alpha_freq, info);
}

mbd_status mbd_plan_destroy(mbd_plan plan) {
  if (!plan) return MBD_OK;
  hipStreamSynchronize(plan->plan.stream);
  for (hipStream_t q : plan->plan.pool)
    if (q) hipStreamSynchronize(q);
  if (plan->plan.gstream) hipStreamSynchronize(plan->plan.gstream);
  for (const mbd::SideStream& s : plan->plan.sides) {
    if (s.side) {
      hipStreamSynchronize(s.side);
      hipStreamDestroy(s.side);
    }
    for (hipEvent_t e : {s.fork, s.pair_done, s.force_done})
      if (e) hipEventDestroy(e);
  }
  for (hipGraphExec_t g : plan->plan.gexec)
    if (g) hipGraphExecDestroy(g);
  for (const auto& v : plan->plan.gpool)
    for (hipGraphExec_t g : v)
      if (g) hipGraphExecDestroy(g);
  if (plan->plan.g_in) hipEventDestroy(plan->plan.g_in);
  if (plan->plan.g_out) hipEventDestroy(plan->plan.g_out);
  if (plan->plan.gstream) hipStreamDestroy(plan->plan.gstream);
  for (hipEvent_t e : plan->plan.timer.pool) hipEventDestroy(e);
  for (hipEvent_t e : plan->plan.pool_done)
    if (e) hipEventDestroy(e);
  if (plan->plan.fork) hipEventDestroy(plan->plan.fork);
  for (hipStream_t q : plan->plan.pool)
    if (q) hipStreamDestroy(q);
  for (void* p : plan->plan.allocations) hipFree(p);
  delete plan;
  return MBD_OK;
}

}  // extern "C"
