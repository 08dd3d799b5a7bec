/*
 * mbd.h - C ABI of the MI355X SPME stochastic-Lanczos many-body dispersion library.
 *
 * What it computes (arXiv 2307.02278):
 *   E_MBD = 1/2 Tr sqrt(C) - 3/2 sum_i omega_i                     (eq. plasmonic2)
 * with the periodic MBD coupling matrix (eq. ham, eqs. vmbd/ccd/gvec)
 *   C = Omega + Diag(g) T^pbc Diag(g),  Omega = diag(omega_i^2 I_3),  g_i = omega_i sqrt(alpha_i),
 * estimated by stochastic Lanczos quadrature: Hutchinson trace over R normalized
 * Rademacher probes (eqs. hutch, dds) and an m-point Gauss quadrature from the
 * Lanczos tridiagonal of each probe (eqs. sl3, sl4, tridiag1, tridiag2; Algorithm 1).
 * Every Lanczos step applies C through generalized dipoles d = g * y and their
 * Ewald field E* = E_dir + E_rec + E_self (eqs. ewalddip, lk3, recurs2; Algorithm 2):
 *   - E_dir: erfc-screened dipole field plus the damping correction -(1 - f) T,
 *            summed over all periodic images within a cutoff (eq. fld_ewald);
 *   - E_rec: smooth particle-mesh Ewald: B-spline spreading of the dipoles,
 *            3D FFT, influence-function convolution, inverse FFT, derivative
 *            gather (eqs. scaledfractional, spme, dipolarr);
 *   - E_self = -(4 tau^3 / (3 sqrt(pi))) d  (eq. fld_ewald1, field coefficient).
 * The damping f is the Fermi function 1 / (1 + exp(-d (r / S_ij - 1))),
 * S_ij = beta (R_vdW,i + R_vdW,j) (the paper defers its explicit form to its
 * stochastic-MBD reference; this is the rsSCS form with range beta).
 *
 * Units: atomic units everywhere (bohr, bohr^3, Hartree, Hartree/bohr).
 * Field sign: "energy convention", E = T d with dipole-dipole energy d_i^T T_ij d_j.
 *
 * Conventions for every entry point:
 *   - Array arguments marked "device" are device pointers on the plan's GPU and
 *     are owned by the caller. The plan owns its workspace (allocated in
 *     mbd_plan_create); mbd_execute and mbd_matvec allocate nothing.
 *   - All work is enqueued on the stream given at plan creation (a hipStream_t,
 *     passed as void*; NULL = the default stream). Calls return once the work is
 *     enqueued unless stated otherwise. A plan is bound to one stream and one
 *     device and is not thread-safe.
 *   - Every call returns an mbd_status; no exception crosses the ABI. Argument
 *     checks happen on the host before any device work and leave the plan
 *     unchanged. mbd_last_error() gives a thread-local message for the last
 *     failure.
 *   - Vectors at the boundary use the caller's atom order, layout [nrhs][n][3],
 *     float64. Internal layouts (atoms sorted by cell, RHS innermost) never leak.
 */
#ifndef MBD_H
#define MBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbd_plan_s* mbd_plan;
typedef int32_t mbd_status;

enum {
  MBD_OK = 0,
  MBD_E_ARG = -1,         /* invalid argument (sizes, parameters, NULL pointers)          */
  MBD_E_CELL = -2,        /* cell vectors not right-handed, or degenerate (zero volume)     */
  MBD_E_GRID = -3,        /* grid size unsupported (see mbd_grid_supported) or < 2p        */
  MBD_E_NOT_POSDEF = -4,  /* a Ritz value theta_k <= 0: C is not positive definite         */
  MBD_E_NONFINITE = -5,   /* NaN/Inf met in a field, a Lanczos scalar or the energy        */
  MBD_E_NODEVICE = -6,    /* no usable GPU                                                 */
  MBD_E_HIP = -7,         /* a HIP runtime call failed                                     */
  MBD_E_OOM = -8,         /* device allocation failed                                      */
  MBD_E_STATE = -9,       /* call out of order (e.g. tridiagonal requested before execute) */
  MBD_E_NOCONV = -10      /* an iterative solve stopped at its iteration limit             */
};

enum { MBD_PREC_FP64 = 0, MBD_PREC_MIXED = 1 /* FP32 SPME + pair kernel, FP64 Lanczos */ };
enum { MBD_REORTH_NONE = 0, MBD_REORTH_LOCAL = 1, MBD_REORTH_FULL = 2 };
enum { MBD_C_DIAG = 1, MBD_C_DIR = 2, MBD_C_REC = 4, MBD_C_SELF = 8, MBD_C_ALL = 15 };

/* One periodic system. Positions may lie in any periodic image. */
typedef struct {
  int32_t n_atoms;      /* N >= 1                                                      */
  const double* pos;    /* device [N][3], bohr                                          */
  double cell[9];       /* host copy, rows a1, a2, a3 in bohr (any right-handed cell)   */
  const double* alpha;  /* device [N], static polarizability alpha_i(0) > 0, bohr^3     */
  const double* omega;  /* device [N], characteristic frequency omega_i > 0, Hartree    */
  const double* r_vdw;  /* device [N], van der Waals radius > 0, bohr                   */
} mbd_system;

/* Launch shape of one system's matvec. It changes how the work is laid out on the GPU:
 * pair_wg_per_cu, pair_subsets (vector pair kernel) and overlap leave every result bit
 * unchanged; grid_chunk changes the summation order inside the spread and the gather,
 * gather_waves the grouping of the partial sums of a_k, and pair_mode (with pair_subsets
 * under it) the order of the direct-space sums, so results agree to rounding across
 * those. A plan is bitwise reproducible for its shape. */
typedef struct {
  int32_t pair_wg_per_cu; /* work-groups per compute unit of the direct-space list kernel;
                             0 => one work-group per 16-atom target group (all resident)  */
  int32_t pair_subsets;   /* vector list kernel: target subsets per wavefront, 1, 2 or 4
                             (at least 64 / block); 0 => the size rule (4096 wavefronts
                             or more). Matrix-core kernel: wavefronts that share one
                             group's candidates, 1, 2 or 4 (at most 4 wavefronts per
                             work-group with block / 64 column wavefronts); 0 => 1      */
  int32_t grid_chunk;     /* right-hand sides per SPME grid chunk: a power of two <= 64
                             that divides block; 0 => 64 (mixed) or 16 (float64)         */
  int32_t overlap;        /* pair kernel on a side stream, concurrent with the grid stages
                             (single-system plans): 1 => forked before the spreads, 2 =>
                             forked after them (beside the transforms only); 0 => one
                             stream                                                       */
  int32_t gather_waves;   /* wavefronts per work-group of the gather and the reciprocal
                             force kernel: 4 or 8; 0 => 4                                 */
  int32_t spread_mode;    /* 0 => spread over 4x4x4 grid tiles, then the forward x
                             transform as its own pass; 1 => spread along whole x-lines
                             fused with the forward x transform (mixed precision, p = 6,
                             64-wide chunks; otherwise 0 is used). Both give the same
                             real grid; the fused form never writes it                  */
  int32_t pair_mode;      /* direct-space list kernel: 0 => vector FMA lanes, one lane per
                             right-hand side, skipping out-of-range pairs; 1 => matrix
                             cores (v_mfma_f32_16x16x4_f32) over the dense per-group
                             product (mixed precision, block a multiple of 64 up to 256;
                             otherwise 0 is used), a wavefront holding 128 right-hand
                             sides where block is a multiple of 128, else 64; 2 => the
                             same with 64 right-hand sides per wavefront (half the
                             accumulator registers). With forces, 1 and 2 also compute
                             the direct force term on the matrix cores when
                             block <= 128                                                 */
} mbd_shape;

enum {
  MBD_TUNE_OFF = 0,       /* built-in shape: pair_wg_per_cu 0, size rule, default chunk,
                             overlap 1                                                    */
  MBD_TUNE_MEASURE = 1,   /* time candidate shapes on each system at plan creation and
                             keep the fastest (reused from tune_cache when it holds one)  */
  MBD_TUNE_GIVEN = 2      /* use params.shape as given, for every system                 */
};
enum { MBD_SHAPE_BUILTIN = 0, MBD_SHAPE_MEASURED = 1, MBD_SHAPE_CACHED = 2, MBD_SHAPE_GIVEN = 3 };

typedef struct {
  double damp_beta;     /* range parameter beta of the Fermi damping (> 0), e.g. 0.83   */
  double damp_d;        /* steepness d of the Fermi damping (> 0), e.g. 6               */
  double ewald_tau;     /* Ewald splitting tau in 1/bohr; <= 0: derived from real_cutoff
                           by erfc(tau r_c) / r_c = 1e-8 with r_c in Angstrom           */
  double real_cutoff;   /* erfc cutoff r_c in bohr (> 0)                               */
  double damp_tol;      /* pair kernel also runs to where 1 - f = damp_tol; 0 => 1e-4;
                           < 0 => only real_cutoff is used                              */
  int32_t grid[3];      /* SPME grid K1..K3; 0 => smallest even 2^a 3^b >= 1.4 / A     */
  int32_t spline_order; /* B-spline order p (support of p points): even, 4..8; 0 => 6   */
  int32_t n_probes;     /* R >= 1 Rademacher probes per system                          */
  int32_t n_steps;      /* m >= 1 Lanczos steps (matvecs, size of the tridiagonal)      */
  int32_t block;        /* probes in flight as one block of right-hand sides; 0 => R   */
  uint64_t seed;        /* probe seed (SplitMix64 counter generator, see below)        */
  int32_t precision;    /* MBD_PREC_FP64 or MBD_PREC_MIXED                              */
  int32_t reorth;       /* MBD_REORTH_NONE / LOCAL / FULL                               */
  int32_t want_forces;  /* 1 => allocate the reverse-sweep workspace so that mbd_execute
                           can return forces (needs block >= 4); 0 => energy only      */
  int32_t deterministic;/* reserved: every reduction already runs in a fixed order, so
                           results are bit-reproducible run to run on one device        */
  double replica_cutoff;/* > 0 => replica method instead of Ewald/SPME (float64 only, no
                           forces): T_ij = sum over images n with |R_j + n - R_i| <
                           replica_cutoff of the damped tensor f T (eq. replica, spherical
                           cutoff centred on atom i; tends to the vacuum boundary
                           condition). 0 => SPME-Ewald                                 */
  int32_t graph;        /* 1 => mbd_execute records its whole launch sequence (all
                           systems, all streams) once into a HIP graph per variant
                           (energy / energy + forces) and replays it afterwards; the
                           positions may change between calls (mbd_set_positions).
                           Stage timing (mbd_set_timing) runs eagerly instead.           */
  int32_t krylov_block; /* 0 or 1 => one Lanczos process per probe. 2, 4 or 8 => block
                           Lanczos on consecutive blocks of that many probes (R and block
                           must be multiples of it; m * krylov_block <= 512; energy only,
                           MBD_REORTH_NONE): per probe block V = Y_0 R_0,
                           A_k = Y_k^T C Y_k, C Y_k - Y_k A_k - Y_{k-1} B_{k-1}^T = Y_{k+1} B_k
                           (Cholesky QR, twice), and
                           Q_l = [R_0^T E_1^T sqrt(T) E_1 R_0]_ll with T the block
                           tridiagonal of the A_k and B_k; the same m matvecs per probe span
                           a Krylov space krylov_block times wider per block.             */
  int32_t tune;         /* MBD_TUNE_OFF / MBD_TUNE_MEASURE / MBD_TUNE_GIVEN               */
  mbd_shape shape;      /* the shape for MBD_TUNE_GIVEN (ignored otherwise)               */
  const char* tune_cache;/* MBD_TUNE_MEASURE: path of a JSON-lines file of measured shapes,
                           one object per line keyed by device architecture, N, grid,
                           block, precision and forces; read at plan creation and
                           appended with each new measurement. NULL => no file.         */
  int32_t store_grids;  /* with want_forces: 1 => keep the real potential grids of every
                           forward Lanczos step of a probe block (n_steps x the grid
                           bytes, e.g. 22.7 GB at N = 24k, K = 96, block 128), so that the
                           reverse force terms read phi of y_k instead of running one
                           more spread and transform per step; 0 => recompute them      */
} mbd_params;

/* Values derived on the host for one system of a plan. */
typedef struct {
  double tau;           /* 1/bohr                                                      */
  double r_pair;        /* direct-space cutoff actually used, bohr                      */
  int32_t grid[3];
  int32_t spline_order;
  int32_t cells[3];     /* cell-list cells per axis                                    */
  int32_t block;        /* right-hand sides per block                                  */
  size_t workspace_bytes;
  int64_t n_pairs;      /* directed (i, j, image) pairs within r_pair at the current positions */
  mbd_shape shape;      /* launch shape in use for this system                         */
  int32_t shape_source; /* MBD_SHAPE_BUILTIN / MEASURED / CACHED / GIVEN                */
  double tune_ms;       /* time of one measured matvec with that shape (0 if not measured) */
} mbd_info;

/* Probe definition (eq. dds): entry (l, i, a) of system s is +-1/sqrt(3N), the sign
 * taken from bit 63 of SplitMix64 output number (l*3N + 3i + a) of the stream seeded
 * with z_s, where z_s is output number s of the stream seeded with `seed`. Output n of
 * a stream seeded with x is mix(x + (n+1) * 0x9E3779B97F4A7C15) (Steele, Lea, Flood 2014).
 * i is the atom's index in the caller's order. */

/* Create a plan for n_sys systems with shared parameters. Validates every argument,
 * derives tau / cutoffs / grids, allocates the whole workspace, sorts atoms into cells
 * and builds B-spline tables and the influence function (device setup, Algorithm 1
 * lines on grid allocation and neighbour lists). `stream` is a hipStream_t or NULL.
 * Returns MBD_E_ARG / MBD_E_CELL / MBD_E_GRID without touching the device on bad input. */
mbd_status mbd_plan_create(mbd_plan* out, const mbd_system* systems, int32_t n_sys,
                           const mbd_params* prm, void* stream);

/* Derived parameters of one system (synchronizes the plan's stream: n_pairs is counted
 * on the device at the current positions). */
mbd_status mbd_plan_info(mbd_plan plan, int32_t sys, mbd_info* info);

/* Re-run the position-dependent device setup (wrap, cell sort, spline tables, tile
 * lists; Algorithm 1 neighbour-list step) with new positions for one system.
 * pos: device [N][3] bohr, caller-owned; it is read during this call's stream work
 * and not retained. The alpha/omega/r_vdw arrays given at plan creation are read
 * again, so they must still be alive. The cell list keeps the cell counts chosen at
 * creation, which stay valid for any positions in the same cell. */
mbd_status mbd_set_positions(mbd_plan plan, int32_t sys, const double* pos);

/* Run Algorithm 1 for every system: R probes in blocks of `block` RHS, m Lanczos steps
 * each, Gauss quadrature per probe, then E = 1/2 (3N/R) sum_l Q_l - 3/2 sum omega
 * (eqs. hutch, sl4, plasmonic2).
 * energy: device [n_sys] float64.
 * forces: NULL, or device [sum of N][3] float64 (systems concatenated, caller atom order)
 *   receiving F = -dE/dR, the exact derivative of the fixed-probe estimator above with
 *   respect to the positions (forces are future work in the paper's conclusions; this is
 *   reverse mode through the Lanczos recurrence and the quadrature, with one adjoint
 *   matvec and the bilinear pair and reciprocal force terms per step). Re-orthogonalization
 *   corrections are not differentiated (exact for MBD_REORTH_NONE). Requires a plan
 *   created with want_forces = 1, else MBD_E_STATE.
 * energy_sd: NULL, or device [n_sys] float64 receiving the standard deviation of the
 *   energy estimate from the spread of the per-probe quadrature values (the Hutchinson
 *   trace estimator of eq. hutch is an average of R independent samples):
 *   sd(E) = 1/2 (3N) s_Q / sqrt(R),  s_Q^2 = sum_l (Q_l - mean Q)^2 / (R - 1);
 *   NaN when R = 1 (no spread to measure; not flagged as an error).
 * The energy, the forces and energy_sd are reduced on the device in a fixed order. */
mbd_status mbd_execute(mbd_plan plan, double* energy, double* forces, double* energy_sd);

/* Synchronize the plan's stream and return the first device-detected error
 * (MBD_E_NOT_POSDEF, MBD_E_NONFINITE) since the last execute, else MBD_OK. */
mbd_status mbd_check(mbd_plan plan);

/* out = C_sel v for nrhs vectors (test and diagnostic hook). v, out: device
 * [nrhs][N][3] float64 in the caller's atom order; 1 <= nrhs <= block.
 * components selects the parts of C: MBD_C_DIAG (Omega v), MBD_C_DIR
 * (g * E_dir(g v)), MBD_C_REC (g * E_rec(g v)), MBD_C_SELF (g * E_self(g v)). */
mbd_status mbd_matvec(mbd_plan plan, int32_t sys, const double* v, double* out,
                      int32_t nrhs, uint32_t components);

/* Lanczos tridiagonals of the last execute (synchronizes; MBD_E_STATE for a plan with
 * krylov_block > 1, whose projection is block tridiagonal). Host arrays:
 * a [R][m] diagonal, b [R][m] with b[l][k] = b_{k+1} (off-diagonal between k and k+1,
 * b[l][m-1] unused), m_eff [R] steps done before a breakdown. */
mbd_status mbd_get_tridiagonal(mbd_plan plan, int32_t sys, double* a, double* b,
                               int32_t* m_eff);

/* Per-probe quadrature values Q_l = sum_k U_1k^2 sqrt(theta_k) of the last execute
 * (synchronizes). q: host [R]. */
mbd_status mbd_get_quadrature(mbd_plan plan, int32_t sys, double* q);

/* ---- Self-consistent screening (range-separated SCS of MBD@rsSCS) -------------------
 *
 * The Review section names the step upstream of the MBD matrix: the polarizabilities are
 * made frequency dependent and screened by a Dyson-like equation solved at a set of
 * imaginary frequencies; the paper does not write it out. Solved here, for one system of a
 * plan at its current positions, with
 *   alpha_i(iu) = alpha_i / (1 + (u / omega_i)^2)                   (one-oscillator model)
 *   (A(iu)^-1 + T_SR(iu)) X_k = E_k,  E_k = unit vector k on every atom, k = 1..3
 *   alpha^SCS_i(iu) = (1/3) sum_k (X_k)_{i,k}     (= (1/3) tr sum_j [(A^-1 + T_SR)^-1]_ij)
 *   T_SR = (1 - f) T_GG,  T_GG = -grad grad (erf(r / sigma_ij) / r),
 *   sigma_ij^2 = sigma_i^2 + sigma_j^2,  sigma_i = (sqrt(2/pi) alpha_i(iu) / 3)^(1/3),
 * f the Fermi damping of the plan (beta, d, the system's unscreened r_vdw), summed over
 * every periodic image within the plan's pair cutoff (mbd_info.r_pair; 1 - f makes T_SR
 * short-ranged, so no Ewald split is involved). Then, with the Casimir-Polder integral on
 * an n-point Gauss-Legendre grid mapped by u = L (1 + x) / (1 - x),
 *   C6_i = (3/pi) sum_q w_q alpha^SCS_i(iu_q)^2,   omega^SCS_i = 4 C6_i / (3 alpha^SCS_i(0)^2),
 *   r_vdw^SCS_i = r_vdw_i (alpha^SCS_i(0) / alpha_i)^(1/3).
 * The 3 (n + 1) right-hand sides (static point plus n nodes) run together through a
 * Jacobi-preconditioned conjugate gradient in float64 on the device, whatever the plan's
 * precision. */
typedef struct {
  int32_t n_freq;       /* quadrature nodes n, 1..31; 0 => 15                              */
  double freq_scale;    /* L of the frequency map, Hartree; <= 0 => 0.6                    */
  double tol;           /* stop when ||r|| <= tol ||E_k|| for every right-hand side;
                           <= 0 => 1e-10                                                    */
  int32_t max_iter;     /* conjugate-gradient iteration limit; <= 0 => 1000                */
} mbd_scs_params;

typedef struct {
  int32_t iterations;       /* conjugate-gradient iterations run                           */
  double max_rel_residual;  /* max over right-hand sides of ||r|| / ||E_k|| at exit        */
} mbd_scs_info;

/* Screened alpha(0), omega and r_vdw of system `sys`, in the caller's atom order:
 * alpha_scs, omega_scs, rvdw_scs: device [N] float64 (required);
 * alpha_freq: device [n][N] float64 alpha^SCS at the quadrature nodes u_q (ascending), or NULL;
 * info: host, or NULL.
 * Synchronous: runs on the plan's stream, allocates a per-call device workspace of
 * 5 x 3 (n + 1) x 3N doubles plus small tables, and frees it before returning. The
 * outputs feed a new plan (MBD@rsSCS): mbd_plan_create with alpha_scs, omega_scs and
 * rvdw_scs as the system's parameters. Errors: MBD_E_ARG (bad arguments),
 * MBD_E_NOT_POSDEF (p^T M p <= 0: the screening matrix is not positive definite at some
 * frequency), MBD_E_NOCONV (max_iter reached; outputs are written from the last iterate),
 * MBD_E_HIP, MBD_E_OOM. The call resets the plan's device status word, so call mbd_check
 * for an execute before calling mbd_scs. */
mbd_status mbd_scs(mbd_plan plan, int32_t sys, const mbd_scs_params* prm, double* alpha_scs,
                   double* omega_scs, double* rvdw_scs, double* alpha_freq, mbd_scs_info* info);

/* The screening solve of mbd_scs without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that forbid it).
 * Same arguments, results and errors as mbd_scs, bit for bit. The workspace is one fixed
 * 64 MiB device array per GPU instead of a per-call allocation: the library holds it on
 * every GPU it runs on until the process ends, and its address is resolved when a plan is
 * first created on that GPU. A system needs 8 (4N + 2N(n+1) + 45N(n+1) + O(n)) bytes,
 * i.e. up to about 11,000 atoms at the default n = 15 frequencies; larger requests fail
 * with MBD_E_ARG before any device work. Every call on one GPU shares the array and
 * leaves its contents behind (each call initializes what it reads), so calls that
 * overlap in time on one GPU, e.g. from two host threads, race and must not be made.
 * Synchronous, like mbd_scs. */
mbd_status mbd_scs_noalloc(mbd_plan plan, int32_t sys, const mbd_scs_params* prm,
                           double* alpha_scs, double* omega_scs, double* rvdw_scs,
                           double* alpha_freq, mbd_scs_info* info);

mbd_status mbd_plan_destroy(mbd_plan plan);

/* 1 if an FFT of length k is compiled in (even 2^a 3^b 5^c in [8, 128]), else 0. */
int32_t mbd_grid_supported(int32_t k);

/* Stage timing (diagnostic). Stages, in pipeline order: */
enum {
  MBD_STAGE_PAIR = 0,      /* direct-space pair kernel                        */
  MBD_STAGE_SPREAD = 1,    /* B-spline spreading of the dipoles               */
  MBD_STAGE_FFT_X = 2,     /* forward real-to-complex transform along x       */
  MBD_STAGE_FFT_Y = 3,     /* forward transform along y                       */
  MBD_STAGE_FFT_Z = 4,     /* transform along z, convolution, inverse along z */
  MBD_STAGE_IFFT_Y = 5,    /* inverse transform along y                       */
  MBD_STAGE_IFFT_X = 6,    /* inverse complex-to-real transform along x       */
  MBD_STAGE_GATHER = 7,    /* derivative gather + epilogue (l = Omega w + g E*) */
  MBD_STAGE_LANCZOS = 8,   /* recurrence update, reductions, quadrature        */
  MBD_STAGE_SETUP = 9,     /* position-dependent setup                         */
  MBD_STAGE_FORCE = 10,    /* pair and reciprocal bilinear force terms         */
  MBD_STAGE_ADJOINT = 11,  /* tridiagonal adjoint and reverse-sweep vector work */
  MBD_N_STAGES = 12
};
/* enable != 0: from now on every stage launch enqueued by this plan is bracketed by
 * HIP events on the plan's stream (adds a few microseconds per launch). */
mbd_status mbd_set_timing(mbd_plan plan, int32_t enable);
/* Synchronize, then return per-stage total milliseconds ms[MBD_N_STAGES] and launch
 * counts launches[MBD_N_STAGES] recorded since the last call (host arrays), and reset. */
mbd_status mbd_get_stage_times(mbd_plan plan, double* ms, int64_t* launches);

const char* mbd_status_string(mbd_status s);
const char* mbd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MBD_H */
