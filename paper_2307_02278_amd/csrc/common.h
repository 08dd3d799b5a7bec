// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mbd.h"

namespace mbd {

constexpr int kMaxOrder = 8;
constexpr int kRedBlocks = 1024;   // blocks (and partial sums) of the row reductions
constexpr int kSpreadTile = 4;     // grid points per spread-tile edge (one wavefront per tile)
constexpr int kMaxSteps = 512;
constexpr int kPartSlots = 8;      // partial-sum slots per reduction block
// Direct-space tensor list: targets per group, stored components per (source,
// target) pair (xx, yy, zz, xy, xz, yz) and values per listed source.
constexpr int kGroup = 16;
constexpr int kTensorWords = 6;
constexpr int kCandStride = kGroup * kTensorWords;

// Device-side error bits (status word).
enum : uint32_t { kErrNotPosdef = 1u, kErrNonfinite = 2u, kErrNoConverge = 4u };

// Everything one kernel launch needs to know about a system's geometry and grid.
struct Geometry {
  int n;                 // atoms
  double L[3];           // cell vector lengths |a_a| (bohr)
  double A[3][3];        // cell vectors a_a (rows, Cartesian bohr)
  double Ar[3][3];       // reciprocal vectors a*_a (rows), a*_a . a_b = delta_ab
  double Mu[3][3];       // K_a a*_a (rows): d u_a / d R, the B-spline chain-rule matrix
  double hv[3][3];       // cell-list shift vectors a_a / nc_a (rows)
  int K[3];              // SPME grid
  int p;                 // spline order
  double tau;            // 1/bohr
  double r_pair;         // direct-space cutoff (bohr)
  int nc[3];             // cells per axis
  double hc[3];          // cell-list cell width per axis, perpendicular to its faces
  int nr[3];             // neighbour-cell range per axis
  int mbits;             // bits per axis of the Morton cell index
  int tile[3];           // spread tile edge per axis (grid points)
  int tiles[3];          // spread tiles per axis
  double beta, damp_d;
  double replica_cut;    // > 0: replica method (damped tensor over images within this cutoff)
  int n_images;          // replica image vectors
  // launch shape of the direct-space list kernels (set by the plan or its tuner)
  int pair_blocks;       // work-groups of a launch; 0 => one per 16-atom group
  int pair_ns;           // target subsets per wavefront (1, 2, 4); 0 => size rule
  int gather_waves;      // wavefronts per work-group of the gather-type kernels (4 or 8)
  int pair_mode;         // 0 => vector list kernel; 1 => matrix-core list kernel (float);
                         // 2 => the same with 64-column wavefronts
  int line_lists;        // 1 => the setup also builds the x-line atom lists (fused spread)
};

// Cells are numbered along a Morton (Z-order) curve so that consecutive sorted
// atoms stay spatially compact; cell_start has 2^(3 mbits) + 1 entries.
__host__ __device__ inline uint32_t morton_spread(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__host__ __device__ inline uint32_t morton_compact(uint32_t v) {
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030C30C3u;
  v = (v ^ (v >> 4)) & 0x0300F00Fu;
  v = (v ^ (v >> 8)) & 0x030000FFu;
  v = (v ^ (v >> 16)) & 0x000003FFu;
  return v;
}
__host__ __device__ inline int cell_index(int cx, int cy, int cz) {
  return (int)(morton_spread((uint32_t)cx) | (morton_spread((uint32_t)cy) << 1) |
               (morton_spread((uint32_t)cz) << 2));
}
__host__ __device__ inline void cell_coords(int c, int& cx, int& cy, int& cz) {
  cx = (int)morton_compact((uint32_t)c);
  cy = (int)morton_compact((uint32_t)c >> 1);
  cz = (int)morton_compact((uint32_t)c >> 2);
}
inline int cell_slots(const Geometry& g) { return 1 << (3 * g.mbits); }

// block Lanczos quadrature (kb probes per Krylov block)
constexpr int kBlockMaxDim = 512;  // largest m kb (dimension of the block tridiagonal)
struct BlockWork {
  int kb = 1;               // probes per Krylov block (2, 4 or 8)
  int nblk = 0;             // row blocks of the Gram reductions
  double* part = nullptr;   // [nblk][B kb] partial Gram sums
  double* G = nullptr;      // [B / kb][kb][kb] Gram matrices
  double* R1 = nullptr;     // [B / kb][kb][kb] Cholesky factor of the current pass
  double* R0 = nullptr;     // [B / kb][kb][kb] probe block = Y_0 R0
  double* Atmp = nullptr;   // [B / kb][kb][kb] A_k of the current step
  double* Bprev = nullptr;  // [B / kb][kb][kb] B_k of the current step
  double* A = nullptr;      // [B / kb][m][kb][kb]
  double* B = nullptr;      // [B / kb][m][kb][kb]
  double* T = nullptr;      // [B / kb][m kb][m kb] eigen workspace
  double* P = nullptr;      // [B / kb][kb][m kb]
  double* d = nullptr;      // [B / kb][m kb]
  double* e = nullptr;      // [B / kb][m kb]
  int* flag = nullptr;      // [B / kb] block ended (rank-deficient residual)
  int* meff = nullptr;      // [B / kb] block steps kept
};
// Device buffers of one system.
struct SysBuffers {
  // sorted atom data
  int* perm = nullptr;         // [n] sorted -> caller index
  int* cell_of = nullptr;      // [n] cell of each caller atom
  int* cell_start = nullptr;   // [cell_slots + 1], Morton-indexed
  int* cell_cursor = nullptr;  // [cell_slots]
  uint32_t* subkey = nullptr;  // [n] Morton code of the atom's sub-cell (order inside a cell)
  double* wpos = nullptr;      // [n][3] wrapped fractional coordinates in [0, 1), caller order
  void* loc = nullptr;         // Real [n][4] cell-local position + damping radius (sorted)
  double* g = nullptr;         // [n] omega sqrt(alpha) (sorted)
  double* om2 = nullptr;       // [n] omega^2 (sorted)
  int* base = nullptr;         // [n][3] spline base indices (sorted)
  int* scell = nullptr;        // [n] Morton cell index of each sorted atom
  void* th = nullptr;          // Real [n][3][p] M_p(w + t)
  void* dth = nullptr;         // Real [n][3][p] M_p'(w + t) (derivative in u_a)
  void* ddth = nullptr;        // Real [n][3][p] M_p''(w + t) (forces only)
  int* tile_count = nullptr;   // [ntiles + 1]
  int* tile_start = nullptr;   // [ntiles + 1]
  int* tile_atoms = nullptr;   // [n * max tiles per stencil]
  // x-line lists of the fused line spread (float plans): for each line y + K2 z, the atoms
  // whose y-z stencil covers it, in atom order, as (s << 8) | (t_y << 4) | t_z
  int* line_count = nullptr;   // [K2 K3 + 1]
  int* line_start = nullptr;   // [K2 K3 + 1]
  int* line_atoms = nullptr;   // [p^2 n]
  void* G = nullptr;           // Real [K3][K2][K1/2 + 1]
  void* Gt = nullptr;          // Real [K2][K1/2 + 1][K3]: G with kz innermost (register z pass)
  void* tw = nullptr;          // Real [2][K1 + K2 + K3] twiddles exp(-2 pi i j / K_a)
  int* images = nullptr;       // [n_images][3] integer lattice vectors (replica method)
  // direct-space tensor list (B >= 16): groups of kGroup sorted targets
  int pg_cap = 0;              // listed sources per group (capacity)
  int* pg_count = nullptr;     // [ngroups] listed sources (may exceed pg_cap: overflow)
  int* pg_max = nullptr;       // [1] max over groups of pg_count
  int2* pg_hdr = nullptr;      // [ngroups][pg_cap] (source index, 16-bit target mask)
  void* pg_T = nullptr;        // Real [ngroups][pg_cap][kGroup][kTensorWords]
  void* pg_zero = nullptr;     // Real [kTensorWords] zeros (matrix-core rows past a list)
  // Lanczos state for one block of right-hand sides
  double* W = nullptr;         // [m][n][3][B] Krylov vectors, unnormalized
  double* Lt = nullptr;        // [n][3][B] C w_k
  void* dv = nullptr;          // Real [n][3][B] generalized dipoles g * w_k
  void* Ed = nullptr;          // Real [n][3][B] direct-space field
  void* grid = nullptr;        // Real [B / BG][K3][K2][K1 + 2][BG]
  double* part = nullptr;      // [kRedBlocks][kPartSlots][B] partial sums
  double* coef = nullptr;      // [B][kMaxSteps] reorthogonalization coefficients
  double* a = nullptr;         // [R][m] Lanczos diagonal
  double* b = nullptr;         // [R][m] nrm[l][k] = ||w_k|| (nrm[l][0] = 1)
  int* meff = nullptr;         // [R]
  double* q = nullptr;         // [R] per-probe quadrature
  double* sum_omega = nullptr; // [1]
  // forces (reverse sweep through the Lanczos recurrence), allocated when requested
  void* pg_F = nullptr;        // Real [ngroups][pg_cap][kGroup][6] r_x, r_y, r_z, B, A'/r, B'/r
  double* ybar = nullptr;      // [3][n][3][B] adjoints of y_{k+1}, y_k, y_{k-1} (rotating)
  double* lbar = nullptr;      // [n][3][B] adjoint of l_k (input of the adjoint matvec)
  void* dq = nullptr;          // Real [n][3][B] g * y_k
  void* phi = nullptr;         // Real [m][K3][K2][K1 + 2][B]: the forward steps' potential grids
  double* tz = nullptr;        // [B][m][m] tridiagonal eigenvectors
  double* abar = nullptr;      // [B][m] dQ/da_k, then the full adjoint of a_k
  double* bbar = nullptr;      // [B][m] dQ/d nrm_k (k >= 1)
  double* adj = nullptr;       // [B][8] per-step adjoint scalars
  double* fsum = nullptr;      // [2][n][3] sums over probes and steps of l-bar^T dC/dR y
                               // (sorted): [0] reciprocal part, [1] direct (pair) part
  BlockWork blk;               // block Lanczos workspace (krylov_block > 1)
};

struct System {
  Geometry geo;
  SysBuffers buf;
  int BG = 64;                 // right-hand sides per grid chunk (divides the block)
  int overlap = 1;             // pair kernel on the side stream: 0 no, 1 forked before the
                               // spreads, 2 forked after them (beside the transforms)
  mbd_shape shape{};           // launch shape in use (reported by mbd_plan_info)
  int shape_source = 0;        // MBD_SHAPE_* : where the shape came from
  double tune_ms = 0.0;        // measured matvec time of that shape (0 if not measured)
  mbd_system src;              // caller's arrays (alpha, omega, r_vdw stay caller-owned)
  double host_cell[9];
  size_t bytes = 0;
};

// Optional per-stage event timing on the plan's stream.
struct StageTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipEvent_t next();
};

// A side stream forked from one of the plan's streams (the caller's or the capture
// stream): each matvec runs its direct-space pair kernel there,
// concurrently with the grid stages on the origin stream, and joins by events.
struct SideStream {
  hipStream_t origin = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, pair_done = nullptr, force_done = nullptr;
};

struct Plan {
  std::vector<System> sys;
  bool forces = false;         // buffers for the reverse sweep exist
  mbd_params prm;
  int prec;                    // MBD_PREC_*
  int B;                       // RHS per block
  int BG;                      // RHS per grid chunk
  hipStream_t stream = nullptr;
  int device = 0;
  int cus = 256;               // compute units of the device
  std::string arch;            // device architecture name (tuning cache key)
  bool batch = false;          // more than one system (per-system streams, no side stream)
  uint32_t* status = nullptr;  // device status word
  bool executed = false;
  std::vector<void*> allocations;
  StageTimer timer;
  // Batches of several systems run concurrently on internal streams (default
  // priority), forked from and joined back to `stream` with events.
  std::vector<hipStream_t> pool;
  std::vector<hipEvent_t> pool_done;
  hipEvent_t fork = nullptr;
  std::vector<int> sys_stream;   // internal stream of each system
  // Graph replay of mbd_execute: [0] energy only, [1] energy + forces. Outputs of a
  // replay land in plan-owned buffers and are copied to the caller's afterwards.
  bool use_graph = false;
  hipStream_t gstream = nullptr;  // capture and replay stream (the caller's may be the null stream)
  hipEvent_t g_in = nullptr, g_out = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<hipGraphExec_t> gpool[2];  // batch plans: one graph per per-system stream
  double* e_out = nullptr;       // [n_sys]
  double* f_out = nullptr;       // [sum n][3] (forces plans)
  double* sd_out = nullptr;      // [n_sys] standard deviation of the energy estimate
  // Side streams of the caller's stream and of the capture stream, created with the
  // plan. The per-system streams of a batch plan have none.
  std::vector<SideStream> sides;
  SideStream* side_of(hipStream_t origin);  // nullptr if origin has no side stream
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files). All enqueue on `st`.
// ---------------------------------------------------------------------------
void launch_line_lists(const Geometry& g, SysBuffers& b, hipStream_t st);
template <typename R>
void launch_setup(const Geometry& g, SysBuffers& b, const double* pos, const double* alpha,
                  const double* omega, const double* rvdw, hipStream_t st);

template <typename R>
void launch_pair(const Geometry& g, const SysBuffers& b, int B, hipStream_t st);

void launch_replica(const Geometry& g, const SysBuffers& b, int B, hipStream_t st);

template <typename R>
void launch_pair_build(const Geometry& g, const SysBuffers& b, bool count_only, hipStream_t st);

template <typename R>
long long count_pairs(const Geometry& g, const SysBuffers& b, hipStream_t st);

template <typename R>
void launch_spread(const Geometry& g, const SysBuffers& b, int B, int BG, int chunk0, int nchunks,
                   hipStream_t st);

template <typename R>
void launch_fft_pass(const Geometry& g, const SysBuffers& b, int B, int BG, int chunk0,
                     int nchunks, int pass, hipStream_t st);
// Spread fused with the forward x pass (float, 64-wide chunks, p = 6); false when this
// case is not compiled (then k_spread and pass 0 run instead).
bool launch_spread_xline(const Geometry& g, const SysBuffers& b, int B, int BG, int chunk0,
                         int nchunks, hipStream_t st);

void fill_int(int* p, int v, int n, hipStream_t st);

template <typename R>
void launch_epilogue(const Geometry& g, const SysBuffers& b, const double* w, int B, int BG,
                     int chunk0, int nchunks, uint32_t comps, hipStream_t st);

void launch_probes(const Geometry& g, const SysBuffers& b, int B, int nb, int probe0,
                   uint64_t seed, int system, bool use_float, hipStream_t st);
void launch_init_scalars(const SysBuffers& b, int nb, int m, int probe0, hipStream_t st);
void launch_update(const Geometry& g, const SysBuffers& b, int B, int nb, int k, int m,
                   int probe0, bool use_float, bool write_d, hipStream_t st);
void launch_reorth(const Geometry& g, const SysBuffers& b, int B, int nb, int k, int m,
                   int probe0, int j0, bool use_float, hipStream_t st);
void launch_finish_a(const SysBuffers& b, int B, int nb, int k, int m, int probe0,
                     uint32_t* status, hipStream_t st);
void launch_finish_norm(const SysBuffers& b, int B, int nb, int k, int m, int probe0,
                        uint32_t* status, hipStream_t st);
void launch_tridiag(const SysBuffers& b, int nb, int m, int probe0, uint32_t* status,
                    hipStream_t st);
void launch_energy(const Geometry& g, const SysBuffers& b, int R, double* energy_out,
                   double* sd_out, uint32_t* status, hipStream_t st);
void launch_pack(const Geometry& g, const SysBuffers& b, const double* v, int nrhs, int B,
                 bool use_float, hipStream_t st);
void launch_unpack(const Geometry& g, const SysBuffers& b, double* out, int nrhs, int B,
                   hipStream_t st);

// forces
template <typename R>
void launch_pair_force(const Geometry& g, const SysBuffers& b, int B, hipStream_t st);
template <typename R>
void launch_spme_force(const Geometry& g, const SysBuffers& b, const void* h, int B, int BG,
                       int chunk0, hipStream_t st, const double* hscale = nullptr);
void launch_tridiag_adjoint(const SysBuffers& b, int nb, int m, int probe0, uint32_t* status,
                            hipStream_t st);
void launch_adjoint_step(const Geometry& g, const SysBuffers& b, int B, int nb, int k, int m,
                         int probe0, bool use_float, hipStream_t st);
void launch_adjoint_accumulate(const Geometry& g, const SysBuffers& b, int B, int k,
                               hipStream_t st);
void launch_forces_finish(const Geometry& g, const SysBuffers& b, int R, double* forces,
                          hipStream_t st);
void fill_double(double* p, double v, size_t n, hipStream_t st);

// self-consistent screening (conjugate gradient over 3 nq right-hand sides)
struct ScsWork {
  int n = 0, nq = 0, ncol = 0, nblk = 0;
  double* locd = nullptr;   // [n][4] sorted cell-local position (float64) and beta R_vdW
  double* ainv = nullptr;   // [n][nq] 1 / alpha_i(iu_q)
  double* sig2 = nullptr;   // [n][nq] sigma_i(u_q)^2
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;  // [n][3][ncol]
  double* part = nullptr;   // [nblk][2][ncol] partial dot products
  double* sums = nullptr;   // [2][ncol] their column sums
  double* sc = nullptr;     // [8][ncol] CG scalars
  int* nact = nullptr;      // [1] columns still iterating
};
void launch_scs_prepare(const Geometry& g, const SysBuffers& b, const double* alpha,
                        const double* omega, const double* rvdw, const double* u,
                        const ScsWork& w, hipStream_t st);
void launch_scs_apply(const Geometry& g, const SysBuffers& b, const ScsWork& w, const double* p,
                      double* q, hipStream_t st);
void launch_scs_init(const ScsWork& w, hipStream_t st);
void launch_scs_iteration(const Geometry& g, const SysBuffers& b, const ScsWork& w, double tol,
                          uint32_t* status, hipStream_t st);
void launch_scs_output(const SysBuffers& b, const ScsWork& w, const double* wq,
                       const double* alpha, const double* rvdw, double* a_out, double* om_out,
                       double* rv_out, double* af_out, hipStream_t st);

void launch_block_start(const Geometry& geo, const SysBuffers& b, const BlockWork& bw, int B,
                        int m, bool use_float, hipStream_t st);
void launch_block_step(const Geometry& geo, const SysBuffers& b, const BlockWork& bw, int B,
                       int k, int m, bool use_float, hipStream_t st);
void launch_block_quadrature(const BlockWork& bw, int nkb, int m, double* q_out,
                             uint32_t* status, hipStream_t st);

bool fft_supported(int k);
void set_error(const std::string& msg);

}  // namespace mbd
