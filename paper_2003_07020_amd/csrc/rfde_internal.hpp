// Internal declarations of the rfde HIP library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "rfde.h"

#define RFDE_HIP(expr)                                  \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return rfde::hip_fail(e_, #expr, __FILE__, __LINE__); \
  } while (0)

#define RFDE_TRY(expr)              \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != RFDE_OK) return rc_; \
  } while (0)

namespace rfde {

int hip_fail(hipError_t e, const char* what, const char* file, int line);

constexpr int TILE = 64;          // factor tile edge (complex entries)
constexpr int TILE_ELEMS = TILE * TILE;

// Number of lower-triangular tiles of a T x T tile grid, and the index of tile (i, j), i >= j.
__host__ __device__ inline size_t lower_tiles(int T) { return (size_t)T * (T + 1) / 2; }
__host__ __device__ inline size_t tile_index(int i, int j) { return (size_t)i * (i + 1) / 2 + j; }

// Shifted-block families handled by one factor or solve launch: a plan's own blocks, or those
// of every instance of a batch wave.  Lives in device memory.
constexpr int MAX_BATCH = 64;
struct BlockSet {
  int count;
  int nb[MAX_BATCH];                 // storage blocks of family k (work items per tile)
  int nfreq[MAX_BATCH];              // frequencies floor(N_t/2)+1 (rows of its z arrays)
  int dual[MAX_BATCH];               // 1: storage block 0 holds the real blocks 0 and N_t/2
  int M[MAX_BATCH];                  // order
  int T[MAX_BATCH];                  // tile count, ceil(M / 64)
  void* fac[MAX_BATCH];              // nf x lower_tiles(T) x 4096 complex
  const double* g[MAX_BATCH];        // g_0..g_{M-1}
  const double2* lambda[MAX_BATCH];  // lambda_0..lambda_{nf-1}
  double coef[MAX_BATCH];            // tau kappa / h^alpha
  const int* live[MAX_BATCH];        // family k is skipped while *live[k] == 0 (NULL: always on)
};

// Work items of one launch, numbered family by family: family fam[k] of the BlockSet owns items
// [start[k], start[k+1]).  Passed by value; it also carries each slot's factor pointer, since
// pointers read from kernel arguments are known to be global-memory pointers (global loads),
// while pointers read from the device-memory BlockSet would be addressed as generic (flat).
struct ItemMap {
  int cnt = 0;
  int start[MAX_BATCH + 1];
  int fam[MAX_BATCH];
  void* fac[MAX_BATCH];
  int total() const { return start[cnt]; }
};

// Bump allocator over one device allocation (a batch keeps one for all its waves, so device
// memory is mapped once instead of per plan and per wave).
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
};

// Tables of a DST-I of length n done by Bluestein's chirp-z form (2(n+1) not a power of two):
// chirp c_m (m = 0..n), twiddles and kernel transform of the cyclic length LB (0: not used).
struct DstBsAxis {
  int n = 0, LB = 0;
  double2* chirp = nullptr;
  float2* chirp32 = nullptr;
  double2* khat = nullptr;
  float2* khat32 = nullptr;
  double2* tw = nullptr;
  float2* tw32 = nullptr;
};

// Workspace of the optional inner solver of the 2D step (b) (k_inner.hip): at most INNER_KMAX
// GMRES steps per frequency.  V: k + 1 basis vectors, Z: their k tau solves, w: the new
// direction (each nf x S complex); per-frequency sums (part: nblk partial sums per frequency,
// h1, h2: reduced, KMAX + 2 entries each) and the small least-squares state.
constexpr int INNER_KMAX = 16;
struct InnerWs {
  double2 *V = nullptr, *Z = nullptr, *w = nullptr, *part = nullptr, *h1 = nullptr,
          *h2 = nullptr, *R = nullptr, *gsn = nullptr, *g = nullptr, *y = nullptr;
  double *gc = nullptr, *beta = nullptr, *scale = nullptr, *res = nullptr;
  int nblk = 0;
};

struct Plan {
  int dim = 1;
  int M = 0, Mx = 0, My = 0, S = 0;   // S = spatial unknowns per time level
  int Nt = 0, nf = 0;                 // nf = Nt/2 + 1
  int Lt = 0;                         // time transform length: Nt, or the Bluestein length
  int L = 0, Lx = 0, Ly = 0;
  int Mp = 0, T = 0;                  // padded order and tile count of the factored blocks
  int nb = 0;                         // storage blocks of the factors (nf, or nf - 1 if dual)
  bool dual = false;                  // even N_t: blocks 0 and N_t/2 (real) share storage block 0
  double alpha = 0, alpha_x = 0, alpha_y = 0;
  double kappa = 0, kappa_x = 0, kappa_y = 0;
  double h = 0, hx = 0, hy = 0, tau = 0, eps = 0;
  double coef = 0, coef_x = 0, coef_y = 0;  // tau kappa / h^alpha
  rfde_opts opts{};
  hipStream_t stream = nullptr;
  int device = 0;
  // Batch member: per-instance kernels of the iteration return at once while *live == 0
  // (the instance has converged in the current restart cycle).  NULL for ordinary plans.
  const int* live = nullptr;
  Arena* arena = nullptr;    // device buffers come from here (not freed by free_plan) if set
  // Launch-shape variants (chosen by the tuner; 0 = the built-in default):
  //   tv_time:   time FFTs with NB >> tv_time transforms per workgroup (tv_time in 0..2)
  //   tv_matvec: 0 default, 1 the other workgroup size, 2 largest FFT radix 8 instead of 16
  //   trsv_cap:  0 one workgroup per block; c > 0 at most c persistent workgroups
  int tv_time = 0, tv_matvec = 0, trsv_cap = 0;

  // setup data (device)
  double* g = nullptr;       // 1D: M; 2D: Mx then My
  double* sym = nullptr;     // 1D: L/2+1; 2D: Lx/2+1 then Ly/2+1 (scaled by coef / L)
  double2* twL = nullptr;    // twiddles exp(-2 pi i m / L); 2D: Lx table then Ly table
  double2* twNt = nullptr;   // twiddles exp(-2 pi i m / Lt)
  float2* twNt32 = nullptr;  // FP32 copy for the FP32 preconditioner
  double2* chirp = nullptr;  // Bluestein (Nt not a power of two): w_k = exp(i pi k^2 / Nt), Nt
  float2* chirp32 = nullptr;
  double2* bhat = nullptr;   // Bluestein: DFT of the conjugate chirp kernel / Lt, Lt entries
  float2* bhat32 = nullptr;
  double* s = nullptr;       // Nt: eps^{j/Nt}
  double2* lambda = nullptr; // nf
  double* sigma = nullptr;   // tau eigenvalues (unscaled): 1D M; 2D Mx then My
  double2* twD = nullptr;    // DST twiddles for length 2(n+1) (tau solver)
  DstBsAxis bs[2];           // tau solver, axes whose DST-I length n has 2(n+1) not a power of
                             // two (1D: bs[0]; 2D: bs[0] x, bs[1] y)
  void* zt = nullptr;        // nf x S complex: the chirp-z DST's first-phase results
  // Toeplitz (Gohberg-Semencul) solver: first columns of the inverses (nf x M), their DFTs of
  // length L divided by L (nf x L), and the two intermediate products (nf x M each)
  double2* gs_x = nullptr;
  double2* gs_xhat = nullptr;
  double2* gs_p = nullptr;
  double2* gs_q = nullptr;
  InnerWs inner;             // 2D with opts.inner_iters > 0
  void* factors = nullptr;   // nf blocks x lower_tiles(T) x 4096 complex (c128 or c64)
  size_t factor_bytes = 0;
  BlockSet* set = nullptr;   // this plan's blocks as a one-family set (device)

  // workspace (device)
  void* zf = nullptr;        // nf x S complex (frequency-domain work, c128 or c64)
  double* vbuf = nullptr;    // (m+1) x N Krylov basis V
  double* zbuf = nullptr;    // m x N preconditioned basis Z
  double* wvec = nullptr;    // N
  double* xvec = nullptr;    // N
  double* Fvec = nullptr;    // N
  double* red = nullptr;     // reduction partials
  double* redout = nullptr;  // reduction results (device)
  double* hred = nullptr;    // pinned host copy of reduction results
  size_t workspace_bytes = 0;
  double ms_setup = 0.0;   // wall time of plan setup
  double ms_factor = 0.0;  // device time of the factorisation launches (HIP events)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

  size_t N() const { return (size_t)Nt * S; }
};

// Family k of a block set = the factor blocks of plan p.
inline void set_family(BlockSet& hs, int k, const Plan& p) {
  hs.nb[k] = p.nb;
  hs.nfreq[k] = p.nf;
  hs.dual[k] = p.dual ? 1 : 0;
  hs.M[k] = p.M;
  hs.T[k] = p.T;
  hs.fac[k] = p.factors;
  hs.g[k] = p.g;
  hs.lambda[k] = p.lambda;
  hs.coef[k] = p.coef;
  hs.live[k] = p.live;
}

// ---- device memory (rfde_mem.hip): a per-device cache of freed blocks ----
int dev_alloc(void** ptr, size_t bytes);
void dev_free(void* ptr);
size_t dev_cached_bytes(int device);

// ---- plan life cycle (rfde_api.hip) ----
int plan_init_1d(Plan* p, double alpha, double kappa, double a, double b, int M, int Nt,
                 double T, rfde_opts o, hipStream_t stream);  // sizes only, no device work
size_t workspace_estimate(const Plan& p);
int plan_allocate_and_setup(Plan* p, bool factor);
void free_plan(Plan* p);
int apply_pinv(Plan& p, const double* v, double* z);
// what: bit 0 time FFTs, bit 1 matvec, bit 2 triangular solves (rfde_tune.hip)
int tune_plan(Plan& p, int what, rfde_tune_report* report);

// Compute units of device dev (queried once per device; 256 if the query fails).
int device_cus(int dev);

// ---- launchers (all enqueue on p.stream) ----
int launch_gk(double alpha, int n, double* g, hipStream_t st);
int launch_twiddles(double2* tw, int n, hipStream_t st);
int launch_twiddles32(float2* tw, int n, hipStream_t st);
int launch_symbol(const double* g, int M, int L, double scale, const double2* tw, double* sym,
                  hipStream_t st);
int launch_time_data(int Nt, double eps, double* s, double2* lambda, hipStream_t st);
int launch_tau_sigma(const double* g, int n, const double2* twD, double* sigma, hipStream_t st);

int launch_matvec(const Plan& p, const double* v, double* y);
int launch_rhs(const Plan& p, const double* u0, const double* f, double* F);

int launch_bluestein_setup(const Plan& p);
int launch_time_fwd(const Plan& p, const double* v, void* z1);
int launch_time_inv(const Plan& p, const void* z2, double* v);
int launch_widen(const Plan& p, const void* zsrc, double2* zdst);  // c64 -> c128 (FP32 plans)
int launch_narrow(const Plan& p, const double2* zsrc, void* zdst); // c128 -> c64

int launch_factorize(Plan& p);
int launch_trsv(const Plan& p, const void* zin, void* zout);
// Factor / solve every block of the families of a set (host copy `hs`, device copy `ds`).
// grid_cap > 0 caps the grid (persistent workgroups looping over the items); 0 launches one
// workgroup per item.  zin/zout: one frequency-domain array per family ([nf][M] complex).
int launch_factorize_set(const BlockSet& hs, const BlockSet* ds, int bits, int grid_cap,
                         hipStream_t st);
int launch_trsv_set(const BlockSet& hs, const BlockSet* ds, const void* const* zin,
                    void* const* zout, int bits, int grid_cap, hipStream_t st);
int launch_tau_solve(const Plan& p, const void* zin, void* zout);
// optional inner solver of the 2D step (b) (k_inner.hip)
int launch_inner_step_b(const Plan& p, const void* z1, void* z2);
int inner_blocks(int S);
size_t inner_workspace_bytes(int k, int nf, int S);
// Toeplitz solver (k_gs.hip): setup (generators and their transforms) and step (b).
int launch_gs_setup(const Plan& p);
int launch_gs_apply(const Plan& p, const void* z1, void* z2);
// DST-I of any length (k_dst_bs.hip): cyclic length, per-axis tables, and the tau solves.
int dstbs_length(int n);
int dstbs_setup_axis(const Plan& p, int axis);
template <typename C> int tau_solve_1d_bs(const Plan& p, const C* zin, C* z);
template <typename C> int tau_rows_2d_bs(const Plan& p, C* z);
template <typename C> int tau_cols_2d_bs(const Plan& p, C* z);
// bhat = DFT_{-1}(b) / LB of the cyclic kernel b_k = conj(w_k) (k < n), b_{LB-k} = conj(w_k)
// (0 < k < n), LB a power of two in 8..8192 (k_timefft.hip).
int launch_bs_spectrum(int n, const double2* w, const double2* tw, int LB, double2* bhat,
                       float2* bhat32, hipStream_t st);
int launch_export_factor(const Plan& p, int index, void* dst);

// BLAS-1 (deterministic fixed-order reductions)
int launch_multi_axpy(const Plan& p, double* w, const double* V, int nvec, const double* coef,
                      double sign);
int launch_nrm2(const Plan& p, const double* x, double* out);
int launch_sub(const Plan& p, const double* a, const double* b, double* out);  // out = a - b

// Logical block index so that each XCD (blocks are dealt round-robin to 8 XCDs) walks a
// contiguous range of logical work: neighbouring work items share operands in one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int x = b & 7, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

}  // namespace rfde
