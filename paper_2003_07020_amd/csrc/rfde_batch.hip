// Batched solves of independent 1D instances with uneven M, N_t, alpha and kappa (the problem of
// Section 2 posed many times), each with its own epsilon-circulant preconditioner (Section 3).
//
// Memory waves: the instances are packed (largest first, first fit) into waves whose factors
// and workspaces fit the device-memory budget; a wave is set up, solved and released before
// the next one starts.
//
// Inside a wave every step runs for all instances at once:
//   * factorisation: one k_ldlt_diag and one k_ldlt_panel launch per tile column for every
//     block of every instance (launch items numbered instance by instance);
//   * FGMRES(m) in lockstep: Arnoldi step j of all instances is one HIP graph (captured at its
//     first use and replayed in later restart cycles): per-instance time FFTs and matvecs, one
//     triangular-solve launch over every block of every instance, then batched CGS2 reductions
//     and a device-side Givens update.  An instance whose residual estimate reaches the
//     tolerance clears its live flag, and every kernel of the graph returns at once for it.
//     The host reads the live flags once per step (one synchronisation for the whole wave).
//   * Each restart cycle ends with the update x += Z y and the true residual F - A x, which
//     decides convergence exactly as the single-instance solver does.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <vector>

#include "rfde_internal.hpp"

namespace rfde {

constexpr int MMAX = 64;  // restart length limit
constexpr int BPI = 64;   // reduction partials per instance and value (one wave sums them)
constexpr int BPA = 64;   // workgroups per instance in the vector kernels
constexpr int DCH = 16;   // vectors per pass of the batched multi-dot

// Device state of one wave.  The first block (live .. est) is copied to the host in one piece.
struct WaveState {
  int live[MAX_BATCH];      // instance takes part in the current launches
  int kdone[MAX_BATCH];     // Arnoldi steps taken in the current cycle
  int bad[MAX_BATCH];       // a non-finite value was met
  int lim[MAX_BATCH];       // step limit of the current cycle
  double beta[MAX_BATCH];   // last residual norm computed
  double bnorm[MAX_BATCH];  // ||F||
  double est[MAX_BATCH][MMAX];
  // device-only part
  int count, m;
  double tol;
  size_t n[MAX_BATCH];
  double* V[MAX_BATCH];     // (m+1) x n: Arnoldi basis; V[0] also holds the residual
  double* Z[MAX_BATCH];     // m x n: preconditioned basis
  double* x[MAX_BATCH];
  double* F[MAX_BATCH];
  double H[MAX_BATCH][(MMAX + 1) * MMAX];  // (i, j) at i * MMAX + j
  double cs[MAX_BATCH][MMAX], sn[MAX_BATCH][MMAX];
  double g[MAX_BATCH][MMAX + 1];
  double y[MAX_BATCH][MMAX];
  double hc[MAX_BATCH][MMAX + 2];
  double part[MAX_BATCH][MMAX + 1][BPI];
};
constexpr size_t HOST_PART = offsetof(WaveState, count);

enum DotSel { DOT_CGS = 0, NRM_NEXT = 1, NRM_V0 = 2, NRM_F = 3 };
enum FinSel { FIN_SET = 0, FIN_ADD = 1, FIN_NEXT = 2, FIN_BETA = 3, FIN_BNORM = 4 };

__device__ __forceinline__ double bsum256(double v, double* sh) {
  const int t = threadIdx.x;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  const double s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return s;
}

// Partials of: DOT_CGS: V[v] . V[j+1] (v < nv); NRM_NEXT: ||V[j+1]||^2; NRM_V0: ||V[0]||^2;
// NRM_F: ||F||^2.  Grid: count x BPI workgroups of 256.
__global__ void __launch_bounds__(256) kb_dot_partial(WaveState* __restrict__ S, int sel, int j,
                                                      int nv) {
  __shared__ double sh[4];
  const int k = blockIdx.x / BPI, b = blockIdx.x % BPI;
  if (k >= S->count || !S->live[k]) return;
  const size_t n = S->n[k];
  const double* t;
  if (sel == DOT_CGS || sel == NRM_NEXT) t = S->V[k] + (size_t)(j + 1) * n;
  else if (sel == NRM_V0) t = S->V[k];
  else t = S->F[k];
  if (sel != DOT_CGS) nv = 1;
  const double* Vk = S->V[k];
  for (int v0 = 0; v0 < nv; v0 += DCH) {
    double acc[DCH];
#pragma unroll
    for (int v = 0; v < DCH; ++v) acc[v] = 0.0;
    for (size_t i = (size_t)b * 256 + threadIdx.x; i < n; i += (size_t)BPI * 256) {
      const double ti = t[i];
      if (sel != DOT_CGS) {
        acc[0] = fma(ti, ti, acc[0]);
      } else {
#pragma unroll
        for (int v = 0; v < DCH; ++v)
          if (v0 + v < nv) acc[v] = fma(Vk[(size_t)(v0 + v) * n + i], ti, acc[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < DCH; ++v) {
      if (v0 + v < nv) {
        const double s = bsum256(acc[v], sh);
        if (threadIdx.x == 0) S->part[k][v0 + v][b] = s;
      }
    }
  }
}

// Sum the BPI partials of each value (one wave per value, fixed tree) and store them.
__global__ void __launch_bounds__(256) kb_dot_final(WaveState* __restrict__ S, int fin, int j,
                                                    int nv) {
  const int k = blockIdx.x;
  if (k >= S->count || !S->live[k]) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (fin >= FIN_NEXT) nv = 1;
  for (int v = w; v < nv; v += 4) {
    double s = S->part[k][v][lane];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (lane != 0) continue;
    if (fin == FIN_SET) {
      S->hc[k][v] = s;
      S->H[k][v * MMAX + j] = s;
    } else if (fin == FIN_ADD) {
      S->hc[k][v] = s;
      S->H[k][v * MMAX + j] += s;
    } else {
      const double r = sqrt(s);
      if (fin == FIN_NEXT) {
        S->hc[k][j + 1] = r;
        S->H[k][(j + 1) * MMAX + j] = r;
      } else if (fin == FIN_BETA) {
        S->beta[k] = r;
      } else {
        S->bnorm[k] = r;
      }
    }
  }
}

// V[j+1] -= sum_{v < nv} hc[v] V[v]
__global__ void __launch_bounds__(256) kb_axpy(WaveState* __restrict__ S, int j, int nv) {
  const int k = blockIdx.x / BPA, b = blockIdx.x % BPA;
  if (k >= S->count || !S->live[k]) return;
  const size_t n = S->n[k];
  const double* Vk = S->V[k];
  double* w = S->V[k] + (size_t)(j + 1) * n;
  const double* h = S->hc[k];
  for (size_t i = (size_t)b * 256 + threadIdx.x; i < n; i += (size_t)BPA * 256) {
    double s = 0.0;
    for (int v = 0; v < nv; ++v) s = fma(h[v], Vk[(size_t)v * n + i], s);
    w[i] -= s;
  }
}

// which = 0: V[j+1] /= hc[j+1];  which = 1: V[0] /= beta.  Skipped when the divisor is not a
// positive finite number (breakdown or failure; the Givens step then stops the instance).
__global__ void __launch_bounds__(256) kb_scale(WaveState* __restrict__ S, int which, int j) {
  const int k = blockIdx.x / BPA, b = blockIdx.x % BPA;
  if (k >= S->count || !S->live[k]) return;
  const size_t n = S->n[k];
  const double d = which == 0 ? S->hc[k][j + 1] : S->beta[k];
  if (!(d > 0.0) || !isfinite(d)) return;
  const double a = 1.0 / d;
  double* w = S->V[k] + (which == 0 ? (size_t)(j + 1) * n : 0);
  for (size_t i = (size_t)b * 256 + threadIdx.x; i < n; i += (size_t)BPA * 256) w[i] *= a;
}

// Givens update of column j (one thread per instance): rotate with the previous rotations,
// form a new one, update g and the residual estimate; stop the instance when the estimate
// reaches tol, at breakdown, at its step limit or on a non-finite value.
__global__ void kb_givens(WaveState* __restrict__ S, int j) {
  const int k = threadIdx.x;
  if (k >= S->count || !S->live[k]) return;
  double* H = S->H[k];
  double* cs = S->cs[k];
  double* sn = S->sn[k];
  double* g = S->g[k];
  const double hn = H[(j + 1) * MMAX + j];
  for (int i = 0; i < j; ++i) {
    const double a = H[i * MMAX + j], b = H[(i + 1) * MMAX + j];
    H[i * MMAX + j] = cs[i] * a + sn[i] * b;
    H[(i + 1) * MMAX + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[j * MMAX + j], b = H[(j + 1) * MMAX + j];
  const double d = hypot(a, b);
  cs[j] = a / d;
  sn[j] = b / d;
  H[j * MMAX + j] = d;
  H[(j + 1) * MMAX + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  const double est = fabs(g[j + 1]) / S->bnorm[k];
  S->est[k][j] = est;
  S->kdone[k] = j + 1;
  const bool finite = isfinite(hn) && isfinite(est) && d > 0.0;
  if (!finite) S->bad[k] = 1;
  if (!finite || est <= S->tol || !(hn > 0.0) || j + 1 >= S->lim[k]) S->live[k] = 0;
}

struct StepLimits {
  int v[MAX_BATCH];
};

// Start of a restart cycle for the instances in `mask`: live, step limits, cleared H and g.
__global__ void kb_cycle_begin(WaveState* __restrict__ S, unsigned long long mask, StepLimits lim) {
  const int k = blockIdx.x;
  if (k >= S->count) return;
  const bool on = (mask >> k) & 1ull;
  for (int e = threadIdx.x; e < (MMAX + 1) * MMAX; e += blockDim.x) S->H[k][e] = 0.0;
  for (int e = threadIdx.x; e <= MMAX; e += blockDim.x) S->g[k][e] = 0.0;
  if (threadIdx.x == 0) {
    S->live[k] = on ? 1 : 0;
    S->kdone[k] = 0;
    S->lim[k] = lim.v[k];
  }
}

// After beta = ||r||: g_0 = beta; the instance iterates if beta / ||F|| > tol.
__global__ void kb_cycle_start(WaveState* __restrict__ S) {
  const int k = threadIdx.x;
  if (k >= S->count || !S->live[k]) return;
  const double beta = S->beta[k];
  if (!isfinite(beta)) {
    S->bad[k] = 1;
    S->live[k] = 0;
    return;
  }
  S->g[k][0] = beta;
  if (!(beta / S->bnorm[k] > S->tol)) S->live[k] = 0;
}

// y = H(0:kd, 0:kd)^{-1} g (back substitution, one thread per instance).
__global__ void kb_solve_y(WaveState* __restrict__ S) {
  const int k = threadIdx.x;
  if (k >= S->count) return;
  const int kd = S->kdone[k];
  const double* H = S->H[k];
  for (int i = kd - 1; i >= 0; --i) {
    double s = S->g[k][i];
    for (int c = i + 1; c < kd; ++c) s -= H[i * MMAX + c] * S->y[k][c];
    S->y[k][i] = s / H[i * MMAX + i];
  }
}

// x += Z y for instances with kdone > 0.
__global__ void __launch_bounds__(256) kb_xupdate(WaveState* __restrict__ S) {
  const int k = blockIdx.x / BPA, b = blockIdx.x % BPA;
  if (k >= S->count) return;
  const int kd = S->kdone[k];
  if (kd == 0) return;
  const size_t n = S->n[k];
  const double* Zk = S->Z[k];
  const double* y = S->y[k];
  double* x = S->x[k];
  for (size_t i = (size_t)b * 256 + threadIdx.x; i < n; i += (size_t)BPA * 256) {
    double s = 0.0;
    for (int v = 0; v < kd; ++v) s = fma(y[v], Zk[(size_t)v * n + i], s);
    x[i] += s;
  }
}

// live = mask (instances that take part in the eager work that follows).
__global__ void kb_set_live(WaveState* __restrict__ S, unsigned long long mask) {
  const int k = threadIdx.x;
  if (k < S->count) S->live[k] = (int)((mask >> k) & 1ull);
}

}  // namespace rfde

using namespace rfde;

struct rfde_batch_ {
  std::vector<rfde_instance> inst;
  rfde_opts opts{};
  std::vector<std::vector<int>> waves;
  std::vector<size_t> bytes;  // device bytes per instance
  size_t budget = 0;
  hipStream_t user = nullptr;
  rfde_batch_info info{};
  int grid_cap_factor = 0, grid_cap_trsv = 0;
  int tune = 0;                    // tune_plan flags for every instance (0: off)
  std::vector<char> conv, failed;  // outcome per instance of the last solve
  Arena arena;                     // device memory of the waves, mapped once, reused
  ~rfde_batch_() {
    dev_free(arena.base);
  }
};

namespace {

struct Wave {
  std::vector<Plan*> plans;
  WaveState* S = nullptr;
  BlockSet* ds = nullptr;
  BlockSet hs{};
  std::vector<hipGraphExec_t> exec;
  hipStream_t st = nullptr;
  WaveState* host = nullptr;  // pinned copy of the leading (host-read) part
  ~Wave() {
    if (host) (void)hipHostFree(host);
    for (auto e : exec)
      if (e) (void)hipGraphExecDestroy(e);
    for (Plan* p : plans) free_plan(p);
    dev_free(S);
    dev_free(ds);
  }
};

int launch_dot(Wave& w, int sel, int j, int nv, int fin) {
  const int cnt = (int)w.plans.size();
  kb_dot_partial<<<cnt * BPI, 256, 0, w.st>>>(w.S, sel, j, nv);
  RFDE_HIP(hipGetLastError());
  kb_dot_final<<<cnt, 256, 0, w.st>>>(w.S, fin, j, nv);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// Arnoldi step j for every live instance (the body of the per-step graph).
int arnoldi_step(Wave& w, int j, int bits, int cap) {
  const int cnt = (int)w.plans.size();
  std::vector<const void*> zin(cnt);
  std::vector<void*> zout(cnt);
  for (int k = 0; k < cnt; ++k) {
    Plan& p = *w.plans[k];
    const size_t N = p.N();
    RFDE_TRY(launch_time_fwd(p, p.vbuf + (size_t)j * N, p.zf));
    zin[k] = p.zf;
    zout[k] = p.zf;
  }
  RFDE_TRY(launch_trsv_set(w.hs, w.ds, zin.data(), zout.data(), bits, cap, w.st));
  for (int k = 0; k < cnt; ++k) {
    Plan& p = *w.plans[k];
    const size_t N = p.N();
    RFDE_TRY(launch_time_inv(p, p.zf, p.zbuf + (size_t)j * N));
    RFDE_TRY(launch_matvec(p, p.zbuf + (size_t)j * N, p.vbuf + (size_t)(j + 1) * N));
  }
  RFDE_TRY(launch_dot(w, DOT_CGS, j, j + 1, FIN_SET));
  kb_axpy<<<cnt * BPA, 256, 0, w.st>>>(w.S, j, j + 1);
  RFDE_HIP(hipGetLastError());
  RFDE_TRY(launch_dot(w, DOT_CGS, j, j + 1, FIN_ADD));
  kb_axpy<<<cnt * BPA, 256, 0, w.st>>>(w.S, j, j + 1);
  RFDE_HIP(hipGetLastError());
  RFDE_TRY(launch_dot(w, NRM_NEXT, j, 1, FIN_NEXT));
  kb_scale<<<cnt * BPA, 256, 0, w.st>>>(w.S, 0, j);
  RFDE_HIP(hipGetLastError());
  kb_givens<<<1, MAX_BATCH, 0, w.st>>>(w.S, j);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int wave_graph(Wave& w, int j, int bits, int cap) {
  if (w.exec[j]) return RFDE_OK;
  RFDE_HIP(hipStreamBeginCapture(w.st, hipStreamCaptureModeThreadLocal));
  const int rc = arnoldi_step(w, j, bits, cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(w.st, &g);
  if (rc != RFDE_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != RFDE_OK) return rc;
    RFDE_HIP(e);
  }
  const hipError_t ei = hipGraphInstantiateWithFlags(&w.exec[j], g, 0);
  (void)hipGraphDestroy(g);
  RFDE_HIP(ei);
  return RFDE_OK;
}

unsigned long long mask_of(const std::vector<char>& on) {
  unsigned long long m = 0;
  for (size_t k = 0; k < on.size(); ++k)
    if (on[k]) m |= 1ull << k;
  return m;
}

// Solve one wave; results for instance wave-slot k go to U[idx[k]], stats[idx[k]].
int solve_wave(rfde_batch_& B, const std::vector<int>& idx, const double* const* u0,
               const double* const* f, double* const* U, rfde_stats* stats, hipStream_t st) {
  const int cnt = (int)idx.size();
  const rfde_opts& o = B.opts;
  const int m = o.restart;
  const int bits = o.precond_bits;
  Wave w;
  w.st = st;
  w.exec.assign(m, nullptr);
  const auto t0 = std::chrono::steady_clock::now();
  B.arena.used = 0;  // the previous wave's plans are gone
  RFDE_TRY(dev_alloc((void**)&w.S, sizeof(WaveState)));
  RFDE_TRY(dev_alloc((void**)&w.ds, sizeof(BlockSet)));
  auto ms_since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
  };
  // plans (setup kernels run, factors allocated but not yet filled)
  for (int k = 0; k < cnt; ++k) {
    const rfde_instance& in = B.inst[idx[k]];
    Plan* p = new (std::nothrow) Plan();
    if (!p) return RFDE_ENOMEM;
    int rc = plan_init_1d(p, in.alpha, in.kappa, in.a, in.b, in.M, in.Nt, in.T, o, st);
    if (rc != RFDE_OK) { delete p; return rc; }
    p->live = reinterpret_cast<const int*>(reinterpret_cast<const char*>(w.S) +
                                           offsetof(WaveState, live)) + k;
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return RFDE_EHIP; }
    p->arena = &B.arena;
    rc = plan_allocate_and_setup(p, false);
    if (rc != RFDE_OK) { free_plan(p); return rc; }
    w.plans.push_back(p);
  }
  // device state and the wave's block set
  std::vector<unsigned char> hbuf(sizeof(WaveState), 0);
  WaveState* hS = reinterpret_cast<WaveState*>(hbuf.data());
  hS->count = cnt;
  hS->m = m;
  hS->tol = o.tol;
  BlockSet& hs = w.hs;
  std::memset(&hs, 0, sizeof(hs));
  hs.count = cnt;
  for (int k = 0; k < cnt; ++k) {
    Plan& p = *w.plans[k];
    hS->n[k] = p.N();
    hS->V[k] = p.vbuf;
    hS->Z[k] = p.zbuf;
    hS->x[k] = p.xvec;
    hS->F[k] = p.Fvec;
    hS->live[k] = 1;
    set_family(hs, k, p);
  }
  RFDE_HIP(hipMemcpy(w.S, hS, sizeof(WaveState), hipMemcpyHostToDevice));
  RFDE_HIP(hipMemcpy(w.ds, &hs, sizeof(BlockSet), hipMemcpyHostToDevice));
  RFDE_HIP(hipHostMalloc((void**)&w.host, HOST_PART, hipHostMallocDefault));
  B.info.ms_plans += ms_since(t0);
  // launch shapes of each instance's time FFTs and matvec (cached per shape)
  const auto tt = std::chrono::steady_clock::now();
  if (B.tune & 3)
    for (Plan* p : w.plans) RFDE_TRY(tune_plan(*p, B.tune & 3, nullptr));
  B.info.ms_tune += ms_since(tt);
  // factorisation of every block of every instance
  hipEvent_t e0, e1;
  RFDE_HIP(hipEventCreate(&e0));
  RFDE_HIP(hipEventCreate(&e1));
  RFDE_HIP(hipEventRecord(e0, st));
  int rc = launch_factorize_set(hs, w.ds, bits, B.grid_cap_factor, st);
  RFDE_HIP(hipEventRecord(e1, st));
  RFDE_HIP(hipStreamSynchronize(st));
  float msf = 0.f;
  (void)hipEventElapsedTime(&msf, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != RFDE_OK) return rc;
  const auto t1 = std::chrono::steady_clock::now();

  // right-hand sides and ||F||
  for (int k = 0; k < cnt; ++k) {
    Plan& p = *w.plans[k];
    RFDE_TRY(launch_rhs(p, u0[idx[k]], f[idx[k]], p.Fvec));
    RFDE_HIP(hipMemsetAsync(p.xvec, 0, p.N() * sizeof(double), st));
  }
  RFDE_TRY(launch_dot(w, NRM_F, 0, 1, FIN_BNORM));
  WaveState* hp = w.host;
  auto pull = [&]() -> int {
    RFDE_HIP(hipMemcpyAsync(hp, w.S, HOST_PART, hipMemcpyDeviceToHost, st));
    RFDE_HIP(hipStreamSynchronize(st));
    return RFDE_OK;
  };
  RFDE_TRY(pull());
  std::vector<char> active(cnt, 1), first(cnt, 1), failed(cnt, 0);
  std::vector<rfde_stats> loc(cnt);
  std::vector<int> total(cnt, 0);
  std::vector<double> rel(cnt, 1.0);
  for (int k = 0; k < cnt; ++k) {
    std::memset(&loc[k], 0, sizeof(rfde_stats));
    const double bn = hp->bnorm[k];
    if (!std::isfinite(bn)) {
      active[k] = 0;
      failed[k] = 1;
    } else if (bn == 0.0) {
      active[k] = 0;
      rel[k] = 0.0;
    } else {
      loc[k].res_hist[0] = 1.0;
      loc[k].n_hist = 1;
    }
  }
  int graph_launches = 0;
  while (true) {
    std::vector<char> run(cnt, 0);
    bool any = false;
    StepLimits lim{};
    for (int k = 0; k < cnt; ++k) {
      if (active[k] && total[k] < o.maxit) {
        run[k] = 1;
        any = true;
        lim.v[k] = std::min(m, o.maxit - total[k]);
      }
    }
    if (!any) break;
    // r = F - A x into V[0] (x = 0 on the first cycle: r = F)
    kb_set_live<<<1, MAX_BATCH, 0, st>>>(w.S, mask_of(run));
    RFDE_HIP(hipGetLastError());
    for (int k = 0; k < cnt; ++k) {
      if (!run[k]) continue;
      Plan& p = *w.plans[k];
      if (first[k]) {
        RFDE_HIP(hipMemcpyAsync(p.vbuf, p.Fvec, p.N() * sizeof(double), hipMemcpyDeviceToDevice,
                                st));
      } else {
        RFDE_TRY(launch_matvec(p, p.xvec, p.wvec));
        RFDE_TRY(launch_sub(p, p.Fvec, p.wvec, p.vbuf));
      }
      first[k] = 0;
    }
    kb_cycle_begin<<<cnt, 256, 0, st>>>(w.S, mask_of(run), lim);
    RFDE_HIP(hipGetLastError());
    RFDE_TRY(launch_dot(w, NRM_V0, 0, 1, FIN_BETA));
    kb_cycle_start<<<1, MAX_BATCH, 0, st>>>(w.S);
    RFDE_HIP(hipGetLastError());
    kb_scale<<<cnt * BPA, 256, 0, st>>>(w.S, 1, 0);
    RFDE_HIP(hipGetLastError());
    RFDE_TRY(pull());
    for (int j = 0; j < m; ++j) {
      bool live_any = false;
      for (int k = 0; k < cnt; ++k) live_any = live_any || hp->live[k];
      if (!live_any) break;
      RFDE_TRY(wave_graph(w, j, bits, B.grid_cap_trsv));
      RFDE_HIP(hipGraphLaunch(w.exec[j], st));
      ++graph_launches;
      RFDE_HIP(hipMemcpyAsync(hp->live, reinterpret_cast<char*>(w.S) + offsetof(WaveState, live),
                              cnt * sizeof(int), hipMemcpyDeviceToHost, st));
      RFDE_HIP(hipStreamSynchronize(st));
    }
    RFDE_TRY(pull());
    // x += Z y, then the true residual of every instance that ran this cycle
    kb_solve_y<<<1, MAX_BATCH, 0, st>>>(w.S);
    RFDE_HIP(hipGetLastError());
    kb_xupdate<<<cnt * BPA, 256, 0, st>>>(w.S);
    RFDE_HIP(hipGetLastError());
    kb_set_live<<<1, MAX_BATCH, 0, st>>>(w.S, mask_of(run));
    RFDE_HIP(hipGetLastError());
    for (int k = 0; k < cnt; ++k) {
      if (!run[k]) continue;
      Plan& p = *w.plans[k];
      RFDE_TRY(launch_matvec(p, p.xvec, p.wvec));
      RFDE_TRY(launch_sub(p, p.Fvec, p.wvec, p.vbuf));
    }
    std::vector<int> kd(cnt);
    for (int k = 0; k < cnt; ++k) kd[k] = hp->kdone[k];
    std::vector<std::vector<double>> est(cnt);
    for (int k = 0; k < cnt; ++k) est[k].assign(hp->est[k], hp->est[k] + kd[k]);
    std::vector<int> bad(cnt);
    for (int k = 0; k < cnt; ++k) bad[k] = hp->bad[k];
    RFDE_TRY(launch_dot(w, NRM_V0, 0, 1, FIN_BETA));
    RFDE_TRY(pull());
    for (int k = 0; k < cnt; ++k) {
      if (!run[k]) continue;
      rfde_stats& s = loc[k];
      for (int i = 0; i < kd[k] && s.n_hist < 256; ++i) s.res_hist[s.n_hist++] = est[k][i];
      total[k] += kd[k];
      ++s.restarts;
      const double beta = hp->beta[k];
      if (bad[k] || !std::isfinite(beta)) {
        active[k] = 0;
        failed[k] = 1;
        continue;
      }
      rel[k] = beta / hp->bnorm[k];
      // done when converged, out of steps, or nothing moved (breakdown at an exact solution)
      if (rel[k] <= o.tol || total[k] >= o.maxit || kd[k] == 0) active[k] = 0;
    }
  }
  // results
  for (int k = 0; k < cnt; ++k) {
    Plan& p = *w.plans[k];
    RFDE_HIP(hipMemcpyAsync(U[idx[k]], p.xvec, p.N() * sizeof(double), hipMemcpyDeviceToDevice,
                            st));
  }
  RFDE_HIP(hipStreamSynchronize(st));
  const auto t2 = std::chrono::steady_clock::now();
  const double ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count();
  const double ms_solve = std::chrono::duration<double, std::milli>(t2 - t1).count();
  for (int k = 0; k < cnt; ++k) {
    rfde_stats& s = loc[k];
    s.iters = total[k];
    s.n_pinv = total[k];
    s.true_rel_res = failed[k] ? NAN : rel[k];
    s.converged = (!failed[k] && rel[k] <= o.tol) ? 1 : 0;
    s.ms_setup = ms_setup;
    s.ms_solve = ms_solve;
    if (stats) stats[idx[k]] = s;
    B.conv[idx[k]] = (char)s.converged;
    B.failed[idx[k]] = failed[k];
  }
  B.info.ms_setup += ms_setup;
  B.info.ms_factor += msf;
  B.info.ms_solve += ms_solve;
  B.info.graph_launches += graph_launches;
  size_t dev = sizeof(WaveState) + sizeof(BlockSet);
  for (Plan* p : w.plans) dev += p->factor_bytes + p->workspace_bytes;
  B.info.device_bytes_max = std::max(B.info.device_bytes_max, dev);
  return RFDE_OK;
}

}  // namespace

extern "C" {

int rfde_batch_create(rfde_batch* batch, int count, const rfde_instance* inst,
                      const rfde_opts* opts, size_t mem_budget, void* hip_stream) {
  if (!batch) return RFDE_EINVAL;
  *batch = nullptr;
  if (count < 1 || !inst) return RFDE_EINVAL;
  rfde_opts o;
  rfde_opts_default(&o);
  if (opts) o = *opts;
  if (o.spatial != RFDE_SPATIAL_EXACT || o.inner_iters > 0) return RFDE_EUNSUPPORTED;
  rfde_batch_* B = new (std::nothrow) rfde_batch_();
  if (!B) return RFDE_ENOMEM;
  B->inst.assign(inst, inst + count);
  B->opts = o;
  B->user = (hipStream_t)hip_stream;
  B->bytes.resize(count);
  B->conv.assign(count, 0);
  B->failed.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    Plan p;
    const rfde_instance& in = inst[i];
    const int rc = plan_init_1d(&p, in.alpha, in.kappa, in.a, in.b, in.M, in.Nt, in.T, o, nullptr);
    if (rc != RFDE_OK) { delete B; return rc; }
    B->bytes[i] = p.factor_bytes + workspace_estimate(p) + ((size_t)1 << 20);
  }
  size_t freeb = 0, totalb = 0;
  int dev = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess || hipGetDevice(&dev) != hipSuccess) {
    delete B;
    return RFDE_EHIP;
  }
  freeb += dev_cached_bytes(dev);
  const size_t fixed = sizeof(WaveState) + sizeof(BlockSet) + ((size_t)64 << 20);
  const size_t cap = freeb > fixed ? (size_t)((freeb - fixed) * 0.95) : 0;
  size_t big = 0;
  for (size_t u : B->bytes) big = std::max(big, u);
  // default: a quarter of the free memory (or the largest instance): small instances share
  // waves, large ones (which fill the GPU alone) take few per wave, and the memory that has to
  // be mapped stays moderate
  B->budget = mem_budget ? std::min(mem_budget, cap) : std::min(cap, std::max(big, cap / 4));
  // first fit, largest first, at most MAX_BATCH instances per wave
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return B->bytes[x] > B->bytes[y]; });
  std::vector<size_t> used;
  for (int i : order) {
    if (B->bytes[i] > B->budget) { delete B; return RFDE_ENOMEM; }
    size_t wsel = used.size();
    for (size_t wv = 0; wv < used.size(); ++wv) {
      if (used[wv] + B->bytes[i] <= B->budget && B->waves[wv].size() < (size_t)MAX_BATCH) {
        wsel = wv;
        break;
      }
    }
    if (wsel == used.size()) {
      used.push_back(0);
      B->waves.emplace_back();
    }
    used[wsel] += B->bytes[i];
    B->waves[wsel].push_back(i);
  }
  for (auto& wv : B->waves) std::sort(wv.begin(), wv.end());
  B->info.count = count;
  B->info.waves = (int)B->waves.size();
  for (auto& wv : B->waves) B->info.max_wave = std::max(B->info.max_wave, (int)wv.size());
  for (size_t u : used) B->info.wave_bytes_max = std::max(B->info.wave_bytes_max, u);
  B->info.budget_bytes = B->budget;
  for (size_t u : B->bytes) B->info.instance_bytes_max = std::max(B->info.instance_bytes_max, u);
  *batch = B;
  return RFDE_OK;
}

int rfde_batch_set_autotune(rfde_batch batch, int what) {
  if (!batch || what < 0 || what > 3) return RFDE_EINVAL;
  batch->tune = what;
  return RFDE_OK;
}

int rfde_batch_set_grid_caps(rfde_batch batch, int factor_cap, int trsv_cap) {
  if (!batch || factor_cap < 0 || trsv_cap < 0) return RFDE_EINVAL;
  batch->grid_cap_factor = factor_cap;
  batch->grid_cap_trsv = trsv_cap;
  return RFDE_OK;
}

int rfde_batch_solve(rfde_batch batch, const double* const* u0, const double* const* f,
                     double* const* U, rfde_stats* stats) {
  if (!batch || !u0 || !f || !U) return RFDE_EINVAL;
  const int count = batch->info.count;
  for (int i = 0; i < count; ++i)
    if (!u0[i] || !f[i] || !U[i]) return RFDE_EINVAL;
  RFDE_HIP(hipStreamSynchronize(batch->user));
  if (!batch->arena.base) {
    RFDE_TRY(dev_alloc((void**)&batch->arena.base, batch->info.wave_bytes_max));
    batch->arena.size = batch->info.wave_bytes_max;
  }
  hipStream_t st = nullptr;
  RFDE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  batch->info.ms_setup = batch->info.ms_factor = batch->info.ms_solve = 0.0;
  batch->info.ms_plans = batch->info.ms_tune = 0.0;
  batch->info.graph_launches = 0;
  int rc = RFDE_OK;
  for (const auto& wv : batch->waves) {
    rc = solve_wave(*batch, wv, u0, f, U, stats, st);
    if (rc != RFDE_OK) break;
  }
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (rc != RFDE_OK) return rc;
  bool all = true, nan = false;
  for (int i = 0; i < count; ++i) {
    all = all && batch->conv[i];
    nan = nan || batch->failed[i];
  }
  if (nan) return RFDE_ENAN;
  return all ? RFDE_OK : RFDE_ENOTCONV;
}

int rfde_batch_get_info(rfde_batch batch, rfde_batch_info* info) {
  if (!batch || !info) return RFDE_EINVAL;
  *info = batch->info;
  return RFDE_OK;
}

int rfde_batch_wave_of(rfde_batch batch, int index) {
  if (!batch || index < 0 || index >= batch->info.count) return RFDE_EINVAL;
  for (size_t w = 0; w < batch->waves.size(); ++w)
    for (int i : batch->waves[w])
      if (i == index) return (int)w;
  return RFDE_EINVAL;
}

int rfde_batch_destroy(rfde_batch batch) {
  delete batch;
  return RFDE_OK;
}

}  // extern "C"
