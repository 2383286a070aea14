// C ABI of the library: plan lifecycle, the individual hot-path steps, and the FGMRES driver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "krylov.hpp"
#include "rfde_internal.hpp"

namespace rfde {

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  if (std::getenv("RFDE_VERBOSE"))
    std::fprintf(stderr, "[rfde] HIP error %s (%d) in %s at %s:%d\n", hipGetErrorString(e), (int)e,
                 what, file, line);
  return e == hipErrorOutOfMemory ? RFDE_ENOMEM : RFDE_EHIP;
}

static int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
// Time levels accepted: powers of two up to 8192 (radix-16 Stockham) and any other count up to
// 4096 (Bluestein, transform length next_pow2(2 Nt - 1) <= 8192).
static bool nt_ok(int Nt) { return Nt >= 2 && (is_pow2(Nt) ? Nt <= 8192 : Nt <= 4096); }
static int time_length(int Nt) { return is_pow2(Nt) ? Nt : next_pow2(2 * Nt - 1); }


void free_plan(Plan* p) {
  if (!p) return;
  void* bufs[] = {p->g,      p->sym,     p->twL,  p->twNt,   p->twNt32, p->chirp, p->chirp32,
                  p->bhat,   p->bhat32,  p->s,    p->lambda, p->sigma,  p->twD,   p->factors,
                  p->zf,     p->vbuf,    p->zbuf, p->wvec,   p->xvec,   p->Fvec,  p->red,
                  p->redout,  p->set,    p->zt,     p->gs_x,  p->gs_xhat, p->gs_p, p->gs_q,
                  p->bs[0].chirp, p->bs[0].chirp32, p->bs[0].khat, p->bs[0].khat32, p->bs[0].tw,
                  p->bs[0].tw32,  p->bs[1].chirp,   p->bs[1].chirp32, p->bs[1].khat,
                  p->bs[1].khat32, p->bs[1].tw,     p->bs[1].tw32,
                  p->inner.V,     p->inner.Z,       p->inner.w,       p->inner.part,
                  p->inner.h1,    p->inner.h2,      p->inner.R,       p->inner.gsn,
                  p->inner.g,     p->inner.y,       p->inner.gc,      p->inner.beta,
                  p->inner.scale, p->inner.res};
  if (!p->arena)
    for (void* b : bufs) dev_free(b);
  if (p->hred) (void)hipHostFree(p->hred);
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

// Device buffer of `bytes` for plan p: from its arena (256-byte aligned) or hipMalloc.
static int palloc(Plan* p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (p->arena) {
    Arena& a = *p->arena;
    const size_t off = (a.used + 255) & ~(size_t)255;
    if (off + bytes > a.size) return RFDE_ENOMEM;
    *ptr = a.base + off;
    a.used = off + bytes;
    return RFDE_OK;
  }
  return dev_alloc(ptr, bytes);
}

template <typename T>
static int dalloc(Plan* p, T** ptr, size_t count, size_t* acc) {
  if (count == 0) count = 1;
  RFDE_TRY(palloc(p, (void**)ptr, count * sizeof(T)));
  if (acc) *acc += count * sizeof(T);
  return RFDE_OK;
}

size_t workspace_estimate(const Plan& p) {
  const size_t N = p.N();
  const size_t m = (size_t)p.opts.restart;
  const size_t csz = p.opts.precond_bits == 32 ? 8 : 16;
  const bool bs = p.bs[0].LB || p.bs[1].LB;
  const size_t gs = p.opts.spatial == RFDE_SPATIAL_TOEPLITZ
                        ? (size_t)p.nf * (3 * (size_t)p.M + p.L) * sizeof(double2) : 0;
  const size_t inner = p.dim == 2 ? inner_workspace_bytes(p.opts.inner_iters, p.nf, p.S) : 0;
  return gs + inner + (2 * m + 1 + 3) * N * 8 + (size_t)p.nf * p.S * csz * (bs ? 2 : 1) +
         ((size_t)70 * 1024) * 8 +
         (size_t)(p.L + p.Lx + p.Ly + 4 * p.Lt + 3 * p.Nt + 2 * (p.bs[0].LB + p.bs[1].LB) +
                  p.M + p.Mx + p.My + 4) * 24;
}

// Axes of a tau plan whose DST-I length n has 2(n+1) not a power of two take the chirp-z
// route: record n and the cyclic length.
static void plan_dst_axes(Plan* p) {
  if (p->opts.spatial != RFDE_SPATIAL_TAU) return;
  const int n0 = p->dim == 1 ? p->M : p->Mx;
  if (!is_pow2(n0 + 1)) { p->bs[0].n = n0; p->bs[0].LB = dstbs_length(n0); }
  if (p->dim == 2 && !is_pow2(p->My + 1)) { p->bs[1].n = p->My; p->bs[1].LB = dstbs_length(p->My); }
}

// Everything common to 1D and 2D plans once the sizes are known.  factor = false leaves the
// factor storage allocated but unfilled (a batch factors its instances together).
int plan_allocate_and_setup(Plan* p, bool factor) {
  const auto t0 = std::chrono::steady_clock::now();
  RFDE_HIP(hipSetDevice(p->device));
  const size_t wsz = workspace_estimate(*p);
  size_t freeb = 0, totalb = 0;
  RFDE_HIP(hipMemGetInfo(&freeb, &totalb));
  if (!p->arena && p->factor_bytes + wsz > freeb + dev_cached_bytes(p->device)) return RFDE_ENOMEM;

  size_t ws = 0;
  const int gl = p->dim == 1 ? p->M : p->Mx + p->My;
  RFDE_TRY(dalloc(p, &p->g, gl, &ws));
  const int symlen = p->dim == 1 ? p->L / 2 + 1 : (p->Lx / 2 + 1) + (p->Ly / 2 + 1);
  RFDE_TRY(dalloc(p, &p->sym, symlen, &ws));
  RFDE_TRY(dalloc(p, &p->twL, p->dim == 1 ? p->L : p->Lx + p->Ly, &ws));
  RFDE_TRY(dalloc(p, &p->twNt, p->Lt, &ws));
  RFDE_TRY(dalloc(p, &p->twNt32, p->Lt, &ws));
  if (p->Lt != p->Nt) {
    RFDE_TRY(dalloc(p, &p->chirp, p->Nt, &ws));
    RFDE_TRY(dalloc(p, &p->chirp32, p->Nt, &ws));
    RFDE_TRY(dalloc(p, &p->bhat, p->Lt, &ws));
    RFDE_TRY(dalloc(p, &p->bhat32, p->Lt, &ws));
  }
  RFDE_TRY(dalloc(p, &p->s, p->Nt, &ws));
  RFDE_TRY(dalloc(p, &p->lambda, p->nf, &ws));
  RFDE_TRY(dalloc(p, &p->sigma, gl, &ws));
  const size_t csz = p->opts.precond_bits == 32 ? 8 : 16;
  RFDE_TRY(palloc(p, &p->zf, (size_t)p->nf * p->S * csz));
  ws += (size_t)p->nf * p->S * csz;
  if (p->opts.spatial == RFDE_SPATIAL_TOEPLITZ) {
    RFDE_TRY(dalloc(p, &p->gs_x, (size_t)p->nf * p->M, &ws));
    RFDE_TRY(dalloc(p, &p->gs_xhat, (size_t)p->nf * p->L, &ws));
    RFDE_TRY(dalloc(p, &p->gs_p, (size_t)p->nf * p->M, &ws));
    RFDE_TRY(dalloc(p, &p->gs_q, (size_t)p->nf * p->M, &ws));
  }
  if (p->dim == 2 && p->opts.inner_iters > 0) {
    InnerWs& I = p->inner;
    const int k = p->opts.inner_iters;
    const size_t vec = (size_t)p->nf * p->S, nfr = p->nf;
    constexpr size_t KS = INNER_KMAX + 1;
    I.nblk = inner_blocks(p->S);
    RFDE_TRY(dalloc(p, &I.V, (k + 1) * vec, &ws));
    RFDE_TRY(dalloc(p, &I.Z, k * vec, &ws));
    RFDE_TRY(dalloc(p, &I.w, vec, &ws));
    RFDE_TRY(dalloc(p, &I.part, nfr * I.nblk * (KS + 1), &ws));
    RFDE_TRY(dalloc(p, &I.h1, nfr * (KS + 1), &ws));
    RFDE_TRY(dalloc(p, &I.h2, nfr * (KS + 1), &ws));
    RFDE_TRY(dalloc(p, &I.R, nfr * INNER_KMAX * KS, &ws));
    RFDE_TRY(dalloc(p, &I.gsn, nfr * INNER_KMAX, &ws));
    RFDE_TRY(dalloc(p, &I.g, nfr * KS, &ws));
    RFDE_TRY(dalloc(p, &I.y, nfr * INNER_KMAX, &ws));
    RFDE_TRY(dalloc(p, &I.gc, nfr * INNER_KMAX, &ws));
    RFDE_TRY(dalloc(p, &I.beta, nfr, &ws));
    RFDE_TRY(dalloc(p, &I.scale, nfr, &ws));
    RFDE_TRY(dalloc(p, &I.res, nfr, &ws));
  }
  for (DstBsAxis& x : p->bs) {
    if (!x.LB) continue;
    RFDE_TRY(dalloc(p, &x.chirp, x.n + 1, &ws));
    RFDE_TRY(dalloc(p, &x.chirp32, x.n + 1, &ws));
    RFDE_TRY(dalloc(p, &x.khat, x.LB, &ws));
    RFDE_TRY(dalloc(p, &x.khat32, x.LB, &ws));
    RFDE_TRY(dalloc(p, &x.tw, x.LB, &ws));
    RFDE_TRY(dalloc(p, &x.tw32, x.LB, &ws));
    if (!p->zt) {
      RFDE_TRY(palloc(p, &p->zt, (size_t)p->nf * p->S * csz));
      ws += (size_t)p->nf * p->S * csz;
    }
  }
  const size_t N = p->N();
  const size_t m = (size_t)p->opts.restart;
  RFDE_TRY(dalloc(p, &p->vbuf, (m + 1) * N, &ws));
  RFDE_TRY(dalloc(p, &p->zbuf, m * N, &ws));
  RFDE_TRY(dalloc(p, &p->wvec, N, &ws));
  RFDE_TRY(dalloc(p, &p->xvec, N, &ws));
  RFDE_TRY(dalloc(p, &p->Fvec, N, &ws));
  RFDE_TRY(dalloc(p, &p->red, CGS2_RED_SIZE, &ws));
  RFDE_TRY(dalloc(p, &p->redout, CGS2_OUT_SIZE, &ws));
  // written by the Arnoldi kernels and read by the host after an event wait: mapped and
  // coherent, so the writes go straight to host memory
  RFDE_HIP(hipHostMalloc((void**)&p->hred, 256 * sizeof(double),
                         hipHostMallocMapped | hipHostMallocCoherent));
  for (auto& e : p->ev) RFDE_HIP(hipEventCreate(&e));
  p->workspace_bytes = ws;
  if (p->factor_bytes) {
    RFDE_TRY(palloc(p, &p->factors, p->factor_bytes));
    BlockSet hs{};
    hs.count = 1;
    set_family(hs, 0, *p);
    RFDE_TRY(dalloc(p, &p->set, 1, &ws));
    p->workspace_bytes = ws;
    RFDE_HIP(hipMemcpy(p->set, &hs, sizeof(BlockSet), hipMemcpyHostToDevice));
  }

  hipStream_t st = p->stream;
  if (p->dim == 1) {
    RFDE_TRY(launch_gk(p->alpha, p->M, p->g, st));
    RFDE_TRY(launch_twiddles(p->twL, p->L, st));
    RFDE_TRY(launch_symbol(p->g, p->M, p->L, p->coef / p->L, p->twL, p->sym, st));
  } else {
    RFDE_TRY(launch_gk(p->alpha_x, p->Mx, p->g, st));
    RFDE_TRY(launch_gk(p->alpha_y, p->My, p->g + p->Mx, st));
    RFDE_TRY(launch_twiddles(p->twL, p->Lx, st));
    RFDE_TRY(launch_twiddles(p->twL + p->Lx, p->Ly, st));
    RFDE_TRY(launch_symbol(p->g, p->Mx, p->Lx, p->coef_x / p->Lx, p->twL, p->sym, st));
    RFDE_TRY(launch_symbol(p->g + p->Mx, p->My, p->Ly, p->coef_y / p->Ly, p->twL + p->Lx,
                           p->sym + (p->Lx / 2 + 1), st));
  }
  if (p->opts.spatial == RFDE_SPATIAL_TAU) {
    // DST twiddles: double tables (length 2(n+1) per axis), then the same in float
    const int P0 = p->dim == 1 ? 2 * (p->M + 1) : 2 * (p->Mx + 1);
    const int P1 = p->dim == 1 ? 0 : 2 * (p->My + 1);
    const int Ptot = P0 + P1;
    RFDE_TRY(palloc(p, (void**)&p->twD, (size_t)Ptot * (sizeof(double2) + sizeof(float2))));
    p->workspace_bytes += (size_t)Ptot * (sizeof(double2) + sizeof(float2));
    float2* tf = reinterpret_cast<float2*>(p->twD + Ptot);
    RFDE_TRY(launch_twiddles(p->twD, P0, st));
    RFDE_TRY(launch_twiddles32(tf, P0, st));
    if (P1) {
      RFDE_TRY(launch_twiddles(p->twD + P0, P1, st));
      RFDE_TRY(launch_twiddles32(tf + P0, P1, st));
    }
    // tau eigenvalues (eq. (3.10)), sines taken from the DST tables
    if (p->dim == 1) {
      RFDE_TRY(launch_tau_sigma(p->g, p->M, p->twD, p->sigma, st));
    } else {
      RFDE_TRY(launch_tau_sigma(p->g, p->Mx, p->twD, p->sigma, st));
      RFDE_TRY(launch_tau_sigma(p->g + p->Mx, p->My, p->twD + P0, p->sigma + p->Mx, st));
    }
    for (int a = 0; a < 2; ++a)
      if (p->bs[a].LB) RFDE_TRY(dstbs_setup_axis(*p, a));
  }
  RFDE_TRY(launch_twiddles(p->twNt, p->Lt, st));
  RFDE_TRY(launch_twiddles32(p->twNt32, p->Lt, st));
  RFDE_TRY(launch_bluestein_setup(*p));
  RFDE_TRY(launch_time_data(p->Nt, p->eps, p->s, p->lambda, st));
  if (p->opts.spatial == RFDE_SPATIAL_TOEPLITZ) {
    RFDE_HIP(hipEventRecord(p->ev[0], st));
    RFDE_TRY(launch_gs_setup(*p));
    RFDE_HIP(hipEventRecord(p->ev[1], st));
  }
  if (p->factor_bytes && factor) {
    RFDE_HIP(hipEventRecord(p->ev[0], st));
    RFDE_TRY(launch_factorize(*p));
    RFDE_HIP(hipEventRecord(p->ev[1], st));
  }
  RFDE_HIP(hipStreamSynchronize(st));
  if ((p->factor_bytes && factor) || p->opts.spatial == RFDE_SPATIAL_TOEPLITZ) {
    float t = 0.f;
    RFDE_HIP(hipEventElapsedTime(&t, p->ev[0], p->ev[1]));
    p->ms_factor = t;
  }
  p->ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return RFDE_OK;
}

static bool opts_ok(const rfde_opts& o) {
  return o.tol > 0 && o.maxit >= 1 && o.restart >= 1 && o.restart <= 64 && o.circ_eps <= 1.0 &&
         (o.precond_bits == 64 || o.precond_bits == 32) &&
         (o.spatial == RFDE_SPATIAL_EXACT || o.spatial == RFDE_SPATIAL_TAU ||
          o.spatial == RFDE_SPATIAL_TOEPLITZ) &&
         o.inner_iters >= 0 && o.inner_iters <= INNER_KMAX && o.inner_tol >= 0.0 &&
         std::isfinite(o.inner_tol);
}

// ---- steps ----
static int pinv_step_b(const Plan& p, const void* z1, void* z2) {
  if (p.dim == 2 && p.opts.inner_iters > 0) return launch_inner_step_b(p, z1, z2);
  if (p.opts.spatial == RFDE_SPATIAL_EXACT) return launch_trsv(p, z1, z2);
  if (p.opts.spatial == RFDE_SPATIAL_TOEPLITZ) return launch_gs_apply(p, z1, z2);
  return launch_tau_solve(p, z1, z2);
}

// z = P^-1 (v * vs[0]) (vs == nullptr: P^-1 v), as step (a) into the plan's frequency buffer
// (pinv_head) and steps (b), (c) from it (pinv_tail)
static int pinv_head(Plan& p, const double* v, const double* vs) {
  return launch_time_fwd_scaled(p, v, p.zf, vs);
}
static int pinv_tail(Plan& p, double* z) {
  RFDE_TRY(pinv_step_b(p, p.zf, p.zf));
  return launch_time_inv(p, p.zf, z);
}

int apply_pinv(Plan& p, const double* v, double* z) {
  RFDE_TRY(pinv_head(p, v, nullptr));
  return pinv_tail(p, z);
}

int plan_init_1d(Plan* p, double alpha, double kappa, double a, double b, int M, int Nt,
                 double T, rfde_opts o, hipStream_t stream) {
  if (!(alpha > 1.0 && alpha <= 2.0) || !(kappa > 0.0) || !(b > a) || M < 1 || M > 4096 ||
      !nt_ok(Nt) || !(T > 0.0) || !opts_ok(o) || !std::isfinite(alpha + kappa + a + b + T))
    return RFDE_EINVAL;
  p->dim = 1;
  p->M = M; p->S = M; p->Nt = Nt; p->nf = Nt / 2 + 1; p->Lt = time_length(Nt);
  p->alpha = alpha; p->kappa = kappa;
  p->h = (b - a) / (M + 1);
  p->tau = T / Nt;
  p->eps = o.circ_eps > 0 ? o.circ_eps : std::min(0.5, 0.5 * p->tau);
  o.circ_eps = p->eps;
  p->coef = p->tau * kappa / std::pow(p->h, alpha);
  p->L = std::max(16, next_pow2(2 * M - 1));
  p->opts = o;
  p->stream = stream;
  plan_dst_axes(p);
  if (o.spatial == RFDE_SPATIAL_TOEPLITZ && o.precond_bits != 64) return RFDE_EUNSUPPORTED;
  if (o.inner_iters > 0) return RFDE_EUNSUPPORTED;  // the inner solver is a 2D option
  if (o.spatial == RFDE_SPATIAL_EXACT) {
    p->T = (M + TILE - 1) / TILE;
    p->Mp = p->T * TILE;
    p->dual = (Nt % 2) == 0;
    p->nb = p->nf - (p->dual ? 1 : 0);
    const size_t csz = o.precond_bits == 32 ? 8 : 16;
    p->factor_bytes = (size_t)p->nb * lower_tiles(p->T) * TILE_ELEMS * csz;
  }
  return RFDE_OK;
}

}  // namespace rfde

using namespace rfde;

extern "C" {

void rfde_opts_default(rfde_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->maxit = 200;
  o->restart = 30;
  o->circ_eps = 0.0;
  o->precond_bits = 64;
  o->spatial = RFDE_SPATIAL_EXACT;
  o->inner_iters = 0;
  o->inner_tol = 0.0;
}

const char* rfde_strerror(int s) {
  switch (s) {
    case RFDE_OK: return "ok";
    case RFDE_ENOTCONV: return "not converged within maxit (best iterate returned)";
    case RFDE_EINVAL: return "invalid argument";
    case RFDE_ENOMEM: return "out of device memory";
    case RFDE_EHIP: return "HIP runtime error";
    case RFDE_ENAN: return "non-finite value encountered";
    case RFDE_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int rfde_gk(double alpha, int n, double* g, void* hip_stream) {
  if (!(alpha > 0.0 && alpha <= 2.0) || n < 1 || !g) return RFDE_EINVAL;
  return launch_gk(alpha, n, g, (hipStream_t)hip_stream);
}

int rfde_plan_create_1d(rfde_plan* plan, double alpha, double kappa, double a, double b, int M,
                        int Nt, double T, const rfde_opts* opts, void* hip_stream) {
  if (!plan) return RFDE_EINVAL;
  *plan = nullptr;
  rfde_opts o;
  rfde_opts_default(&o);
  if (opts) o = *opts;
  Plan* p = new (std::nothrow) Plan();
  if (!p) return RFDE_ENOMEM;
  int rc = plan_init_1d(p, alpha, kappa, a, b, M, Nt, T, o, (hipStream_t)hip_stream);
  if (rc != RFDE_OK) { delete p; return rc; }
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return RFDE_EHIP; }
  rc = plan_allocate_and_setup(p, true);
  if (rc != RFDE_OK) { free_plan(p); return rc; }
  *plan = reinterpret_cast<rfde_plan>(p);
  return RFDE_OK;
}

int rfde_plan_create_2d(rfde_plan* plan, double alpha_x, double alpha_y, double kappa_x,
                        double kappa_y, double ax, double bx, double ay, double by, int Mx, int My,
                        int Nt, double T, const rfde_opts* opts, void* hip_stream) {
  if (!plan) return RFDE_EINVAL;
  *plan = nullptr;
  rfde_opts o;
  rfde_opts_default(&o);
  if (opts) o = *opts;
  o.spatial = RFDE_SPATIAL_TAU;
  if (!(alpha_x > 1.0 && alpha_x <= 2.0) || !(alpha_y > 1.0 && alpha_y <= 2.0) ||
      !(kappa_x > 0.0) || !(kappa_y > 0.0) || !(bx > ax) || !(by > ay) || Mx < 1 || My < 1 ||
      Mx > 4096 || My > 4096 || !nt_ok(Nt) || !(T > 0.0) || !opts_ok(o) ||
      !std::isfinite(alpha_x + alpha_y + kappa_x + kappa_y + ax + bx + ay + by + T))
    return RFDE_EINVAL;
  if (o.inner_iters > 0 && o.precond_bits != 64) return RFDE_EUNSUPPORTED;
  Plan* p = new (std::nothrow) Plan();
  if (!p) return RFDE_ENOMEM;
  p->dim = 2;
  p->Mx = Mx; p->My = My; p->M = Mx * My; p->S = Mx * My;
  p->Nt = Nt; p->nf = Nt / 2 + 1; p->Lt = time_length(Nt);
  p->alpha_x = alpha_x; p->alpha_y = alpha_y; p->kappa_x = kappa_x; p->kappa_y = kappa_y;
  p->hx = (bx - ax) / (Mx + 1);
  p->hy = (by - ay) / (My + 1);
  p->tau = T / Nt;
  p->eps = o.circ_eps > 0 ? o.circ_eps : std::min(0.5, 0.5 * p->tau);
  o.circ_eps = p->eps;
  p->coef_x = p->tau * kappa_x / std::pow(p->hx, alpha_x);
  p->coef_y = p->tau * kappa_y / std::pow(p->hy, alpha_y);
  p->Lx = std::max(16, next_pow2(2 * Mx - 1));
  p->Ly = std::max(16, next_pow2(2 * My - 1));
  p->opts = o;
  p->stream = (hipStream_t)hip_stream;
  plan_dst_axes(p);
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return RFDE_EHIP; }
  const int rc = plan_allocate_and_setup(p, true);
  if (rc != RFDE_OK) { free_plan(p); return rc; }
  *plan = reinterpret_cast<rfde_plan>(p);
  return RFDE_OK;
}

int rfde_plan_destroy(rfde_plan plan) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return RFDE_OK;
  (void)hipStreamSynchronize(p->stream);
  free_plan(p);
  return RFDE_OK;
}

int rfde_plan_get_info(rfde_plan plan, rfde_plan_info* info) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !info) return RFDE_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->dim = p->dim;
  info->M = p->M; info->Mx = p->Mx; info->My = p->My;
  info->Nt = p->Nt; info->n_freq = p->nf;
  info->L = p->L; info->Lx = p->Lx; info->Ly = p->Ly;
  info->Mp = p->Mp;
  info->h = p->h; info->hx = p->hx; info->hy = p->hy;
  info->tau = p->tau; info->circ_eps = p->eps;
  info->coef = p->coef; info->coef_x = p->coef_x; info->coef_y = p->coef_y;
  info->factor_bytes = p->factor_bytes;
  info->workspace_bytes = p->workspace_bytes;
  info->precond_bits = p->opts.precond_bits;
  info->spatial = p->opts.spatial;
  info->ms_setup = p->ms_setup;
  info->ms_factor = p->ms_factor;
  return RFDE_OK;
}

int rfde_plan_export(rfde_plan plan, int what, int index, void* dst) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !dst) return RFDE_EINVAL;
  hipStream_t st = p->stream;
  const int gl = p->dim == 1 ? p->M : p->Mx + p->My;
  switch (what) {
    case RFDE_EXPORT_GK:
      RFDE_HIP(hipMemcpyAsync(dst, p->g, gl * sizeof(double), hipMemcpyDeviceToDevice, st));
      return RFDE_OK;
    case RFDE_EXPORT_SYMBOL: {
      const int n = p->dim == 1 ? p->L / 2 + 1 : (p->Lx / 2 + 1) + (p->Ly / 2 + 1);
      RFDE_HIP(hipMemcpyAsync(dst, p->sym, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      return RFDE_OK;
    }
    case RFDE_EXPORT_LAMBDA:
      RFDE_HIP(hipMemcpyAsync(dst, p->lambda, p->nf * sizeof(double2), hipMemcpyDeviceToDevice, st));
      return RFDE_OK;
    case RFDE_EXPORT_SCALE:
      RFDE_HIP(hipMemcpyAsync(dst, p->s, p->Nt * sizeof(double), hipMemcpyDeviceToDevice, st));
      return RFDE_OK;
    case RFDE_EXPORT_FACTOR:
      if (!p->factor_bytes || index < 0 || index >= p->nf) return RFDE_EINVAL;
      return launch_export_factor(*p, index, dst);
    case RFDE_EXPORT_TOEPLITZ_X:
      if (p->opts.spatial != RFDE_SPATIAL_TOEPLITZ || index < 0 || index >= p->nf)
        return RFDE_EINVAL;
      RFDE_HIP(hipMemcpyAsync(dst, p->gs_x + (size_t)index * p->M, p->M * sizeof(double2),
                              hipMemcpyDeviceToDevice, st));
      return RFDE_OK;
    case RFDE_EXPORT_TAU_SIGMA:
      if (p->opts.spatial != RFDE_SPATIAL_TAU) return RFDE_EINVAL;  // only tau plans hold sigma
      RFDE_HIP(hipMemcpyAsync(dst, p->sigma, gl * sizeof(double), hipMemcpyDeviceToDevice, st));
      return RFDE_OK;
    default:
      return RFDE_EINVAL;
  }
}

int rfde_build_rhs(rfde_plan plan, const double* u0, const double* f, double* F) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !u0 || !f || !F) return RFDE_EINVAL;
  return launch_rhs(*p, u0, f, F);
}

int rfde_apply_A(rfde_plan plan, const double* v, double* y) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !v || !y || v == y) return RFDE_EINVAL;
  return launch_matvec(*p, v, y);
}

int rfde_pinv_step_a(rfde_plan plan, const double* v, void* z1) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !v || !z1) return RFDE_EINVAL;
  if (p->opts.precond_bits == 32) {
    RFDE_TRY(launch_time_fwd(*p, v, p->zf));
    return launch_widen(*p, p->zf, (double2*)z1);
  }
  return launch_time_fwd(*p, v, z1);
}

int rfde_pinv_step_b(rfde_plan plan, const void* z1, void* z2) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !z1 || !z2) return RFDE_EINVAL;
  if (p->opts.precond_bits == 32) {
    RFDE_TRY(launch_narrow(*p, (const double2*)z1, p->zf));
    RFDE_TRY(pinv_step_b(*p, p->zf, p->zf));
    return launch_widen(*p, p->zf, (double2*)z2);
  }
  return pinv_step_b(*p, z1, z2);
}

int rfde_pinv_step_c(rfde_plan plan, const void* z2, double* v) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !z2 || !v) return RFDE_EINVAL;
  if (p->opts.precond_bits == 32) {
    RFDE_TRY(launch_narrow(*p, (const double2*)z2, p->zf));
    return launch_time_inv(*p, p->zf, v);
  }
  return launch_time_inv(*p, z2, v);
}

int rfde_apply_Pinv(rfde_plan plan, const double* v, double* z) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !v || !z) return RFDE_EINVAL;
  return apply_pinv(*p, v, z);
}

int rfde_solve(rfde_plan plan, const double* u0, const double* f, const double* U_init, double* U,
               double tol, rfde_stats* stats) {
  Plan* pp = reinterpret_cast<Plan*>(plan);
  if (!pp || !u0 || !f || !U) return RFDE_EINVAL;
  Plan& p = *pp;
  const auto t0 = std::chrono::steady_clock::now();
  if (!(tol > 0)) tol = p.opts.tol;
  const int m = p.opts.restart;
  const size_t N = p.N();
  hipStream_t st = p.stream;
  double* hr = p.hred;
  double* hr_dev = nullptr;  // the same pinned buffer in the device address space
  RFDE_HIP(hipHostGetDevicePointer((void**)&hr_dev, hr, 0));
  // marks the end of an Arnoldi step's column in the stream (no timing: a timed event stalls
  // the queue for a few microseconds)
  hipEvent_t ev_col = nullptr;
  RFDE_HIP(hipEventCreateWithFlags(&ev_col, hipEventDisableTiming));
  struct EventGuard {
    hipEvent_t e;
    ~EventGuard() { (void)hipEventDestroy(e); }
  } ev_guard{ev_col};
  rfde_stats loc;
  std::memset(&loc, 0, sizeof(loc));
  // Only the first preconditioner application and the first matvec of a solve are timed (an
  // event pair in the stream costs a few microseconds of idle GPU per step); the reported
  // estimates are those times multiplied by the number of applications.
  float t_pinv = -1.f, t_mv = -1.f;
  int n_pinv = 0, n_mv = 0;

  auto fetch = [&](int count) -> int {
    RFDE_HIP(hipMemcpyAsync(hr, p.redout, count * sizeof(double), hipMemcpyDeviceToHost, st));
    RFDE_HIP(hipStreamSynchronize(st));
    return RFDE_OK;
  };
  auto timed_matvec = [&](const double* v, double* y) -> int {
    if (n_mv++ == 0) RFDE_HIP(hipEventRecord(p.ev[2], st));
    RFDE_TRY(launch_matvec(p, v, y));
    if (n_mv == 1) RFDE_HIP(hipEventRecord(p.ev[3], st));
    return RFDE_OK;
  };
  // after a synchronisation: read the first application's times once
  auto read_times = [&]() -> int {
    if (t_mv < 0.f && n_mv > 0) RFDE_HIP(hipEventElapsedTime(&t_mv, p.ev[2], p.ev[3]));
    if (t_pinv < 0.f && n_pinv > 0) RFDE_HIP(hipEventElapsedTime(&t_pinv, p.ev[0], p.ev[1]));
    return RFDE_OK;
  };

  RFDE_TRY(launch_rhs(p, u0, f, p.Fvec));
  RFDE_TRY(launch_nrm2(p, p.Fvec, p.redout));
  RFDE_TRY(fetch(1));
  const double bnorm = hr[0];
  if (!std::isfinite(bnorm)) return RFDE_ENAN;
  if (bnorm == 0.0) {
    RFDE_HIP(hipMemsetAsync(U, 0, N * sizeof(double), st));
    RFDE_HIP(hipStreamSynchronize(st));
    loc.converged = 1;
    if (stats) *stats = loc;
    return RFDE_OK;
  }
  // x = U_init (or 0); r = F - A x
  double* x = p.xvec;
  double* r = p.vbuf;  // first basis vector slot holds r, normalised in place
  if (U_init) {
    RFDE_HIP(hipMemcpyAsync(x, U_init, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    RFDE_TRY(timed_matvec(x, p.wvec));
    RFDE_TRY(launch_sub(p, p.Fvec, p.wvec, r));
  } else {
    RFDE_HIP(hipMemsetAsync(x, 0, N * sizeof(double), st));
    RFDE_HIP(hipMemcpyAsync(r, p.Fvec, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  RFDE_TRY(launch_nrm2(p, r, p.redout));
  RFDE_TRY(fetch(1));
  RFDE_TRY(read_times());
  double beta = hr[0];
  if (U_init && !(beta < bnorm)) {
    // the guess does not reduce the residual: fall back to the zero start
    RFDE_HIP(hipMemsetAsync(x, 0, N * sizeof(double), st));
    RFDE_HIP(hipMemcpyAsync(r, p.Fvec, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    RFDE_HIP(hipMemcpyAsync(p.redout, &bnorm, sizeof(double), hipMemcpyHostToDevice, st));
    beta = bnorm;
  }
  if (!std::isfinite(beta)) return RFDE_ENAN;
  loc.res_hist[0] = beta / bnorm;
  loc.n_hist = 1;
  int total = 0;
  double rel = beta / bnorm;
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gvec(m + 1), y(m);
  while (rel > tol && total < p.opts.maxit) {
    // u_0 = r (already in the first basis slot), |u_0| = beta
    RFDE_TRY(launch_cgs2_start(p, beta, p.redout));
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gvec.begin(), gvec.end(), 0.0);
    gvec[0] = beta;
    int k = 0;
    bool breakdown = false;
    bool head_done = false;  // step (a) of this step's P^-1 already queued
    for (int j = 0; j < m; ++j) {
      double* vj = p.vbuf + (size_t)j * N;
      double* zj = p.zbuf + (size_t)j * N;
      double* vn = p.vbuf + (size_t)(j + 1) * N;
      // z_j = P^-1 (u_j / |u_j|), the direction of step j (the flexible variant allows any)
      if (n_pinv == 0) RFDE_HIP(hipEventRecord(p.ev[0], st));
      if (!head_done) RFDE_TRY(pinv_head(p, vj, p.redout + CGS2_VS + j));
      RFDE_TRY(pinv_tail(p, zj));
      if (n_pinv++ == 0) RFDE_HIP(hipEventRecord(p.ev[1], st));
      RFDE_TRY(timed_matvec(zj, vn));
      // classical Gram-Schmidt, twice (CGS2), in two sweeps over the stored vectors; the
      // kernels leave h1, h2 and n in the mapped host buffer
      RFDE_TRY(launch_cgs2(p, p.vbuf, j + 1, vn, p.redout, hr_dev));
      RFDE_HIP(hipEventRecord(ev_col, st));
      // Step (a) of the next step needs only u_{j+1} and its scale, both on the device: queue
      // it before waiting for the column, so the GPU works while the host reads it (wasted only
      // if this step turns out to be the last)
      head_done = j + 1 < m && total + 1 < p.opts.maxit;
      if (head_done) RFDE_TRY(pinv_head(p, vn, p.redout + CGS2_VS + j + 1));
      RFDE_HIP(hipEventSynchronize(ev_col));
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hr[i] + hr[CGS2_H2 + i];
      const double hn = hr[CGS2_NRM];
      RFDE_TRY(read_times());
      if (!std::isfinite(hn)) return RFDE_ENAN;
      H[(size_t)(j + 1) * m + j] = hn;
      if (!(hn > 0.0)) breakdown = true;
      // apply previous rotations, then a new one
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
      const double d = std::hypot(a, b);
      cs[j] = a / d;
      sn[j] = b / d;
      H[(size_t)j * m + j] = d;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = cs[j] * gvec[j];
      ++total;
      k = j + 1;
      const double est = std::fabs(gvec[j + 1]) / bnorm;
      if (loc.n_hist < 256) loc.res_hist[loc.n_hist++] = est;
      if (est <= tol || total >= p.opts.maxit || breakdown) break;
    }
    // y = H(0:k,0:k)^{-1} g; x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double s = gvec[i];
      for (int c = i + 1; c < k; ++c) s -= H[(size_t)i * m + c] * y[c];
      y[i] = s / H[(size_t)i * m + i];
    }
    RFDE_HIP(hipMemcpyAsync(p.redout, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
    RFDE_TRY(launch_multi_axpy(p, x, p.zbuf, k, p.redout, 1.0));
    // true residual
    RFDE_TRY(timed_matvec(x, p.wvec));
    RFDE_TRY(launch_sub(p, p.Fvec, p.wvec, r));
    RFDE_TRY(launch_nrm2(p, r, p.redout));
    RFDE_TRY(fetch(1));
    beta = hr[0];
    if (!std::isfinite(beta)) return RFDE_ENAN;
    rel = beta / bnorm;
    ++loc.restarts;
    if (breakdown) break;
  }
  RFDE_HIP(hipMemcpyAsync(U, x, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  RFDE_HIP(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  loc.iters = total;
  loc.true_rel_res = rel;
  loc.converged = rel <= tol ? 1 : 0;
  loc.ms_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
  loc.n_pinv = n_pinv;
  loc.n_matvec = n_mv;
  loc.ms_pinv_est = n_pinv > 0 ? (double)t_pinv * n_pinv : 0.0;
  loc.ms_setup = p.ms_setup;
  loc.ms_matvec_est = n_mv > 0 ? (double)t_mv * n_mv : 0.0;
  if (stats) *stats = loc;
  return loc.converged ? RFDE_OK : RFDE_ENOTCONV;
}

}  // extern "C"
