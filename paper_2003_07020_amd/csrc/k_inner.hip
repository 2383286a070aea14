// Optional inner solver of the 2D preconditioner step (b).  The paper solves the shifted
// systems of eq. (4.5) with the tau approximation only; with opts.inner_iters = k > 0 each
// frequency n instead takes up to k GMRES steps on the exact shifted operator
//   B_n = lambda_n I - tau A = lambda_n I + coef_x T_x (on x) + coef_y T_y (on y),
// from a zero start, right-preconditioned by that frequency's tau solve (the flexible outer
// iteration absorbs the change of preconditioner between applications).
//
// All frequencies advance in lockstep on the [nf][My][Mx] complex array:
//   z_j = P_tau^{-1} v_j (the tau solve of every frequency), w = B z_j (two FFT passes),
//   classical Gram-Schmidt applied twice against v_0..v_j with Hermitian inner products
//   (per-frequency sums in a fixed order), h_{j+1,j} = ||w|| by Pythagoras after the second
//   projection, v_{j+1} = w / h_{j+1,j};
// each frequency's Hessenberg column is reduced by complex Givens rotations (one thread per
// frequency), which also gives its residual estimate |g_{j+1}|; after the last step
// x_n = sum_j y_j z_j with y = R^{-1} g.  With opts.inner_tol > 0 every frequency stops after
// the first step at which all of them have |g_{j+1}| <= inner_tol ||z1_n|| (the host reads
// the estimates after each step).
#include <algorithm>
#include <vector>

#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

constexpr int DOT_NT = 256;
constexpr int KS = INNER_KMAX + 1;  // per-frequency stride of the Hessenberg column and g

__device__ __forceinline__ double2 cmul_conj(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// x direction: y[r] = lambda_{r / My} v[r] + coef_x T_x v[r] for the complex rows r of the
// [nf][My][Mx] array (T_x v by circulant embedding: the symbol carries coef_x / L), NB rows
// per workgroup.
template <int L, int NB, int NT, int MAXR>
__global__ void __launch_bounds__(NT) k_inner_rows(const double2* __restrict__ v,
                                                   double2* __restrict__ y,
                                                   const double* __restrict__ sym,
                                                   const double2* __restrict__ tw,
                                                   const double2* __restrict__ lambda, int Mx,
                                                   int My, int nrows) {
  __shared__ double2 buf[NB * L];
  const int r0 = blockIdx.x * NB;
  auto load = [&](int f, int idx) -> double2 {
    const int r = r0 + f;
    return (r < nrows && idx < Mx) ? v[(size_t)r * Mx + idx] : make_double2(0.0, 0.0);
  };
  auto store_scaled = [&](int f, int k, double2 c) {
    const double s = sym[k <= L / 2 ? k : L - k];
    buf[f * L + k] = make_double2(c.x * s, c.y * s);
  };
  fft_io<L, -1, NT, NB, L, false, true, true, MAXR>(buf, tw, load, store_scaled);
  __syncthreads();
  auto store_out = [&](int f, int idx, double2 c) {
    const int r = r0 + f;
    if (r < nrows && idx < Mx) {
      const size_t i = (size_t)r * Mx + idx;
      y[i] = cadd(cmul(lambda[r / My], v[i]), c);
    }
  };
  NoLoad nl;
  fft_io<L, +1, NT, NB, L, false, false, true, MAXR>(buf, tw, nl, store_out);
}

// y direction: y += coef_y T_y v along the columns of every frequency, NB adjacent complex
// columns per workgroup (batch index fastest, so the row segments are contiguous).
template <int L, int NB, int NT, int MAXR>
__global__ void __launch_bounds__(NT) k_inner_cols(const double2* __restrict__ v,
                                                   double2* __restrict__ y,
                                                   const double* __restrict__ sym,
                                                   const double2* __restrict__ tw, int Mx,
                                                   int My) {
  constexpr int LDN = L + 1;
  __shared__ double2 buf[NB * LDN];
  const int ntile = (Mx + NB - 1) / NB;
  const int n = blockIdx.x / ntile, x0 = (blockIdx.x % ntile) * NB;
  const size_t base = (size_t)n * Mx * My;
  auto load = [&](int f, int iy) -> double2 {
    const int x = x0 + f;
    return (iy < My && x < Mx) ? v[base + (size_t)iy * Mx + x] : make_double2(0.0, 0.0);
  };
  auto store_scaled = [&](int f, int k, double2 c) {
    const double s = sym[k <= L / 2 ? k : L - k];
    buf[f * LDN + k] = make_double2(c.x * s, c.y * s);
  };
  fft_io<L, -1, NT, NB, LDN, true, true, true, MAXR>(buf, tw, load, store_scaled);
  __syncthreads();
  auto store_out = [&](int f, int iy, double2 c) {
    const int x = x0 + f;
    if (iy < My && x < Mx) {
      const size_t i = base + (size_t)iy * Mx + x;
      y[i] = cadd(y[i], c);
    }
  };
  NoLoad nl;
  fft_io<L, +1, NT, NB, LDN, true, false, true, MAXR>(buf, tw, nl, store_out);
}

// Block b's share of frequency n's sums: conj(V_j) . w for j < nv and |w|^2, written to
// part[((n * nblk) + b) * KS1 + j] (j = nv: the squared norm in .x).  Strided per-thread sums,
// wave shuffles, then the four wave totals: a fixed order.
constexpr int KS1 = KS + 1;
__global__ void __launch_bounds__(DOT_NT) k_inner_dots(const double2* __restrict__ V,
                                                       size_t vstride, int nv,
                                                       const double2* __restrict__ w, int S,
                                                       int nblk, double2* __restrict__ part) {
  const int n = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  double2 acc[KS];
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < KS; ++j) acc[j] = make_double2(0.0, 0.0);
  const size_t off = (size_t)n * S;
  for (int i = b * DOT_NT + t; i < S; i += nblk * DOT_NT) {
    const double2 wv = w[off + i];
    nrm = fma(wv.x, wv.x, fma(wv.y, wv.y, nrm));
#pragma unroll
    for (int j = 0; j < KS; ++j)
      if (j < nv) acc[j] = cadd(acc[j], cmul_conj(V[j * vstride + off + i], wv));
  }
  __shared__ double2 red[DOT_NT / 64][KS1];
  const int lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int j = 0; j <= KS; ++j) {
    if (j <= nv) {  // nv is uniform
      double2 v = j < nv ? acc[j < KS ? j : KS - 1] : make_double2(nrm, 0.0);
      for (int m = 32; m >= 1; m >>= 1) {
        v.x += __shfl_xor(v.x, m);
        v.y += __shfl_xor(v.y, m);
      }
      if (lane == 0) red[wv][j] = v;
    }
  }
  __syncthreads();
  if (t <= nv) {
    double2 s = red[0][t];
    for (int q = 1; q < DOT_NT / 64; ++q) s = cadd(s, red[q][t]);
    part[((size_t)n * nblk + b) * KS1 + t] = s;
  }
}

// out[n * KS1 + j] = sum over the blocks of part (j <= nv), in block order.
__global__ void k_inner_reduce(const double2* __restrict__ part, int nblk, int nv, int nf,
                               double2* __restrict__ out) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nf * (nv + 1)) return;
  const int n = id / (nv + 1), j = id % (nv + 1);
  double2 s = make_double2(0.0, 0.0);
  for (int b = 0; b < nblk; ++b) s = cadd(s, part[((size_t)n * nblk + b) * KS1 + j]);
  out[(size_t)n * KS1 + j] = s;
}

// dst = (init ? dst : 0) + sign * sum_{j < nv} c[n][j] V_j over all frequencies; c has stride
// cstride per frequency.
__global__ void k_inner_comb(double2* __restrict__ dst, int init, double sign,
                             const double2* __restrict__ V, size_t vstride, int nv,
                             const double2* __restrict__ c, int cstride, int S, int nf) {
  const size_t N = (size_t)nf * S;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(i / S);
    double2 acc = init ? dst[i] : make_double2(0.0, 0.0);
    for (int j = 0; j < nv; ++j) {
      const double2 t = cmul(c[(size_t)n * cstride + j], V[j * vstride + i]);
      acc = make_double2(acc.x + sign * t.x, acc.y + sign * t.y);
    }
    dst[i] = acc;
  }
}

// dst = src * scale[n] (per frequency).
__global__ void k_inner_scale(double2* __restrict__ dst, const double2* __restrict__ src,
                              const double* __restrict__ scale, int S, int nf) {
  const size_t N = (size_t)nf * S;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double s = scale[i / S];
    dst[i] = make_double2(src[i].x * s, src[i].y * s);
  }
}

// Per-frequency state of the small least-squares problem.
struct InnerState {
  double2* R;      // nf x KMAX columns of KS: the rotated Hessenberg matrix
  double* gc;      // nf x KMAX: Givens cosines (real)
  double2* gsn;    // nf x KMAX: Givens sines
  double2* g;      // nf x KS: rotated beta e_1
  double* beta;    // nf
  double* scale;   // nf: 1 / (norm of the next basis vector), 0 at a breakdown
  double* res;     // nf: |g_{j+1}| / beta (0 for a zero right-hand side)
  double2* y;      // nf x KMAX
};

// beta_n = ||z1_n|| from the reduced norm sums (index 0 of out), g = beta e_1.
__global__ void k_inner_start(const double2* __restrict__ out, InnerState st, int nf) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  const double b = sqrt(out[(size_t)n * KS1].x);
  st.beta[n] = b;
  st.scale[n] = b > 0.0 ? 1.0 / b : 0.0;
  for (int i = 0; i < KS; ++i) st.g[(size_t)n * KS + i] = make_double2(0.0, 0.0);
  st.g[(size_t)n * KS] = make_double2(b, 0.0);
  st.res[n] = b > 0.0 ? 1.0 : 0.0;
}

// Column j of the Hessenberg matrix: h_i = h1_i + h2_i (i <= j), h_{j+1} = sqrt(s - |h2|^2)
// with s = ||w||^2 before the second projection; apply the earlier rotations, form the new
// one, rotate g, record the residual estimate and the scale of v_{j+1}.
__global__ void k_inner_givens(const double2* __restrict__ h1, const double2* __restrict__ h2,
                               InnerState st, int j, int nf) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  double2 h[KS];
  double p2 = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double2 b = h2[(size_t)n * KS1 + i];
    h[i] = cadd(h1[(size_t)n * KS1 + i], b);
    p2 += b.x * b.x + b.y * b.y;
  }
  const double s2 = h2[(size_t)n * KS1 + j + 1].x - p2;
  const double hn = s2 > 0.0 ? sqrt(s2) : 0.0;
  st.scale[n] = hn > 0.0 ? 1.0 / hn : 0.0;
  // earlier rotations: [h_i; h_{i+1}] <- [c h_i + s h_{i+1}; -conj(s) h_i + c h_{i+1}]
  for (int i = 0; i < j; ++i) {
    const double c = st.gc[(size_t)n * INNER_KMAX + i];
    const double2 s = st.gsn[(size_t)n * INNER_KMAX + i];
    const double2 a = h[i], b = h[i + 1];
    h[i] = cadd(make_double2(c * a.x, c * a.y), cmul(s, b));
    h[i + 1] = csub(make_double2(c * b.x, c * b.y), cmul_conj(s, a));
  }
  // new rotation zeroing the real h_{j+1,j} = hn below a = h_j
  const double2 a = h[j];
  const double aa = sqrt(a.x * a.x + a.y * a.y);
  const double rho = sqrt(aa * aa + hn * hn);
  double c = 1.0;
  double2 s = make_double2(0.0, 0.0);
  double2 r = a;
  if (rho > 0.0) {
    const double2 ph = aa > 0.0 ? make_double2(a.x / aa, a.y / aa) : make_double2(1.0, 0.0);
    c = aa / rho;
    s = make_double2(ph.x * hn / rho, ph.y * hn / rho);
    r = make_double2(ph.x * rho, ph.y * rho);
  }
  st.gc[(size_t)n * INNER_KMAX + j] = c;
  st.gsn[(size_t)n * INNER_KMAX + j] = s;
  for (int i = 0; i < j; ++i) st.R[((size_t)n * INNER_KMAX + j) * KS + i] = h[i];
  st.R[((size_t)n * INNER_KMAX + j) * KS + j] = r;
  const double2 gj = st.g[(size_t)n * KS + j];
  st.g[(size_t)n * KS + j] = make_double2(c * gj.x, c * gj.y);
  const double2 gn = cmul_conj(s, gj);
  st.g[(size_t)n * KS + j + 1] = make_double2(-gn.x, -gn.y);
  const double b = st.beta[n];
  st.res[n] = b > 0.0 ? sqrt(gn.x * gn.x + gn.y * gn.y) / b : 0.0;
}

// y = R^{-1} g over the first `steps` columns (a zero pivot, from a breakdown or a zero
// right-hand side, gives a zero component).
__global__ void k_inner_backsolve(InnerState st, int steps, int nf) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  for (int i = steps - 1; i >= 0; --i) {
    double2 t = st.g[(size_t)n * KS + i];
    for (int m = i + 1; m < steps; ++m)
      t = csub(t, cmul(st.R[((size_t)n * INNER_KMAX + m) * KS + i], st.y[(size_t)n * INNER_KMAX + m]));
    const double2 d = st.R[((size_t)n * INNER_KMAX + i) * KS + i];
    const double dd = d.x * d.x + d.y * d.y;
    st.y[(size_t)n * INNER_KMAX + i] =
        dd > 0.0 ? make_double2((t.x * d.x + t.y * d.y) / dd, (t.y * d.x - t.x * d.y) / dd)
                 : make_double2(0.0, 0.0);
  }
}

constexpr int inner_nb(int L) { return L >= 4096 ? 1 : (4096 / L > 8 ? 8 : 4096 / L); }
constexpr int inner_maxr(int L) { return L <= 512 ? 8 : 16; }
constexpr int inner_nt(int L, int NB) {
  return (NB * L / inner_maxr(L) < 64) ? 64
                                       : (NB * L / inner_maxr(L) > 512 ? 512 : NB * L / inner_maxr(L));
}

template <int L>
static int inner_rows_t(const Plan& p, const double2* v, double2* y) {
  constexpr int NB = inner_nb(L), MAXR = inner_maxr(L), NT = inner_nt(L, NB);
  const int nrows = p.nf * p.My;
  k_inner_rows<L, NB, NT, MAXR><<<(nrows + NB - 1) / NB, NT, 0, p.stream>>>(
      v, y, p.sym, p.twL, p.lambda, p.Mx, p.My, nrows);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int L>
static int inner_cols_t(const Plan& p, const double2* v, double2* y) {
  constexpr int NB = inner_nb(L), MAXR = inner_maxr(L), NT = inner_nt(L, NB);
  const int ntile = (p.Mx + NB - 1) / NB;
  k_inner_cols<L, NB, NT, MAXR><<<p.nf * ntile, NT, 0, p.stream>>>(
      v, y, p.sym + (p.Lx / 2 + 1), p.twL + p.Lx, p.Mx, p.My);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

#define RFDE_INNER_L_SWITCH(Lval, FN, ...)      \
  switch (Lval) {                               \
    case 16: return FN<16>(__VA_ARGS__);        \
    case 32: return FN<32>(__VA_ARGS__);        \
    case 64: return FN<64>(__VA_ARGS__);        \
    case 128: return FN<128>(__VA_ARGS__);      \
    case 256: return FN<256>(__VA_ARGS__);      \
    case 512: return FN<512>(__VA_ARGS__);      \
    case 1024: return FN<1024>(__VA_ARGS__);    \
    case 2048: return FN<2048>(__VA_ARGS__);    \
    case 4096: return FN<4096>(__VA_ARGS__);    \
    case 8192: return FN<8192>(__VA_ARGS__);    \
    default: return RFDE_EINVAL;                \
  }

// w = B_n z for every frequency n
static int inner_apply_B(const Plan& p, const double2* z, double2* w) {
  const int rc = [&]() -> int { RFDE_INNER_L_SWITCH(p.Lx, inner_rows_t, p, z, w); }();
  if (rc != RFDE_OK) return rc;
  RFDE_INNER_L_SWITCH(p.Ly, inner_cols_t, p, z, w);
}

int inner_blocks(int S) { return std::max(1, std::min(64, (S + DOT_NT * 8 - 1) / (DOT_NT * 8))); }

size_t inner_workspace_bytes(int k, int nf, int S) {
  if (k <= 0) return 0;
  const size_t vec = (size_t)nf * S * sizeof(double2);
  const size_t nblk = inner_blocks(S);
  return (2 * (size_t)k + 2) * vec + (size_t)nf * nblk * KS1 * sizeof(double2) +
         (size_t)nf * (3 * KS1 + INNER_KMAX * (KS + 3) + KS + 4) * sizeof(double2);
}

static InnerState inner_state(const Plan& p) {
  const InnerWs& I = p.inner;
  return InnerState{I.R, I.gc, I.gsn, I.g, I.beta, I.scale, I.res, I.y};
}

// part -> out: per-frequency sums conj(V_j) . src (j < nv) and |src|^2
static int inner_sums(const Plan& p, const double2* V, int nv, const double2* src,
                      double2* out) {
  const InnerWs& I = p.inner;
  const size_t vs = (size_t)p.nf * p.S;
  k_inner_dots<<<dim3(I.nblk, p.nf), DOT_NT, 0, p.stream>>>(V, vs, nv, src, p.S, I.nblk, I.part);
  RFDE_HIP(hipGetLastError());
  const int tot = p.nf * (nv + 1);
  k_inner_reduce<<<(tot + 255) / 256, 256, 0, p.stream>>>(I.part, I.nblk, nv, p.nf, out);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

static int elementwise_grid(const Plan& p) {
  const size_t N = (size_t)p.nf * p.S;
  return (int)std::min<size_t>((N + 255) / 256, 8192);
}

int launch_inner_step_b(const Plan& p, const void* z1v, void* z2v) {
  const InnerWs& I = p.inner;
  const int k = p.opts.inner_iters, nf = p.nf, S = p.S;
  const size_t vs = (size_t)nf * S;
  const double2* z1 = (const double2*)z1v;
  double2* z2 = (double2*)z2v;
  const InnerState st = inner_state(p);
  const int eg = elementwise_grid(p), pg = (nf + 63) / 64;
  // beta and v_0 = z1 / beta (z1 may alias z2: it is not read after this)
  RFDE_TRY(inner_sums(p, I.V, 0, z1, I.h1));
  k_inner_start<<<pg, 64, 0, p.stream>>>(I.h1, st, nf);
  RFDE_HIP(hipGetLastError());
  k_inner_scale<<<eg, 256, 0, p.stream>>>(I.V, z1, I.scale, S, nf);
  RFDE_HIP(hipGetLastError());
  int steps = k;
  std::vector<double> hres(p.opts.inner_tol > 0 ? nf : 0);
  for (int j = 0; j < k; ++j) {
    double2* Vj = I.V + j * vs;
    double2* Zj = I.Z + j * vs;
    RFDE_TRY(launch_tau_solve(p, Vj, Zj));
    RFDE_TRY(inner_apply_B(p, Zj, I.w));
    // classical Gram-Schmidt twice: h1 = V^H w, w -= V h1; h2 = V^H w (with ||w||^2),
    // w -= V h2
    RFDE_TRY(inner_sums(p, I.V, j + 1, I.w, I.h1));
    k_inner_comb<<<eg, 256, 0, p.stream>>>(I.w, 1, -1.0, I.V, vs, j + 1, I.h1, KS1, S, nf);
    RFDE_HIP(hipGetLastError());
    RFDE_TRY(inner_sums(p, I.V, j + 1, I.w, I.h2));
    k_inner_comb<<<eg, 256, 0, p.stream>>>(I.w, 1, -1.0, I.V, vs, j + 1, I.h2, KS1, S, nf);
    RFDE_HIP(hipGetLastError());
    k_inner_givens<<<pg, 64, 0, p.stream>>>(I.h1, I.h2, st, j, nf);
    RFDE_HIP(hipGetLastError());
    if (j + 1 < k) {
      k_inner_scale<<<eg, 256, 0, p.stream>>>(I.V + (j + 1) * vs, I.w, I.scale, S, nf);
      RFDE_HIP(hipGetLastError());
    }
    if (p.opts.inner_tol > 0 && j + 1 < k) {
      RFDE_HIP(hipMemcpyAsync(hres.data(), I.res, nf * sizeof(double), hipMemcpyDeviceToHost,
                              p.stream));
      RFDE_HIP(hipStreamSynchronize(p.stream));
      if (*std::max_element(hres.begin(), hres.end()) <= p.opts.inner_tol) {
        steps = j + 1;
        break;
      }
    }
  }
  k_inner_backsolve<<<pg, 64, 0, p.stream>>>(st, steps, nf);
  RFDE_HIP(hipGetLastError());
  k_inner_comb<<<eg, 256, 0, p.stream>>>(z2, 0, 1.0, I.Z, vs, steps, I.y, INNER_KMAX, S, nf);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // namespace rfde
