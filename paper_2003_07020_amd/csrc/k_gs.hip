// Preconditioner step (b), exact 1D variant without factors: every shifted block
//     B_n = lambda_n I + coef T,   T[r][c] = g_|r-c|   (eq. (3.5))
// is itself a symmetric Toeplitz matrix (complex, since lambda_n is), so its inverse is fixed by
// one vector, the first column x = B_n^{-1} e_0, through the Gohberg-Semencul formula for
// symmetric Toeplitz matrices:
//     B^{-1} = (L(x) L(x)^T - L(u) L(u)^T) / x_0,   u = (0, x_{n-1}, ..., x_1),
// with L(v) the lower-triangular Toeplitz matrix of first column v.  Setup computes x for every
// frequency by the Levinson-Durbin recursion (O(M^2) per block instead of the O(M^3)
// factorisation) and keeps its DFT; each application is four products with triangular Toeplitz
// matrices, each a truncated linear convolution done by FFT of the circulant-embedding length L.
//
// Durbin's recursion on the normalised matrix R = B / t_0 (t_0 = lambda_n + coef g_0,
// r_k = coef g_k / t_0): y^(1) = -r_1; for k = 1..n-2: beta <- (1 - a^2) beta,
// a = -(r_{k+1} + sum_{i=1}^{k} r_{k+1-i} y_i) / beta, y_i <- y_i + a y_{k+1-i} (i <= k),
// y_{k+1} = a; then x = gamma / t_0 (1, y), gamma = 1 / (1 + sum_i r_i y_i).  No conjugation:
// B is complex symmetric, not Hermitian.  Every leading principal submatrix is nonsingular
// (the Hermitian part Re(lambda_n) I + coef T is positive definite for eps < 1), so the
// recursion does not break down.
//
// Products: L(v) w is the first n entries of the cyclic convolution of v and w padded to L
// (L >= 2n - 1); L(v)^T w = J L(v) J w with J the reversal.  With X = DFT(x) (padded),
// DFT(u)_k = w^{nk} (X_{-k} - x_0), w = exp(-2 pi i / L), so only X is stored.  One application:
//     p = J L(x) J b,  q = J L(u) J b         (launch 1: two transform pairs on J b)
//     z = (L(x) p - L(u) q) / x_0              (launch 2: two transform pairs)
// one workgroup per frequency row, except a last row that would run alone in a round of its
// own: its products are then formed as direct sums by all the other rows' workgroups.
#include "buf_io.hpp"
#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

// Arithmetic of a work item: complex, or componentwise on (.x, .y) for the dual item, which
// runs the real recursions of the two real blocks (frequencies 0 and N_t/2 of an even N_t,
// whose lambda are real) side by side, so an even N_t gives N_t/2 equal work items.
template <bool D> __device__ __forceinline__ double2 gmul(double2 a, double2 b) {
  if constexpr (D) return make_double2(a.x * b.x, a.y * b.y);
  else return cmul(a, b);
}
template <bool D> __device__ __forceinline__ double2 gdiv(double2 a, double2 b) {
  if constexpr (D) return make_double2(a.x / b.x, a.y / b.y);
  else return cdiv(a, b);
}
template <bool D> __device__ __forceinline__ double2 gone() {
  return make_double2(1.0, D ? 1.0 : 0.0);
}
// c + a b with every product fused into an FMA
template <bool D> __device__ __forceinline__ double2 gfma(double2 a, double2 b, double2 c) {
  if constexpr (D) return make_double2(fma(a.x, b.x, c.x), fma(a.y, b.y, c.y));
  else
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// 1 / b: one real division (of |b|^2) for a complex b
template <bool D> __device__ __forceinline__ double2 grcp(double2 b) {
  if constexpr (D) return make_double2(1.0 / b.x, 1.0 / b.y);
  else {
    const double r = 1.0 / fma(b.x, b.x, b.y * b.y);
    return make_double2(b.x * r, -b.y * r);
  }
}

// Work items of the setup launch: with an even N_t (dual), item 0 holds rows 0 and N_t/2 and
// item n >= 1 holds row n, so there are nf - 1 items; otherwise item n = row n.  (The
// application treats every row as complex: its convolutions of the two real rows would need
// both kernels in one transform, which cost more than the extra work item.)

// v plus the value DPP control C routes to this lane, on both halves of the double, in the rows
// of ROWS (the other rows' results are unspecified: the moves leave those lanes unwritten, and
// with no old value to keep they need no zeroed register)
template <int C, int ROWS = 0xf>
__device__ __forceinline__ double dpp_add(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)bits, C, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), C, ROWS, 0xf, true);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave in a fixed order, returned uniform: quad swaps (xor 1, xor 2),
// row half-mirror and mirror (each 16-lane row then holds its row sum), then the row broadcasts
// of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3, which leave the total in lane
// 63 (the only lane read: rows left out of a broadcast hold unspecified values).  Data moves
// lane to lane through DPP, not through LDS.
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1>(v);        // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4E>(v);        // quad_perm [2, 3, 0, 1]
  v = dpp_add<0x141>(v);       // row_half_mirror
  v = dpp_add<0x140>(v);       // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, 63);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One workgroup per item: x[n][0..M-1] = first column of B_n^{-1}.  y lives in LDS (64 KB at
// M = 4096, so two items share a CU) and in registers: y_i with 2i <= k+1 (the lower half at
// step k) stays in a register of the thread that updates the pair (i, k+1-i) from the step it
// enters the lower half on, so a pair costs one LDS read and one write (of its upper element).
// A step is one pass: the thread that updates the pair also adds the new pair's terms of the
// next step's sum
//   sum_{m=1}^{k+1} g_m y_{k+2-m} = g_{k+2-i} y_i + g_{k+2-j} y_j + ... + g_1 y_{k+1}
// (j = k+1-i), so the sum needs no second pass and the step one barrier (the reduction's, which
// also orders this step's writes of y before the next step's reads).  A thread issues all of its
// pairs' LDS reads before any write (the pairs of a step are disjoint) and before the division
// that gives a.  The partner weights g_{k+2-i} of the next step are loaded one step ahead
// through a buffer descriptor of g (indices outside it, which only slots not yet active use,
// read zero).  The
// per-thread partial sums are reduced in a fixed order (strided sums, the wave sum, then the
// wave totals, which alternate between two buffers by step parity), so the result does not
// depend on scheduling.  With two items per CU each SIMD runs one wave of each, and a step is
// bound by the vector instructions it issues (every slot's complex updates and sums, the wave
// sums, the division), so the step keeps its instruction count low: products fused into FMAs,
// one real division for the complex reciprocal, DPP moves that need no zeroed register, and
// the weights loaded rather than passed between threads.  (Two items per workgroup, at one
// workgroup per CU, were slower.)
constexpr int LEV_NT = 256;
// pair slots per thread: at step k <= M - 2 <= 4094 the pairs are i = 1 .. (k+1)/2 <= 2047
constexpr int LEV_S = 2048 / LEV_NT;
template <bool D>
__device__ __forceinline__ void levinson_item(const double* __restrict__ g, double coef,
                                              double2 lam, int M, double2* __restrict__ out0,
                                              double2* __restrict__ out1, double2* y,
                                              double2 (*part)[LEV_NT / 64]) {
  const int t = threadIdx.x, w = t >> 6;
  // t_0 = lambda + coef g_0 (dual: lam = (lambda_0, lambda_{N_t/2}), both real)
  const double2 t0 = D ? make_double2(lam.x + coef * g[0], lam.y + coef * g[0])
                       : make_double2(lam.x + coef * g[0], lam.y);
  const double2 it0 = gdiv<D>(gone<D>(), t0);
  // r_k = (coef g_k) / t_0 = rs g_k
  const double2 rs = make_double2(coef * it0.x, coef * it0.y);
  auto store = [&](int i, double2 v) {
    if constexpr (D) {
      out0[i] = make_double2(v.x, 0.0);
      out1[i] = make_double2(v.y, 0.0);
    } else {
      out0[i] = v;
    }
  };
  if (M == 1) {
    if (t == 0) store(0, it0);
    return;
  }
  // block sum of a per-thread value, identical in every thread
  auto block_sum = [&](double2 v, int par) -> double2 {
    v = make_double2(wave_sum(v.x), wave_sum(v.y));
    if ((t & 63) == 0) part[par][w] = v;
    __syncthreads();
    double2 s = part[par][0];
#pragma unroll
    for (int q = 1; q < LEV_NT / 64; ++q) s = cadd(s, part[par][q]);
    return s;
  };
  // slot q of thread t is the pair with i = 1 + t + LEV_NT q: its weight g_{i+1} is fixed, the
  // weight g_{k+2-i} = g[k + 1 - t - LEV_NT q] of its partner moves by one per step (read as
  // zero outside [0, M), for the slots not yet active, whose values are never used)
  const __amdgpu_buffer_rsrc_t gr = make_rsrc(g, M * 8);
  double gi[LEV_S], gj[LEV_S];
#pragma unroll
  for (int q = 0; q < LEV_S; ++q) {
    gi[q] = buf_load(gr, 2 + t + LEV_NT * q);
    gj[q] = buf_load(gr, 2 - t - LEV_NT * q);
  }
  // y_i of slot q once it is in the lower half (from step 2i - 1 on, when its pair is (i, i))
  double2 yr[LEV_S];
#pragma unroll
  for (int q = 0; q < LEV_S; ++q) yr[q] = make_double2(0.0, 0.0);
  const double g1 = g[1];
  double2 a = make_double2(-rs.x * g1, -rs.y * g1);  // -r_1
  if (t == 0) y[0] = a;
  // beta_1 = 1 - a_0^2 and its inverse
  double2 beta = csub(gone<D>(), gmul<D>(a, a));
  double2 ib = grcp<D>(beta);
  double2 dot = make_double2(g1 * a.x, g1 * a.y);  // the step-1 sum g_1 y_1
  double gnext = M > 2 ? g[2] : 0.0;
  __syncthreads();
  for (int k = 1; k <= M - 2; ++k) {
    // partners y_j (j = k+1-i >= i) from LDS; they do not depend on a
    double2 yj[LEV_S];
#pragma unroll
    for (int q = 0; q < LEV_S; ++q) {
      const int i = 1 + t + LEV_NT * q;
      if (2 * i <= k + 1) yj[q] = y[k - i];
    }
    const double gk1 = gnext;
    if (k + 2 < M) gnext = g[k + 2];
    // partner weights of step k + 1
    double gn[LEV_S];
#pragma unroll
    for (int q = 0; q < LEV_S; ++q) gn[q] = buf_load(gr, k + 2 - t - LEV_NT * q);
    // a = -(r_{k+1} + sum_m r_m y_{k+1-m}) / beta_k, by the inverse computed a step ahead
    const double2 s = D ? make_double2(rs.x * (dot.x + gk1), rs.y * (dot.y + gk1))
                        : cmul(rs, make_double2(dot.x + gk1, dot.y));
    a = gmul<D>(s, ib);
    a = make_double2(-a.x, -a.y);
    // beta_{k+1} = (1 - a^2) beta_k and its inverse: needed only by the next step, so the
    // division runs beside this step's update and sum instead of on the path from sum to a
    beta = gmul<D>(csub(gone<D>(), gmul<D>(a, a)), beta);
    ib = grcp<D>(beta);
    // y_i <- y_i + a y_j, y_j <- y_j + a y_i; the new values' terms of the next sum,
    // g_{k+2-i} y_i + g_{i+1} y_j (y_i once when i = j)
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < LEV_S; ++q) {
      const int i = 1 + t + LEV_NT * q;
      if (2 * i <= k + 1) {
        const bool first = 2 * i == k + 1;  // i = j: y_i moves from LDS into its register
        const double2 yi = first ? yj[q] : yr[q];
        const double2 ni = gfma<D>(a, yj[q], yi);
        const double2 nj = gfma<D>(a, yi, yj[q]);
        yr[q] = ni;
        if (!first) y[k - i] = nj;
        const double wj = first ? 0.0 : gi[q];
        acc.x = fma(gj[q], ni.x, fma(wj, nj.x, acc.x));
        acc.y = fma(gj[q], ni.y, fma(wj, nj.y, acc.y));
      }
    }
    if (t == 0) y[k] = a;
    const double2 sg = block_sum(acc, k & 1);
#pragma unroll
    for (int q = 0; q < LEV_S; ++q) gj[q] = gn[q];
    dot = make_double2(sg.x + g1 * a.x, sg.y + g1 * a.y);
  }
  // the lower half back into LDS beside the upper half
#pragma unroll
  for (int q = 0; q < LEV_S; ++q) {
    const int i = 1 + t + LEV_NT * q;
    if (2 * i <= M - 1) y[i - 1] = yr[q];
  }
  __syncthreads();
  // gamma = 1 / (1 + sum_{m=1}^{M-1} r_m y_m)
  double2 acc = make_double2(0.0, 0.0);
  for (int m = 1 + t; m <= M - 1; m += LEV_NT) {
    const double2 yv = y[m - 1];
    const double gm = g[m];
    acc.x = fma(gm, yv.x, acc.x);
    acc.y = fma(gm, yv.y, acc.y);
  }
  const double2 sg = block_sum(acc, (M - 1) & 1);
  const double2 den = cadd(gone<D>(), gmul<D>(rs, sg));
  const double2 sc = gdiv<D>(it0, den);  // gamma / t_0
  if (t == 0) store(0, sc);
  for (int i = 1 + t; i <= M - 1; i += LEV_NT) store(i, gmul<D>(sc, y[i - 1]));
}

__global__ void __launch_bounds__(LEV_NT) k_levinson(const double* __restrict__ g, double coef,
                                                     const double2* __restrict__ lambda, int M,
                                                     int nf, int dual,
                                                     double2* __restrict__ xgen) {
  extern __shared__ double2 y[];         // M - 1 entries (y[i-1] holds y_i)
  __shared__ double2 part[2][LEV_NT / 64];
  const int item = blockIdx.x;
  if (dual && item == 0) {
    const double2 lam = make_double2(lambda[0].x, lambda[nf - 1].x);
    levinson_item<true>(g, coef, lam, M, xgen, xgen + (size_t)(nf - 1) * M, y, part);
  } else {
    levinson_item<false>(g, coef, lambda[item], M, xgen + (size_t)item * M, nullptr, y, part);
  }
}

// Xhat[n][k] = DFT_L(x[n] padded)_k / L, one workgroup per frequency.
template <int L, int NT>
__global__ void __launch_bounds__(NT) k_gs_spectrum(const double2* __restrict__ xgen, int M,
                                                    const double2* __restrict__ tw,
                                                    double2* __restrict__ xhat) {
  __shared__ double2 buf[L];
  const int n = blockIdx.x;
  const double2* x = xgen + (size_t)n * M;
  double2* X = xhat + (size_t)n * L;
  auto load = [&](int, int idx) -> double2 { return idx < M ? x[idx] : make_double2(0.0, 0.0); };
  auto store = [&](int, int k, double2 c) { X[k] = make_double2(c.x / L, c.y / L); };
  fft_io<L, -1, NT, 1, L, false, true, true, 16>(buf, tw, load, store);
}

// Kernel transforms of the two generators at frequency index k (the tables hold 1/L):
//   DFT(x)_k / L = X[k],   DFT(u)_k / L = w^{Mk} (X[-k] - x_0 / L).
template <int L>
__device__ __forceinline__ double2 gs_kernel(const double2* __restrict__ X,
                                             const double2* __restrict__ tw, int M, double2 x0L,
                                             int which, int k) {
  if (which == 0) return X[k];
  const double2 xm = X[(L - k) & (L - 1)];
  const double2 wk = tw[(int)(((long long)M * k) & (L - 1))];
  return cmul(wk, csub(xm, x0L));
}

// One transform pair per generator on a row held in LDS: out(idx) for idx < M receives the
// first M entries of the cyclic convolution of the row (from load) with generator `which`.
template <int L, int NT, typename Load, typename Store>
__device__ __forceinline__ void gs_conv(double2* buf, const double2* __restrict__ tw,
                                        const double2* __restrict__ X, int M, double2 x0L,
                                        int which, Load& load, Store& store) {
  auto mul = [&](int, int k, double2 c) {
    buf[k] = cmul(c, gs_kernel<L>(X, tw, M, x0L, which, k));
  };
  fft_io<L, -1, NT, 1, L, false, true, true, 16>(buf, tw, load, mul);
  __syncthreads();
  NoLoad nl;
  fft_io<L, +1, NT, 1, L, false, false, true, 16>(buf, tw, nl, store);
  __syncthreads();  // buf is reused by the next pair
}

// The last row by direct sums (when it would otherwise take a round of workgroups of its own):
// every workgroup forms a few consecutive entries, one wave per entry, the lanes taking every
// 64th term and the wave sum adding them in a fixed order, with the row's vectors staged in the
// (not yet used) transform buffer, two at a time (2M <= L).  Entries of this workgroup:
// [blockIdx.x * per, (blockIdx.x + 1) * per) within [0, M).
template <int NT, typename Entry>
__device__ __forceinline__ void gs_direct_rows(int M, Entry& entry) {
  constexpr int NW = NT / 64;
  const int per = (M + gridDim.x - 1) / gridDim.x;
  const int m0 = blockIdx.x * per, m1 = m0 + per < M ? m0 + per : M;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int m = m0 + wv; m < m1; m += NW) entry(m, lane);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {  // c + a b
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// This lane's share of sum_{t < n} term(t): t = lane, lane + 64, ... in four interleaved partial
// sums (independent LDS reads in flight), added in a fixed order.
template <typename F>
__device__ __forceinline__ double2 lane_sum(int n, int lane, F term) {
  double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0, s3 = s0;
  int t = lane;
  for (; t + 192 < n; t += 256) {
    s0 = term(t, s0);
    s1 = term(t + 64, s1);
    s2 = term(t + 128, s2);
    s3 = term(t + 192, s3);
  }
  for (; t < n; t += 64) s0 = term(t, s0);
  return cadd(cadd(s0, s1), cadd(s2, s3));
}

// Launch 1: p = J L(x) J b, q = J L(u) J b for row n of b (one workgroup per row); with
// ndir >= 0, row ndir by direct sums: p_m = sum_{l >= m} x_{l-m} b_l, q_m = sum_{l > m}
// x_{M-(l-m)} b_l (u_0 = 0, u_d = x_{M-d}).
template <int L, int NT>
__global__ void __launch_bounds__(NT) k_gs_apply1(const double2* __restrict__ b,
                                                  double2* __restrict__ P,
                                                  double2* __restrict__ Q,
                                                  const double2* __restrict__ xhat,
                                                  const double2* __restrict__ xgen, int M,
                                                  const double2* __restrict__ tw, int ndir) {
  __shared__ double2 buf[L];
  if (ndir >= 0) {
    double2* xd = buf;      // x of row ndir
    double2* bd = buf + M;  // b of row ndir
    for (int e = threadIdx.x; e < M; e += NT) {
      xd[e] = xgen[(size_t)ndir * M + e];
      bd[e] = b[(size_t)ndir * M + e];
    }
    __syncthreads();
    auto entry = [&](int m, int lane) {
      // terms l = m + d: x_d b_l (d >= 0), x_{M-d} b_l (d >= 1)
      double2 sp = lane_sum(M - m, lane, [&](int d, double2 s) {
        return cfma(xd[d], bd[m + d], s);
      });
      double2 sq = lane_sum(M - m - 1, lane, [&](int e, double2 s) {
        return cfma(xd[M - 1 - e], bd[m + 1 + e], s);
      });
      sp = make_double2(wave_sum(sp.x), wave_sum(sp.y));
      sq = make_double2(wave_sum(sq.x), wave_sum(sq.y));
      if (lane == 0) {
        P[(size_t)ndir * M + m] = sp;
        Q[(size_t)ndir * M + m] = sq;
      }
    };
    gs_direct_rows<NT>(M, entry);
    __syncthreads();  // buf is the transforms' next
  }
  const int n = blockIdx.x;
  const double2* bn = b + (size_t)n * M;
  const double2* X = xhat + (size_t)n * L;
  const double2 x0 = xgen[(size_t)n * M];
  const double2 x0L = make_double2(x0.x / L, x0.y / L);
  auto load_rev = [&](int, int idx) -> double2 {
    return idx < M ? bn[M - 1 - idx] : make_double2(0.0, 0.0);
  };
  double2* Pn = P + (size_t)n * M;
  double2* Qn = Q + (size_t)n * M;
  auto store_p = [&](int, int idx, double2 c) { if (idx < M) Pn[M - 1 - idx] = c; };
  auto store_q = [&](int, int idx, double2 c) { if (idx < M) Qn[M - 1 - idx] = c; };
  gs_conv<L, NT>(buf, tw, X, M, x0L, 0, load_rev, store_p);
  gs_conv<L, NT>(buf, tw, X, M, x0L, 1, load_rev, store_q);
}

// Launch 2: z = (L(x) p - L(u) q) / x_0 for row n.  The second pair's store subtracts from the
// value the same thread stored in the first (the store pattern of the last pass is fixed per
// thread).  With ndir >= 0, row ndir by direct sums:
// z_i = (sum_{j <= i} x_{i-j} p_j - sum_{j < i} x_{M-(i-j)} q_j) / x_0.
template <int L, int NT>
__global__ void __launch_bounds__(NT) k_gs_apply2(const double2* __restrict__ P,
                                                  const double2* __restrict__ Q,
                                                  double2* __restrict__ z,
                                                  const double2* __restrict__ xhat,
                                                  const double2* __restrict__ xgen, int M,
                                                  const double2* __restrict__ tw, int ndir) {
  __shared__ double2 buf[L];
  if (ndir >= 0) {
    // first the sums with p (x and p staged), then with q (q over p); the entry's lane 0 keeps
    // the first sum in z between the two
    double2* xd = buf;
    double2* vd = buf + M;
    double2* zd = z + (size_t)ndir * M;
    for (int e = threadIdx.x; e < M; e += NT) {
      xd[e] = xgen[(size_t)ndir * M + e];
      vd[e] = P[(size_t)ndir * M + e];
    }
    __syncthreads();
    auto entry1 = [&](int i, int lane) {
      double2 s = lane_sum(i + 1, lane, [&](int j, double2 a) {
        return cfma(xd[i - j], vd[j], a);
      });
      s = make_double2(wave_sum(s.x), wave_sum(s.y));
      if (lane == 0) zd[i] = s;
    };
    gs_direct_rows<NT>(M, entry1);
    __syncthreads();
    for (int e = threadIdx.x; e < M; e += NT) vd[e] = Q[(size_t)ndir * M + e];
    __syncthreads();
    const double2 ix0d = cdiv(make_double2(1.0, 0.0), xd[0]);
    auto entry2 = [&](int i, int lane) {
      double2 s = lane_sum(i, lane, [&](int j, double2 a) {
        return cfma(xd[M - (i - j)], vd[j], a);
      });
      s = make_double2(wave_sum(s.x), wave_sum(s.y));
      if (lane == 0) zd[i] = cmul(csub(zd[i], s), ix0d);
    };
    gs_direct_rows<NT>(M, entry2);
    __syncthreads();  // buf is the transforms' next
  }
  const int n = blockIdx.x;
  const double2* X = xhat + (size_t)n * L;
  const double2 x0 = xgen[(size_t)n * M];
  const double2 x0L = make_double2(x0.x / L, x0.y / L);
  const double2 ix0 = cdiv(make_double2(1.0, 0.0), x0);
  const double2* Pn = P + (size_t)n * M;
  const double2* Qn = Q + (size_t)n * M;
  double2* zn = z + (size_t)n * M;
  auto load_p = [&](int, int idx) -> double2 { return idx < M ? Pn[idx] : make_double2(0.0, 0.0); };
  auto load_q = [&](int, int idx) -> double2 { return idx < M ? Qn[idx] : make_double2(0.0, 0.0); };
  auto store1 = [&](int, int idx, double2 c) { if (idx < M) zn[idx] = c; };
  auto store2 = [&](int, int idx, double2 c) {
    if (idx < M) zn[idx] = cmul(csub(zn[idx], c), ix0);
  };
  gs_conv<L, NT>(buf, tw, X, M, x0L, 0, load_p, store1);
  gs_conv<L, NT>(buf, tw, X, M, x0L, 1, load_q, store2);
}

template <int L> constexpr int gs_threads() { return L >= 2048 ? 512 : (L >= 256 ? 256 : 64); }

template <int L>
static int gs_setup_t(const Plan& p) {
  constexpr int NT = gs_threads<L>();
  k_gs_spectrum<L, NT><<<p.nf, NT, 0, p.stream>>>(p.gs_x, p.M, p.twL, p.gs_xhat);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// Even N_t: the real rows 0 and N_t/2 form one work item of the setup (nf - 1 items in all).
static int gs_dual(const Plan& p) { return (p.Nt % 2 == 0 && p.nf >= 2) ? 1 : 0; }

// Row split of the application: one workgroup per row by transforms, except that the last row
// goes to the direct sums when it alone would start another round of workgroups (the rows
// before it fill whole rounds of the resident slots, as 512 rows do on 256 CUs at one
// workgroup per CU, L = 8192).  Returns that row, or -1.
template <int L, int NT>
static int gs_direct_row(const Plan& p) {
  if (p.nf < 2) return -1;
  // resident workgroups per CU (queried once per instantiation)
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_gs_apply1<L, NT>, NT, 0) !=
        hipSuccess)
      v = 0;
    return v;
  }();
  if (per_cu <= 0) return -1;
  const int slots = per_cu * device_cus(p.device);
  return (p.nf - 1) % slots == 0 ? p.nf - 1 : -1;
}

template <int L>
static int gs_apply_t(const Plan& p, const double2* z1, double2* z2) {
  constexpr int NT = gs_threads<L>();
  const int ndir = gs_direct_row<L, NT>(p);
  const int rows = ndir >= 0 ? p.nf - 1 : p.nf;
  k_gs_apply1<L, NT><<<rows, NT, 0, p.stream>>>(z1, p.gs_p, p.gs_q, p.gs_xhat, p.gs_x, p.M,
                                                p.twL, ndir);
  RFDE_HIP(hipGetLastError());
  k_gs_apply2<L, NT><<<rows, NT, 0, p.stream>>>(p.gs_p, p.gs_q, z2, p.gs_xhat, p.gs_x, p.M,
                                                p.twL, ndir);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

#define RFDE_GSL_SWITCH(FN, ...)                 \
  switch (p.L) {                                 \
    case 16: return FN<16>(__VA_ARGS__);         \
    case 32: return FN<32>(__VA_ARGS__);         \
    case 64: return FN<64>(__VA_ARGS__);         \
    case 128: return FN<128>(__VA_ARGS__);       \
    case 256: return FN<256>(__VA_ARGS__);       \
    case 512: return FN<512>(__VA_ARGS__);       \
    case 1024: return FN<1024>(__VA_ARGS__);     \
    case 2048: return FN<2048>(__VA_ARGS__);     \
    case 4096: return FN<4096>(__VA_ARGS__);     \
    case 8192: return FN<8192>(__VA_ARGS__);     \
    default: return RFDE_EINVAL;                 \
  }

// Setup of the Toeplitz solver: generators by Levinson-Durbin, then their transforms.
int launch_gs_setup(const Plan& p) {
  const size_t lds = (size_t)(p.M > 1 ? p.M - 1 : 1) * sizeof(double2);
  const int dual = gs_dual(p);
  k_levinson<<<p.nf - dual, LEV_NT, lds, p.stream>>>(p.g, p.coef, p.lambda, p.M, p.nf, dual,
                                                     p.gs_x);
  RFDE_HIP(hipGetLastError());
  RFDE_GSL_SWITCH(gs_setup_t, p);
}

// z2_n = B_n^{-1} z1_n for every frequency (z1 may alias z2: launch 1 reads z1 and writes
// only the work arrays; launch 2 writes z2).
int launch_gs_apply(const Plan& p, const void* z1, void* z2) {
  RFDE_GSL_SWITCH(gs_apply_t, p, (const double2*)z1, (double2*)z2);
}

}  // namespace rfde
