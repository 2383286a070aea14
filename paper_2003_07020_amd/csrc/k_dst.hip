// Preconditioner step (b) with the tau approximation of the Toeplitz blocks (eq. (3.9)-(3.11)
// in 1D, eq. (4.4)-(4.5) in 2D): the tau matrix is Q diag(sigma) Q with the DST-I matrix
// Q[i][j] = sqrt(2/(n+1)) sin(pi i j/(n+1)) (symmetric, Q Q = I), so
//     1D: z2_n = Q diag(1 / (lambda_n + coef sigma_i)) Q z1_n
//     2D: z2_n = (Qy kron Qx) diag(1 / (lambda_n + coef_x sigma^x_i + coef_y sigma^y_j)) (Qy kron Qx) z1_n.
// A length-n DST-I is computed by a complex FFT of length P = 2(n+1) of the odd extension
// (0, x_1..x_n, 0, -x_n..-x_1): FFT_k = -2i sum_j x_j sin(pi j k/(n+1)), hence
// (Q x)_k = sqrt(2/(n+1)) (i/2) FFT_k.  P must be a power of two here (other lengths take the
// chirp-z DST of k_dst_bs.hip).  1D rows in FP64 with P >= 512 take a complex FFT of length
// P / 2 instead (k_dst_half).
#include <type_traits>

#include "buf_io.hpp"
#include "fft3.hpp"
#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

// buf holds FFT output; return sqrt(2/(n+1)) (i/2) buf[k] as the DST coefficient k.
template <typename C>
__device__ __forceinline__ C dst_coef(C y, typename cplx_traits<C>::real sc) {
  // (i/2) y = (-y.y/2, y.x/2)
  return cmk<C>(-0.5f * sc * y.y, 0.5f * sc * y.x);
}

// Rows: `nrows` contiguous rows of length n; NB rows per block.  DST along the row; with
// SCALE, divide coefficient k by (lambda_f + coef sigma_k) and apply the DST again
// (f = row / rows_per_freq).  The odd extension is formed by the first FFT pass's loads and the
// coefficients are written by the last pass's stores.
template <int P, int NB, int NT, typename C, bool SCALE, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_dst_rows(C* __restrict__ z, int nrows, int rows_per_freq,
                                                 const double2* __restrict__ lambda,
                                                 const double* __restrict__ sigma, double coef,
                                                 const C* __restrict__ tw) {
  using R = typename cplx_traits<C>::real;
  constexpr int n = P / 2 - 1;
  __shared__ C buf[NB * P];
  const int row0 = xcd_remap(blockIdx.x, gridDim.x) * NB;
  const R sc = (R)sqrt(2.0 / (n + 1));
  auto load = [&](int f, int idx) -> C {
    const int row = row0 + f;
    if (row >= nrows || idx == 0 || idx == n + 1) return cmk<C>((R)0, (R)0);
    if (idx <= n) return z[(size_t)row * n + idx - 1];
    const C x = z[(size_t)row * n + (P - idx) - 1];
    return cmk<C>(-x.x, -x.y);
  };
  auto store_out = [&](int f, int idx, C y) {
    const int row = row0 + f;
    if (row < nrows && idx >= 1 && idx <= n) z[(size_t)row * n + idx - 1] = dst_coef(y, sc);
  };
  if constexpr (SCALE) {
    auto store_scaled = [&](int f, int idx, C y) {
      const int row = row0 + f;
      C* B = buf + f * P;
      if (idx == 0 || idx == n + 1) {
        B[idx] = cmk<C>((R)0, (R)0);
      } else if (idx <= n) {
        C wv = cmk<C>((R)0, (R)0);
        if (row < nrows) {
          const double2 lam = lambda[row / rows_per_freq];
          const double dr = lam.x + coef * sigma[idx - 1], di = lam.y;
          const double den = dr * dr + di * di;
          wv = cmul(dst_coef(y, sc), cmk<C>((R)(dr / den), (R)(-di / den)));
        }
        B[idx] = wv;
        B[P - idx] = cmk<C>(-wv.x, -wv.y);
      }
    };
    fft_io<P, -1, NT, NB, P, false, true, true, MAXR>(buf, tw, load, store_scaled);
    __syncthreads();
    NoLoad nl;
    fft_io<P, -1, NT, NB, P, false, false, true, MAXR>(buf, tw, nl, store_out);
  } else {
    fft_io<P, -1, NT, NB, P, false, true, true, MAXR>(buf, tw, load, store_out);
  }
}

// 1D tau solve of whole rows on the three-stage register FFT (P >= 256): row r of z (complex,
// length n = P/2 - 1) is odd-extended, transformed, scaled and transformed back without leaving
// registers.  X = DFT(odd(z)) is odd, so the scaled coefficients W_k = X_k d_m (m = min(k, P-k))
// are odd too and the second DST-I, sc (i/2) DFT(W), equals -sc (i/2) times the unnormalised
// inverse DFT of W; with the first DST's sc (i/2) the product of the constants is sc^2 / 4:
//     d_m = (sc^2 / 4) / (lambda_r + coef sigma_m),  d_0 = d_{P/2} = 0.
// With DUAL (N_t even) the real rows 0 and N_t/2 (real lambda, real data) share one transform
// as its real and imaginary parts: the DFT of a real odd sequence is imaginary, so in
// X = DFT(odd(a + i b)) the imaginary part carries a's coefficients and the real part b's, and
// each is scaled by its own row's (real) d_m; the work list is then nrows - 1 transforms, N_t/2
// of them for N_t even (no lone last row on the grid).
// Rows are read and written through buffer descriptors covering exactly the row, so the odd
// extension's zeros (indices 0 and P/2) come from the hardware range check.
template <int P, typename C, int WAVES, bool DUAL>
__global__ void __launch_bounds__(256, WAVES) k_dst3_scale(const C* zin, C* zout, int nrows,
                                                           const double2* __restrict__ lambda,
                                                           const double* __restrict__ sigma,
                                                           double coef, const C* __restrict__ tw) {
  using E = Fft3WideMid<P, 256>;
  using R = typename cplx_traits<C>::real;
  constexpr int n = P / 2 - 1;
  __shared__ R lds[E::LDS];
  const int nitems = DUAL ? nrows - 1 : nrows;
  // item = row; with DUAL item 0 is the pair of rows 0 and nrows - 1
  const int item0 = xcd_remap(blockIdx.x, gridDim.x) * E::NB;
  const double sc2 = 2.0 / (n + 1) / 4.0;
  auto rowr = [&](const C* z, int r) {
    const bool ok = r >= 0 && r < nrows;
    return make_rsrc(z + (ok ? (size_t)r * n : 0), ok ? n * (int)sizeof(C) : 0);
  };
  // rows read (rs, rs2) and written (ws, ws2); zin == zout is allowed (each workgroup reads all
  // of its rows before it writes any)
  __amdgpu_buffer_rsrc_t rs[E::B1], rs2[E::B1], ws[E::B1], ws2[E::B1];
  bool dual[E::B1];
#pragma unroll
  for (int b = 0; b < E::B1; ++b) {
    const int it = item0 + E::f_of_b1(b);
    dual[b] = DUAL && it == 0;
    rs[b] = rowr(zin, it < nitems ? it : -1);
    rs2[b] = rowr(zin, dual[b] ? nrows - 1 : -1);
    ws[b] = rowr(zout, it < nitems ? it : -1);
    ws2[b] = rowr(zout, dual[b] ? nrows - 1 : -1);
  }
  auto load = [&](int b, int, int idx, int n1) -> C {
    const int j = n1 < E::N1 / 2 ? idx - 1 : P - idx - 1;
    const R sg = n1 < E::N1 / 2 ? (R)1 : (R)-1;
    C x;
    if (DUAL && dual[b]) x = cmk<C>(buf_load_re<C>(rs[b], j), buf_load_re<C>(rs2[b], j));
    else x = buf_load_c<C>(rs[b], j);
    return cmk<C>(sg * x.x, sg * x.y);
  };
  // d_m of row r as a complex number; 1 / |den|^2 by the hardware reciprocal refined with two
  // Newton steps r <- r + r (1 - q r) (each at least doubles the correct bits)
  auto scale = [&](int r, int m) -> double2 {
    const double2 lm = lambda[r];
    const bool in = m >= 1 && m <= n;
    const double dr = lm.x + coef * sigma[in ? m - 1 : 0], di = lm.y;
    const double q = dr * dr + di * di;
    double rq = __builtin_amdgcn_rcp(q);
    rq = fma(rq, fma(-q, rq, 1.0), rq);
    rq = fma(rq, fma(-q, rq, 1.0), rq);
    const double s = in ? sc2 * rq : 0.0;
    return make_double2(dr * s, -di * s);
  };
  auto pw = [&](int f, int k, C& c) {
    const int it = min(item0 + f, nitems - 1), m = k <= P / 2 ? k : P - k;
    if (DUAL && it == 0) {
      const double da = scale(0, m).x, db = scale(nrows - 1, m).x;
      c = cmk<C>((R)(c.x * db), (R)(c.y * da));
    } else {
      const double2 d = scale(it, m);
      c = cmk<C>((R)(c.x * d.x - c.y * d.y), (R)(c.x * d.y + c.y * d.x));
    }
  };
  auto store = [&](int b, int, int idx, int n1, C c) {
    if (n1 >= E::N1 / 2) return;
    if (DUAL && dual[b]) {
      buf_store_c<C>(ws[b], idx - 1, cmk<C>(c.x, (R)0));
      buf_store_c<C>(ws2[b], idx - 1, cmk<C>(c.y, (R)0));
    } else {
      buf_store_c<C>(ws[b], idx - 1, c);
    }
  };
  E::run(lds, tw, load, pw, store);
}

// 1D tau solve of whole rows on a transform of half that length (N = n + 1 = P / 2 >= 256).
// For x_1..x_{N-1} (x_0 = x_N = 0) let c_j = sin(pi j / N) (x_j + x_{N-j}) + (x_j - x_{N-j}) / 2
// and F_k = sum_j c_j exp(+2 pi i j k / N).  With O_k = (F_k + F_{N-k}) / 2 and
// E_k = -i (F_k - F_{N-k}) / 2 the sine sums S_m = sum_j x_j sin(pi j m / N) are S_{2k} = E_k
// and S_{2k+1} = O_0 + ... + O_k - O_0 / 2 (the identity for real sequences, applied to the
// real and imaginary parts at once since every coefficient is real).  The solve is
// z2 = (2 / N) S(d S(z1)) with d_m = 1 / (lambda_r + coef sigma_m).  The first transform runs
// as the forward stages on conj(c), which give conj(F); the second as the inverse stages, which
// form the +i sums directly from the stage-3 layout.  Between and after the transforms the
// spectrum sits in LDS (one complex slot of padding per 8 entries, so that a lane's run of 8
// consecutive entries starts on a different bank group than its neighbour's); the prefix sums
// take a fixed order: a thread's KT consecutive entries, then a scan over the lanes of the row.
// DUAL: rows 0 and nrows - 1 (real lambda, real data) share item 0 as real and imaginary parts,
// each scaled by its own row's d.
template <int N, typename C, int WAVES, bool DUAL>
__global__ void __launch_bounds__(256, WAVES) k_dst_half(const C* zin, C* zout, int nrows,
                                                         const double2* __restrict__ lambda,
                                                         const double* __restrict__ sigma,
                                                         double coef, const C* __restrict__ tw) {
  using S3 = Split3<N>;
  using E = Fft3<S3::N1, S3::N2, S3::N3, S3::NB, 256, 2>;
  using R = typename cplx_traits<C>::real;
  constexpr int n = N - 1, NB = E::NB, T = 256 / NB, KT = N / 2 / T;
  constexpr int LDN = N + N / 8;
  constexpr int CPLX = NB * LDN * 2;
  constexpr int LDSR = E::LDS > CPLX ? E::LDS : CPLX;
  static_assert(KT >= 1 && KT * T == N / 2, "whole runs of the prefix sums per thread");
  static_assert(T % 32 == 0 && T <= 256, "lanes per row");
  __shared__ R lds[LDSR];
  __shared__ R wsum[2][4];
  C* buf = reinterpret_cast<C*>(lds);
  auto at = [](int f, int k) { return f * LDN + k + (k >> 3); };
  const int nitems = DUAL ? nrows - 1 : nrows;
  const int item0 = xcd_remap(blockIdx.x, gridDim.x) * E::NB;
  auto rowr = [&](const C* z, int r) {
    const bool ok = r >= 0 && r < nrows;
    return make_rsrc(z + (ok ? (size_t)r * n : 0), ok ? n * (int)sizeof(C) : 0);
  };
  __amdgpu_buffer_rsrc_t rs[E::B1], rs2[E::B1];
  bool dual[E::B1];
#pragma unroll
  for (int b = 0; b < E::B1; ++b) {
    const int it = item0 + E::f_of_b1(b);
    dual[b] = DUAL && it == 0;
    rs[b] = rowr(zin, it < nitems ? it : -1);
    rs2[b] = rowr(zin, dual[b] ? nrows - 1 : -1);
  }
  // x_j of the item, j = 0..N (zero outside 1..n through the descriptor's range)
  auto xval = [&](int b, int j) -> C {
    if (DUAL && dual[b]) return cmk<C>(buf_load_re<C>(rs[b], j - 1), buf_load_re<C>(rs2[b], j - 1));
    return buf_load_c<C>(rs[b], j - 1);
  };
  auto sinN = [&](int j) -> R { return -tw[j].y; };  // sin(pi j / N) = sin(2 pi j / P)
  // stage-1 input: conj(c_idx)
  auto load = [&](int b, int, int idx, int) -> C {
    const C x = xval(b, idx), y = xval(b, N - idx);
    const R sj = sinN(idx);
    const R cx = sj * (x.x + y.x) + (R)0.5 * (x.x - y.x);
    const R cy = sj * (x.y + y.y) + (R)0.5 * (x.y - y.y);
    return cmk<C>(cx, -cy);
  };

  // Exclusive prefix over the lanes of a row (T consecutive threads) of a per-thread (vx, vy).
  auto lane_scan = [&](R vx, R vy, R& ex, R& ey) {
    constexpr int SEG = T < 64 ? T : 64;
    const int lane = threadIdx.x & 63, sl = lane & (SEG - 1);
    R ix = vx, iy = vy;
#pragma unroll
    for (int d = 1; d < SEG; d <<= 1) {
      const R tx = __shfl_up(ix, d, SEG), ty = __shfl_up(iy, d, SEG);
      if (sl >= d) {
        ix += tx;
        iy += ty;
      }
    }
    R px = __shfl_up(ix, 1, SEG), py = __shfl_up(iy, 1, SEG);
    if (sl == 0) px = py = (R)0;
    if constexpr (T > 64) {
      const int w = threadIdx.x >> 6;
      if (lane == 63) {
        wsum[0][w] = ix;
        wsum[1][w] = iy;
      }
      __syncthreads();
      const int w0 = (threadIdx.x / T) * (T / 64);
      R ox = (R)0, oy = (R)0;
      for (int q = w0; q < w; ++q) {
        ox += wsum[0][q];
        oy += wsum[1][q];
      }
      px = ox + px;
      py = oy + py;
    }
    ex = px;
    ey = py;
  };
  // Sine sums S_m of row f from F in buf; emit(f, m, S_m) for the thread's m = 2k, 2k + 1,
  // k = tl KT .. tl KT + KT - 1 (m = 0 is emitted as zero), after a barrier (emit may write buf).
  const int fs = threadIdx.x / T, tl = threadIdx.x % T;
  auto sine_sums = [&](auto emit) {
    const C F0 = buf[at(fs, 0)];
    C O[KT], Ev[KT];
    R tx = (R)0, ty = (R)0;
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      const int k = tl * KT + i;
      const C Fk = buf[at(fs, k)], Fm = buf[at(fs, (N - k) & (N - 1))];
      O[i] = cmk<C>((R)0.5 * (Fk.x + Fm.x), (R)0.5 * (Fk.y + Fm.y));
      Ev[i] = cmk<C>((R)0.5 * (Fk.y - Fm.y), (R)-0.5 * (Fk.x - Fm.x));
      tx += O[i].x;
      ty += O[i].y;
    }
    R sx, sy;
    lane_scan(tx, ty, sx, sy);
    sx -= (R)0.5 * F0.x;
    sy -= (R)0.5 * F0.y;
    C Sodd[KT];
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      sx += O[i].x;
      sy += O[i].y;
      Sodd[i] = cmk<C>(sx, sy);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      const int k = tl * KT + i;
      emit(fs, 2 * k, k == 0 ? cmk<C>((R)0, (R)0) : Ev[i]);
      emit(fs, 2 * k + 1, Sodd[i]);
    }
  };
  // d_m (times 2 / N) of row r as a complex number
  const double sc = 2.0 / N;
  auto scale = [&](int r, int m) -> double2 {
    const double2 lm = lambda[r];
    const double dr = lm.x + coef * sigma[m - 1], di = lm.y;
    const double q = dr * dr + di * di;
    const double s = sc / q;
    return make_double2(dr * s, -di * s);
  };

  C v[E::P];
  // first transform: forward stages on conj(c); F = conj of the result, to LDS
  E::fwd1(v, tw, load);
  {
    auto s1a = [](int i) { return E::a_of_s1(i); };
    auto s2a = [](int i) { return E::a_of_s2(i); };
    auto s2b = [](int i) { return E::b_of_s2(i); };
    auto s3b = [](int i) { return E::b_of_s3(i); };
    E::template exchange<C>(lds, v, s1a, s2a);
    E::fwd2(v, tw);
    E::template exchange<C>(lds, v, s2b, s3b);
  }
#pragma unroll
  for (int b = 0; b < E::B3; ++b) {
    int f, k1, k2;
    E::dec3(threadIdx.x + b * 256, f, k1, k2);
    C* x = v + b * E::N3;
    dft_any<E::N3, -1>(x);
#pragma unroll
    for (int k3 = 0; k3 < E::N3; ++k3)
      buf[at(f, k1 + E::N1 * k2 + E::N1 * E::N2 * k3)] = cconj(x[k3]);
  }
  __syncthreads();
  // W = d S(z1) (times 2 / N), in place
  {
    const int it = min(item0 + fs, nitems - 1);
    auto emit_w = [&](int f, int m, C Sm) {
      C w = cmk<C>((R)0, (R)0);
      if (m >= 1) {
        if (DUAL && it == 0) {
          const double da = scale(0, m).x, db = scale(nrows - 1, m).x;
          w = cmk<C>((R)(Sm.x * da), (R)(Sm.y * db));
        } else {
          const double2 d = scale(it, m);
          w = cmk<C>((R)(Sm.x * d.x - Sm.y * d.y), (R)(Sm.x * d.y + Sm.y * d.x));
        }
      }
      buf[at(f, m)] = w;
    };
    sine_sums(emit_w);
  }
  __syncthreads();
  // second transform: c'_k of W into the stage-3 layout, then the inverse stages
#pragma unroll
  for (int b = 0; b < E::B3; ++b) {
    int f, k1, k2;
    E::dec3(threadIdx.x + b * 256, f, k1, k2);
    C* x = v + b * E::N3;
#pragma unroll
    for (int k3 = 0; k3 < E::N3; ++k3) {
      const int k = k1 + E::N1 * k2 + E::N1 * E::N2 * k3;
      const C a = buf[at(f, k)];
      const C c = k == 0 ? cmk<C>((R)0, (R)0) : buf[at(f, N - k)];
      const R sk = sinN(k);
      x[k3] = cmk<C>(sk * (a.x + c.x) + (R)0.5 * (a.x - c.x), sk * (a.y + c.y) + (R)0.5 * (a.y - c.y));
    }
    dft_any<E::N3, +1>(x);
  }
  __syncthreads();
  {
    auto s1a = [](int i) { return E::a_of_s1(i); };
    auto s2a = [](int i) { return E::a_of_s2(i); };
    auto s2b = [](int i) { return E::b_of_s2(i); };
    auto s3b = [](int i) { return E::b_of_s3(i); };
    E::template exchange<C>(lds, v, s3b, s2b);
    E::inv2(v, tw);
    E::template exchange<C>(lds, v, s2a, s1a);
  }
  auto store_f = [&](int, int f, int idx, int, C c) { buf[at(f, idx)] = c; };
  E::inv1(v, tw, store_f);
  __syncthreads();
  // z2 = S(W): to LDS, then written out row by row
  auto emit_out = [&](int f, int m, C Sm) { buf[at(f, m)] = Sm; };
  sine_sums(emit_out);
  __syncthreads();
  for (int e = threadIdx.x; e < NB * n; e += 256) {
    const int f = e / n, m = e - f * n + 1;
    const int it = item0 + f;
    if (it >= nitems) continue;
    const C val = buf[at(f, m)];
    if (DUAL && it == 0) {
      zout[m - 1] = cmk<C>(val.x, (R)0);
      zout[(size_t)(nrows - 1) * n + m - 1] = cmk<C>(val.y, (R)0);
    } else {
      zout[(size_t)it * n + m - 1] = val;
    }
  }
}

// Columns of [nf][My][Mx] planes: one block per (frequency, tile of NB columns), columns taken
// fastest by the threads.  DST along y, divide by lambda_n + coef_x sigma^x_ix +
// coef_y sigma^y_iy (the x-direction DST has already been applied to the rows), DST again.
template <int P, int NB, int NT, typename C, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_dst_cols(C* __restrict__ z, int Mx,
                                                 const double2* __restrict__ lambda,
                                                 const double* __restrict__ sigx,
                                                 const double* __restrict__ sigy, double cx,
                                                 double cy, const C* __restrict__ tw) {
  using R = typename cplx_traits<C>::real;
  constexpr int n = P / 2 - 1;  // My
  constexpr int LDN = P + 1;
  __shared__ C buf[NB * LDN];
  const int ntile = (Mx + NB - 1) / NB;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);  // neighbouring tiles share cache lines
  const int fq = bid / ntile, x0 = (bid % ntile) * NB;
  C* plane = z + (size_t)fq * n * Mx;
  const R sc = (R)sqrt(2.0 / (n + 1));
  const double2 lam = lambda[fq];
  auto load = [&](int b, int idx) -> C {
    const int x = x0 + b;
    if (x >= Mx || idx == 0 || idx == n + 1) return cmk<C>((R)0, (R)0);
    if (idx <= n) return plane[(size_t)(idx - 1) * Mx + x];
    const C v = plane[(size_t)(P - idx - 1) * Mx + x];
    return cmk<C>(-v.x, -v.y);
  };
  auto store_scaled = [&](int b, int idx, C y) {
    const int x = x0 + b;
    C* B = buf + b * LDN;
    if (idx == 0 || idx == n + 1) {
      B[idx] = cmk<C>((R)0, (R)0);
    } else if (idx <= n) {
      C wv = cmk<C>((R)0, (R)0);
      if (x < Mx) {
        const double dr = lam.x + cx * sigx[x] + cy * sigy[idx - 1], di = lam.y;
        const double den = dr * dr + di * di;
        wv = cmul(dst_coef(y, sc), cmk<C>((R)(dr / den), (R)(-di / den)));
      }
      B[idx] = wv;
      B[P - idx] = cmk<C>(-wv.x, -wv.y);
    }
  };
  fft_io<P, -1, NT, NB, LDN, true, true, true, MAXR>(buf, tw, load, store_scaled);
  __syncthreads();
  auto store_out = [&](int b, int idx, C y) {
    const int x = x0 + b;
    if (x < Mx && idx >= 1 && idx <= n) plane[(size_t)(idx - 1) * Mx + x] = dst_coef(y, sc);
  };
  NoLoad nl;
  fft_io<P, -1, NT, NB, LDN, true, false, true, MAXR>(buf, tw, nl, store_out);
}

template <int P, typename C>
constexpr int dst_nb() {
  constexpr int target = (int)sizeof(C) == 16 ? 8 : 16;
  constexpr int cap = 135168 / ((P + 1) * (int)sizeof(C));
  return cap < 1 ? 1 : (cap < target ? cap : target);
}
// Largest radix: 8 up to P = 512 (twice the threads of radix 16 for the same LDS, so more waves
// per CU hide the global-memory latency of these short transforms), 16 above.
template <int P> constexpr int dst_maxr() { return P <= 512 ? 8 : 16; }
// one largest-radix butterfly per thread (NB P / MAXR, between 64 and 512)
template <int P, typename C>
constexpr int dst_nt() {
  constexpr int t = dst_nb<P, C>() * P / dst_maxr<P>();
  return t < 64 ? 64 : (t > 512 ? 512 : t);
}

template <int P, typename C>
static int dst3_scale(const Plan& p, const C* zin, C* z, int nrows, const double* sigma,
                      double coef, const C* tw) {
  using E = Fft3WideMid<P, 256>;
  // P = 8192 in FP64 needs more than 256 registers per lane at one wave per SIMD; two waves
  // with a few spills run faster (71 vs 77 us at M = 4095)
  constexpr int W = (P >= 8192 && sizeof(C) == 16) ? 2 : 1;
  const bool dual = p.Nt % 2 == 0 && nrows == p.Nt / 2 + 1 && nrows >= 2;
  const int items = dual ? nrows - 1 : nrows;
  const int grid = (items + E::NB - 1) / E::NB;
  if (dual)
    k_dst3_scale<P, C, W, true><<<grid, 256, 0, p.stream>>>(zin, z, nrows, p.lambda, sigma, coef,
                                                            tw);
  else
    k_dst3_scale<P, C, W, false><<<grid, 256, 0, p.stream>>>(zin, z, nrows, p.lambda, sigma, coef,
                                                             tw);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

template <int P, typename C, bool SCALE>
static int dst_rows(const Plan& p, C* z, int nrows, int rows_per_freq, const double* sigma,
                    double coef, const C* tw) {
  constexpr int NB = dst_nb<P, C>();
  constexpr int NT = dst_nt<P, C>();
  k_dst_rows<P, NB, NT, C, SCALE, dst_maxr<P>()><<<(nrows + NB - 1) / NB, NT, 0, p.stream>>>(
      z, nrows, rows_per_freq, p.lambda, sigma, coef, tw);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

template <int P, typename C>
static int dst_cols(const Plan& p, C* z, const C* tw) {
  constexpr int NB = dst_nb<P, C>();
  constexpr int NT = dst_nt<P, C>();
  const int ntile = (p.Mx + NB - 1) / NB;
  k_dst_cols<P, NB, NT, C, dst_maxr<P>()><<<p.nf * ntile, NT, 0, p.stream>>>(z, p.Mx, p.lambda, p.sigma,
                                                              p.sigma + p.Mx, p.coef_x, p.coef_y,
                                                              tw);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

#define RFDE_P_SWITCH(Pval, FN, ...)           \
  switch (Pval) {                              \
    case 4: return FN<4, __VA_ARGS__;          \
    case 8: return FN<8, __VA_ARGS__;          \
    case 16: return FN<16, __VA_ARGS__;        \
    case 32: return FN<32, __VA_ARGS__;        \
    case 64: return FN<64, __VA_ARGS__;        \
    case 128: return FN<128, __VA_ARGS__;      \
    case 256: return FN<256, __VA_ARGS__;      \
    case 512: return FN<512, __VA_ARGS__;      \
    case 1024: return FN<1024, __VA_ARGS__;    \
    case 2048: return FN<2048, __VA_ARGS__;    \
    case 4096: return FN<4096, __VA_ARGS__;    \
    case 8192: return FN<8192, __VA_ARGS__;    \
    default: return RFDE_EUNSUPPORTED;         \
  }

// Twiddle tables for the DST lengths live after the L tables: they are built on demand by the
// plan (p.twD holds 2 (Mx+1) entries then 2 (My+1) in 2D; 2 (M+1) in 1D), double and float.
template <int P, typename C>
static int dst_half(const Plan& p, const C* zin, C* z, const C* tw) {
  constexpr int N = P / 2;
  using E = Fft3<Split3<N>::N1, Split3<N>::N2, Split3<N>::N3, Split3<N>::NB, 256, 2>;
  // two workgroups per CU: the padded spectrum takes 73.7 KB of LDS
  constexpr int W = 2;
  const int nrows = p.nf;
  const bool dual = p.Nt % 2 == 0 && nrows == p.Nt / 2 + 1 && nrows >= 2;
  const int items = dual ? nrows - 1 : nrows;
  const int grid = (items + E::NB - 1) / E::NB;
  if (dual)
    k_dst_half<N, C, W, true><<<grid, 256, 0, p.stream>>>(zin, z, nrows, p.lambda, p.sigma,
                                                         p.coef, tw);
  else
    k_dst_half<N, C, W, false><<<grid, 256, 0, p.stream>>>(zin, z, nrows, p.lambda, p.sigma,
                                                          p.coef, tw);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// FP64 rows of P >= 512 take the half-length transform.  In FP32 its prefix sums over N / 2
// entries lose more than the full-length transform does (5.6e-5 relative at M = 4095,
// alpha = 1.8, where the full length stays within 2e-5), so FP32 keeps the full length.
template <int P, typename C>
static int dst_1d(const Plan& p, const C* zin, C* z, const C* tw) {
  if constexpr (P >= 512 && sizeof(C) == 16) {
    return dst_half<P, C>(p, zin, z, tw);
  } else if constexpr (P >= 256) {
    return dst3_scale<P, C>(p, zin, z, p.nf, p.sigma, p.coef, tw);
  } else {
    if (zin != z)
      RFDE_HIP(hipMemcpyAsync(z, zin, (size_t)p.nf * p.S * sizeof(C), hipMemcpyDeviceToDevice,
                              p.stream));
    return dst_rows<P, C, true>(p, z, p.nf, 1, p.sigma, p.coef, tw);
  }
}

template <typename C>
static int tau_solve_t(const Plan& p, const void* zinv, void* zio) {
  C* z = (C*)zio;
  const C* zin = (const C*)zinv;
  const bool f32 = std::is_same<C, float2>::value;
  if (p.dim == 1) {
    if (p.bs[0].LB) return tau_solve_1d_bs<C>(p, zin, z);
    const int P = 2 * (p.M + 1);
    const C* tw = f32 ? (const C*)((double2*)p.twD + P) : (const C*)p.twD;
    RFDE_P_SWITCH(P, dst_1d, C>(p, zin, z, tw));
  }
  if (zin != z)
    RFDE_HIP(hipMemcpyAsync(z, zin, (size_t)p.nf * p.S * sizeof(C), hipMemcpyDeviceToDevice,
                            p.stream));
  const int Px = 2 * (p.Mx + 1), Py = 2 * (p.My + 1);
  const double2* twd = p.twD;
  const C* twx = f32 ? (const C*)(twd + Px + Py) : (const C*)twd;
  const C* twy = f32 ? (const C*)((const float2*)(twd + Px + Py) + Px) : (const C*)(twd + Px);
  // axes whose 2(n+1) is not a power of two take the chirp-z DST (k_dst_bs.hip)
  auto rows = [&]() -> int {
    if (p.bs[0].LB) return tau_rows_2d_bs<C>(p, z);
    RFDE_P_SWITCH(Px, dst_rows, C, false>(p, z, p.nf * p.My, p.My, p.sigma, 0.0, twx));
  };
  auto cols = [&]() -> int {
    if (p.bs[1].LB) return tau_cols_2d_bs<C>(p, z);
    RFDE_P_SWITCH(Py, dst_cols, C>(p, z, twy));
  };
  int rc = rows();
  if (rc != RFDE_OK) return rc;
  rc = cols();
  if (rc != RFDE_OK) return rc;
  return rows();
}

int launch_tau_solve(const Plan& p, const void* zin, void* zout) {
  if (p.opts.precond_bits == 32) return tau_solve_t<float2>(p, zin, zout);
  return tau_solve_t<double2>(p, zin, zout);
}

}  // namespace rfde
