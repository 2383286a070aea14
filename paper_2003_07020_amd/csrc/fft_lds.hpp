// LDS-resident power-of-two FFT building blocks for gfx950 (wave64).
//
// Transforms are radix-{2,4,8,16} Stockham passes on a double2 (or float2) buffer in LDS:
// each pass reads R points at stride N/R, applies the twiddles w^(t k) of its sub-length,
// does an in-register radix-R DFT and, after a barrier, writes the R outputs at stride Ns
// (Govindaraju et al., "High performance discrete Fourier transforms on graphics
// processors", SC'08, Stockham autosort formulation).  The result is in natural order.
//
// Sign convention: SIGN = -1 computes X_m = sum_j x_j exp(-2 pi i j m / N),
//                  SIGN = +1 computes X_m = sum_j x_j exp(+2 pi i j m / N)   (no 1/N).
// Twiddles come from a table tw[m] = exp(-2 pi i m / N), m = 0..N-1, held in global memory
// (read through the vector L1/L2 caches); the +1 direction uses its conjugate.
#pragma once
#include <hip/hip_runtime.h>

namespace rfde {

template <typename C> struct cplx_traits;
template <> struct cplx_traits<double2> { using real = double; };
template <> struct cplx_traits<float2> { using real = float; };

template <typename C> __device__ __forceinline__ C cmk(typename cplx_traits<C>::real x,
                                                       typename cplx_traits<C>::real y) {
  C r; r.x = x; r.y = y; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
// multiply by i^SIGN: SIGN=-1 -> -i, SIGN=+1 -> +i
template <int SIGN, typename C> __device__ __forceinline__ C mul_i(C a) {
  return SIGN < 0 ? cmk<C>(a.y, -a.x) : cmk<C>(-a.y, a.x);
}

// In-register DFTs (natural order in, natural order out).
template <int SIGN, typename C> __device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a; a = cadd(t, b); b = csub(t, b);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft4(C* v) {
  C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  C b0 = cadd(v[1], v[3]), b1 = mul_i<SIGN>(csub(v[1], v[3]));
  v[0] = cadd(a0, b0); v[2] = csub(a0, b0);
  v[1] = cadd(a1, b1); v[3] = csub(a1, b1);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft8(C* v) {
  using R = typename cplx_traits<C>::real;
  const R s = (R)0.70710678118654752440084436210484903928;
  C e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
  dft4<SIGN>(e); dft4<SIGN>(o);
  // o[k] *= exp(SIGN 2 pi i k / 8)
  o[1] = cmk<C>(s * (o[1].x - SIGN * o[1].y), s * (o[1].y + SIGN * o[1].x));
  o[2] = mul_i<SIGN>(o[2]);
  o[3] = cmk<C>(-s * (o[3].x + SIGN * o[3].y), s * (SIGN * o[3].x - o[3].y));
#pragma unroll
  for (int k = 0; k < 4; ++k) { v[k] = cadd(e[k], o[k]); v[k + 4] = csub(e[k], o[k]); }
}

template <int SIGN, typename C> __device__ __forceinline__ void dft16(C* v) {
  using R = typename cplx_traits<C>::real;
  // 16 = 4 x 4: DFT4 over stride-4 groups, twiddle, DFT4 over the other index.
  C a[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int p = 0; p < 4; ++p) a[q][p] = v[q + 4 * p];
    dft4<SIGN>(a[q]);
  }
  // twiddle a[q][p] *= exp(SIGN 2 pi i q p / 16)
  const R c1 = (R)0.92387953251128675612818318939678828682, s1 = (R)0.38268343236508977172845998403039886676;
  const R c2 = (R)0.70710678118654752440084436210484903928;
#pragma unroll
  for (int q = 1; q < 4; ++q) {
#pragma unroll
    for (int p = 1; p < 4; ++p) {
      const int e = q * p;  // 1..9
      R wc, ws;
      switch (e) {
        case 1: wc = c1; ws = s1; break;
        case 2: wc = c2; ws = c2; break;
        case 3: wc = s1; ws = c1; break;
        case 4: wc = 0; ws = 1; break;
        case 6: wc = -c2; ws = c2; break;
        default: wc = -c1; ws = -s1; break;  // 9: angle 9pi/8 -> cos = -c1, sin = -s1
      }
      C w = cmk<C>(wc, SIGN * ws);
      a[q][p] = cmul(a[q][p], w);
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    C t[4] = {a[0][p], a[1][p], a[2][p], a[3][p]};
    dft4<SIGN>(t);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[p + 4 * q] = t[q];
  }
}

template <int R, int SIGN, typename C> __device__ __forceinline__ void dft_r(C* v) {
  if constexpr (R == 2) dft2<SIGN>(v[0], v[1]);
  else if constexpr (R == 4) dft4<SIGN>(v);
  else if constexpr (R == 8) dft8<SIGN>(v);
  else dft16<SIGN>(v);
}

// Radix chosen for the pass that follows a sub-length Ns of a length-N transform (largest
// radix MAXR, 16 or 8; the last pass takes what remains).
__host__ __device__ constexpr int pass_radix(int N, int Ns, int MAXR = 16) {
  return (N / Ns) >= MAXR ? MAXR : (N / Ns);
}

// Placeholder functors for passes that stay inside LDS.
struct NoLoad {};
struct NoStore {};

// One Stockham pass over NB batched transforms held in LDS (transform f at buf + f * LDN).
//   FIRST: the pass reads its inputs through load(f, idx) instead of from buf (no LDS read);
//   LAST:  the pass hands its outputs to store(f, idx, value) instead of writing buf.
//   BFAST: consecutive threads take consecutive transforms (batch index fastest), which makes
//          strided global loads/stores of the FIRST/LAST passes coalesced when the transforms
//          are adjacent columns of a row-major array; LDN should then be odd (N + 1).
// Twiddles: w = tw[k * step] is read once per butterfly (tw[m] = exp(-2 pi i m / N)) and its
// powers w^t are formed by repeated multiplication.
// Barriers: after the reads when they came from buf (the pass is in place), and after the
// writes when they went to buf.  A caller must synchronise before reusing buf after a LAST
// pass whose store writes buf.
template <int N, int R, int Ns, int SIGN, int NT, int NB, int LDN, bool BFAST, bool FIRST,
          bool LAST, typename C, typename Load, typename Store>
__device__ __forceinline__ void stockham_pass_io(C* buf, const C* __restrict__ tw, Load& load,
                                                 Store& store) {
  constexpr int NBF = N / R;               // butterflies per transform
  constexpr int TOT = NBF * NB;            // butterflies in the block
  constexpr int BPT = (TOT + NT - 1) / NT; // butterflies per thread
  constexpr int step = N / (Ns * R);
  C v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jj = tid + b * NT;
    if (TOT % NT == 0 || jj < TOT) {
      const int f = BFAST ? jj % NB : jj / NBF;
      const int j = BFAST ? jj / NB : jj - f * NBF;
      const int k = j & (Ns - 1);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        if constexpr (FIRST) v[b][t] = load(f, j + t * NBF);
        else v[b][t] = buf[f * LDN + j + t * NBF];
      }
      if constexpr (Ns > 1) {
        C w = tw[k * step];
        if (SIGN > 0) w = cconj(w);
        C wt = w;
        v[b][1] = cmul(v[b][1], wt);
#pragma unroll
        for (int t = 2; t < R; ++t) {
          wt = cmul(wt, w);
          v[b][t] = cmul(v[b][t], wt);
        }
      }
      dft_r<R, SIGN>(v[b]);
    }
  }
  if constexpr (!FIRST) __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jj = tid + b * NT;
    if (TOT % NT == 0 || jj < TOT) {
      const int f = BFAST ? jj % NB : jj / NBF;
      const int j = BFAST ? jj / NB : jj - f * NBF;
      const int k = j & (Ns - 1);
      const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        if constexpr (LAST) store(f, idxD + t * Ns, v[b][t]);
        else buf[f * LDN + idxD + t * Ns] = v[b][t];
      }
    }
  }
  if constexpr (!LAST) __syncthreads();
}

template <int N, int Ns, int SIGN, int NT, int NB, int LDN, bool BFAST, bool FIRST_EXT,
          bool LAST_EXT, int MAXR, typename C, typename Load, typename Store>
__device__ __forceinline__ void fft_passes(C* buf, const C* __restrict__ tw, Load& load,
                                           Store& store) {
  constexpr int R = pass_radix(N, Ns, MAXR);
  constexpr bool last = (Ns * R >= N);
  stockham_pass_io<N, R, Ns, SIGN, NT, NB, LDN, BFAST, FIRST_EXT && Ns == 1, LAST_EXT && last>(
      buf, tw, load, store);
  if constexpr (!last) {
    fft_passes<N, Ns * R, SIGN, NT, NB, LDN, BFAST, FIRST_EXT, LAST_EXT, MAXR>(buf, tw, load,
                                                                               store);
  }
}

// Length-N transform of NB sequences, first inputs from load(f, idx) (or buf), last outputs to
// store(f, idx, value) (or buf, natural order).  N must be a power of two >= 2.
template <int N, int SIGN, int NT, int NB, int LDN, bool BFAST, bool FIRST_EXT, bool LAST_EXT,
          int MAXR = 16, typename C, typename Load, typename Store>
__device__ __forceinline__ void fft_io(C* buf, const C* __restrict__ tw, Load& load, Store& store) {
  fft_passes<N, 1, SIGN, NT, NB, LDN, BFAST, FIRST_EXT, LAST_EXT, MAXR>(buf, tw, load, store);
}

// Full length-N transform of NB batched sequences held in LDS (natural order in and out,
// transform f at buf + f * N).  The caller must __syncthreads() after filling buf.
template <int N, int SIGN, int NT, int NB, typename C>
__device__ __forceinline__ void fft_lds(C* buf, const C* __restrict__ tw) {
  NoLoad nl;
  NoStore ns;
  fft_passes<N, 1, SIGN, NT, NB, N, false, false, false, 16>(buf, tw, nl, ns);
}

}  // namespace rfde
