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

// Radix chosen for the pass that follows a sub-length Ns of a length-N transform.
__host__ __device__ constexpr int pass_radix(int N, int Ns) {
  return (N / Ns) >= 16 ? 16 : (N / Ns);
}

// One Stockham pass over `nb` batched transforms stored back to back in `buf` (stride N).
// All NT threads of the block participate; includes the two barriers.
template <int N, int R, int SIGN, int NT, int NB, typename C>
__device__ __forceinline__ void stockham_pass(C* buf, int Ns, const C* __restrict__ tw) {
  constexpr int NBF = N / R;               // butterflies per transform
  constexpr int TOT = NBF * NB;            // butterflies in the block
  constexpr int BPT = (TOT + NT - 1) / NT; // butterflies per thread
  C v[BPT][R];
  const int tid = threadIdx.x;
  const int step = N / (Ns * R);
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jj = tid + b * NT;
    if (TOT % NT == 0 || jj < TOT) {
      const int f = jj / NBF, j = jj - f * NBF;
      const int k = j % Ns;
      C* src = buf + f * N;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = src[j + t * NBF];
      if (Ns > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          C w = tw[t * k * step];
          if (SIGN > 0) w = cconj(w);
          v[b][t] = cmul(v[b][t], w);
        }
      }
      dft_r<R, SIGN>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int jj = tid + b * NT;
    if (TOT % NT == 0 || jj < TOT) {
      const int f = jj / NBF, j = jj - f * NBF;
      const int k = j % Ns;
      C* dst = buf + f * N;
      const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) dst[idxD + t * Ns] = v[b][t];
    }
  }
  __syncthreads();
}

// Full length-N transform of NB batched sequences held in LDS (natural order in and out).
// The caller must __syncthreads() after filling buf.
template <int N, int SIGN, int NT, int NB, typename C>
__device__ __forceinline__ void fft_lds(C* buf, const C* __restrict__ tw) {
  if constexpr (N >= 2) {
    constexpr int R0 = pass_radix(N, 1);
    stockham_pass<N, R0, SIGN, NT, NB>(buf, 1, tw);
    if constexpr (N / R0 >= 2) {
      constexpr int Ns1 = R0;
      constexpr int R1 = pass_radix(N, Ns1);
      stockham_pass<N, R1, SIGN, NT, NB>(buf, Ns1, tw);
      if constexpr (N / (Ns1 * R1) >= 2) {
        constexpr int Ns2 = Ns1 * R1;
        constexpr int R2 = pass_radix(N, Ns2);
        stockham_pass<N, R2, SIGN, NT, NB>(buf, Ns2, tw);
        if constexpr (N / (Ns2 * R2) >= 2) {
          constexpr int Ns3 = Ns2 * R2;
          constexpr int R3 = pass_radix(N, Ns3);
          stockham_pass<N, R3, SIGN, NT, NB>(buf, Ns3, tw);
          if constexpr (N / (Ns3 * R3) >= 2) {
            constexpr int Ns4 = Ns3 * R3;
            constexpr int R4 = pass_radix(N, Ns4);
            stockham_pass<N, R4, SIGN, NT, NB>(buf, Ns4, tw);
            static_assert(N / (Ns4 * R4) < 2, "FFT length beyond 16^5");
          }
        }
      }
    }
  }
}

}  // namespace rfde
