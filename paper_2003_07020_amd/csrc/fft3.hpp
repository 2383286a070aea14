// Three-stage register FFT for gfx950: NB transforms of length N = N1 N2 N3 per workgroup of
// NT threads, every thread holding P = N NB / NT points in registers for the whole transform.
//
// Forward transform (decimation in frequency) with n = n1 N2 N3 + n2 N3 + n3 and
// k = k1 + N1 k2 + N1 N2 k3, w = exp(-2 pi i / N):
//   stage 1, over n1 for each (n2, n3): DFT of length N1, then times w^((n2 N3 + n3) k1);
//   stage 2, over n2 for each (k1, n3): DFT of length N2, then times w^(N1 n3 k2);
//   stage 3, over n3 for each (k1, k2): DFT of length N3, giving X[k] in registers.
// A pointwise product is applied there and the unnormalised inverse runs the same stages in
// reverse (decimation in time: conjugate twiddles before each DFT), so the spectrum is never
// brought into natural order and the middle of the transform pair needs no exchange at all.
//
// Between stages the points move through LDS one real component at a time (half the LDS of a
// complex exchange, so two or more workgroups share a CU), in two layouts per transform f:
//   A(k1, n2, n3) = f ZA + k1 SA + n2 N3 + n3,        SA = N3 (N2 + 1), ZA = N1 SA
//   B(k1, k2, n3) = f ZB + k1 SB + k2 (N3 + 1) + n3,  SB = N2 (N3 + 1), ZB = N1 SB
// Consecutive lanes take consecutive n3 (writes of A and B, reads of A) or consecutive k2
// (reads of B, odd stride N3 + 1); the paddings keep the 16 and 32 consecutive lanes of one
// 8-byte access in distinct banks for the radix splits instantiated here.
#pragma once
#include <type_traits>

#include "fft_lds.hpp"

namespace rfde {

// Length-32 DFT in registers from two length-16 DFTs (even and odd samples).
template <int SIGN, typename C> __device__ __forceinline__ void dft32(C* v) {
  using R = typename cplx_traits<C>::real;
  // cos(pi k / 16), k = 0..8
  constexpr R cs[9] = {(R)1.0,
                       (R)0.98078528040323044912618223613424,
                       (R)0.92387953251128675612818318939679,
                       (R)0.83146961230254523707878837761791,
                       (R)0.70710678118654752440084436210485,
                       (R)0.55557023301960222474283081394853,
                       (R)0.38268343236508977172845998403040,
                       (R)0.19509032201612826784828486847702,
                       (R)0.0};
  C e[16], o[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    e[m] = v[2 * m];
    o[m] = v[2 * m + 1];
  }
  dft16<SIGN>(e);
  dft16<SIGN>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    // o[k] times exp(SIGN 2 pi i k / 32) = (cos(pi k / 16), SIGN sin(pi k / 16))
    C t;
    if (k == 0) {
      t = o[0];
    } else if (k == 8) {
      t = mul_i<SIGN>(o[8]);
    } else {
      const R c = k < 8 ? cs[k] : -cs[16 - k];
      const R s = k < 8 ? cs[8 - k] : cs[k - 8];
      t = cmul(o[k], cmk<C>(c, SIGN * s));
    }
    v[k] = cadd(e[k], t);
    v[k + 16] = csub(e[k], t);
  }
}

template <int R, int SIGN, typename C> __device__ __forceinline__ void dft_any(C* v) {
  if constexpr (R == 32) dft32<SIGN>(v);
  else dft_r<R, SIGN>(v);
}

// v[k] *= w^k for k = 1..R-1, w = tw[e] (conjugated for SIGN > 0), tw[m] = exp(-2 pi i m / N).
// The powers are formed by repeated multiplication and restarted from the table at k = 16
// (tw[16 e]), which keeps the rounding of the chain to at most 15 products.
template <int R, int SIGN, typename C>
__device__ __forceinline__ void twiddle_pow(C* v, const C* __restrict__ tw, int e) {
  if constexpr (R > 1) {
    C w = tw[e];
    if (SIGN > 0) w = cconj(w);
    C wk = w;
    v[1] = cmul(v[1], wk);
#pragma unroll
    for (int k = 2; k < R; ++k) {
      if (k == 16) {
        wk = tw[16 * e];
        if (SIGN > 0) wk = cconj(wk);
      } else {
        wk = cmul(wk, w);
      }
      v[k] = cmul(v[k], wk);
    }
  }
}

// TWS: stride of the twiddle table, tw[m TWS] = exp(-2 pi i m / N) (a table of a multiple of the
// length serves).
template <int N1_, int N2_, int N3_, int NB_, int NT_, int TWS = 1>
struct Fft3 {
  static constexpr int N1 = N1_, N2 = N2_, N3 = N3_, NB = NB_, NT = NT_;
  static constexpr int N = N1 * N2 * N3;
  static constexpr int T1 = N2 * N3;  // stage-1 butterflies per transform
  static constexpr int SA = N3 * (N2 + 1), SB = N2 * (N3 + 1);
  static constexpr int ZA = N1 * SA, ZB = N1 * SB;
  static constexpr int LDS = NB * (ZA > ZB ? ZA : ZB);  // reals
  static constexpr int P = N * NB / NT;                 // points per thread
  static constexpr int B1 = NB * N2 * N3 / NT, B2 = NB * N1 * N3 / NT, B3 = NB * N1 * N2 / NT;
  static_assert(B1 * NT == NB * N2 * N3 && B2 * NT == NB * N1 * N3 && B3 * NT == NB * N1 * N2,
                "every stage must give each thread a whole number of butterflies");

  // butterfly u of stage 1: transform f, t = n2 N3 + n3
  __device__ static __forceinline__ void dec1(int u, int& f, int& t) {
    f = u / T1;
    t = u % T1;
  }
  // butterfly u of stage 2: transform f, (k1, n3)
  __device__ static __forceinline__ void dec2(int u, int& f, int& k1, int& n3) {
    f = u / (N1 * N3);
    const int r = u % (N1 * N3);
    k1 = r / N3;
    n3 = r % N3;
  }
  // butterfly u of stage 3: transform f, (k1, k2)
  __device__ static __forceinline__ void dec3(int u, int& f, int& k1, int& k2) {
    f = u / (N1 * N2);
    const int r = u % (N1 * N2);
    k1 = r / N2;
    k2 = r % N2;
  }
  __device__ static __forceinline__ int addrA(int f, int k1, int n2, int n3) {
    return f * ZA + k1 * SA + n2 * N3 + n3;
  }
  __device__ static __forceinline__ int addrB(int f, int k1, int k2, int n3) {
    return f * ZB + k1 * SB + k2 * (N3 + 1) + n3;
  }

  // Move the P points through LDS, real parts then imaginary parts: register i leaves from
  // address wa(i) and register i is refilled from address ra(i).
  template <typename C, typename WA, typename RA>
  __device__ static __forceinline__ void exchange(typename cplx_traits<C>::real* lds, C* v,
                                                  WA wa, RA ra) {
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int i = 0; i < P; ++i) lds[wa(i)] = part ? v[i].y : v[i].x;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < P; ++i) (part ? v[i].y : v[i].x) = lds[ra(i)];
      __syncthreads();
    }
  }
  // register i in stage 1: butterfly i / N1, index k1 (or n1) = i % N1
  __device__ static __forceinline__ int a_of_s1(int i) {
    int f, t;
    dec1(threadIdx.x + (i / N1) * NT, f, t);
    return f * ZA + (i % N1) * SA + t;
  }
  // register i in stage 2 (layout A): butterfly i / N2, index n2 = i % N2
  __device__ static __forceinline__ int a_of_s2(int i) {
    int f, k1, n3;
    dec2(threadIdx.x + (i / N2) * NT, f, k1, n3);
    return addrA(f, k1, i % N2, n3);
  }
  // register i in stage 2 (layout B): butterfly i / N2, index k2 = i % N2
  __device__ static __forceinline__ int b_of_s2(int i) {
    int f, k1, n3;
    dec2(threadIdx.x + (i / N2) * NT, f, k1, n3);
    return addrB(f, k1, i % N2, n3);
  }
  // register i in stage 3: butterfly i / N3, index n3 = i % N3
  __device__ static __forceinline__ int b_of_s3(int i) {
    int f, k1, k2;
    dec3(threadIdx.x + (i / N3) * NT, f, k1, k2);
    return addrB(f, k1, k2, i % N3);
  }

  // Transform of stage-1 butterfly b of this thread, as a wave-uniform (scalar) value: T1 is a
  // multiple of 64, so every lane of a wave works on the same transform.
  __device__ static __forceinline__ int f_of_b1(int b) {
    static_assert(T1 % 64 == 0 && NT % 64 == 0, "stage-1 transforms must be wave-uniform");
    return __builtin_amdgcn_readfirstlane(((int)threadIdx.x + b * NT) / T1);
  }

  // Forward stage 1: inputs from load(b, f, idx, n1), idx = n1 T1 + t the natural index of
  // transform f (wave-uniform), b the thread's butterfly.
  template <typename C, typename Load>
  __device__ static __forceinline__ void fwd1(C* v, const C* __restrict__ tw, Load& load) {
#pragma unroll
    for (int b = 0; b < B1; ++b) {
      const int t = (threadIdx.x + b * NT) % T1;
      const int f = f_of_b1(b);
      C* x = v + b * N1;
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) x[n1] = load(b, f, n1 * T1 + t, n1);
      dft_any<N1, -1>(x);
      twiddle_pow<N1, -1>(x, tw, TWS * t);
    }
  }
  template <typename C>
  __device__ static __forceinline__ void fwd2(C* v, const C* __restrict__ tw) {
#pragma unroll
    for (int b = 0; b < B2; ++b) {
      int f, k1, n3;
      dec2(threadIdx.x + b * NT, f, k1, n3);
      C* x = v + b * N2;
      dft_any<N2, -1>(x);
      twiddle_pow<N2, -1>(x, tw, TWS * N1 * n3);
    }
  }
  // Stage 3 forward, pointwise(f, k, value&) on every X[k], stage 3 inverse.
  template <typename C, typename PW>
  __device__ static __forceinline__ void mid(C* v, PW& pw) {
#pragma unroll
    for (int b = 0; b < B3; ++b) {
      int f, k1, k2;
      dec3(threadIdx.x + b * NT, f, k1, k2);
      C* x = v + b * N3;
      dft_any<N3, -1>(x);
#pragma unroll
      for (int k3 = 0; k3 < N3; ++k3) pw(f, k1 + N1 * k2 + N1 * N2 * k3, x[k3]);
      dft_any<N3, +1>(x);
    }
  }
  template <typename C>
  __device__ static __forceinline__ void inv2(C* v, const C* __restrict__ tw) {
#pragma unroll
    for (int b = 0; b < B2; ++b) {
      int f, k1, n3;
      dec2(threadIdx.x + b * NT, f, k1, n3);
      C* x = v + b * N2;
      twiddle_pow<N2, +1>(x, tw, TWS * N1 * n3);
      dft_any<N2, +1>(x);
    }
  }
  // Inverse stage 1: outputs to store(b, f, idx, n1, value), as for fwd1.
  template <typename C, typename Store>
  __device__ static __forceinline__ void inv1(C* v, const C* __restrict__ tw, Store& store) {
#pragma unroll
    for (int b = 0; b < B1; ++b) {
      const int t = (threadIdx.x + b * NT) % T1;
      const int f = f_of_b1(b);
      C* x = v + b * N1;
      twiddle_pow<N1, +1>(x, tw, TWS * t);
      dft_any<N1, +1>(x);
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) store(b, f, n1 * T1 + t, n1, x[n1]);
    }
  }

  // y = IDFT(pw(DFT(x))) without the 1/N of the inverse: load -> 4 exchanges -> store.
  template <typename C, typename Load, typename PW, typename Store>
  __device__ static __forceinline__ void run(typename cplx_traits<C>::real* lds,
                                             const C* __restrict__ tw, Load& load, PW& pw,
                                             Store& store) {
    C v[P];
    fwd1(v, tw, load);
    auto s1a = [](int i) { return a_of_s1(i); };
    auto s2a = [](int i) { return a_of_s2(i); };
    auto s2b = [](int i) { return b_of_s2(i); };
    auto s3b = [](int i) { return b_of_s3(i); };
    exchange<C>(lds, v, s1a, s2a);
    fwd2(v, tw);
    exchange<C>(lds, v, s2b, s3b);
    mid(v, pw);
    exchange<C>(lds, v, s3b, s2b);
    inv2(v, tw);
    exchange<C>(lds, v, s2a, s1a);
    inv1(v, tw, store);
  }
};

// Radix split used for a transform of length N (N >= 256).
template <int N> struct Split3;
template <> struct Split3<256> { static constexpr int N1 = 4, N2 = 8, N3 = 8, NB = 8; };
template <> struct Split3<512> { static constexpr int N1 = 8, N2 = 8, N3 = 8, NB = 8; };
template <> struct Split3<1024> { static constexpr int N1 = 16, N2 = 8, N3 = 8, NB = 4; };
template <> struct Split3<2048> { static constexpr int N1 = 8, N2 = 16, N3 = 16, NB = 2; };
template <> struct Split3<4096> { static constexpr int N1 = 16, N2 = 16, N3 = 16, NB = 1; };
template <> struct Split3<8192> { static constexpr int N1 = 16, N2 = 16, N3 = 32, NB = 1; };

template <int N, int NT = 256>
using Fft3For = Fft3<Split3<N>::N1, Split3<N>::N2, Split3<N>::N3, Split3<N>::NB, NT>;

// Split with the radix-32 stage first for N = 8192: a pointwise step that needs many registers
// of its own then runs on two 16-point butterflies instead of one 32-point one.
template <int N, int NT = 256>
using Fft3WideMid = typename std::conditional<N == 8192, Fft3<32, 16, 16, 1, NT>,
                                              Fft3For<N, NT>>::type;

}  // namespace rfde
