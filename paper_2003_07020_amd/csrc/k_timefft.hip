// Preconditioner steps (a) and (c) (Section 3.1): the scaled DFT over the time index.
//
// step (a): z1_n = sum_j theta^{n j} s_j v_j,  theta = exp(+2 pi i / Nt), s_j = eps^{j/Nt},
//           for n = 0..Nt/2 (the other half is the complex conjugate, Section 3.2).
// step (c): v_j = (1 / (Nt s_j)) sum_n theta^{-n j} z2_n with z2_{Nt-n} = conj(z2_n).
//
// Layout: v is [Nt][S] (space fastest), z is [Nt/2+1][S] complex.  A block owns a tile of
// TS = 2 NB adjacent spatial points and all Nt time levels.  Two real sequences (points 2p and
// 2p+1 of the tile) share one complex transform and are separated with the conjugate symmetry
// of real-input DFTs: X = (Z_n + conj(Z_{Nt-n})) / 2, Y = (Z_n - conj(Z_{Nt-n})) / (2i).
// Threads take the NB transforms fastest, so every global access is a contiguous row segment
// of TS values (128 bytes where the LDS budget allows); the first pass of step (a) reads v
// straight from memory and the last pass of step (c) writes v straight to memory.
//
// Nt not a power of two: Bluestein's chirp-z form.  With w_k = exp(i pi k^2 / Nt),
// theta^{n j} = w_n w_j conj(w_{n-j}), so X_n = w_n sum_j (x_j w_j) conj(w_{n-j}) is a linear
// convolution of length-Nt sequences, done exactly as a cyclic one of power-of-two length
// Lt >= 2 Nt - 1 (forward FFT, product with the precomputed DFT of the kernel, inverse FFT),
// all in LDS.  Step (c) uses sum_n Z_n theta^{-n j} = conj(sum_n conj(Z_n) theta^{n j}).
#include "fft_lds.hpp"
#include "krylov.hpp"
#include "rfde_internal.hpp"

namespace rfde {

template <int N, int NB, int NT, typename C, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_time_fwd(const double* __restrict__ v, C* __restrict__ z1,
                                                 const double* __restrict__ s,
                                                 const double* __restrict__ vs,
                                                 const C* __restrict__ tw, int S,
                                                 const int* __restrict__ live) {
  if (live && *live == 0) return;
  using R = typename cplx_traits<C>::real;
  const double vsc = vs ? vs[0] : 1.0;
  constexpr int LDN = N + 1;
  __shared__ C buf[NB * LDN];
  constexpr int TS = 2 * NB;
  const int i0 = xcd_remap(blockIdx.x, gridDim.x) * TS;  // neighbours share lines: one XCD
  auto load = [&](int f, int j) -> C {
    const int i = i0 + 2 * f;
    const double* row = v + (size_t)j * S;
    const double sj = s[j] * vsc;
    const R a = (i < S) ? (R)(sj * row[i]) : (R)0;
    const R b = (i + 1 < S) ? (R)(sj * row[i + 1]) : (R)0;
    return cmk<C>(a, b);
  };
  NoStore ns;
  fft_io<N, +1, NT, NB, LDN, true, true, false, MAXR>(buf, tw, load, ns);
  for (int e = threadIdx.x; e < (N / 2 + 1) * TS; e += NT) {
    const int n = e / TS, q = e - n * TS;
    const int i = i0 + q;
    if (i >= S) continue;
    const C a = buf[(q >> 1) * LDN + n];
    const C b = cconj(buf[(q >> 1) * LDN + ((N - n) & (N - 1))]);
    C out;
    if ((q & 1) == 0) out = cmk<C>((R)0.5 * (a.x + b.x), (R)0.5 * (a.y + b.y));
    else out = cmk<C>((R)0.5 * (a.y - b.y), (R)-0.5 * (a.x - b.x));
    z1[(size_t)n * S + i] = out;
  }
}

template <int N, int NB, int NT, typename C, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_time_inv(const C* __restrict__ z2, double* __restrict__ v,
                                                 const double* __restrict__ s,
                                                 const C* __restrict__ tw, int S,
                                                 const int* __restrict__ live) {
  if (live && *live == 0) return;
  using R = typename cplx_traits<C>::real;
  constexpr int LDN = N + 1;
  __shared__ C buf[NB * LDN];
  constexpr int TS = 2 * NB;
  const int i0 = xcd_remap(blockIdx.x, gridDim.x) * TS;  // neighbours share lines: one XCD
  // Z_n = P_n + i Q_n with P, Q the half spectra of points 2p, 2p+1, extended by
  // P_{N-n} = conj(P_n); imaginary parts at n = 0 and n = N/2 are dropped.
  auto load = [&](int f, int n) -> C {
    const int ia = i0 + 2 * f, ib = ia + 1;
    const int nn = n <= N / 2 ? n : N - n;
    C P = cmk<C>((R)0, (R)0), Q = cmk<C>((R)0, (R)0);
    if (ia < S) P = z2[(size_t)nn * S + ia];
    if (ib < S) Q = z2[(size_t)nn * S + ib];
    if (nn == 0 || nn == N / 2) { P.y = (R)0; Q.y = (R)0; }
    if (n <= N / 2) return cmk<C>(P.x - Q.y, P.y + Q.x);
    return cmk<C>(P.x + Q.y, Q.x - P.y);
  };
  auto store = [&](int f, int j, C c) {
    const int i = i0 + 2 * f;
    double* row = v + (size_t)j * S;
    const double sc = 1.0 / ((double)N * s[j]);
    if (i < S) row[i] = (double)c.x * sc;
    if (i + 1 < S) row[i + 1] = (double)c.y * sc;
  };
  fft_io<N, -1, NT, NB, LDN, true, true, true, MAXR>(buf, tw, load, store);
}

// ---- Bluestein variants (Nt not a power of two, LB = Lt) ----
template <int LB, int NB, int NT, typename C, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_time_fwd_bs(const double* __restrict__ v, C* __restrict__ z1,
                                                    const double* __restrict__ s,
                                                    const double* __restrict__ vs,
                                                    const C* __restrict__ tw,
                                                    const C* __restrict__ chirp,
                                                    const C* __restrict__ bhat, int S, int Nt,
                                                    const int* __restrict__ live) {
  if (live && *live == 0) return;
  using R = typename cplx_traits<C>::real;
  const double vsc = vs ? vs[0] : 1.0;
  constexpr int LDN = LB + 1;
  __shared__ C buf[NB * LDN];
  constexpr int TS = 2 * NB;
  const int i0 = xcd_remap(blockIdx.x, gridDim.x) * TS;  // neighbours share lines: one XCD
  auto load = [&](int f, int j) -> C {
    if (j >= Nt) return cmk<C>((R)0, (R)0);
    const int i = i0 + 2 * f;
    const double* row = v + (size_t)j * S;
    const double sj = s[j] * vsc;
    const R a = (i < S) ? (R)(sj * row[i]) : (R)0;
    const R b = (i + 1 < S) ? (R)(sj * row[i + 1]) : (R)0;
    return cmul(cmk<C>(a, b), chirp[j]);
  };
  NoLoad nl;
  NoStore ns;
  fft_io<LB, -1, NT, NB, LDN, true, true, false, MAXR>(buf, tw, load, ns);
  for (int e = threadIdx.x; e < NB * LB; e += NT) {
    const int f = e % NB, k = e / NB;
    buf[f * LDN + k] = cmul(buf[f * LDN + k], bhat[k]);
  }
  __syncthreads();
  fft_io<LB, +1, NT, NB, LDN, true, false, false, MAXR>(buf, tw, nl, ns);
  const int nf = Nt / 2 + 1;
  for (int e = threadIdx.x; e < nf * TS; e += NT) {
    const int n = e / TS, q = e - n * TS;
    const int i = i0 + q;
    if (i >= S) continue;
    const int m = n == 0 ? 0 : Nt - n;
    const C a = cmul(chirp[n], buf[(q >> 1) * LDN + n]);
    const C b = cconj(cmul(chirp[m], buf[(q >> 1) * LDN + m]));
    C out;
    if ((q & 1) == 0) out = cmk<C>((R)0.5 * (a.x + b.x), (R)0.5 * (a.y + b.y));
    else out = cmk<C>((R)0.5 * (a.y - b.y), (R)-0.5 * (a.x - b.x));
    z1[(size_t)n * S + i] = out;
  }
}

template <int LB, int NB, int NT, typename C, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_time_inv_bs(const C* __restrict__ z2, double* __restrict__ v,
                                                    const double* __restrict__ s,
                                                    const C* __restrict__ tw,
                                                    const C* __restrict__ chirp,
                                                    const C* __restrict__ bhat, int S, int Nt,
                                                    const int* __restrict__ live) {
  if (live && *live == 0) return;
  using R = typename cplx_traits<C>::real;
  constexpr int LDN = LB + 1;
  __shared__ C buf[NB * LDN];
  constexpr int TS = 2 * NB;
  const int i0 = xcd_remap(blockIdx.x, gridDim.x) * TS;  // neighbours share lines: one XCD
  const int half = Nt / 2;
  // y_n = conj(Z_n) w_n with Z_n = P_n + i Q_n rebuilt from the half spectra as in k_time_inv
  // (only an even Nt has a self-conjugate n = Nt/2).
  auto load = [&](int f, int n) -> C {
    if (n >= Nt) return cmk<C>((R)0, (R)0);
    const int ia = i0 + 2 * f, ib = ia + 1;
    const int nn = n <= half ? n : Nt - n;
    C P = cmk<C>((R)0, (R)0), Q = cmk<C>((R)0, (R)0);
    if (ia < S) P = z2[(size_t)nn * S + ia];
    if (ib < S) Q = z2[(size_t)nn * S + ib];
    if (nn == 0 || 2 * nn == Nt) { P.y = (R)0; Q.y = (R)0; }
    const C Z = n <= half ? cmk<C>(P.x - Q.y, P.y + Q.x) : cmk<C>(P.x + Q.y, Q.x - P.y);
    return cmul(cconj(Z), chirp[n]);
  };
  // R_j = w_j conv_j = sum_n conj(Z_n) theta^{n j}; v_{2p} + i v_{2p+1} = conj(R_j) / (Nt s_j)
  auto store = [&](int f, int j, C c) {
    if (j >= Nt) return;
    const C Rj = cmul(chirp[j], c);
    const int i = i0 + 2 * f;
    double* row = v + (size_t)j * S;
    const double sc = 1.0 / ((double)Nt * s[j]);
    if (i < S) row[i] = (double)Rj.x * sc;
    if (i + 1 < S) row[i + 1] = -(double)Rj.y * sc;
  };
  NoStore ns;
  fft_io<LB, -1, NT, NB, LDN, true, true, false, MAXR>(buf, tw, load, ns);
  for (int e = threadIdx.x; e < NB * LB; e += NT) {
    const int f = e % NB, k = e / NB;
    buf[f * LDN + k] = cmul(buf[f * LDN + k], bhat[k]);
  }
  __syncthreads();
  NoLoad nl;
  fft_io<LB, +1, NT, NB, LDN, true, false, true, MAXR>(buf, tw, nl, store);
}

// w_k = exp(i pi (k^2 mod 2 Nt) / Nt) in both precisions (the integer reduction keeps the
// angle exact before rounding).
__global__ void k_bs_chirp(int Nt, double2* __restrict__ w, float2* __restrict__ w32) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Nt) return;
  const long long r = ((long long)k * k) % (2LL * Nt);
  double sn, cs;
  sincospi((double)r / Nt, &sn, &cs);
  w[k] = make_double2(cs, sn);
  w32[k] = make_float2((float)cs, (float)sn);
}

// bhat = DFT_{-1}(b) / LB with the cyclic kernel b_k = conj(w_k) (k < Nt),
// b_{LB-k} = conj(w_k) (0 < k < Nt), zero elsewhere.  One block.
template <int LB>
__global__ void __launch_bounds__(256) k_bs_kernel(int Nt, const double2* __restrict__ w,
                                                   const double2* __restrict__ tw,
                                                   double2* __restrict__ bhat,
                                                   float2* __restrict__ bhat32) {
  __shared__ double2 buf[LB];
  for (int k = threadIdx.x; k < LB; k += 256) {
    double2 b = make_double2(0.0, 0.0);
    if (k < Nt) b = make_double2(w[k].x, -w[k].y);
    else if (LB - k < Nt) b = make_double2(w[LB - k].x, -w[LB - k].y);
    buf[k] = b;
  }
  __syncthreads();
  fft_lds<LB, -1, 256, 1>(buf, tw);
  for (int k = threadIdx.x; k < LB; k += 256) {
    const double2 c = make_double2(buf[k].x / LB, buf[k].y / LB);
    bhat[k] = c;
    bhat32[k] = make_float2((float)c.x, (float)c.y);
  }
}

// Transforms per block: 128-byte row segments (NB = 8 complex128 / 16 complex64 pairs) unless
// the ~130 KB LDS budget forces fewer; variants 1 and 2 halve NB once and twice (more, smaller
// workgroups); variant 3 keeps NB with 1024 threads and radix-8 passes (more waves in flight).
template <int N, typename C, int V = 0>
constexpr int time_nb() {
  constexpr int target = (int)sizeof(C) == 16 ? 8 : 16;
  constexpr int cap = 135168 / ((N + 1) * (int)sizeof(C));
  constexpr int nb = cap < 1 ? 1 : (cap < target ? cap : target);
  constexpr int sh = V == 3 ? 0 : V;
  return (nb >> sh) < 1 ? 1 : (nb >> sh);
}
// Largest radix: 8 for variant 3 and for N <= 512 (twice the threads of radix 16 for the same
// LDS, so more waves per CU hide the global-memory latency of these short transforms), else 16.
template <int N, int V> constexpr int time_maxr() { return (V == 3 || N <= 512) ? 8 : 16; }
// Threads: one largest-radix butterfly each (NB N / MAXR, between 64 and 512); variant 3: 1024
// threads for NB N >= 8192.
template <int N, typename C, int V = 0>
constexpr int time_nt() {
  if (V == 3 && time_nb<N, C, V>() * N >= 8192) return 1024;
  constexpr int t = time_nb<N, C, V>() * N / time_maxr<N, V>();
  return t < 64 ? 64 : (t > 512 ? 512 : t);
}

template <int N, typename C, int V>
static int tf_fwd_v(const Plan& p, const double* v, void* z1, const C* tw, const double* vs) {
  constexpr int NB = time_nb<N, C, V>();
  constexpr int NT = time_nt<N, C, V>();
  const int blocks = (p.S + 2 * NB - 1) / (2 * NB);
  k_time_fwd<N, NB, NT, C, time_maxr<N, V>()><<<blocks, NT, 0, p.stream>>>(v, (C*)z1, p.s, vs, tw,
                                                                         p.S, p.live);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int N, typename C, int V>
static int tf_inv_v(const Plan& p, const void* z2, double* v, const C* tw) {
  constexpr int NB = time_nb<N, C, V>();
  constexpr int NT = time_nt<N, C, V>();
  const int blocks = (p.S + 2 * NB - 1) / (2 * NB);
  k_time_inv<N, NB, NT, C, time_maxr<N, V>()><<<blocks, NT, 0, p.stream>>>((const C*)z2, v, p.s, tw,
                                                                         p.S, p.live);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
// Compute units of the plan's device (queried once per device).
int device_cus(int dev) {
  static int cached[64] = {0};
  if (dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        c <= 0)
      return 256;
    cached[dev] = c;
  }
  return cached[dev];
}
// Variant 0 takes the half-width shape (variant 1) when the full width would leave CUs without
// a workgroup (e.g. complex64 at 32 columns per workgroup: 128 workgroups for 4095 columns).
template <int N, typename C>
static bool time_narrow(const Plan& p) {
  constexpr int NB = time_nb<N, C, 0>();
  return NB >= 2 && (p.S + 2 * NB - 1) / (2 * NB) < device_cus(p.device);
}
template <int N, typename C>
static int tf_fwd(const Plan& p, const double* v, void* z1, const C* tw, const double* vs) {
  if (p.tv_time == 1 || (p.tv_time == 0 && time_narrow<N, C>(p)))
    return tf_fwd_v<N, C, 1>(p, v, z1, tw, vs);
  if (p.tv_time == 2) return tf_fwd_v<N, C, 2>(p, v, z1, tw, vs);
  // variant 3 by default for the FP64 forward transform at N >= 1024 (M = 4095, N_t = 1024:
  // 20.2 against 22.5 us; the inverse is faster in the default shape, 20.4 against 21.1 us)
  constexpr bool fwd3 = N >= 1024 && sizeof(C) == 16;
  if (p.tv_time == 3 || (p.tv_time == 0 && fwd3)) return tf_fwd_v<N, C, 3>(p, v, z1, tw, vs);
  return tf_fwd_v<N, C, 0>(p, v, z1, tw, vs);
}
template <int N, typename C>
static int tf_inv(const Plan& p, const void* z2, double* v, const C* tw) {
  if (p.tv_time == 1 || (p.tv_time == 0 && time_narrow<N, C>(p)))
    return tf_inv_v<N, C, 1>(p, z2, v, tw);
  if (p.tv_time == 2) return tf_inv_v<N, C, 2>(p, z2, v, tw);
  if (p.tv_time == 3) return tf_inv_v<N, C, 3>(p, z2, v, tw);
  return tf_inv_v<N, C, 0>(p, z2, v, tw);
}

template <int LB, typename C, int V>
static int tf_fwd_bs_v(const Plan& p, const double* v, void* z1, const C* tw, const C* w,
                       const C* bh, const double* vs) {
  constexpr int NB = time_nb<LB, C, V>();
  constexpr int NT = time_nt<LB, C, V>();
  const int blocks = (p.S + 2 * NB - 1) / (2 * NB);
  k_time_fwd_bs<LB, NB, NT, C, time_maxr<LB, V>()><<<blocks, NT, 0, p.stream>>>(v, (C*)z1, p.s, vs, tw, w, bh, p.S,
                                                            p.Nt, p.live);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int LB, typename C, int V>
static int tf_inv_bs_v(const Plan& p, const void* z2, double* v, const C* tw, const C* w,
                       const C* bh) {
  constexpr int NB = time_nb<LB, C, V>();
  constexpr int NT = time_nt<LB, C, V>();
  const int blocks = (p.S + 2 * NB - 1) / (2 * NB);
  k_time_inv_bs<LB, NB, NT, C, time_maxr<LB, V>()><<<blocks, NT, 0, p.stream>>>((const C*)z2, v, p.s, tw, w, bh, p.S,
                                                             p.Nt, p.live);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int LB, typename C>
static int tf_fwd_bs(const Plan& p, const double* v, void* z1, const C* tw, const C* w,
                     const C* bh, const double* vs) {
  // (variant 3 has no Bluestein instantiation: it runs the default shape)
  if (p.tv_time == 1) return tf_fwd_bs_v<LB, C, 1>(p, v, z1, tw, w, bh, vs);
  if (p.tv_time == 2) return tf_fwd_bs_v<LB, C, 2>(p, v, z1, tw, w, bh, vs);
  return tf_fwd_bs_v<LB, C, 0>(p, v, z1, tw, w, bh, vs);
}
template <int LB, typename C>
static int tf_inv_bs(const Plan& p, const void* z2, double* v, const C* tw, const C* w,
                     const C* bh) {
  if (p.tv_time == 1) return tf_inv_bs_v<LB, C, 1>(p, z2, v, tw, w, bh);
  if (p.tv_time == 2) return tf_inv_bs_v<LB, C, 2>(p, z2, v, tw, w, bh);
  return tf_inv_bs_v<LB, C, 0>(p, z2, v, tw, w, bh);
}
template <int LB, typename C>
static int bs_kernel(const Plan& p) {
  k_bs_kernel<LB><<<1, 256, 0, p.stream>>>(p.Nt, p.chirp, p.twNt, p.bhat, p.bhat32);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

#define RFDE_LB_SWITCH(FN, C, ...)                 \
  switch (p.Lt) {                                  \
    case 8: return FN<8, C>(__VA_ARGS__);          \
    case 16: return FN<16, C>(__VA_ARGS__);        \
    case 32: return FN<32, C>(__VA_ARGS__);        \
    case 64: return FN<64, C>(__VA_ARGS__);        \
    case 128: return FN<128, C>(__VA_ARGS__);      \
    case 256: return FN<256, C>(__VA_ARGS__);      \
    case 512: return FN<512, C>(__VA_ARGS__);      \
    case 1024: return FN<1024, C>(__VA_ARGS__);    \
    case 2048: return FN<2048, C>(__VA_ARGS__);    \
    case 4096: return FN<4096, C>(__VA_ARGS__);    \
    case 8192: return FN<8192, C>(__VA_ARGS__);    \
    default: return RFDE_EINVAL;                   \
  }

template <int LB>
static int bs_spectrum(int n, const double2* w, const double2* tw, double2* bhat, float2* bhat32,
                       hipStream_t st) {
  k_bs_kernel<LB><<<1, 256, 0, st>>>(n, w, tw, bhat, bhat32);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int launch_bs_spectrum(int n, const double2* w, const double2* tw, int LB, double2* bhat,
                       float2* bhat32, hipStream_t st) {
  if (LB < 2 * n - 1) return RFDE_EINVAL;
  switch (LB) {
    case 8: return bs_spectrum<8>(n, w, tw, bhat, bhat32, st);
    case 16: return bs_spectrum<16>(n, w, tw, bhat, bhat32, st);
    case 32: return bs_spectrum<32>(n, w, tw, bhat, bhat32, st);
    case 64: return bs_spectrum<64>(n, w, tw, bhat, bhat32, st);
    case 128: return bs_spectrum<128>(n, w, tw, bhat, bhat32, st);
    case 256: return bs_spectrum<256>(n, w, tw, bhat, bhat32, st);
    case 512: return bs_spectrum<512>(n, w, tw, bhat, bhat32, st);
    case 1024: return bs_spectrum<1024>(n, w, tw, bhat, bhat32, st);
    case 2048: return bs_spectrum<2048>(n, w, tw, bhat, bhat32, st);
    case 4096: return bs_spectrum<4096>(n, w, tw, bhat, bhat32, st);
    case 8192: return bs_spectrum<8192>(n, w, tw, bhat, bhat32, st);
    default: return RFDE_EINVAL;
  }
}

int launch_bluestein_setup(const Plan& p) {
  if (p.Lt == p.Nt) return RFDE_OK;
  k_bs_chirp<<<(p.Nt + 255) / 256, 256, 0, p.stream>>>(p.Nt, p.chirp, p.chirp32);
  RFDE_HIP(hipGetLastError());
  RFDE_LB_SWITCH(bs_kernel, double2, p);
}

#define RFDE_NT_SWITCH(FN, C, ...)                 \
  switch (p.Nt) {                                  \
    case 2: return FN<2, C>(__VA_ARGS__);          \
    case 4: return FN<4, C>(__VA_ARGS__);          \
    case 8: return FN<8, C>(__VA_ARGS__);          \
    case 16: return FN<16, C>(__VA_ARGS__);        \
    case 32: return FN<32, C>(__VA_ARGS__);        \
    case 64: return FN<64, C>(__VA_ARGS__);        \
    case 128: return FN<128, C>(__VA_ARGS__);      \
    case 256: return FN<256, C>(__VA_ARGS__);      \
    case 512: return FN<512, C>(__VA_ARGS__);      \
    case 1024: return FN<1024, C>(__VA_ARGS__);    \
    case 2048: return FN<2048, C>(__VA_ARGS__);    \
    case 4096: return FN<4096, C>(__VA_ARGS__);    \
    case 8192: return FN<8192, C>(__VA_ARGS__);    \
    default: return RFDE_EINVAL;                   \
  }

int launch_time_fwd_scaled(const Plan& p, const double* v, void* z1, const double* vs) {
  if (p.Lt != p.Nt) {
    if (p.opts.precond_bits == 32) {
      RFDE_LB_SWITCH(tf_fwd_bs, float2, p, v, z1, p.twNt32, p.chirp32, p.bhat32, vs);
    }
    RFDE_LB_SWITCH(tf_fwd_bs, double2, p, v, z1, p.twNt, p.chirp, p.bhat, vs);
  }
  if (p.opts.precond_bits == 32) { RFDE_NT_SWITCH(tf_fwd, float2, p, v, z1, p.twNt32, vs); }
  RFDE_NT_SWITCH(tf_fwd, double2, p, v, z1, p.twNt, vs);
}

int launch_time_fwd(const Plan& p, const double* v, void* z1) {
  return launch_time_fwd_scaled(p, v, z1, nullptr);
}

int launch_time_inv(const Plan& p, const void* z2, double* v) {
  if (p.Lt != p.Nt) {
    if (p.opts.precond_bits == 32) {
      RFDE_LB_SWITCH(tf_inv_bs, float2, p, z2, v, p.twNt32, p.chirp32, p.bhat32);
    }
    RFDE_LB_SWITCH(tf_inv_bs, double2, p, z2, v, p.twNt, p.chirp, p.bhat);
  }
  if (p.opts.precond_bits == 32) { RFDE_NT_SWITCH(tf_inv, float2, p, z2, v, p.twNt32); }
  RFDE_NT_SWITCH(tf_inv, double2, p, z2, v, p.twNt);
}

__global__ void k_widen(const float2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_double2((double)a[i].x, (double)a[i].y);
}
__global__ void k_narrow(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

int launch_widen(const Plan& p, const void* zsrc, double2* zdst) {
  const size_t n = (size_t)p.nf * p.S;
  k_widen<<<(int)std::min<size_t>((n + 255) / 256, 8192), 256, 0, p.stream>>>((const float2*)zsrc,
                                                                               zdst, n);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
int launch_narrow(const Plan& p, const double2* zsrc, void* zdst) {
  const size_t n = (size_t)p.nf * p.S;
  k_narrow<<<(int)std::min<size_t>((n + 255) / 256, 8192), 256, 0, p.stream>>>(zsrc,
                                                                                (float2*)zdst, n);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // namespace rfde
