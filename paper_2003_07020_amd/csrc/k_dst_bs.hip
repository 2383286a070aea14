// DST-I of any length n for preconditioner step (b) with the tau approximation (eq. (3.9)-(3.11)
// in 1D, eq. (4.5) in 2D) when 2(n+1) is not a power of two.
//
// With w = exp(i pi / (n+1)) the sine sums split into two exponential sums,
//     S_k = sum_{j=1}^{n} x_j sin(pi j k / (n+1)) = (P_k - Q_k) / (2i),
//     P_k = sum_j x_j w^{jk},  Q_k = sum_j x_j w^{-jk},   k = 1..n,
// and each is a chirp-z (Bluestein) sum: with c_m = w^{m^2/2} = exp(i pi m^2 / (2(n+1))),
// jk = (j^2 + k^2 - (k-j)^2)/2 gives w^{jk} = c_j c_k conj(c_{k-j}), so
//     P_k = c_k sum_j (x_j c_j) conj(c_{k-j}),   Q_k = conj(c_k) sum_j (x_j conj(c_j)) c_{k-j},
// two linear convolutions with kernels of lags |k - j| <= n - 1, done as cyclic convolutions of
// the power-of-two length LB >= 2n - 1 in LDS: forward FFT, product with the transform of the
// kernel (precomputed once per plan, divided by LB), unnormalised inverse FFT.  The transform of
// the kernel c_m is conj(Khat[(LB - k) mod LB]) when Khat is that of conj(c_m), so one table
// serves both.  The chirp angles are reduced exactly (m^2 mod 4(n+1)) before rounding.
//
// A DST of a set of sequences takes two launches: phase 0 forms P and parks it in a work array
// of the data's shape; phase 1 forms Q, combines sc (P - Q)/(2i) with sc = sqrt(2/(n+1)) (the
// orthonormal DST-I Q of the tau matrix) and, with SCALE, divides coefficient k by the shifted
// eigenvalue before the store.  The tau solves then chain DST, scaled DST (1D: 4 launches;
// 2D: rows, columns with the division, rows).
#include <type_traits>

#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

// Sequences of a launch: sequence s lies in plane s / spp at index s % spp of that plane;
// element j (1..n) of it is at plane * plane_stride + idx * seq_stride + (j - 1) * elem_stride.
struct DstSeqs {
  int n, nseq, spp;
  long long seq_stride, elem_stride, plane_stride;
};

// c_m = exp(i pi (m^2 mod 4(n+1)) / (2(n+1))), m = 0..n, in both precisions.
__global__ void k_dstbs_chirp(int n, double2* __restrict__ c, float2* __restrict__ c32) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m > n) return;
  const long long per = 4LL * (n + 1);
  const long long r = ((long long)m * m) % per;
  double sn, cs;
  sincospi((double)r / (2.0 * (n + 1)), &sn, &cs);
  c[m] = make_double2(cs, sn);
  c32[m] = make_float2((float)cs, (float)sn);
}

template <int LB, int NB, int NT, typename C, bool BFAST, int PH, bool SCALE, int MAXR>
__global__ void __launch_bounds__(NT) k_dstbs(const C* in, C* tmp, C* out, DstSeqs q,
                                              const C* __restrict__ chirp,
                                              const C* __restrict__ khat, const C* __restrict__ tw,
                                              const double2* __restrict__ lambda,
                                              const double* __restrict__ sigA, double coefA,
                                              const double* __restrict__ sigB, double coefB,
                                              double sc) {
  using R = typename cplx_traits<C>::real;
  constexpr int LDN = BFAST ? LB + 1 : LB;
  __shared__ C buf[NB * LDN];
  const int s0 = xcd_remap(blockIdx.x, gridDim.x) * NB;
  auto addr = [&](int s, int j) -> size_t {
    const int plane = s / q.spp, idx = s - plane * q.spp;
    return (size_t)plane * q.plane_stride + (size_t)idx * q.seq_stride +
           (size_t)(j - 1) * q.elem_stride;
  };
  auto load = [&](int f, int j) -> C {
    const int s = s0 + f;
    if (s >= q.nseq || j < 1 || j > q.n) return cmk<C>((R)0, (R)0);
    const C x = in[addr(s, j)];
    return PH == 0 ? cmul(x, chirp[j]) : cmul(x, cconj(chirp[j]));
  };
  auto mul_kernel = [&](int f, int k, C v) {
    const C K = PH == 0 ? khat[k] : cconj(khat[(LB - k) & (LB - 1)]);
    buf[f * LDN + k] = cmul(v, K);
  };
  fft_io<LB, -1, NT, NB, LDN, BFAST, true, true, MAXR>(buf, tw, load, mul_kernel);
  __syncthreads();
  auto store = [&](int f, int k, C v) {
    const int s = s0 + f;
    if (s >= q.nseq || k < 1 || k > q.n) return;
    const size_t a = addr(s, k);
    if constexpr (PH == 0) {
      tmp[a] = cmul(v, chirp[k]);
    } else {
      const C d = csub(tmp[a], cmul(v, cconj(chirp[k])));
      // sc (P - Q) / (2i) = sc (d.y, -d.x) / 2
      C y = cmk<C>((R)(0.5 * sc) * d.y, -(R)(0.5 * sc) * d.x);
      if constexpr (SCALE) {
        const int plane = s / q.spp, idx = s - plane * q.spp;
        const double2 lam = lambda[plane];
        double dr = lam.x + coefA * sigA[k - 1];
        if (sigB) dr += coefB * sigB[idx];
        const double di = lam.y, den = dr * dr + di * di;
        y = cmul(y, cmk<C>((R)(dr / den), (R)(-di / den)));
      }
      out[a] = y;
    }
  };
  NoLoad nl;
  fft_io<LB, +1, NT, NB, LDN, BFAST, false, true, MAXR>(buf, tw, nl, store);
}

// Sequences per workgroup: about 64 KB of LDS for contiguous sequences; for strided ones
// (columns, batch index fastest) up to 16 so that rows of adjacent columns are read together.
template <int LB, typename C, bool BFAST>
constexpr int dstbs_nb() {
  constexpr int cap = 65536 / ((LB + (BFAST ? 1 : 0)) * (int)sizeof(C));
  constexpr int target = BFAST ? ((int)sizeof(C) == 16 ? 8 : 16) : 8;
  return cap < 1 ? 1 : (cap < target ? cap : target);
}
template <int LB> constexpr int dstbs_maxr() { return LB <= 512 ? 8 : 16; }
template <int LB, typename C, bool BFAST>
constexpr int dstbs_nt() {
  constexpr int t = dstbs_nb<LB, C, BFAST>() * LB / dstbs_maxr<LB>();
  return t < 64 ? 64 : (t > 512 ? 512 : t);
}

template <int LB, typename C, bool BFAST, int PH, bool SCALE>
static int dstbs_launch(hipStream_t st, const C* in, C* tmp, C* out, const DstSeqs& q,
                        const C* chirp, const C* khat, const C* tw, const double2* lambda,
                        const double* sigA, double coefA, const double* sigB, double coefB) {
  constexpr int NB = dstbs_nb<LB, C, BFAST>();
  constexpr int NT = dstbs_nt<LB, C, BFAST>();
  const int grid = (q.nseq + NB - 1) / NB;
  k_dstbs<LB, NB, NT, C, BFAST, PH, SCALE, dstbs_maxr<LB>()><<<grid, NT, 0, st>>>(
      in, tmp, out, q, chirp, khat, tw, lambda, sigA, coefA, sigB, coefB,
      std::sqrt(2.0 / (q.n + 1)));
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// One DST (phases 0 and 1) of the sequences q, in -> out through tmp, optionally scaled.
template <int LB, typename C, bool BFAST, bool SCALE>
static int dstbs_pair(hipStream_t st, const C* in, C* tmp, C* out, const DstSeqs& q,
                      const C* chirp, const C* khat, const C* tw, const double2* lambda,
                      const double* sigA, double coefA, const double* sigB, double coefB) {
  RFDE_TRY((dstbs_launch<LB, C, BFAST, 0, false>(st, in, tmp, out, q, chirp, khat, tw, lambda,
                                                  sigA, coefA, sigB, coefB)));
  return dstbs_launch<LB, C, BFAST, 1, SCALE>(st, in, tmp, out, q, chirp, khat, tw, lambda, sigA,
                                               coefA, sigB, coefB);
}

// Length LB of the cyclic convolutions for a DST-I of length n.
int dstbs_length(int n) {
  int lb = 8;
  while (lb < 2 * n - 1) lb <<= 1;
  return lb;
}

// Tables of axis a (0: the 1D axis or x, 1: y) inside the plan's DST-I table block.
template <typename C>
static void dstbs_tables(const Plan& p, int a, const C** chirp, const C** khat, const C** tw) {
  const DstBsAxis& x = p.bs[a];
  if constexpr (std::is_same<C, float2>::value) {
    *chirp = x.chirp32; *khat = x.khat32; *tw = x.tw32;
  } else {
    *chirp = x.chirp; *khat = x.khat; *tw = x.tw;
  }
}

#define RFDE_LBS_SWITCH(LBval, FN, ...)         \
  switch (LBval) {                              \
    case 8: return FN<8, __VA_ARGS__;           \
    case 16: return FN<16, __VA_ARGS__;         \
    case 32: return FN<32, __VA_ARGS__;         \
    case 64: return FN<64, __VA_ARGS__;         \
    case 128: return FN<128, __VA_ARGS__;       \
    case 256: return FN<256, __VA_ARGS__;       \
    case 512: return FN<512, __VA_ARGS__;       \
    case 1024: return FN<1024, __VA_ARGS__;     \
    case 2048: return FN<2048, __VA_ARGS__;     \
    case 4096: return FN<4096, __VA_ARGS__;     \
    case 8192: return FN<8192, __VA_ARGS__;     \
    default: return RFDE_EUNSUPPORTED;          \
  }

// 1D: z = Q diag(1 / (lambda_r + coef sigma_k)) Q zin for every row r of the half spectrum.
template <typename C>
int tau_solve_1d_bs(const Plan& p, const C* zin, C* z) {
  const C *ch, *kh, *tw;
  dstbs_tables<C>(p, 0, &ch, &kh, &tw);
  C* tmp = (C*)p.zt;
  DstSeqs q{p.M, p.nf, 1, 0, 1, p.M};
  const int LB = p.bs[0].LB;
  auto first = [&]() -> int {
    RFDE_LBS_SWITCH(LB, dstbs_pair, C, false, true>(p.stream, zin, tmp, z, q, ch, kh, tw,
                                                    p.lambda, p.sigma, p.coef, nullptr, 0.0));
  };
  auto second = [&]() -> int {
    RFDE_LBS_SWITCH(LB, dstbs_pair, C, false, false>(p.stream, z, tmp, z, q, ch, kh, tw,
                                                     p.lambda, nullptr, 0.0, nullptr, 0.0));
  };
  RFDE_TRY(first());
  return second();
}

// 2D, x direction (rows of every plane), in place, unscaled.
template <typename C>
int tau_rows_2d_bs(const Plan& p, C* z) {
  const C *ch, *kh, *tw;
  dstbs_tables<C>(p, 0, &ch, &kh, &tw);
  DstSeqs q{p.Mx, p.nf * p.My, p.My, p.Mx, 1, (long long)p.Mx * p.My};
  auto run = [&]() -> int {
    RFDE_LBS_SWITCH(p.bs[0].LB, dstbs_pair, C, false, false>(p.stream, z, (C*)p.zt, z, q, ch, kh,
                                                             tw, p.lambda, nullptr, 0.0, nullptr,
                                                             0.0));
  };
  return run();
}

// 2D, y direction (columns of every plane), in place: DST, division by
// lambda_f + coef_x sigma^x_i + coef_y sigma^y_k, DST.
template <typename C>
int tau_cols_2d_bs(const Plan& p, C* z) {
  const C *ch, *kh, *tw;
  dstbs_tables<C>(p, 1, &ch, &kh, &tw);
  DstSeqs q{p.My, p.nf * p.Mx, p.Mx, 1, p.Mx, (long long)p.Mx * p.My};
  C* tmp = (C*)p.zt;
  const int LB = p.bs[1].LB;
  auto first = [&]() -> int {
    RFDE_LBS_SWITCH(LB, dstbs_pair, C, true, true>(p.stream, z, tmp, z, q, ch, kh, tw, p.lambda,
                                                   p.sigma + p.Mx, p.coef_y, p.sigma, p.coef_x));
  };
  auto second = [&]() -> int {
    RFDE_LBS_SWITCH(LB, dstbs_pair, C, true, false>(p.stream, z, tmp, z, q, ch, kh, tw, p.lambda,
                                                    nullptr, 0.0, nullptr, 0.0));
  };
  RFDE_TRY(first());
  return second();
}

template int tau_solve_1d_bs<double2>(const Plan&, const double2*, double2*);
template int tau_solve_1d_bs<float2>(const Plan&, const float2*, float2*);
template int tau_rows_2d_bs<double2>(const Plan&, double2*);
template int tau_rows_2d_bs<float2>(const Plan&, float2*);
template int tau_cols_2d_bs<double2>(const Plan&, double2*);
template int tau_cols_2d_bs<float2>(const Plan&, float2*);

// Tables of one axis: chirp (n + 1 entries), twiddles of LB, transform of the kernel / LB.
int dstbs_setup_axis(const Plan& p, int a) {
  const DstBsAxis& x = p.bs[a];
  k_dstbs_chirp<<<(x.n + 1 + 255) / 256, 256, 0, p.stream>>>(x.n, x.chirp, x.chirp32);
  RFDE_HIP(hipGetLastError());
  RFDE_TRY(launch_twiddles(x.tw, x.LB, p.stream));
  RFDE_TRY(launch_twiddles32(x.tw32, x.LB, p.stream));
  return launch_bs_spectrum(x.n, x.chirp, x.tw, x.LB, x.khat, x.khat32, p.stream);
}

}  // namespace rfde
