// Vector kernels of the FGMRES outer iteration (FP64).  Reductions are deterministic: a fixed
// grid writes one partial per block in a fixed order, and a single block sums the partials
// with a fixed tree, so repeated runs are bitwise identical.
#include <cstdint>

#include "krylov.hpp"
#include "rfde_internal.hpp"

namespace rfde {

constexpr int RED_BLOCKS = 1024;  // partials per reduced quantity
constexpr int VCHUNK = 4;         // vectors handled per pass of k_dot_partial

__device__ __forceinline__ double block_sum_256(double v, double* sh) {
  const int t = threadIdx.x;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return s;
}

// partial[v * RED_BLOCKS + b] = sum over block b's share of V[v0+v][i] * w[i], v < nv (<= VCHUNK)
__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ V, size_t ld,
                                                     int nv, const double* __restrict__ w,
                                                     size_t n, double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc[VCHUNK] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)RED_BLOCKS * 256) {
    const double wi = w[i];
#pragma unroll
    for (int v = 0; v < VCHUNK; ++v)
      if (v < nv) acc[v] = fma(V[v * ld + i], wi, acc[v]);
  }
#pragma unroll
  for (int v = 0; v < VCHUNK; ++v) {
    if (v < nv) {
      const double s = block_sum_256(acc[v], sh);
      if (threadIdx.x == 0) partial[v * RED_BLOCKS + blockIdx.x] = s;
    }
  }
}

// out[v] = sum_b partial[v * RED_BLOCKS + b] (fixed order), one block per v.
__global__ void __launch_bounds__(256) k_dot_final(const double* __restrict__ partial,
                                                   double* __restrict__ out, int do_sqrt) {
  __shared__ double sh[4];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < RED_BLOCKS; b += 256) acc += partial[v * RED_BLOCKS + b];
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) out[v] = do_sqrt ? sqrt(s) : s;
}

// ---- CGS2 in two sweeps over the stored basis U (the scheme is described in krylov.hpp) ----
constexpr int CGS_ACC = 16;  // dot products accumulated per sweep
enum { CGS_DOT = 0, CGS_AXPY_DOT = 1 };

// MODE CGS_DOT:      partial[v][b] = sum_i U[v][i] w[i], v < nv.
// MODE CGS_AXPY_DOT: w[i] -= sum_{v < nall} c[v] U[v][i]; partial[v][b] = sum_i U[v][i] w[i]
//                    (the updated w), v < nv; pnrm[b] = sum_i w[i]^2 (the updated w).
// U holds the vectors at stride n.  NV > 0: nv = NV and, for the correcting mode, nall = NV,
// known at compile time so every basis value of an element is loaded before any is used (all
// loads in flight together); NV = 0: any nall (> CGS_ACC) with nv = CGS_ACC, by loops.
// Elements are read in pairs (16-byte loads) from the first 16-byte boundary of w.
template <int MODE, int NV>
__global__ void __launch_bounds__(256) k_cgs(double* __restrict__ w, const double* __restrict__ V,
                                             size_t n, int nall, const double* __restrict__ c,
                                             double* __restrict__ partial,
                                             double* __restrict__ pnrm) {
  constexpr int NACC = NV > 0 ? NV : CGS_ACC;
  constexpr int NOUT = MODE == CGS_AXPY_DOT ? NACC + 1 : NACC;  // the last: |w|^2
  double acc[NOUT];
#pragma unroll
  for (int v = 0; v < NOUT; ++v) acc[v] = 0.0;
  auto element = [&](size_t i, double wi) -> double {
    double vv[NACC];
    if constexpr (NV > 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) vv[v] = V[(size_t)v * n + i];
      if constexpr (MODE != CGS_DOT) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s = fma(c[v], vv[v], s);
        wi -= s;
      }
    } else {
      static_assert(MODE != CGS_DOT, "dot sweeps take at most CGS_ACC vectors per launch");
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < CGS_ACC; ++v) {
        vv[v] = V[(size_t)v * n + i];
        s = fma(c[v], vv[v], s);
      }
      for (int v = CGS_ACC; v < nall; ++v) s = fma(c[v], V[(size_t)v * n + i], s);
      wi -= s;
    }
#pragma unroll
    for (int v = 0; v < NACC; ++v) acc[v] = fma(vv[v], wi, acc[v]);
    if constexpr (MODE == CGS_AXPY_DOT) acc[NACC] = fma(wi, wi, acc[NACC]);
    return wi;
  };
  // pairs start where w is 16-byte aligned (w is a basis slot at offset j N: 8-byte aligned
  // only when N is odd); the element before them and an odd last element are done alone
  const size_t off = (reinterpret_cast<uintptr_t>(w) & 15) ? 1 : 0;
  const size_t n2 = (n - off) / 2;
  double2* wp = reinterpret_cast<double2*>(w + off);
  for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < n2; k += (size_t)RED_BLOCKS * 256) {
    const double2 wv = wp[k];
    const double a = element(off + 2 * k, wv.x), b = element(off + 2 * k + 1, wv.y);
    if constexpr (MODE != CGS_DOT) wp[k] = make_double2(a, b);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (off) {
      const double a = element(0, w[0]);
      if constexpr (MODE != CGS_DOT) w[0] = a;
    }
    if (off + 2 * n2 < n) {
      const double a = element(n - 1, w[n - 1]);
      if constexpr (MODE != CGS_DOT) w[n - 1] = a;
    }
  }
  // per-wave sums of every accumulator, then one barrier and the four wave sums per value in
  // the fixed order (w0 + w1) + (w2 + w3)
  __shared__ double shv[4][NOUT];
#pragma unroll
  for (int v = 0; v < NOUT; ++v) {
    double r = acc[v];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) r += __shfl_xor(r, m);
    if ((threadIdx.x & 63) == 0) shv[threadIdx.x >> 6][v] = r;
  }
  __syncthreads();
  if ((int)threadIdx.x < NOUT) {
    const int v = threadIdx.x;
    const double t = (shv[0][v] + shv[1][v]) + (shv[2][v] + shv[3][v]);
    if (v < NACC) partial[v * RED_BLOCKS + blockIdx.x] = t;
    else pnrm[blockIdx.x] = t;
  }
}

// launch of mode MODE over nv (1..CGS_ACC) vectors known at compile time, or NV = 0
template <int MODE>
static int cgs_launch(const Plan& p, double* w, const double* V, int nall, int nv,
                      const double* c, double* partial, double* pnrm) {
  const size_t n = p.N();
#define RFDE_CGS_CASE(K)                                                                     \
  case K:                                                                                    \
    k_cgs<MODE, K><<<RED_BLOCKS, 256, 0, p.stream>>>(w, V, n, nall, c, partial, pnrm);       \
    break;
  if (MODE != CGS_DOT && nall > CGS_ACC) {
    if constexpr (MODE != CGS_DOT)
      k_cgs<MODE, 0><<<RED_BLOCKS, 256, 0, p.stream>>>(w, V, n, nall, c, partial, pnrm);
  } else {
    switch (nv) {
      RFDE_CGS_CASE(1) RFDE_CGS_CASE(2) RFDE_CGS_CASE(3) RFDE_CGS_CASE(4)
      RFDE_CGS_CASE(5) RFDE_CGS_CASE(6) RFDE_CGS_CASE(7) RFDE_CGS_CASE(8)
      RFDE_CGS_CASE(9) RFDE_CGS_CASE(10) RFDE_CGS_CASE(11) RFDE_CGS_CASE(12)
      RFDE_CGS_CASE(13) RFDE_CGS_CASE(14) RFDE_CGS_CASE(15) RFDE_CGS_CASE(16)
      default: return RFDE_EINVAL;
    }
  }
#undef RFDE_CGS_CASE
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// Sum over the 64 lanes of a wave in a fixed butterfly order (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// The factor is kept as its inverse Q = R^{-1} (upper triangular, column-major, leading
// dimension CGS2_R_LD): the coefficient maps are then products, one lane per entry, each a
// sum in a fixed order.  Lane i < nvec returns (Q^T y)_i = sum_{k <= i} Q(k, i) y_k.
__device__ __forceinline__ double qt_times(const double* __restrict__ Q, const double* ys,
                                           int nvec) {
  const int i = threadIdx.x;
  double t = 0.0;
  if (i < nvec)
    for (int k = 0; k <= i; ++k) t = fma(Q[k + CGS2_R_LD * i], ys[k], t);
  return t;
}
// Lane i < nvec returns (Q y)_i = sum_{i <= k < nvec} Q(i, k) y_k.
__device__ __forceinline__ double q_times(const double* __restrict__ Q, const double* ys,
                                          int nvec) {
  const int i = threadIdx.x;
  double t = 0.0;
  if (i < nvec)
    for (int k = i; k < nvec; ++k) t = fma(Q[i + CGS2_R_LD * k], ys[k], t);
  return t;
}

// ys[v] = sum of the RED_BLOCKS partials of value v < nvec (256 threads, fixed order: four
// strided partials per thread, then the wave sums, then (w0 + w1) + (w2 + w3)).
__device__ __forceinline__ void sum_partials(const double* __restrict__ partial, int nvec,
                                             double (*sh)[4], double* ys) {
  const int t = threadIdx.x;
  for (int v = 0; v < nvec; ++v) {
    const double* pv = partial + (size_t)v * RED_BLOCKS;
    double a = (pv[t] + pv[t + 256]) + (pv[t + 512] + pv[t + 768]);
    a = wave_sum(a);
    if ((t & 63) == 0) sh[v][t >> 6] = a;
  }
  __syncthreads();
  if (t < 64) ys[t] = t < nvec ? (sh[t][0] + sh[t][1]) + (sh[t][2] + sh[t][3]) : 0.0;
  __syncthreads();
}

// Sweep A's coefficients: a = U^T w from the sweep's partials, h1 = Q^T a (= V^T w) to the
// host-visible h1, c1 = Q h1 to the device.
__global__ void __launch_bounds__(256) k_cgs2_fin_a(const double* __restrict__ partial,
                                                    const double* __restrict__ Q, int nvec,
                                                    double* h1, double* __restrict__ c1) {
  static_assert(RED_BLOCKS == 1024, "sum_partials reads four partials per thread");
  __shared__ double sh[64][4], ys[64], hs[64];
  sum_partials(partial, nvec, sh, ys);
  const int lane = threadIdx.x;
  double h = 0.0;
  if (lane < 64) {
    h = qt_times(Q, ys, nvec);
    hs[lane] = h;
  }
  __syncthreads();
  if (lane < nvec) {
    h1[lane] = h;
    c1[lane] = q_times(Q, hs, nvec);
  }
}

// Sweep B's coefficients: b = U^T w1 and s = |w1|^2 from the partials, h2 = Q^T b, n =
// sqrt(s - |h2|^2); h2 and n to the host-visible h2 / nrm; appends column nvec of R^{-1},
// (-Q h2 / n, 1 / n), and vs[nvec] = 1 / sqrt(s).  n = 0 (breakdown: the cycle ends at this
// step) leaves the column 0.
__global__ void __launch_bounds__(256) k_cgs2_fin_b(const double* __restrict__ partial,
                                                    const double* __restrict__ pnrm,
                                                    double* __restrict__ Q, int nvec, double* h2,
                                                    double* nrm, double* __restrict__ vs) {
  __shared__ double sh[65][4], ys[64], hs[64];
  sum_partials(partial, nvec, sh, ys);
  const int lane = threadIdx.x;
  {  // s: the same fixed order, kept in sh[64]
    double a = (pnrm[lane] + pnrm[lane + 256]) + (pnrm[lane + 512] + pnrm[lane + 768]);
    a = wave_sum(a);
    if ((lane & 63) == 0) sh[64][lane >> 6] = a;
  }
  double h = 0.0;
  if (lane < 64) {
    h = qt_times(Q, ys, nvec);
    hs[lane] = h;
  }
  __syncthreads();
  if (lane < 64) {
    const double s = (sh[64][0] + sh[64][1]) + (sh[64][2] + sh[64][3]);
    const double hh = wave_sum(lane < nvec ? h * h : 0.0);
    const double n2 = s - hh;
    const double nv = n2 > 0.0 ? sqrt(n2) : 0.0;
    const double qh = q_times(Q, hs, nvec);
    if (lane < nvec) {
      h2[lane] = h;
      Q[lane + CGS2_R_LD * nvec] = nv > 0.0 ? -qh / nv : 0.0;
    }
    if (lane == 0) {
      Q[nvec + CGS2_R_LD * nvec] = nv > 0.0 ? 1.0 / nv : 0.0;
      *nrm = nv;
      vs[nvec] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    }
  }
}

__global__ void __launch_bounds__(64) k_cgs2_start(double* __restrict__ Q,
                                                   double* __restrict__ vs, double beta) {
  if (threadIdx.x == 0) {
    Q[0] = 1.0 / beta;
    vs[0] = 1.0 / beta;
  }
}

int launch_cgs2_start(const Plan& p, double beta, double* out) {
  k_cgs2_start<<<1, 64, 0, p.stream>>>(p.red + CGS2_R_OFF, out + CGS2_VS, beta);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int launch_cgs2(const Plan& p, const double* U, int nvec, double* w, double* out,
                double* hout) {
  if (nvec < 1 || nvec > 64) return RFDE_EINVAL;
  const size_t n = p.N();
  double* Q = p.red + CGS2_R_OFF;                // R^{-1}
  double* pn = p.red + (size_t)64 * RED_BLOCKS;  // partials of |w1|^2
  // sweep A: a = U^T w -> h1, c1
  for (int v0 = 0; v0 < nvec; v0 += CGS_ACC) {
    const int nv = std::min(CGS_ACC, nvec - v0);
    RFDE_TRY(cgs_launch<CGS_DOT>(p, w, U + (size_t)v0 * n, nv, nv, nullptr,
                                 p.red + (size_t)v0 * RED_BLOCKS, nullptr));
  }
  k_cgs2_fin_a<<<1, 256, 0, p.stream>>>(p.red, Q, nvec, hout, out + CGS2_C);
  RFDE_HIP(hipGetLastError());
  // sweep B: w1 = w - U c1 with its dot products with the first CGS_ACC vectors and |w1|^2;
  // the rest (if any) by dot sweeps; then h2, n and the new column of R^{-1}
  RFDE_TRY(cgs_launch<CGS_AXPY_DOT>(p, w, U, nvec, std::min(CGS_ACC, nvec), out + CGS2_C, p.red,
                                    pn));
  for (int v0 = CGS_ACC; v0 < nvec; v0 += CGS_ACC) {
    const int nv = std::min(CGS_ACC, nvec - v0);
    RFDE_TRY(cgs_launch<CGS_DOT>(p, w, U + (size_t)v0 * n, nv, nv, nullptr,
                                 p.red + (size_t)v0 * RED_BLOCKS, nullptr));
  }
  k_cgs2_fin_b<<<1, 256, 0, p.stream>>>(p.red, pn, Q, nvec, hout + CGS2_H2, hout + CGS2_NRM,
                                        out + CGS2_VS);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int launch_nrm2(const Plan& p, const double* x, double* out) {
  const size_t n = p.N();
  k_dot_partial<<<RED_BLOCKS, 256, 0, p.stream>>>(x, n, 1, x, n, p.red);
  RFDE_HIP(hipGetLastError());
  k_dot_final<<<1, 256, 0, p.stream>>>(p.red, out, 1);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// w[i] += sign * sum_v coef[v] V[v][i]; NV > 0: nvec = NV known at compile time (all loads of an
// element in flight together), NV = 0: any nvec by a loop.
template <int NV>
__global__ void __launch_bounds__(256) k_multi_axpy(double* __restrict__ w,
                                                   const double* __restrict__ V, size_t n,
                                                   int nvec, const double* __restrict__ coef,
                                                   double sign) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    if constexpr (NV > 0) {
      double vv[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) vv[v] = V[(size_t)v * n + i];
#pragma unroll
      for (int v = 0; v < NV; ++v) s = fma(coef[v], vv[v], s);
    } else {
      for (int v = 0; v < nvec; ++v) s = fma(coef[v], V[(size_t)v * n + i], s);
    }
    w[i] = fma(sign, s, w[i]);
  }
}

int launch_multi_axpy(const Plan& p, double* w, const double* V, int nvec, const double* coef,
                      double sign) {
  const size_t n = p.N();
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
#define RFDE_AXPY_CASE(K)                                                                    \
  case K:                                                                                    \
    k_multi_axpy<K><<<blocks, 256, 0, p.stream>>>(w, V, n, nvec, coef, sign);                \
    break;
  switch (nvec) {
    RFDE_AXPY_CASE(1) RFDE_AXPY_CASE(2) RFDE_AXPY_CASE(3) RFDE_AXPY_CASE(4)
    RFDE_AXPY_CASE(5) RFDE_AXPY_CASE(6) RFDE_AXPY_CASE(7) RFDE_AXPY_CASE(8)
    RFDE_AXPY_CASE(9) RFDE_AXPY_CASE(10) RFDE_AXPY_CASE(11) RFDE_AXPY_CASE(12)
    RFDE_AXPY_CASE(13) RFDE_AXPY_CASE(14) RFDE_AXPY_CASE(15) RFDE_AXPY_CASE(16)
    default: k_multi_axpy<0><<<blocks, 256, 0, p.stream>>>(w, V, n, nvec, coef, sign);
  }
#undef RFDE_AXPY_CASE
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b, double* out,
                      size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

int launch_sub(const Plan& p, const double* a, const double* b, double* out) {
  const size_t n = p.N();
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  k_sub<<<blocks, 256, 0, p.stream>>>(a, b, out, n);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // namespace rfde
