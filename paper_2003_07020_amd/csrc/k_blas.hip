// Vector kernels of the FGMRES outer iteration (FP64).  Reductions are deterministic: a fixed
// grid writes one partial per block in a fixed order, and a single block sums the partials
// with a fixed tree, so repeated runs are bitwise identical.
#include "krylov.hpp"
#include "rfde_internal.hpp"

namespace rfde {

constexpr int RED_BLOCKS = 1024;  // partials per reduced quantity
constexpr int VCHUNK = 4;         // vectors handled per pass of the multi-dot kernel

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

int launch_multi_dot(const Plan& p, const double* V, int nvec, const double* w, double* out) {
  const size_t n = p.N();
  for (int v0 = 0; v0 < nvec; v0 += VCHUNK) {
    const int nv = std::min(VCHUNK, nvec - v0);
    k_dot_partial<<<RED_BLOCKS, 256, 0, p.stream>>>(V + (size_t)v0 * n, n, nv, w, n,
                                                     p.red + (size_t)v0 * RED_BLOCKS);
    RFDE_HIP(hipGetLastError());
  }
  k_dot_final<<<nvec, 256, 0, p.stream>>>(p.red, out, 0);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// ---- CGS2 in three sweeps over the basis (classical Gram-Schmidt applied twice) ----
// Sweep A: h1 = V^T w.  Sweep B: w1 = w - V h1, and h2 = V^T w1 accumulated in the same sweep
// (each element of w1 is formed in registers, then multiplied by the basis values just read).
// Sweep C: w2 = w1 - V h2 and |w2|^2.  The arithmetic is that of CGS2; one sweep over V and w is
// saved, and the host reads h1, h2 and |w2| once per Arnoldi step.
constexpr int CGS_ACC = 16;  // dot products accumulated per sweep
enum { CGS_DOT = 0, CGS_AXPY_DOT = 1, CGS_AXPY_NRM = 2 };

// MODE CGS_DOT:      partial[v][b] = sum_i V[v][i] w[i], v < nv.
// MODE CGS_AXPY_DOT: w[i] -= sum_{v < nall} h[v] V[v][i]; partial[v][b] = sum_i V[v][i] w[i]
//                    (the updated w), v < nv.
// MODE CGS_AXPY_NRM: w[i] -= sum_{v < nall} h[v] V[v][i]; partial[0][b] = sum_i w[i]^2.
// V holds the vectors at stride n.  NV > 0: nv = NV and, for the correcting modes, nall = NV,
// known at compile time so every basis value of an element is loaded before any is used (all
// loads in flight together); NV = 0: any nall (> CGS_ACC) with nv = CGS_ACC, by loops.
// Elements are read in pairs (16-byte loads) with the last element of an odd n done alone.
template <int MODE, int NV>
__global__ void __launch_bounds__(256) k_cgs(double* __restrict__ w, const double* __restrict__ V,
                                             size_t n, int nall, const double* __restrict__ h,
                                             double* __restrict__ partial) {
  constexpr int NACC = MODE == CGS_AXPY_NRM ? 1 : (NV > 0 ? NV : CGS_ACC);
  double acc[NACC];
#pragma unroll
  for (int v = 0; v < NACC; ++v) acc[v] = 0.0;
  auto element = [&](size_t i, double wi) -> double {
    if constexpr (NV > 0) {
      double vv[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) vv[v] = V[(size_t)v * n + i];
      if constexpr (MODE != CGS_DOT) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s = fma(h[v], vv[v], s);
        wi -= s;
      }
      if constexpr (MODE == CGS_AXPY_NRM) {
        acc[0] = fma(wi, wi, acc[0]);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = fma(vv[v], wi, acc[v]);
      }
    } else {
      static_assert(MODE != CGS_DOT, "dot sweeps take at most CGS_ACC vectors per launch");
      double vv[CGS_ACC];
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < CGS_ACC; ++v) {
        vv[v] = V[(size_t)v * n + i];
        s = fma(h[v], vv[v], s);
      }
      for (int v = CGS_ACC; v < nall; ++v) s = fma(h[v], V[(size_t)v * n + i], s);
      wi -= s;
      if constexpr (MODE == CGS_AXPY_NRM) {
        acc[0] = fma(wi, wi, acc[0]);
      } else {
#pragma unroll
        for (int v = 0; v < CGS_ACC; ++v) acc[v] = fma(vv[v], wi, acc[v]);
      }
    }
    return wi;
  };
  const size_t n2 = n / 2;
  for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < n2; k += (size_t)RED_BLOCKS * 256) {
    const double2 wv = reinterpret_cast<const double2*>(w)[k];
    const double a = element(2 * k, wv.x), b = element(2 * k + 1, wv.y);
    if constexpr (MODE != CGS_DOT) reinterpret_cast<double2*>(w)[k] = make_double2(a, b);
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double a = element(n - 1, w[n - 1]);
    if constexpr (MODE != CGS_DOT) w[n - 1] = a;
  }
  // per-wave sums of every accumulator, then one barrier and the four wave sums per value in
  // the fixed order (w0 + w1) + (w2 + w3)
  __shared__ double shv[4][NACC];
#pragma unroll
  for (int v = 0; v < NACC; ++v) {
    double r = acc[v];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) r += __shfl_xor(r, m);
    if ((threadIdx.x & 63) == 0) shv[threadIdx.x >> 6][v] = r;
  }
  __syncthreads();
  if ((int)threadIdx.x < NACC) {
    const int v = threadIdx.x;
    partial[v * RED_BLOCKS + blockIdx.x] = (shv[0][v] + shv[1][v]) + (shv[2][v] + shv[3][v]);
  }
}

// launch of mode MODE over nv (1..CGS_ACC) vectors known at compile time, or NV = 0
template <int MODE>
static int cgs_launch(const Plan& p, double* w, const double* V, int nall, int nv,
                      const double* h, double* partial) {
  const size_t n = p.N();
#define RFDE_CGS_CASE(K)                                                                     \
  case K:                                                                                    \
    k_cgs<MODE, K><<<RED_BLOCKS, 256, 0, p.stream>>>(w, V, n, nall, h, partial);             \
    break;
  if (MODE != CGS_DOT && nall > CGS_ACC) {
    if constexpr (MODE != CGS_DOT)
      k_cgs<MODE, 0><<<RED_BLOCKS, 256, 0, p.stream>>>(w, V, n, nall, h, partial);
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

int launch_cgs2(const Plan& p, const double* V, int nvec, double* w, double* out) {
  const size_t n = p.N();
  // sweep A: h1 -> out[0 .. nvec)
  for (int v0 = 0; v0 < nvec; v0 += CGS_ACC) {
    const int nv = std::min(CGS_ACC, nvec - v0);
    RFDE_TRY(cgs_launch<CGS_DOT>(p, w, V + (size_t)v0 * n, nv, nv, nullptr,
                                 p.red + (size_t)v0 * RED_BLOCKS));
  }
  k_dot_final<<<nvec, 256, 0, p.stream>>>(p.red, out, 0);
  RFDE_HIP(hipGetLastError());
  // sweep B: w -= V h1 and the dot products with the first CGS_ACC vectors; the rest (if any)
  // by dot sweeps; h2 -> out[CGS2_H2 ..)
  RFDE_TRY(cgs_launch<CGS_AXPY_DOT>(p, w, V, nvec, std::min(CGS_ACC, nvec), out, p.red));
  for (int v0 = CGS_ACC; v0 < nvec; v0 += CGS_ACC) {
    const int nv = std::min(CGS_ACC, nvec - v0);
    RFDE_TRY(cgs_launch<CGS_DOT>(p, w, V + (size_t)v0 * n, nv, nv, nullptr,
                                 p.red + (size_t)v0 * RED_BLOCKS));
  }
  k_dot_final<<<nvec, 256, 0, p.stream>>>(p.red, out + CGS2_H2, 0);
  RFDE_HIP(hipGetLastError());
  // sweep C: w -= V h2 and |w| -> out[CGS2_NRM]
  RFDE_TRY(cgs_launch<CGS_AXPY_NRM>(p, w, V, nvec, std::min(CGS_ACC, nvec), out + CGS2_H2,
                                    p.red));
  k_dot_final<<<1, 256, 0, p.stream>>>(p.red, out + CGS2_NRM, 1);
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

// y = x * s (inv = 0) or y = x / s (inv = 1), s a device scalar
__global__ void k_scale_copy(const double* x, double* y, size_t n,
                             const double* __restrict__ s, int inv) {
  const double a = inv ? 1.0 / s[0] : s[0];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i] * a;
}

int launch_scale_copy(const Plan& p, const double* x, double* y, const double* scal_dev, int inv) {
  const size_t n = p.N();
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  k_scale_copy<<<blocks, 256, 0, p.stream>>>(x, y, n, scal_dev, inv);
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
