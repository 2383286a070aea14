// Vector kernels of the FGMRES outer iteration (FP64).  Reductions are deterministic: a fixed
// grid writes one partial per block in a fixed order, and a single block sums the partials
// with a fixed tree, so repeated runs are bitwise identical.
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

int launch_nrm2(const Plan& p, const double* x, double* out) {
  const size_t n = p.N();
  k_dot_partial<<<RED_BLOCKS, 256, 0, p.stream>>>(x, n, 1, x, n, p.red);
  RFDE_HIP(hipGetLastError());
  k_dot_final<<<1, 256, 0, p.stream>>>(p.red, out, 1);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// w[i] += sign * sum_v coef[v] V[v][i]
__global__ void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, size_t n,
                             int nvec, const double* __restrict__ coef, double sign) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int v = 0; v < nvec; ++v) s = fma(coef[v], V[v * n + i], s);
    w[i] = fma(sign, s, w[i]);
  }
}

int launch_multi_axpy(const Plan& p, double* w, const double* V, int nvec, const double* coef,
                      double sign) {
  const size_t n = p.N();
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  k_multi_axpy<<<blocks, 256, 0, p.stream>>>(w, V, n, nvec, coef, sign);
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
