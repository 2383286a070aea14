// Hardware peak probe for the measurement: a kernel that issues nothing but matrix-core
// instructions on register-resident operands, so its rate is the chip's sustained MFMA peak for
// one instruction form.  Used beside a device copy to state the roofline the solver's kernels
// are measured against on the machine at hand (the published figures are the reference).
#include "rfde_internal.hpp"

namespace rfde {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int PROBE_CHAINS = 8;  // independent accumulators per wave (covers the MFMA latency)

// KIND 0: v_mfma_f64_16x16x4f64; 1: v_mfma_f32_16x16x4f32; 2: v_mfma_f32_16x16x16bf16_1k;
// 3: v_mfma_f32_16x16x32_bf16.  Every lane writes one value so nothing is optimised away.
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_mfma(int iters, float seed, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const float x = seed + 1e-3f * (float)lane;
  if constexpr (KIND == 0) {
    v4d acc[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
    const double a = (double)x, b = 1.0 - (double)x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = (float)s;
  } else if constexpr (KIND == 1) {
    v4f acc[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = (v4f){0.f, 0.f, 0.f, 0.f};
    const float a = x, b = 1.f - x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
  } else if constexpr (KIND == 2) {
    v4f acc[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = (v4f){0.f, 0.f, 0.f, 0.f};
    const short h = (short)(__float_as_uint(x) >> 16);
    const v4s a = (v4s){h, h, h, h}, b = (v4s){h, h, h, h};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
  } else {
    v4f acc[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = (v4f){0.f, 0.f, 0.f, 0.f};
    const __bf16 h = (__bf16)x;
    const v8bf a = (v8bf){h, h, h, h, h, h, h, h};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
  }
}

}  // namespace rfde

using namespace rfde;

extern "C" {

int rfde_probe_mfma(int kind, int iters, double* tflops, void* stream) {
  if (kind < 0 || kind > 3 || iters < 1 || iters > (1 << 20) || !tflops) return RFDE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  constexpr int blocks = 2048;  // 8 waves per CU on 256 CUs
  float* out = nullptr;
  RFDE_HIP(hipMallocAsync((void**)&out, (size_t)blocks * 256 * sizeof(float), st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = RFDE_OK;
  auto launch = [&](int it) {
    switch (kind) {
      case 0: k_probe_mfma<0><<<blocks, 256, 0, st>>>(it, 0.5f, out); break;
      case 1: k_probe_mfma<1><<<blocks, 256, 0, st>>>(it, 0.5f, out); break;
      case 2: k_probe_mfma<2><<<blocks, 256, 0, st>>>(it, 0.5f, out); break;
      default: k_probe_mfma<3><<<blocks, 256, 0, st>>>(it, 0.5f, out); break;
    }
    return hipGetLastError();
  };
  do {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { rc = RFDE_EHIP; break; }
    if (launch(iters) != hipSuccess) { rc = RFDE_EHIP; break; }  // warm-up (clocks, code load)
    if (hipEventRecord(e0, st) != hipSuccess || launch(iters) != hipSuccess ||
        hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = RFDE_EHIP;
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) { rc = RFDE_EHIP; break; }
    // flops per instruction: 2 * 16 * 16 * K with K = 4, 4, 16, 32
    const double K = kind <= 1 ? 4.0 : (kind == 2 ? 16.0 : 32.0);
    const double flops = (double)blocks * 4 * (double)iters * PROBE_CHAINS * 2.0 * 16 * 16 * K;
    *tflops = flops / (ms * 1e-3) / 1e12;
  } while (0);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFreeAsync(out, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

}  // extern "C"
