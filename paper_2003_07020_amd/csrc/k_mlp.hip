// Learned initial guess: forward, backward and Adam kernels of the guess network, the guess
// assembly and the sine-mode projection used to build its training targets.
//
// Network (per sample): phat = (p - mu)/sd; h1 = tanh(W1 phat + b1); h2 = tanh(W2 h1 + b2);
// g = W3t h2 + b3 with W3t [NOUT x H2].  The output layer is the large one (NOUT = nsrc Nt Ks,
// 524288 at M = 1023, N_t = 512, Ks = 64); its two products run on BF16 MFMAs
// (v_mfma_f32_16x16x16_bf16, FP32 accumulate) with BF16 copies of W3t, h2 and dg, while the
// weight gradient dW3t = dg^T h2 is formed in FP32 inside the Adam update.  Loss = mean (g - y)^2.
#include <cmath>
#include <mutex>

#include "rfde_internal.hpp"

namespace rfde {

typedef float mf4_t __attribute__((ext_vector_type(4)));
typedef short ms4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

// accumulator element e of lane l sits at row 4*(l/16) + e, column l%16 of the 16x16 block
__device__ __forceinline__ int bf_row(int l, int e) { return 4 * (l >> 4) + e; }

// ---- hidden layers: one block per sample -----------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_hidden(const float* __restrict__ feats,
                                                    const float* __restrict__ mu,
                                                    const float* __restrict__ sd,
                                                    const float* __restrict__ W1,
                                                    const float* __restrict__ b1,
                                                    const float* __restrict__ W2,
                                                    const float* __restrict__ b2, int Pin, int H1,
                                                    int H2, float* __restrict__ phat_out,
                                                    float* __restrict__ h1, float* __restrict__ h2,
                                                    unsigned short* __restrict__ h2b) {
  __shared__ float ph[64];
  __shared__ float a1[256];
  const int b = blockIdx.x, t = threadIdx.x;
  if (t < Pin) {
    const float v = (feats[(size_t)b * Pin + t] - mu[t]) / sd[t];
    ph[t] = v;
    phat_out[(size_t)b * Pin + t] = v;
  }
  __syncthreads();
  if (t < H1) {
    float s = b1[t];
    for (int q = 0; q < Pin; ++q) s = fmaf(W1[t * Pin + q], ph[q], s);
    const float v = tanhf(s);
    a1[t] = v;
    h1[(size_t)b * H1 + t] = v;
  }
  __syncthreads();
  if (t < H2) {
    float s = b2[t];
    for (int q = 0; q < H1; ++q) s = fmaf(W2[t * H1 + q], a1[q], s);
    const float v = tanhf(s);
    h2[(size_t)b * H2 + t] = v;
    h2b[(size_t)b * H2 + t] = f2bf(v);
  }
}

// ---- output layer: g[b][o] = sum_h h2[b][h] W3t[o][h] + b3[o] --------------------------------
// One wave per 16 output columns and all batch rows (B <= 64, padded to 16-row blocks).  VEC:
// h2's BF16 copy and W3t's are 8-byte aligned, and a lane's four consecutive values of a k step
// come as one 8-byte load (one access per lane instead of four).
template <int RB, bool VEC>
__global__ void __launch_bounds__(256) k_mlp_out(const unsigned short* __restrict__ h2b,
                                                 const unsigned short* __restrict__ W3b,
                                                 const float* __restrict__ b3, int B, int H2,
                                                 int NOUT, float* __restrict__ g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int o0 = (blockIdx.x * 4 + w) * 16;
  if (o0 >= NOUT) return;
  const int l16 = lane & 15, lq = lane >> 4;
  mf4_t acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = (mf4_t){0.f, 0.f, 0.f, 0.f};
  const unsigned short* wrow = W3b + (size_t)(o0 + l16) * H2;
  for (int k0 = 0; k0 < H2; k0 += 16) {
    const int kk = k0 + 4 * lq;
    ms4_t bv;
    if constexpr (VEC) {
      bv = *reinterpret_cast<const ms4_t*>(wrow + kk);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = (short)wrow[kk + j];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int bb = r * 16 + l16;
      ms4_t av = (ms4_t){0, 0, 0, 0};
      if (bb < B) {
        const unsigned short* hrow = h2b + (size_t)bb * H2 + kk;
        if constexpr (VEC) {
          av = *reinterpret_cast<const ms4_t*>(hrow);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) av[j] = (short)hrow[j];
        }
      }
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[r], 0, 0, 0);
    }
  }
  const int o = o0 + l16;
  const float bias = b3[o];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int bb = r * 16 + bf_row(lane, e);
      if (bb < B) g[(size_t)bb * NOUT + o] = acc[r][e] + bias;
    }
}

// ---- loss and dg ---------------------------------------------------------------------------------
constexpr int MLP_RED = 1024;
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ g,
                                                  const float* __restrict__ y, size_t n,
                                                  float* __restrict__ dg,
                                                  unsigned short* __restrict__ dgb,
                                                  double* __restrict__ partial) {
  __shared__ double sh[4];
  const float scale = 2.0f / (float)n;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)MLP_RED * 256) {
    const float d = g[i] - y[i];
    acc += (double)d * d;
    const float gr = scale * d;
    dg[i] = gr;
    dgb[i] = f2bf(gr);
  }
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void __launch_bounds__(256) k_mlp_loss_final(const double* __restrict__ partial,
                                                        size_t n, float* __restrict__ loss) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int b = threadIdx.x; b < MLP_RED; b += 256) acc += partial[b];
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = (float)(((sh[0] + sh[1]) + (sh[2] + sh[3])) / (double)n);
}

// ---- dh2[b][h] = sum_o dg[b][o] W3t[o][h], split over chunks of KCH output columns -----------------
// VEC: dg's BF16 copy is 8-byte aligned and a lane's four consecutive dg values of a k step come
// as one 8-byte load.
constexpr int KCH = 1024;
template <int RB, bool VEC>
__global__ void __launch_bounds__(256) k_mlp_dh2(const unsigned short* __restrict__ dgb,
                                                 const unsigned short* __restrict__ W3b, int B,
                                                 int H2, int NOUT, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int c0 = blockIdx.x * KCH;
  const int nhb = H2 / 16;
  for (int hb = w; hb < nhb; hb += 4) {
    mf4_t acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = (mf4_t){0.f, 0.f, 0.f, 0.f};
    const int h = hb * 16 + l16;
    for (int k0 = c0; k0 < c0 + KCH && k0 < NOUT; k0 += 16) {
      const int kk = k0 + 4 * lq;
      ms4_t bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = (short)W3b[(size_t)(kk + j) * H2 + h];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int bb = r * 16 + l16;
        ms4_t av = (ms4_t){0, 0, 0, 0};
        if (bb < B) {
          const unsigned short* drow = dgb + (size_t)bb * NOUT + kk;
          if constexpr (VEC) {
            av = *reinterpret_cast<const ms4_t*>(drow);
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) av[j] = (short)drow[j];
          }
        }
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[r], 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int bb = r * 16 + bf_row(lane, e);
        if (bb < B) part[((size_t)blockIdx.x * B + bb) * H2 + h] = acc[r][e];
      }
  }
}

__global__ void k_mlp_dh2_reduce(const float* __restrict__ part, int nchunk, int BH,
                                 float* __restrict__ dh2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= BH) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * BH + i];
  dh2[i] = s;
}

// ---- Adam ----------------------------------------------------------------------------------------
struct AdamCfg {
  float lr, b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};
__device__ __forceinline__ void adam_apply(float& w, float& m, float& v, float grad,
                                           const AdamCfg& a) {
  m = a.b1 * m + (1.f - a.b1) * grad;
  v = a.b2 * v + (1.f - a.b2) * grad * grad;
  w -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

// dW3t[o][h] = sum_b dg[b][o] h2[b][h] (FP32), db3[o] = sum_b dg[b][o]; Adam update of W3t and
// its BF16 copy (mode 0) or plain gradient output (mode 1).  A thread owns a 4 x 4 block of
// weights: four consecutive outputs o (NOUT % 16 == 0) by four consecutive h (H2 % 16 == 0), so
// each row's 16-byte h2 load feeds sixteen sums and each dg value four, and consecutive threads
// take consecutive h (row accesses stay contiguous); the batch loop is unrolled so that several
// rows' loads are in flight, and every sum still runs over b in order.  VEC: h2, the parameter
// arrays (and the gradient output) are 16-byte aligned and are moved four values per access;
// otherwise one value per access.
template <bool VEC>
__global__ void __launch_bounds__(256) k_mlp_w3(const float* __restrict__ dg,
                                                const float* __restrict__ h2, int B, int H2,
                                                int NOUT, float* __restrict__ W3t,
                                                unsigned short* __restrict__ W3b,
                                                float* __restrict__ mW, float* __restrict__ vW,
                                                float* __restrict__ b3, float* __restrict__ mb,
                                                float* __restrict__ vb, AdamCfg a, int mode,
                                                float* __restrict__ gW, float* __restrict__ gb) {
  const int qr = H2 / 4;
  const size_t units = (size_t)(NOUT / 4) * qr;
  const size_t u = blockIdx.x * (size_t)256 + threadIdx.x;
  if (u >= units) return;
  const int h = 4 * (int)(u % qr);
  const int o0 = 4 * (int)(u / qr);
  float sm[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) sm[i][c] = 0.f;
#pragma unroll 4
  for (int b = 0; b < B; ++b) {
    const float* hb = h2 + (size_t)b * H2 + h;
    float4 x;
    if constexpr (VEC) x = *reinterpret_cast<const float4*>(hb);
    else x = make_float4(hb[0], hb[1], hb[2], hb[3]);
    const float* db = dg + (size_t)b * NOUT + o0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float d = db[i];
      sm[i][0] = fmaf(d, x.x, sm[i][0]);
      sm[i][1] = fmaf(d, x.y, sm[i][1]);
      sm[i][2] = fmaf(d, x.z, sm[i][2]);
      sm[i][3] = fmaf(d, x.w, sm[i][3]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const size_t e = (size_t)(o0 + i) * H2 + h;
    if (mode == 1) {
      if constexpr (VEC) {
        *reinterpret_cast<float4*>(gW + e) = make_float4(sm[i][0], sm[i][1], sm[i][2], sm[i][3]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) gW[e + c] = sm[i][c];
      }
    } else if constexpr (VEC) {
      float4 w = *reinterpret_cast<const float4*>(W3t + e);
      float4 m = *reinterpret_cast<const float4*>(mW + e);
      float4 v = *reinterpret_cast<const float4*>(vW + e);
      adam_apply(w.x, m.x, v.x, sm[i][0], a);
      adam_apply(w.y, m.y, v.y, sm[i][1], a);
      adam_apply(w.z, m.z, v.z, sm[i][2], a);
      adam_apply(w.w, m.w, v.w, sm[i][3], a);
      *reinterpret_cast<float4*>(W3t + e) = w;
      *reinterpret_cast<float4*>(mW + e) = m;
      *reinterpret_cast<float4*>(vW + e) = v;
      const unsigned int lo = f2bf(w.x) | ((unsigned int)f2bf(w.y) << 16);
      const unsigned int hi = f2bf(w.z) | ((unsigned int)f2bf(w.w) << 16);
      *reinterpret_cast<uint2*>(W3b + e) = make_uint2(lo, hi);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float w = W3t[e + c], m = mW[e + c], v = vW[e + c];
        adam_apply(w, m, v, sm[i][c], a);
        W3t[e + c] = w; mW[e + c] = m; vW[e + c] = v;
        W3b[e + c] = f2bf(w);
      }
    }
  }
  if (h == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = o0 + i;
      float sb = 0.f;
      for (int b = 0; b < B; ++b) sb += dg[(size_t)b * NOUT + o];
      if (mode == 1) {
        gb[o] = sb;
      } else {
        float w = b3[o], m = mb[o], v = vb[o];
        adam_apply(w, m, v, sb, a);
        b3[o] = w; mb[o] = m; vb[o] = v;
      }
    }
  }
}

// Hidden layers backward from dh2, with Adam (mode 0) or gradient output (mode 1), in three
// launches over the elements: da2 = dh2 (1 - h2^2); da1 = (da2 W2) (1 - h1^2), which reads W2
// before its update; then every small-layer parameter (W2, b2, W1, b1, in that index order)
// forms its gradient as a sum over the batch in order and takes its Adam step.
struct SmallParams {
  float *W1, *b1, *W2, *b2;
  float *mW1, *vW1, *mb1, *vb1, *mW2, *vW2, *mb2, *vb2;
  float *gW1, *gb1, *gW2, *gb2;
};
__global__ void __launch_bounds__(256) k_mlp_da2(const float* __restrict__ h2,
                                                 const float* __restrict__ dh2, int n,
                                                 float* __restrict__ da2) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n) da2[e] = dh2[e] * (1.f - h2[e] * h2[e]);
}
__global__ void __launch_bounds__(256) k_mlp_da1(const float* __restrict__ h1,
                                                 const float* __restrict__ da2,
                                                 const float* __restrict__ W2, int B, int H1,
                                                 int H2, float* __restrict__ da1) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= B * H1) return;
  const int b = e / H1, q = e % H1;
  float s = 0.f;
  for (int r = 0; r < H2; ++r) s = fmaf(da2[b * H2 + r], W2[r * H1 + q], s);
  da1[e] = s * (1.f - h1[e] * h1[e]);
}
__global__ void __launch_bounds__(256) k_mlp_small_update(const float* __restrict__ phat,
                                                          const float* __restrict__ h1,
                                                          const float* __restrict__ da2,
                                                          const float* __restrict__ da1, int B,
                                                          int Pin, int H1, int H2,
                                                          SmallParams P, AdamCfg a, int mode) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e < H2 * H1) {
    const int r = e / H1, q = e % H1;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s = fmaf(da2[b * H2 + r], h1[b * H1 + q], s);
    if (mode == 1) P.gW2[e] = s;
    else adam_apply(P.W2[e], P.mW2[e], P.vW2[e], s, a);
    return;
  }
  e -= H2 * H1;
  if (e < H2) {
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += da2[b * H2 + e];
    if (mode == 1) P.gb2[e] = s;
    else adam_apply(P.b2[e], P.mb2[e], P.vb2[e], s, a);
    return;
  }
  e -= H2;
  if (e < H1 * Pin) {
    const int q = e / Pin, c = e % Pin;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s = fmaf(da1[b * H1 + q], phat[b * Pin + c], s);
    if (mode == 1) P.gW1[e] = s;
    else adam_apply(P.W1[e], P.mW1[e], P.vW1[e], s, a);
    return;
  }
  e -= H1 * Pin;
  if (e < H1) {
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += da1[b * H1 + e];
    if (mode == 1) P.gb1[e] = s;
    else adam_apply(P.b1[e], P.mb1[e], P.vb1[e], s, a);
  }
}

// ---- guess assembly and projection -----------------------------------------------------------
__global__ void k_sine_table(double* __restrict__ S, int M, int Ks) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * Ks) return;
  const int i = e / Ks, s = e % Ks;
  const long long ph = (long long)(i + 1) * (s + 1) % (2 * (M + 1));
  S[e] = sinpi((double)ph / (M + 1));
}

// U[t][i] = sum_s Y[t][s] S[i][s], Y[t][s] = sum_k cs[k] g[k][t][s]; one block per t.
__global__ void __launch_bounds__(256) k_guess_assemble(const float* __restrict__ g,
                                                        const double* __restrict__ cs, int nsrc,
                                                        int Nt, int Ks, int M,
                                                        const double* __restrict__ S,
                                                        double* __restrict__ U) {
  __shared__ double Y[256];
  const int t = blockIdx.x;
  for (int s = threadIdx.x; s < Ks; s += 256) {
    double acc = 0.0;
    for (int k = 0; k < nsrc; ++k) acc += cs[k] * (double)g[((size_t)k * Nt + t) * Ks + s];
    Y[s] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < M; i += 256) {
    double acc = 0.0;
    for (int s = 0; s < Ks; ++s) acc = fma(Y[s], S[(size_t)i * Ks + s], acc);
    U[(size_t)t * M + i] = acc;
  }
}

// Y[t][s] = factor (2/(M+1)) sum_i U[t][i] S[i][s]; one block per t, one thread per s.
__global__ void __launch_bounds__(256) k_project_sine(const double* __restrict__ U, int M, int Ks,
                                                      const double* __restrict__ S, double factor,
                                                      float* __restrict__ Y) {
  const int t = blockIdx.x, s = threadIdx.x;
  if (s >= Ks) return;
  const double* row = U + (size_t)t * M;
  double acc = 0.0;
  for (int i = 0; i < M; ++i) acc = fma(row[i], S[(size_t)i * Ks + s], acc);
  Y[(size_t)t * Ks + s] = (float)(acc * factor * 2.0 / (M + 1));
}

}  // namespace rfde

using namespace rfde;

extern "C" {

static bool mlp_ok(const rfde_mlp* m, int B) {
  return m && B >= 1 && B <= 64 && m->Pin >= 1 && m->Pin <= 64 && m->H1 >= 1 && m->H1 <= 256 &&
         m->H2 >= 16 && m->H2 <= 256 && m->H2 % 16 == 0 && m->NOUT >= 16 && m->NOUT % 16 == 0 &&
         m->W1 && m->b1 && m->W2 && m->b2 && m->W3t && m->b3 && m->W3t_bf16 && m->mu && m->sd;
}

size_t rfde_mlp_workspace_bytes(const rfde_mlp* m, int B) {
  if (!m) return 0;
  const size_t nchunk = ((size_t)m->NOUT + KCH - 1) / KCH;
  size_t b = 0;
  b += (size_t)B * m->Pin * 4 + (size_t)B * m->H1 * 4 + (size_t)B * m->H2 * 4;  // phat, h1, h2
  b += (size_t)B * m->H2 * 2;                                                  // h2 bf16
  b += (size_t)B * m->NOUT * 4 + (size_t)B * m->NOUT * 2;                      // dg, dg bf16
  b += nchunk * B * m->H2 * 4 + (size_t)B * m->H2 * 4;                         // dh2 parts, dh2
  b += (size_t)B * m->H2 * 4 + (size_t)B * m->H1 * 4;                          // da2, da1
  b += MLP_RED * 8 + 256;                                                      // loss partials
  return b + 64 * 16;  // alignment slack
}

struct MlpWs {
  float *phat, *h1, *h2, *dg, *dh2part, *dh2, *da2, *da1;
  unsigned short *h2b, *dgb;
  double* part;
};
static inline size_t carve_round(size_t bytes) { return (bytes + 63) & ~(size_t)63; }
// Bytes of the forward pass's part of the workspace (phat, h1, h2, h2 in BF16), which carve()
// places first.
static size_t forward_ws_bytes(const rfde_mlp* m, int B) {
  return carve_round((size_t)B * m->Pin * 4) + carve_round((size_t)B * m->H1 * 4) +
         carve_round((size_t)B * m->H2 * 4) + carve_round((size_t)B * m->H2 * 2);
}
static MlpWs carve(const rfde_mlp* m, int B, void* ws, bool forward_only = false) {
  unsigned char* p = (unsigned char*)ws;
  auto take = [&](size_t bytes) {
    unsigned char* r = p;
    p += carve_round(bytes);
    return (void*)r;
  };
  const size_t nchunk = ((size_t)m->NOUT + KCH - 1) / KCH;
  MlpWs w{};
  w.phat = (float*)take((size_t)B * m->Pin * 4);
  w.h1 = (float*)take((size_t)B * m->H1 * 4);
  w.h2 = (float*)take((size_t)B * m->H2 * 4);
  w.h2b = (unsigned short*)take((size_t)B * m->H2 * 2);
  if (forward_only) return w;
  w.dg = (float*)take((size_t)B * m->NOUT * 4);
  w.dgb = (unsigned short*)take((size_t)B * m->NOUT * 2);
  w.dh2part = (float*)take(nchunk * B * m->H2 * 4);
  w.dh2 = (float*)take((size_t)B * m->H2 * 4);
  w.da2 = (float*)take((size_t)B * m->H2 * 4);
  w.da1 = (float*)take((size_t)B * m->H1 * 4);
  w.part = (double*)take(MLP_RED * 8);
  return w;
}

static int mlp_forward_impl(const rfde_mlp* m, const float* feats, int B, float* g, MlpWs& w,
                            hipStream_t st) {
  k_mlp_hidden<<<B, 256, 0, st>>>(feats, m->mu, m->sd, m->W1, m->b1, m->W2, m->b2, m->Pin, m->H1,
                                  m->H2, w.phat, w.h1, w.h2, w.h2b);
  RFDE_HIP(hipGetLastError());
  const int blocks = (m->NOUT / 16 + 3) / 4;
  const int RB = (B + 15) / 16;
  const bool vec = ((uintptr_t)m->W3t_bf16 & 7) == 0 && ((uintptr_t)w.h2b & 7) == 0;
#define RFDE_MLP_OUT(R, V) \
  k_mlp_out<R, V><<<blocks, 256, 0, st>>>(w.h2b, m->W3t_bf16, m->b3, B, m->H2, m->NOUT, g)
  switch (RB) {
    case 1: if (vec) RFDE_MLP_OUT(1, true); else RFDE_MLP_OUT(1, false); break;
    case 2: if (vec) RFDE_MLP_OUT(2, true); else RFDE_MLP_OUT(2, false); break;
    case 3: if (vec) RFDE_MLP_OUT(3, true); else RFDE_MLP_OUT(3, false); break;
    default: if (vec) RFDE_MLP_OUT(4, true); else RFDE_MLP_OUT(4, false); break;
  }
#undef RFDE_MLP_OUT
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int rfde_mlp_forward(const rfde_mlp* m, const float* feats, int B, float* g, void* ws,
                     void* stream) {
  if (!mlp_ok(m, B) || !feats || !g || !ws) return RFDE_EINVAL;
  MlpWs w = carve(m, B, ws);
  return mlp_forward_impl(m, feats, B, g, w, (hipStream_t)stream);
}

// ---- forward pass without a caller workspace ---------------------------------------------------
// The activations live in `scratch`, a fixed device array of each GPU.  Host code never uses the
// array's name as an address: its device address is looked up once per device with
// hipGetSymbolAddress and kept in scratch_dev[].  Every call on one device shares the array, so
// calls on that device must not overlap (they race); nothing in it needs clearing, since the
// forward pass writes every activation before reading it.
constexpr size_t MLP_SCRATCH_BYTES = 256 * 1024;
constexpr int MLP_SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[MLP_SCRATCH_BYTES];
static void* scratch_dev[MLP_SCRATCH_MAX_DEVICES];
static std::mutex scratch_mu;

static int scratch_ptr(void** out) {
  int dev = -1;
  RFDE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MLP_SCRATCH_MAX_DEVICES) return RFDE_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    RFDE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return RFDE_EHIP;
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return RFDE_OK;
}

size_t rfde_mlp_forward_noalloc_max_bytes(void) { return MLP_SCRATCH_BYTES; }

int rfde_mlp_forward_noalloc(const rfde_mlp* m, const float* feats, int B, float* g,
                             void* stream) {
  if (!mlp_ok(m, B) || !feats || !g) return RFDE_EINVAL;
  if (forward_ws_bytes(m, B) > MLP_SCRATCH_BYTES) return RFDE_EINVAL;
  void* ptr = nullptr;
  const int rc = scratch_ptr(&ptr);
  if (rc != RFDE_OK) return rc;
  MlpWs w = carve(m, B, ptr, /*forward_only=*/true);
  return mlp_forward_impl(m, feats, B, g, w, (hipStream_t)stream);
}

// forward + loss + backward; mode 0: Adam step, mode 1: gradients into grads (flat, parameter
// order W1, b1, W2, b2, W3t, b3).
static int mlp_backward(const rfde_mlp* m, const float* feats, const float* y, int B, float* g,
                        float lr, int t, float* loss, int mode, float* grads, void* ws,
                        hipStream_t st) {
  MlpWs w = carve(m, B, ws);
  {
    const int rc = mlp_forward_impl(m, feats, B, g, w, st);
    if (rc != RFDE_OK) return rc;
  }
  const size_t n = (size_t)B * m->NOUT;
  k_mlp_loss<<<MLP_RED, 256, 0, st>>>(g, y, n, w.dg, w.dgb, w.part);
  RFDE_HIP(hipGetLastError());
  k_mlp_loss_final<<<1, 256, 0, st>>>(w.part, n, loss);
  RFDE_HIP(hipGetLastError());
  const int nchunk = (m->NOUT + KCH - 1) / KCH;
  const int RB = (B + 15) / 16;
  const bool dvec = ((uintptr_t)w.dgb & 7) == 0;
#define RFDE_MLP_DH2(R, V) \
  k_mlp_dh2<R, V><<<nchunk, 256, 0, st>>>(w.dgb, m->W3t_bf16, B, m->H2, m->NOUT, w.dh2part)
  switch (RB) {
    case 1: if (dvec) RFDE_MLP_DH2(1, true); else RFDE_MLP_DH2(1, false); break;
    case 2: if (dvec) RFDE_MLP_DH2(2, true); else RFDE_MLP_DH2(2, false); break;
    case 3: if (dvec) RFDE_MLP_DH2(3, true); else RFDE_MLP_DH2(3, false); break;
    default: if (dvec) RFDE_MLP_DH2(4, true); else RFDE_MLP_DH2(4, false); break;
  }
#undef RFDE_MLP_DH2
  RFDE_HIP(hipGetLastError());
  const int BH = B * m->H2;
  k_mlp_dh2_reduce<<<(BH + 255) / 256, 256, 0, st>>>(w.dh2part, nchunk, BH, w.dh2);
  RFDE_HIP(hipGetLastError());
  AdamCfg a;
  a.lr = lr; a.b1 = 0.9f; a.b2 = 0.999f; a.eps = 1e-8f;
  a.c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
  a.c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
  // parameter offsets in the flat gradient buffer
  const size_t oW1 = 0, ob1 = oW1 + (size_t)m->H1 * m->Pin, oW2 = ob1 + m->H1,
               ob2 = oW2 + (size_t)m->H2 * m->H1, oW3 = ob2 + m->H2,
               ob3 = oW3 + (size_t)m->NOUT * m->H2;
  // small layers first: their backward reads W2 before the update
  SmallParams P;
  P.W1 = m->W1; P.b1 = m->b1; P.W2 = m->W2; P.b2 = m->b2;
  P.mW1 = m->mW1; P.vW1 = m->vW1; P.mb1 = m->mb1; P.vb1 = m->vb1;
  P.mW2 = m->mW2; P.vW2 = m->vW2; P.mb2 = m->mb2; P.vb2 = m->vb2;
  P.gW1 = grads ? grads + oW1 : nullptr; P.gb1 = grads ? grads + ob1 : nullptr;
  P.gW2 = grads ? grads + oW2 : nullptr; P.gb2 = grads ? grads + ob2 : nullptr;
  const int nda2 = B * m->H2, nda1 = B * m->H1;
  const int nsmall = m->H2 * m->H1 + m->H2 + m->H1 * m->Pin + m->H1;
  k_mlp_da2<<<(nda2 + 255) / 256, 256, 0, st>>>(w.h2, w.dh2, nda2, w.da2);
  RFDE_HIP(hipGetLastError());
  k_mlp_da1<<<(nda1 + 255) / 256, 256, 0, st>>>(w.h1, w.da2, m->W2, B, m->H1, m->H2, w.da1);
  RFDE_HIP(hipGetLastError());
  k_mlp_small_update<<<(nsmall + 255) / 256, 256, 0, st>>>(w.phat, w.h1, w.da2, w.da1, B,
                                                            m->Pin, m->H1, m->H2, P, a, mode);
  RFDE_HIP(hipGetLastError());
  const size_t quads = (size_t)(m->NOUT / 4) * (m->H2 / 4);  // 4 x 4 weight blocks
  float* gW3 = grads ? grads + oW3 : nullptr;
  auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  const bool vec = al16(w.h2) &&
                   (mode == 1 ? al16(gW3)
                              : (al16(m->W3t) && al16(m->mW3) && al16(m->vW3) &&
                                 ((uintptr_t)m->W3t_bf16 & 7) == 0));
  if (vec)
    k_mlp_w3<true><<<(unsigned)((quads + 255) / 256), 256, 0, st>>>(
        w.dg, w.h2, B, m->H2, m->NOUT, m->W3t, m->W3t_bf16, m->mW3, m->vW3, m->b3, m->mb3,
        m->vb3, a, mode, gW3, grads ? grads + ob3 : nullptr);
  else
    k_mlp_w3<false><<<(unsigned)((quads + 255) / 256), 256, 0, st>>>(
        w.dg, w.h2, B, m->H2, m->NOUT, m->W3t, m->W3t_bf16, m->mW3, m->vW3, m->b3, m->mb3,
        m->vb3, a, mode, gW3, grads ? grads + ob3 : nullptr);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int rfde_mlp_grads(const rfde_mlp* m, const float* feats, const float* y, int B, float* g,
                   float* grads, float* loss, void* ws, void* stream) {
  if (!mlp_ok(m, B) || !feats || !y || !g || !grads || !loss || !ws) return RFDE_EINVAL;
  return mlp_backward(m, feats, y, B, g, 0.f, 1, loss, 1, grads, ws, (hipStream_t)stream);
}

int rfde_mlp_train_step(const rfde_mlp* m, const float* feats, const float* y, int B, float* g,
                        float lr, int t, float* loss, void* ws, void* stream) {
  if (!mlp_ok(m, B) || !feats || !y || !g || !loss || !ws || t < 1 || !(lr > 0.f) || !m->mW1 ||
      !m->vW1 || !m->mb1 || !m->vb1 || !m->mW2 || !m->vW2 || !m->mb2 || !m->vb2 || !m->mW3 ||
      !m->vW3 || !m->mb3 || !m->vb3)
    return RFDE_EINVAL;
  return mlp_backward(m, feats, y, B, g, lr, t, loss, 0, nullptr, ws, (hipStream_t)stream);
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, unsigned short* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = f2bf(a[i]);
}

int rfde_f32_to_bf16(size_t n, const float* src, unsigned short* dst, void* stream) {
  if (!src || !dst) return RFDE_EINVAL;
  if (n == 0) return RFDE_OK;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 16384);
  k_f32_to_bf16<<<blocks, 256, 0, (hipStream_t)stream>>>(src, dst, n);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int rfde_sine_table(int M, int Ks, double* S, void* stream) {
  if (M < 1 || Ks < 1 || Ks > 256 || !S) return RFDE_EINVAL;
  k_sine_table<<<(M * Ks + 255) / 256, 256, 0, (hipStream_t)stream>>>(S, M, Ks);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int rfde_guess_assemble(int nsrc, int Nt, int Ks, int M, const float* g, const double* coef_scaled,
                        const double* S, double* U, void* stream) {
  if (nsrc < 1 || Nt < 1 || Ks < 1 || Ks > 256 || M < 1 || !g || !coef_scaled || !S || !U)
    return RFDE_EINVAL;
  k_guess_assemble<<<Nt, 256, 0, (hipStream_t)stream>>>(g, coef_scaled, nsrc, Nt, Ks, M, S, U);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int rfde_project_sine(int Nt, int M, int Ks, const double* U, const double* S, double factor,
                      float* Y, void* stream) {
  if (Nt < 1 || M < 1 || Ks < 1 || Ks > 256 || !U || !S || !Y) return RFDE_EINVAL;
  k_project_sine<<<Nt, 256, 0, (hipStream_t)stream>>>(U, M, Ks, S, factor, Y);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // extern "C"
