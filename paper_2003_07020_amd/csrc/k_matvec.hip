// All-at-once matvec y = (C kron I - tau I kron A) v (Section 3.2: vec(V C^T) - tau vec(A V)),
// and the right-hand side F of eq. (2.11).
//
// -tau A = coef T with coef = tau kappa / h^alpha, T symmetric Toeplitz.  T v is the first M
// entries of the symmetric circulant of order L applied to v padded with zeros; that circulant
// is diagonalised by the DFT with the real symbol `sym` (which already carries coef / L).
// Because the symbol is real, one complex transform applies it to two real time levels at
// once: the real part carries level k, the imaginary part level k+1.
//
// Time stencil (rows of C, eq. (2.12)): level 0: v_0; level 1: 3/2 v_1 - 2 v_0;
// level k >= 2: 3/2 v_k - 2 v_{k-1} + 1/2 v_{k-2}.
#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

__device__ __forceinline__ double time_stencil(const double* __restrict__ v, int k, size_t S,
                                               size_t idx) {
  // idx = k * S + i
  if (k == 0) return v[idx];
  if (k == 1) return 1.5 * v[idx] - 2.0 * v[idx - S];
  return 1.5 * v[idx] - 2.0 * v[idx - S] + 0.5 * v[idx - 2 * S];
}

// One block per pair of time levels (2b, 2b+1).
template <int L>
__global__ void __launch_bounds__(256) k_matvec_1d(const double* __restrict__ v,
                                                   double* __restrict__ y,
                                                   const double* __restrict__ sym,
                                                   const double2* __restrict__ tw, int M, int Nt) {
  __shared__ double2 buf[L];
  const int k0 = 2 * blockIdx.x, k1 = k0 + 1;
  const bool has1 = k1 < Nt;
  const size_t S = (size_t)M;
  for (int i = threadIdx.x; i < L; i += 256) {
    double a = 0.0, b = 0.0;
    if (i < M) {
      a = v[(size_t)k0 * S + i];
      if (has1) b = v[(size_t)k1 * S + i];
    }
    buf[i] = make_double2(a, b);
  }
  __syncthreads();
  fft_lds<L, -1, 256, 1>(buf, tw);
  for (int m = threadIdx.x; m < L; m += 256) {
    const double s = sym[m <= L / 2 ? m : L - m];
    buf[m].x *= s;
    buf[m].y *= s;
  }
  __syncthreads();
  fft_lds<L, +1, 256, 1>(buf, tw);
  for (int i = threadIdx.x; i < M; i += 256) {
    const size_t i0 = (size_t)k0 * S + i;
    y[i0] = time_stencil(v, k0, S, i0) + buf[i].x;
    if (has1) {
      const size_t i1 = i0 + S;
      y[i1] = time_stencil(v, k1, S, i1) + buf[i].y;
    }
  }
}

// 2D, x direction: rows of length Mx (contiguous).  There are Nt*My rows; one block per pair of
// rows.  Writes y = time stencil + (tau c_x T_x along x) v.
template <int L>
__global__ void __launch_bounds__(256) k_matvec_2d_x(const double* __restrict__ v,
                                                     double* __restrict__ y,
                                                     const double* __restrict__ sym,
                                                     const double2* __restrict__ tw, int Mx,
                                                     int My, int Nt) {
  __shared__ double2 buf[L];
  const int rows = Nt * My;
  const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
  const bool has1 = r1 < rows;
  const size_t S = (size_t)Mx * My;
  for (int i = threadIdx.x; i < L; i += 256) {
    double a = 0.0, b = 0.0;
    if (i < Mx) {
      a = v[(size_t)r0 * Mx + i];
      if (has1) b = v[(size_t)r1 * Mx + i];
    }
    buf[i] = make_double2(a, b);
  }
  __syncthreads();
  fft_lds<L, -1, 256, 1>(buf, tw);
  for (int m = threadIdx.x; m < L; m += 256) {
    const double s = sym[m <= L / 2 ? m : L - m];
    buf[m].x *= s;
    buf[m].y *= s;
  }
  __syncthreads();
  fft_lds<L, +1, 256, 1>(buf, tw);
  const int ka = r0 / My, kb = r1 / My;
  for (int i = threadIdx.x; i < Mx; i += 256) {
    const size_t i0 = (size_t)r0 * Mx + i;
    y[i0] = time_stencil(v, ka, S, i0) + buf[i].x;
    if (has1) {
      const size_t i1 = (size_t)r1 * Mx + i;
      y[i1] = time_stencil(v, kb, S, i1) + buf[i].y;
    }
  }
}

// 2D, y direction: for one time level and a tile of 2*NB adjacent columns, NB complex transforms
// of length L along y (column pairs packed as real/imaginary parts).  Adds (tau c_y T_y along y) v
// into y.
template <int L, int NB>
__global__ void __launch_bounds__(256) k_matvec_2d_y(const double* __restrict__ v,
                                                     double* __restrict__ y,
                                                     const double* __restrict__ sym,
                                                     const double2* __restrict__ tw, int Mx,
                                                     int My) {
  __shared__ double2 buf[NB * L];
  constexpr int TS = 2 * NB;
  const int ntile = (Mx + TS - 1) / TS;
  const int k = blockIdx.x / ntile, tile = blockIdx.x % ntile;
  const int x0 = tile * TS;
  const size_t base = (size_t)k * Mx * My;
  // zero-fill, then gather rows of TS contiguous values
  for (int e = threadIdx.x; e < NB * L; e += 256) buf[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int e = threadIdx.x; e < My * TS; e += 256) {
    const int iy = e / TS, q = e % TS, x = x0 + q;
    if (x < Mx) {
      const double val = v[base + (size_t)iy * Mx + x];
      double2* slot = &buf[(q >> 1) * L + iy];
      if (q & 1) slot->y = val; else slot->x = val;
    }
  }
  __syncthreads();
  fft_lds<L, -1, 256, NB>(buf, tw);
  for (int e = threadIdx.x; e < NB * L; e += 256) {
    const int m = e % L;
    const double s = sym[m <= L / 2 ? m : L - m];
    buf[e].x *= s;
    buf[e].y *= s;
  }
  __syncthreads();
  fft_lds<L, +1, 256, NB>(buf, tw);
  for (int e = threadIdx.x; e < My * TS; e += 256) {
    const int iy = e / TS, q = e % TS, x = x0 + q;
    if (x < Mx) {
      const double2 c = buf[(q >> 1) * L + iy];
      y[base + (size_t)iy * Mx + x] += (q & 1) ? c.y : c.x;
    }
  }
}

template <int L>
static int mv1d(const Plan& p, const double* v, double* y) {
  k_matvec_1d<L><<<(p.Nt + 1) / 2, 256, 0, p.stream>>>(v, y, p.sym, p.twL, p.M, p.Nt);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int L>
static int mv2dx(const Plan& p, const double* v, double* y) {
  const int rows = p.Nt * p.My;
  k_matvec_2d_x<L><<<(rows + 1) / 2, 256, 0, p.stream>>>(v, y, p.sym, p.twL, p.Mx, p.My, p.Nt);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int L>
static int mv2dy(const Plan& p, const double* v, double* y) {
  constexpr int NB = (L >= 4096) ? 1 : (L >= 2048 ? 2 : (4096 / L < 8 ? 4096 / L : 8));
  const int ntile = (p.Mx + 2 * NB - 1) / (2 * NB);
  const double* symy = p.sym + (p.Lx / 2 + 1);
  const double2* twy = p.twL + p.Lx;
  k_matvec_2d_y<L, NB><<<p.Nt * ntile, 256, 0, p.stream>>>(v, y, symy, twy, p.Mx, p.My);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

#define RFDE_L_SWITCH(Lval, FN, ...)            \
  switch (Lval) {                               \
    case 16: return FN<16>(__VA_ARGS__);        \
    case 32: return FN<32>(__VA_ARGS__);        \
    case 64: return FN<64>(__VA_ARGS__);        \
    case 128: return FN<128>(__VA_ARGS__);      \
    case 256: return FN<256>(__VA_ARGS__);      \
    case 512: return FN<512>(__VA_ARGS__);      \
    case 1024: return FN<1024>(__VA_ARGS__);    \
    case 2048: return FN<2048>(__VA_ARGS__);    \
    case 4096: return FN<4096>(__VA_ARGS__);    \
    case 8192: return FN<8192>(__VA_ARGS__);    \
    default: return RFDE_EINVAL;                \
  }

static int mv2d(const Plan& p, const double* v, double* y) {
  int rc;
  switch (p.Lx) {
    case 16: rc = mv2dx<16>(p, v, y); break;
    case 32: rc = mv2dx<32>(p, v, y); break;
    case 64: rc = mv2dx<64>(p, v, y); break;
    case 128: rc = mv2dx<128>(p, v, y); break;
    case 256: rc = mv2dx<256>(p, v, y); break;
    case 512: rc = mv2dx<512>(p, v, y); break;
    case 1024: rc = mv2dx<1024>(p, v, y); break;
    case 2048: rc = mv2dx<2048>(p, v, y); break;
    case 4096: rc = mv2dx<4096>(p, v, y); break;
    case 8192: rc = mv2dx<8192>(p, v, y); break;
    default: return RFDE_EINVAL;
  }
  if (rc != RFDE_OK) return rc;
  RFDE_L_SWITCH(p.Ly, mv2dy, p, v, y);
}

int launch_matvec(const Plan& p, const double* v, double* y) {
  if (p.dim == 2) return mv2d(p, v, y);
  RFDE_L_SWITCH(p.L, mv1d, p, v, y);
}

// F_1 = tau f^1 + u0; F_2 = tau f^2 - u0/2; F_k = tau f^k.
__global__ void k_rhs(const double* __restrict__ u0, const double* f, double* F, size_t S,
                      int Nt, double tau) {
  const size_t N = S * Nt;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < N;
       idx += (size_t)gridDim.x * blockDim.x) {
    double val = tau * f[idx];
    if (idx < S) val += u0[idx];
    else if (idx < 2 * S) val -= 0.5 * u0[idx - S];
    F[idx] = val;
  }
}

int launch_rhs(const Plan& p, const double* u0, const double* f, double* F) {
  const size_t N = p.N();
  const int blocks = (int)std::min<size_t>((N + 255) / 256, 8192);
  k_rhs<<<blocks, 256, 0, p.stream>>>(u0, f, F, (size_t)p.S, p.Nt, p.tau);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // namespace rfde
