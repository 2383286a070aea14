// Setup kernels: weights g_k (eq. (2.4)), FFT twiddle tables, the circulant-embedding symbol of
// the Toeplitz block (Section 2.1: T_x is symmetric Toeplitz and is applied by FFT), the
// time-circulant data s_j and lambda_n (eq. (3.3)), and tau-approximation eigenvalues (eq. (3.10)).
#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

// g_{k+1} = g_k (k - a/2) / (k + 1 + a/2), g_0 = Gamma(1+a) / Gamma(1+a/2)^2.  One block: each
// thread owns a contiguous chunk; the chunk products are prefix-multiplied, then each thread
// walks its chunk.
__global__ void __launch_bounds__(256) k_gk(double a, int n, double* __restrict__ g) {
  __shared__ double part[256];
  const int t = threadIdx.x;
  const int chunk = (n + 255) / 256;
  const int k0 = min(n, t * chunk), k1 = min(n, k0 + chunk);
  const double h = 0.5 * a;
  double p = 1.0;
  for (int k = k0; k < k1; ++k) p *= (k - h) / (k + 1.0 + h);
  part[t] = p;
  __syncthreads();
  if (t == 0) {
    double acc = 1.0;
    for (int i = 0; i < 256; ++i) { const double q = part[i]; part[i] = acc; acc *= q; }
  }
  __syncthreads();
  const double g0 = tgamma(1.0 + a) / (tgamma(1.0 + h) * tgamma(1.0 + h));
  double gj = g0 * part[t];
  for (int j = k0; j < k1; ++j) { g[j] = gj; gj *= (j - h) / (j + 1.0 + h); }
}

int launch_gk(double alpha, int n, double* g, hipStream_t st) {
  k_gk<<<1, 256, 0, st>>>(alpha, n, g);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// tw[m] = exp(-2 pi i m / n)
__global__ void k_twiddles(double2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    double s, c;
    sincospi(-2.0 * m / n, &s, &c);
    tw[m] = make_double2(c, s);
  }
}
__global__ void k_twiddles32(float2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    double s, c;
    sincospi(-2.0 * m / n, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
  }
}
int launch_twiddles(double2* tw, int n, hipStream_t st) {
  k_twiddles<<<(n + 255) / 256, 256, 0, st>>>(tw, n);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
int launch_twiddles32(float2* tw, int n, hipStream_t st) {
  k_twiddles32<<<(n + 255) / 256, 256, 0, st>>>(tw, n);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// Symbol of the symmetric circulant of order L whose first column is
// (g_0, g_1, ..., g_{M-1}, 0, ..., 0, g_{M-1}, ..., g_1) (L >= 2M - 1): its eigenvalues are the
// DFT of that column, real because the column is even.  Stored for m = 0..L/2 times `scale`.
template <int L>
__global__ void __launch_bounds__(256) k_symbol(const double* __restrict__ g, int M, double scale,
                                                const double2* __restrict__ tw,
                                                double* __restrict__ sym) {
  __shared__ double2 buf[L];
  for (int m = threadIdx.x; m < L; m += 256) {
    double c = 0.0;
    if (m < M) c = g[m];
    else if (m > L - M) c = g[L - m];
    buf[m] = make_double2(c, 0.0);
  }
  __syncthreads();
  fft_lds<L, -1, 256, 1>(buf, tw);
  for (int m = threadIdx.x; m <= L / 2; m += 256) sym[m] = buf[m].x * scale;
}

template <int L>
static int symbol_for(const double* g, int M, double scale, const double2* tw, double* sym,
                      hipStream_t st) {
  k_symbol<L><<<1, 256, 0, st>>>(g, M, scale, tw, sym);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int launch_symbol(const double* g, int M, int L, double scale, const double2* tw, double* sym,
                  hipStream_t st) {
  switch (L) {
    case 16: return symbol_for<16>(g, M, scale, tw, sym, st);
    case 32: return symbol_for<32>(g, M, scale, tw, sym, st);
    case 64: return symbol_for<64>(g, M, scale, tw, sym, st);
    case 128: return symbol_for<128>(g, M, scale, tw, sym, st);
    case 256: return symbol_for<256>(g, M, scale, tw, sym, st);
    case 512: return symbol_for<512>(g, M, scale, tw, sym, st);
    case 1024: return symbol_for<1024>(g, M, scale, tw, sym, st);
    case 2048: return symbol_for<2048>(g, M, scale, tw, sym, st);
    case 4096: return symbol_for<4096>(g, M, scale, tw, sym, st);
    case 8192: return symbol_for<8192>(g, M, scale, tw, sym, st);
    default: return RFDE_EINVAL;
  }
}

// s_j = eps^{j/Nt} = exp((j/Nt) ln eps), each power evaluated on its own.
// lambda_n = 3/2 - 2 eps^{1/Nt} theta^n + 1/2 eps^{2/Nt} theta^{2n}, theta = exp(2 pi i / Nt).
__global__ void k_time_data(int Nt, double eps, double* __restrict__ s,
                            double2* __restrict__ lam) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const double le = log(eps);
  if (j < Nt) s[j] = exp(((double)j / Nt) * le);
  if (j <= Nt / 2) {
    const double x1 = exp(le / Nt), x2 = exp(2.0 * le / Nt);
    double s1, c1, s2, c2;
    sincospi(2.0 * (double)(j % Nt) / Nt, &s1, &c1);
    sincospi(2.0 * (double)((2 * j) % Nt) / Nt, &s2, &c2);
    lam[j] = make_double2(1.5 - 2.0 * x1 * c1 + 0.5 * x2 * c2, -2.0 * x1 * s1 + 0.5 * x2 * s2);
  }
}

int launch_time_data(int Nt, double eps, double* s, double2* lambda, hipStream_t st) {
  k_time_data<<<(Nt + 255) / 256, 256, 0, st>>>(Nt, eps, s, lambda);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

// Eigenvalues of the natural tau approximation of the symmetric Toeplitz matrix with first
// column g_0..g_{n-1}: chat_k = g_k - g_{k+2} (k <= n-3), chat_{n-2} = g_{n-2}, chat_{n-1} = g_{n-1};
// sigma_i = sum_{j=1}^{n} chat_{j-1} sin(pi i j/(n+1)) / sin(pi i/(n+1)), i = 1..n (eq. (3.10)).
// One workgroup per i; the sines come from the twiddle table of length P = 2(n+1)
// (tw[m] = exp(-2 pi i m / P), so sin(pi i j / (n+1)) = -Im tw[(i j) mod P]) and the partial
// sums are combined in a fixed order (the result does not depend on scheduling).
__global__ void __launch_bounds__(256) k_tau_sigma(const double* __restrict__ g, int n,
                                                   const double2* __restrict__ tw,
                                                   double* __restrict__ sigma) {
  __shared__ double part[256];
  const int i = blockIdx.x + 1;
  const int P = 2 * (n + 1);
  const int step = (int)((256LL * i) % P);
  int m = (int)((long long)i * (threadIdx.x + 1) % P);
  double acc = 0.0;
  for (int j = threadIdx.x + 1; j <= n; j += 256) {
    const int k = j - 1;
    const double c = (k <= n - 3) ? g[k] - g[k + 2] : g[k];
    acc += c * -tw[m].y;
    m += step;
    if (m >= P) m -= P;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[i - 1] = part[0] / -tw[i].y;
}

int launch_tau_sigma(const double* g, int n, const double2* tw, double* sigma, hipStream_t st) {
  k_tau_sigma<<<n, 256, 0, st>>>(g, n, tw, sigma);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // namespace rfde
