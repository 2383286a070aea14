// All-at-once matvec y = (C kron I - tau I kron A) v (Section 3.2: vec(V C^T) - tau vec(A V)),
// and the right-hand side F of eq. (2.11).
//
// -tau A = coef T with coef = tau kappa / h^alpha, T symmetric Toeplitz.  T v is the first M
// entries of the symmetric circulant of order L applied to v padded with zeros; that circulant
// is diagonalised by the DFT with the real symbol `sym` (which already carries coef / L).
// Because the symbol is real, one complex transform applies it to two real vectors at once:
// the real part carries one, the imaginary part the other.
//
// The transforms run in LDS with the first pass reading global memory directly, the symbol
// applied as the last forward pass writes, and the BDF2 time stencil fused into the store of
// the last inverse pass, so v is read and y written once per element.
//
// Time stencil (rows of C, eq. (2.12)): level 0: v_0; level 1: 3/2 v_1 - 2 v_0;
// level k >= 2: 3/2 v_k - 2 v_{k-1} + 1/2 v_{k-2}.
#include "buf_io.hpp"
#include "fft3.hpp"
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

template <int L> constexpr int mv_threads() { return L >= 2048 ? 512 : 256; }

// Rows of length n (contiguous): one block per pair of rows (r0, r0+1) of the flattened
// [rows][n] array; row r belongs to time level r / rows_per_level.  Writes
// y = time stencil + (symbol-circulant product) v for both rows.
template <int L, int NT, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_matvec_rows(const double* __restrict__ v,
                                                    double* __restrict__ y,
                                                    const double* __restrict__ sym,
                                                    const double2* __restrict__ tw, int n,
                                                    int rows, int rows_per_level, size_t S,
                                                    const int* __restrict__ live) {
  if (live && *live == 0) return;
  __shared__ double2 buf[L];
  const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
  const bool has1 = r1 < rows;
  const double* v0 = v + (size_t)r0 * n;
  const double* v1 = v + (size_t)r1 * n;
  auto load = [&](int, int idx) -> double2 {
    double a = 0.0, b = 0.0;
    if (idx < n) {
      a = v0[idx];
      if (has1) b = v1[idx];
    }
    return make_double2(a, b);
  };
  auto store_scaled = [&](int, int idx, double2 x) {
    const double s = sym[idx <= L / 2 ? idx : L - idx];
    buf[idx] = make_double2(x.x * s, x.y * s);
  };
  fft_io<L, -1, NT, 1, L, false, true, true, MAXR>(buf, tw, load, store_scaled);
  __syncthreads();
  const int ka = r0 / rows_per_level, kb = r1 / rows_per_level;
  auto store_out = [&](int, int idx, double2 x) {
    if (idx < n) {
      const size_t i0 = (size_t)r0 * n + idx;
      y[i0] = time_stencil(v, ka, S, i0) + x.x;
      if (has1) {
        const size_t i1 = (size_t)r1 * n + idx;
        y[i1] = time_stencil(v, kb, S, i1) + x.y;
      }
    }
  };
  NoLoad nl;
  fft_io<L, +1, NT, 1, L, false, false, true, MAXR>(buf, tw, nl, store_out);
}

// Same product for L >= 256 on the three-stage register FFT: NB row pairs per workgroup, the
// forward transform, the symbol and the inverse transform in registers with four LDS exchanges.
// Only inputs below n (<= L/2) are non-zero and only outputs below n are kept, so the first
// stage's upper half of inputs and the last stage's upper half of outputs are pruned at
// compile time.  Rows are addressed through buffer descriptors whose range is the row (or
// empty for a row past the end or a level before the first), so the hardware range check
// replaces every bounds test: loads outside read zero and stores outside are dropped.
// A pair is the same spatial row (index y within a level of rows_per_level rows) at two
// consecutive levels 2kp and 2kp + 1, pair q = y K2 + kp with K2 = ceil(N_t / 2): the BDF2
// stencil of the pair then needs only the rows of levels 2kp - 1 and 2kp - 2, which are the
// rows of the previous pair, read moments before by the same workgroup (NB consecutive pairs)
// or by its neighbour in the same XCD (pairs are dealt so that each XCD takes a contiguous
// range).
template <int L, int WAVES>
__global__ void __launch_bounds__(256, WAVES)
    k_matvec3(const double* __restrict__ v, double* __restrict__ y,
              const double* __restrict__ sym, const double2* __restrict__ tw, int n, int rows,
              int rows_per_level, const int* __restrict__ live) {
  using E = Fft3For<L, 256>;
  if (live && *live == 0) return;
  __shared__ double lds[E::LDS];
  const int pair0 = xcd_remap(blockIdx.x, gridDim.x) * E::NB;
  const int nbytes = n * 8;
  const int rpl = rows_per_level;
  const int K2 = (rows / rpl + 1) / 2;
  const int npairs = rpl * K2;
  // row r of v (or y) as a buffer; empty when r is outside [0, rows)
  auto row = [&](const double* base, int r) {
    const bool ok = r >= 0 && r < rows;
    return make_rsrc(base + (ok ? (size_t)r * n : 0), ok ? nbytes : 0);
  };
  // Per stage-1 butterfly of this thread (one row pair each): the rows it reads and writes and
  // the BDF2 rows of C (eq. (2.12)): level 0: v_0; level k >= 1: 3/2 v_k - 2 v_{k-1} + 1/2
  // v_{k-2} (missing levels read zero through empty descriptors).
  struct Rows {
    __amdgpu_buffer_rsrc_t a, b, a1, a2, ya, yb;
    double ca;
  };
  Rows rs[E::B1];
#pragma unroll
  for (int b = 0; b < E::B1; ++b) {
    const int q = pair0 + E::f_of_b1(b);
    // past the last pair: every row (and its stencil rows) lies before the first
    const int r0 = q < npairs ? 2 * (q % K2) * rpl + q / K2 : -3 * rpl - 1;
    const int r1 = r0 + rpl;
    rs[b].a = row(v, r0);
    rs[b].b = row(v, r1);
    rs[b].a1 = row(v, r0 - rpl);
    rs[b].a2 = row(v, r0 - 2 * rpl);
    rs[b].ya = row(y, r0);
    rs[b].yb = row(y, r1);
    rs[b].ca = r0 < rpl ? 1.0 : 1.5;
  }
  auto load = [&](int b, int, int idx, int n1) -> double2 {
    if (n1 >= E::N1 / 2) return make_double2(0.0, 0.0);
    return make_double2(buf_load(rs[b].a, idx), buf_load(rs[b].b, idx));
  };
  auto pw = [&](int, int k, double2& c) {
    const double s = sym[k <= L / 2 ? k : L - k];
    c.x *= s;
    c.y *= s;
  };
  auto store = [&](int b, int, int idx, int n1, double2 c) {
    if (n1 >= E::N1 / 2) return;
    const Rows& r = rs[b];
    const double va = buf_load(r.a, idx), va1 = buf_load(r.a1, idx);
    const double s0 = r.ca * va - 2.0 * va1 + 0.5 * buf_load(r.a2, idx);
    const double s1 = 1.5 * buf_load(r.b, idx) - 2.0 * va + 0.5 * va1;
    buf_store(r.ya, idx, s0 + c.x);
    buf_store(r.yb, idx, s1 + c.y);
  };
  E::run(lds, tw, load, pw, store);
}

// 2D, y direction: for one time level and a tile of 2*NB adjacent columns, NB complex transforms
// of length L along y (column pairs packed as real/imaginary parts, batch index fastest so the
// row segments are read and written contiguously).  Adds (tau c_y T_y along y) v into y.
template <int L, int NB, int NT, int MAXR = 16>
__global__ void __launch_bounds__(NT) k_matvec_2d_y(const double* __restrict__ v,
                                                    double* __restrict__ y,
                                                    const double* __restrict__ sym,
                                                    const double2* __restrict__ tw, int Mx,
                                                    int My) {
  constexpr int LDN = L + 1;
  __shared__ double2 buf[NB * LDN];
  constexpr int TS = 2 * NB;
  const int ntile = (Mx + TS - 1) / TS;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);  // neighbouring tiles share cache lines
  const int k = bid / ntile, tile = bid % ntile;
  const int x0 = tile * TS;
  const size_t base = (size_t)k * Mx * My;
  auto load = [&](int f, int iy) -> double2 {
    double a = 0.0, b = 0.0;
    const int x = x0 + 2 * f;
    if (iy < My) {
      const double* row = v + base + (size_t)iy * Mx;
      if (x < Mx) a = row[x];
      if (x + 1 < Mx) b = row[x + 1];
    }
    return make_double2(a, b);
  };
  auto store_scaled = [&](int f, int idx, double2 c) {
    const double s = sym[idx <= L / 2 ? idx : L - idx];
    buf[f * LDN + idx] = make_double2(c.x * s, c.y * s);
  };
  fft_io<L, -1, NT, NB, LDN, true, true, true, MAXR>(buf, tw, load, store_scaled);
  __syncthreads();
  auto store_out = [&](int f, int iy, double2 c) {
    const int x = x0 + 2 * f;
    if (iy < My) {
      double* row = y + base + (size_t)iy * Mx;
      if (x < Mx) row[x] += c.x;
      if (x + 1 < Mx) row[x + 1] += c.y;
    }
  };
  NoLoad nl;
  fft_io<L, +1, NT, NB, LDN, true, false, true, MAXR>(buf, tw, nl, store_out);
}

// Variants: 0 = three-stage register FFT (L >= 256; smaller L: the Stockham kernel);
// 1 = Stockham passes with the default workgroup size and radix 16; 2 = the other workgroup size
// (256 <-> 512); 3 = radix-8 passes (1024 threads for L >= 8192).
template <int L>
static int mv_rows(const Plan& p, const double* v, double* y, int n, int rows, int rpl,
                   const int* live) {
  using E = Fft3For<L, 256>;
  // L = 8192 needs more than 256 registers per lane at one wave per SIMD; bounding it to two
  // waves costs a few spills but hides latency better (measured 35 vs 44 us at M = 4095).
  // L <= 512 fits four waves (128 registers) without spills.
  constexpr int WAVES = L >= 8192 ? 2 : (L <= 512 ? 4 : 1);
  const int npairs = rpl * ((rows / rpl + 1) / 2);
  const int groups = (npairs + E::NB - 1) / E::NB;
  k_matvec3<L, WAVES><<<groups, 256, 0, p.stream>>>(v, y, p.sym, p.twL, n, rows, rpl, live);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}
template <int L, int V>
static int mv1d_v(const Plan& p, const double* v, double* y) {
  if constexpr (V == 0 && L >= 256) {
    return mv_rows<L>(p, v, y, p.M, p.Nt, 1, p.live);
  } else {
    constexpr int NT0 = mv_threads<L>();
    constexpr int NT = V == 2 ? (NT0 == 512 ? 256 : 512) : (V == 3 && L >= 8192 ? 1024 : NT0);
    constexpr int MAXR = V == 3 ? 8 : 16;
    k_matvec_rows<L, NT, MAXR><<<(p.Nt + 1) / 2, NT, 0, p.stream>>>(v, y, p.sym, p.twL, p.M, p.Nt,
                                                                    1, (size_t)p.M, p.live);
    RFDE_HIP(hipGetLastError());
    return RFDE_OK;
  }
}
template <int L>
static int mv1d(const Plan& p, const double* v, double* y) {
  if (p.tv_matvec == 1) return mv1d_v<L, 1>(p, v, y);
  if (p.tv_matvec == 2) return mv1d_v<L, 2>(p, v, y);
  if (p.tv_matvec == 3) return mv1d_v<L, 3>(p, v, y);
  return mv1d_v<L, 0>(p, v, y);
}
template <int L>
static int mv2dx(const Plan& p, const double* v, double* y) {
  const int rows = p.Nt * p.My;
  if constexpr (L >= 256) {
    return mv_rows<L>(p, v, y, p.Mx, rows, p.My, nullptr);
  } else {
    constexpr int NT = mv_threads<L>();
    k_matvec_rows<L, NT><<<(rows + 1) / 2, NT, 0, p.stream>>>(v, y, p.sym, p.twL, p.Mx, rows,
                                                              p.My, (size_t)p.Mx * p.My, nullptr);
    RFDE_HIP(hipGetLastError());
    return RFDE_OK;
  }
}
template <int L>
static int mv2dy(const Plan& p, const double* v, double* y) {
  // tile of 2*NB columns: 128-byte row segments where the LDS budget (~130 KB) allows
  constexpr int NB = (8 * (L + 1) * 16 <= 135168) ? 8 : ((4 * (L + 1) * 16 <= 135168) ? 4 : ((2 * (L + 1) * 16 <= 135168) ? 2 : 1));
  // radix 8 up to L = 512 (twice the threads per LDS byte: more waves to hide latency)
  constexpr int MAXR = L <= 512 ? 8 : 16;
  constexpr int NT = (NB * L / MAXR < 64) ? 64 : (NB * L / MAXR > 512 ? 512 : NB * L / MAXR);
  const int ntile = (p.Mx + 2 * NB - 1) / (2 * NB);
  const double* symy = p.sym + (p.Lx / 2 + 1);
  const double2* twy = p.twL + p.Lx;
  k_matvec_2d_y<L, NB, NT, MAXR><<<p.Nt * ntile, NT, 0, p.stream>>>(v, y, symy, twy, p.Mx, p.My);
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

static int mv2dx_dispatch(const Plan& p, const double* v, double* y) {
  RFDE_L_SWITCH(p.Lx, mv2dx, p, v, y);
}

int launch_matvec(const Plan& p, const double* v, double* y) {
  if (p.dim == 2) {
    const int rc = mv2dx_dispatch(p, v, y);
    if (rc != RFDE_OK) return rc;
    RFDE_L_SWITCH(p.Ly, mv2dy, p, v, y);
  }
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
