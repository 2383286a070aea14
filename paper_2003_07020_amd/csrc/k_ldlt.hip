// Preconditioner step (b), exact 1D variant: factor the floor(Nt/2)+1 shifted blocks
//     B_n = lambda_n I + coef T,   coef = tau kappa / h^alpha,  T[r][c] = g_|r-c|   (eq. (3.5))
// once, then solve B_n z2_n = z1_n for every n in each preconditioner application.
//
// B_n is complex symmetric (B_n^T = B_n) and its Hermitian part Re(lambda_n) I + coef T is
// positive definite (Re lambda_n >= 0 by Proposition 3.1, T SPD), so every leading principal
// submatrix is nonsingular and Gaussian elimination needs no pivoting.  For a symmetric matrix
// that elimination gives U = D L^T, so only B_n = L D L^T (L unit lower, D diagonal) is kept:
// the factor memory and flops are half those of a general LU.
//
// Storage: the order is padded to Mp = 64 T (padding rows/columns are identity rows/columns).
// Per block n, the lower-triangular 64x64 tiles (i, j), i >= j, are stored one after another
// (tile index i(i+1)/2 + j), each tile column-major (entry (r, c) at c*64 + r).
//   off-diagonal tile (i, j):  L_ij
//   diagonal tile (j, j):      strict lower part: inverse of the unit-lower diagonal block L_jj;
//                              diagonal: d (the entries of D); strict upper part: L_jj transposed.
//
// Factorisation: left-looking (Crout) over tile columns j = 0..T-1.  Two launches per column:
//   k_ldlt_diag:  unblocked LDL^T in LDS of the pending diagonal tile and the inverse of its
//                 unit-lower factor;
//   k_ldlt_panel: for i > j, S = B_ij - sum_{k<j} (L_ik D_k) L_jk^T (MFMA), then
//                 L_ij = S L_jj^{-T} D_j^{-1} (a second MFMA product with the stored inverse),
//                 then the pending diagonal tile (i, i) -= (L_ij D_j) L_ij^T (a third), so the
//                 diagonal launches, which have only one workgroup per block, do no GEMM work.
// B_ij is generated from g, coef and lambda_n in the accumulator initialisation, so the
// assembled matrices are never stored.
//
// Real blocks: for an even N_t, lambda_0 and lambda_{N_t/2} are real, so B_0 and B_{N_t/2} are
// real symmetric (positive definite).  Their factors share one storage block (the "dual" block,
// stored first): the .x components hold B_0's factor and the .y components B_{N_t/2}'s, with
// componentwise arithmetic.  A plan then has N_t/2 storage blocks instead of N_t/2 + 1, each of
// the same size, which divides evenly over the workgroup slots of the GPU (513 blocks of work on
// 512 slots left one block running alone at the end of every launch).
#include <algorithm>
#include <type_traits>

#include "fft_lds.hpp"
#include "rfde_internal.hpp"

namespace rfde {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename C> struct mma;
template <> struct mma<double2> {
  using R = double;
  using V = d4_t;
  __device__ static __forceinline__ V fma(R a, R b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row (within the 16x16 block) of accumulator element e held by lane l
  __device__ static __forceinline__ int row(int l, int e) { return (l >> 4) + 4 * e; }
};
template <> struct mma<float2> {
  using R = float;
  using V = f4_t;
  __device__ static __forceinline__ V fma(R a, R b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
};

constexpr int LDSLD = 65;  // padded leading dimension of 64x64 tiles staged in LDS

// Entry (R, Cc) of B_n, padded with identity beyond M.  D (dual block): lam = (lambda_0,
// lambda_{N_t/2}) and the entry is (B_0[R][Cc], B_{N_t/2}[R][Cc]).
template <bool D>
__device__ __forceinline__ double2 shifted_entry(const double* __restrict__ g, double coef,
                                                 double2 lam, int M, int R, int Cc) {
  if (R >= M || Cc >= M) {
    const double e = R == Cc ? 1.0 : 0.0;
    return make_double2(e, D ? e : 0.0);
  }
  const int d = R > Cc ? R - Cc : Cc - R;
  const double t = coef * g[d];
  if constexpr (D) return make_double2(t + (d == 0 ? lam.x : 0.0), t + (d == 0 ? lam.y : 0.0));
  return make_double2(t + (d == 0 ? lam.x : 0.0), d == 0 ? lam.y : 0.0);
}

// Products and inverses in the arithmetic of a block: complex, or componentwise (dual block).
template <bool D, typename C> __device__ __forceinline__ C xmul(C a, C b) {
  if constexpr (D) return cmk<C>(a.x * b.x, a.y * b.y);
  else return cmul(a, b);
}
template <bool D, typename C> __device__ __forceinline__ C xinv(C d) {
  using R = typename cplx_traits<C>::real;
  if constexpr (D) {
    return cmk<C>((R)1 / d.x, (R)1 / d.y);
  } else {
    const R den = d.x * d.x + d.y * d.y;
    return cmk<C>(d.x / den, -d.y / den);
  }
}

// lambda of storage block n of family fm (the dual block 0 takes lambda_0 and lambda_{N_t/2}).
template <bool D>
__device__ __forceinline__ double2 block_lambda(const BlockSet* __restrict__ set, int fm, int n) {
  if constexpr (D) return make_double2(set->lambda[fm][0].x, set->lambda[fm][set->nfreq[fm] - 1].x);
  else return set->lambda[fm][n];
}

// Family slot k of an item map holding `item` (binary search over the start offsets).
__device__ __forceinline__ int find_slot(const ItemMap& m, int item) {
  int lo = 0, hi = m.cnt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (m.start[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Accumulators of one wave: 2x2 blocks of 16x16, real and imaginary parts.
template <typename C> struct WaveAcc {
  typename mma<C>::V re[2][2], im[2][2];
};

// The long K loop of the tile update forms complex products with three real products instead
// of four (the 3M method): for x = a b with a = ar + i ai, b = br + i bi,
//   p1 = ar br,  p2 = ai bi,  p3 = (ar + ai)(br + bi),  Re x = p1 - p2,  Im x = p3 - p1 - p2,
// accumulated separately over K.  The initial value B_ij enters as p1 = Re B, p2 = 0,
// p3 = Re B + Im B.  Rounding stays normwise at the unit roundoff times the operand norms.
template <typename C> struct WaveAcc3 {
  typename mma<C>::V p1[2][2], p2[2][2], p3[2][2];
};

// Dual blocks need two real products per entry: p1 accumulates the .x (B_0) part and p2 the
// .y (B_{N_t/2}) part; p3 is unused.
template <typename C, bool D>
__device__ __forceinline__ void acc3_init(WaveAcc3<C>& a, int i, int j,
                                          const double* __restrict__ g, double coef, double2 lam,
                                          int M) {
  using R = typename mma<C>::R;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1, l16 = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr * 32 + bi * 16 + mma<C>::row(lane, e);
        const int c = wc * 32 + bj * 16 + l16;
        const double2 b = shifted_entry<D>(g, coef, lam, M, i * TILE + r, j * TILE + c);
        a.p1[bi][bj][e] = (R)b.x;
        if constexpr (D) {
          a.p2[bi][bj][e] = (R)b.y;
        } else {
          a.p2[bi][bj][e] = (R)0;
          a.p3[bi][bj][e] = (R)(b.x + b.y);
        }
      }
}

template <typename C>
__device__ __forceinline__ void acc3_zero(WaveAcc3<C>& a) {
  using R = typename mma<C>::R;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a.p1[bi][bj][e] = (R)0;
        a.p2[bi][bj][e] = (R)0;
        a.p3[bi][bj][e] = (R)0;
      }
}

template <typename C, bool D>
__device__ __forceinline__ void acc3_finish(const WaveAcc3<C>& a, WaveAcc<C>& acc) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      if constexpr (D) {
        acc.re[bi][bj] = a.p1[bi][bj];
        acc.im[bi][bj] = a.p2[bi][bj];
      } else {
        acc.re[bi][bj] = a.p1[bi][bj] - a.p2[bi][bj];
        acc.im[bi][bj] = a.p3[bi][bj] - a.p1[bi][bj] - a.p2[bi][bj];
      }
    }
}

// One K step of 4: A entries na (the -(L_ik d_k) values) for the wave's two row blocks, B
// entries b (L_jk) for its two column blocks.
template <typename C, bool D>
__device__ __forceinline__ void acc3_step(WaveAcc3<C>& a, const typename mma<C>::R (&nar)[2],
                                          const typename mma<C>::R (&nai)[2],
                                          const typename mma<C>::R (&br)[2],
                                          const typename mma<C>::R (&bim)[2]) {
  using R = typename mma<C>::R;
  if constexpr (D) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        a.p1[bi][bj] = mma<C>::fma(nar[bi], br[bj], a.p1[bi][bj]);
        a.p2[bi][bj] = mma<C>::fma(nai[bi], bim[bj], a.p2[bi][bj]);
      }
    return;
  }
  R sa[2], sb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    sa[q] = nar[q] + nai[q];
    sb[q] = br[q] + bim[q];
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      a.p1[bi][bj] = mma<C>::fma(nar[bi], br[bj], a.p1[bi][bj]);
      a.p2[bi][bj] = mma<C>::fma(nai[bi], bim[bj], a.p2[bi][bj]);
      a.p3[bi][bj] = mma<C>::fma(sa[bi], sb[bj], a.p3[bi][bj]);
    }
}

// acc = B_ij - sum_{k<j} (L_ik D_k) L_jk^T for the 64x64 tile (i, j) of block n, operands
// staged through LDS (used for FP32).  The K dimension (j tiles of 64 columns) is walked in chunks of KC = 16 columns.  A chunk of
// L_ik, of L_jk (16 contiguous tile columns each, column-major tiles) and the 16 matching d_k
// are copied by the whole workgroup into one of two LDS buffers while the four waves run the
// MFMAs of the previous chunk from the other buffer, so every operand byte crosses the
// global-memory path once per workgroup instead of once per wave.
constexpr int KC = 16;
template <typename C> struct StageBuf {
  C A[2][KC * TILE];
  C B[2][KC * TILE];
  C D[2][KC];
};

template <typename C, bool D>
__device__ __forceinline__ void tile_update_staged(WaveAcc<C>& acc, const C* __restrict__ fac,
                                                   int i, int j, const double* __restrict__ g,
                                                   double coef, double2 lam, int M,
                                                   StageBuf<C>& sb) {
  using R = typename mma<C>::R;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  WaveAcc3<C> a3;
  acc3_init<C, D>(a3, i, j, g, coef, lam, M);
  const int nchunk = j * (TILE / KC);
  if (nchunk == 0) {
    acc3_finish<C, D>(a3, acc);
    return;
  }
  // per thread: PER entries of each operand chunk (KC*64 = PER x 256) and one d
  constexpr int PER = KC * TILE / 256;
  static_assert(PER * 256 == KC * TILE && KC <= 256 && KC % 4 == 0, "chunk shape");
  const C* Arow = fac + tile_index(i, 0) * TILE_ELEMS;
  const C* Brow = fac + tile_index(j, 0) * TILE_ELEMS;
  C ra[PER], rb[PER], rd;
  auto gload = [&](int c) {
    const int k = c / (TILE / KC), c0 = (c % (TILE / KC)) * KC;
    const size_t off = (size_t)k * TILE_ELEMS + (size_t)c0 * TILE;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      ra[u] = Arow[off + tid + 256 * u];
      rb[u] = Brow[off + tid + 256 * u];
    }
    if (tid < KC) rd = fac[tile_index(k, k) * TILE_ELEMS + (size_t)(c0 + tid) * (TILE + 1)];
  };
  auto lstore = [&](int bsel) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      sb.A[bsel][tid + 256 * u] = ra[u];
      sb.B[bsel][tid + 256 * u] = rb[u];
    }
    if (tid < KC) sb.D[bsel][tid] = rd;
  };
  gload(0);
  lstore(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int cur = c & 1;
    if (c + 1 < nchunk) gload(c + 1);
#pragma unroll
    for (int q = 0; q < KC / 4; ++q) {
      const int kk = 4 * q + lq;
      const C d = sb.D[cur][kk];
      R nar[2], nai[2], br[2], bim[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const C a = sb.A[cur][kk * TILE + wr * 32 + bi * 16 + l16];
        // na = -(a d)
        if constexpr (D) {
          nar[bi] = -(a.x * d.x);
          nai[bi] = -(a.y * d.y);
        } else {
          nar[bi] = -(a.x * d.x - a.y * d.y);
          nai[bi] = -(a.x * d.y + a.y * d.x);
        }
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const C b = sb.B[cur][kk * TILE + wc * 32 + bj * 16 + l16];
        br[bj] = b.x;
        bim[bj] = b.y;
      }
      acc3_step<C, D>(a3, nar, nai, br, bim);
    }
    if (c + 1 < nchunk) lstore(cur ^ 1);
    __syncthreads();
  }
  acc3_finish<C, D>(a3, acc);
}

// acc = B_ij - sum_{k<j} (L_ik D_k) L_jk^T, operands read by each wave straight from global
// memory in the MFMA lane layout (used for FP64, whose MFMAs are slow enough to hide the loads).
template <typename C, bool D>
__device__ __forceinline__ void tile_update_direct(WaveAcc<C>& acc, const C* __restrict__ fac, int i,
                                            int j, const double* __restrict__ g, double coef,
                                            double2 lam, int M) {
  using R = typename mma<C>::R;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int l16 = lane & 15, lq = lane >> 4;
  WaveAcc3<C> a3;
  acc3_init<C, D>(a3, i, j, g, coef, lam, M);
  for (int k = 0; k < j; ++k) {
    const C* Lik = fac + tile_index(i, k) * TILE_ELEMS;
    const C* Ljk = fac + tile_index(j, k) * TILE_ELEMS;
    const C* Dk = fac + tile_index(k, k) * TILE_ELEMS;
#pragma unroll 2
    for (int q = 0; q < 16; ++q) {
      const int kk = 4 * q + lq;
      const C d = Dk[kk * (TILE + 1)];
      R nar[2], nai[2], br[2], bim[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const C a = Lik[kk * TILE + wr * 32 + bi * 16 + l16];
        // na = -(a d)
        if constexpr (D) {
          nar[bi] = -(a.x * d.x);
          nai[bi] = -(a.y * d.y);
        } else {
          nar[bi] = -(a.x * d.x - a.y * d.y);
          nai[bi] = -(a.x * d.y + a.y * d.x);
        }
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const C b = Ljk[kk * TILE + wc * 32 + bj * 16 + l16];
        br[bj] = b.x;
        bim[bj] = b.y;
      }
      acc3_step<C, D>(a3, nar, nai, br, bim);
    }
  }
  acc3_finish<C, D>(a3, acc);
}

// Write the wave accumulators into an LDS tile (column-major, leading dimension LDSLD).
template <typename C>
__device__ __forceinline__ void acc_to_lds(const WaveAcc<C>& acc, C* __restrict__ S) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1, l16 = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr * 32 + bi * 16 + mma<C>::row(lane, e);
        const int c = wc * 32 + bj * 16 + l16;
        S[c * LDSLD + r] = cmk<C>(acc.re[bi][bj][e], acc.im[bi][bj][e]);
      }
}

// Diagonal tile of column j.  Its pending value S = B_jj - sum_{k<j} (L_jk D_k) L_jk^T has been
// accumulated in the tile's own slot by the panel launches of columns 0..j-1 (j = 0: B_00 is
// generated here).  Unblocked LDL^T of S in LDS, then the inverse of the unit-lower factor by
// forward substitution, kept in the (free) upper triangle of the same LDS tile: thread c writes
// column c of L^{-1} transposed, S[r*LD + c] = Linv[r][c] for r > c.  The stored tile (entry
// (rr, cc) at cc*64 + rr) is then exactly S read transposed: Linv below the diagonal, d on it,
// L transposed above it.
// Items: the blocks n of every family with more than j tile columns.
template <typename C, bool P>
__global__ void __launch_bounds__(256) k_ldlt_diag(const BlockSet* __restrict__ set, ItemMap map,
                                                   int j) {
  using R = typename mma<C>::R;
  __shared__ C S[TILE * LDSLD];
  auto body = [&](int slot, int fm, int n, auto dtag) {
  constexpr bool D = decltype(dtag)::value;
  const int M = set->M[fm];
  const double* __restrict__ g = set->g[fm];
  const double coef = set->coef[fm];
  C* fac = (C*)map.fac[slot] + (size_t)n * lower_tiles(set->T[fm]) * TILE_ELEMS;
  C* Djj = fac + tile_index(j, j) * TILE_ELEMS;
  const int t = threadIdx.x;
  if (j == 0) {
    const double2 lam = block_lambda<D>(set, fm, n);
    for (int e = t; e < TILE_ELEMS; e += 256) {
      const int c = e >> 6, r = e & 63;
      const double2 b = shifted_entry<D>(g, coef, lam, M, r, c);
      S[c * LDSLD + r] = cmk<C>((R)b.x, (R)b.y);
    }
  } else {
    for (int e = t; e < TILE_ELEMS; e += 256) S[(e >> 6) * LDSLD + (e & 63)] = Djj[e];
  }
  __syncthreads();
  const int r = t & 63, cg = t >> 6;
  // column p: d = S[p][p]; S[r][c] -= S[r][p] S[c][p] / d for r >= c > p; S[r][p] /= d, r > p.
  for (int p = 0; p < TILE; ++p) {
    const C dinv = xinv<D>(S[p * LDSLD + p]);
    if (r > p) {
      const C ur = S[p * LDSLD + r];
      const C lr = xmul<D>(ur, dinv);
      for (int c = p + 1 + cg; c <= r; c += 4) {
        const C uc = S[p * LDSLD + c];
        S[c * LDSLD + r] = csub(S[c * LDSLD + r], xmul<D>(lr, uc));
      }
    }
    __syncthreads();
    if (cg == 0 && r > p) S[p * LDSLD + r] = xmul<D>(S[p * LDSLD + r], dinv);
    __syncthreads();
  }
  // x = L^{-1} e_c: x_c = 1, x_rr = -(L[rr][c] + sum_{c<m<rr} L[rr][m] x_m); L[rr][m] lives at
  // S[m*LD + rr] (lower), x_m at S[m*LD + c] (upper, written earlier by this thread).
  if (t < TILE) {
    const int c = t;
    for (int rr = c + 1; rr < TILE; ++rr) {
      C s = S[c * LDSLD + rr];
      for (int m = c + 1; m < rr; ++m) s = cadd(s, xmul<D>(S[m * LDSLD + rr], S[m * LDSLD + c]));
      S[rr * LDSLD + c] = cmk<C>(-s.x, -s.y);
    }
  }
  __syncthreads();
  for (int e = t; e < TILE_ELEMS; e += 256) Djj[e] = S[(e & 63) * LDSLD + (e >> 6)];
  __syncthreads();  // S is reused by the next item
  };
  auto run = [&](int item) {
    const int slot = find_slot(map, item);
    const int fm = map.fam[slot];
    const int n = item - map.start[slot];
    if (n == 0 && set->dual[fm]) body(slot, fm, n, std::true_type{});
    else body(slot, fm, n, std::false_type{});
  };
  if constexpr (P) {
    for (int item = blockIdx.x; item < map.start[map.cnt]; item += gridDim.x) run(item);
  } else {
    run(blockIdx.x);
  }
}

// Items: (block n, tile row i > j) of every family with more than j + 1 tile columns, i
// fastest.  Each round of gridDim.x items is dealt through xcd_remap so that every XCD takes a
// contiguous range (the tiles of one block share their row-j operands in that XCD's L2).
template <typename C, bool P>
__global__ void __launch_bounds__(256) k_ldlt_panel(const BlockSet* __restrict__ set, ItemMap map,
                                                    int j) {
  using R = typename mma<C>::R;
  // LDS: operand staging during the K loop, then the 64x64 tile S for the epilogue
  constexpr size_t SB = sizeof(StageBuf<C>), ST = sizeof(C) * TILE * LDSLD;
  __shared__ __align__(16) unsigned char smem[SB > ST ? SB : ST];
  StageBuf<C>& sb = *reinterpret_cast<StageBuf<C>*>(smem);
  C* S = reinterpret_cast<C*>(smem);
  auto body = [&](int slot, int fm, int n, int i, auto dtag) {
  constexpr bool D = decltype(dtag)::value;
  const int T = set->T[fm], M = set->M[fm];
  const double* __restrict__ g = set->g[fm];
  const double coef = set->coef[fm];
  const double2 lamn = block_lambda<D>(set, fm, n);
  C* fac = (C*)map.fac[slot] + (size_t)n * lower_tiles(T) * TILE_ELEMS;
  {
    WaveAcc<C> acc;
    if constexpr (sizeof(C) == 8) {
      tile_update_staged<C, D>(acc, fac, i, j, g, coef, lamn, M, sb);
      __syncthreads();  // staging buffers are reused as S
    } else {
      tile_update_direct<C, D>(acc, fac, i, j, g, coef, lamn, M);
    }
    acc_to_lds<C>(acc, S);
  }
  __syncthreads();
  // X = S L_jj^{-T}:  X[r][c] = sum_m S[r][m] Linv[c][m], Linv[c][m] = Djj[m*64 + c] (c > m),
  // 1 (c == m), 0 (c < m).
  const C* Djj = fac + tile_index(j, j) * TILE_ELEMS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1, l16 = lane & 15, lq = lane >> 4;
  // (three real MFMA products per complex product, as in the K loop; two for a dual block)
  WaveAcc<C> x;
  {
    WaveAcc3<C> x3;
    acc3_zero<C>(x3);
#pragma unroll 2
    for (int q = 0; q < 16; ++q) {
      const int m = 4 * q + lq;
      R sr[2], si[2], br[2], bim[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const C s = S[m * LDSLD + wr * 32 + bi * 16 + l16];
        sr[bi] = s.x; si[bi] = s.y;
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int c = wc * 32 + bj * 16 + l16;
        C b;
        if (c > m) b = Djj[m * TILE + c];
        else b = cmk<C>((R)(c == m ? 1 : 0), (R)(D && c == m ? 1 : 0));
        br[bj] = b.x; bim[bj] = b.y;
      }
      acc3_step<C, D>(x3, sr, si, br, bim);
    }
    acc3_finish<C, D>(x3, x);
  }
  __syncthreads();  // everyone is done reading S
  // L_ij[r][c] = X[r][c] / d_c, staged through LDS for coalesced stores
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int c = wc * 32 + bj * 16 + l16;
      const C dinv = xinv<D>(Djj[c * (TILE + 1)]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr * 32 + bi * 16 + mma<C>::row(lane, e);
        S[c * LDSLD + r] = xmul<D>(cmk<C>(x.re[bi][bj][e], x.im[bi][bj][e]), dinv);
      }
    }
  __syncthreads();
  C* Lij = fac + tile_index(i, j) * TILE_ELEMS;
  for (int e = threadIdx.x; e < TILE_ELEMS; e += 256) Lij[e] = S[(e >> 6) * LDSLD + (e & 63)];
  // This column's contribution to the pending diagonal tile (i, i):
  //   P_ii -= (L_ij D_j) L_ij^T,  P_ii = B_ii before column 0.
  // Only the lower triangle is used later, so the wave owning the upper-right quadrant skips.
  WaveAcc<C> dl;
  const bool active = !(wr == 0 && wc == 1);
  {
    WaveAcc3<C> d3;
    acc3_zero<C>(d3);
    if (active) {
#pragma unroll 2
      for (int q = 0; q < 16; ++q) {
        const int m = 4 * q + lq;
        const C d = Djj[m * (TILE + 1)];
        R ar[2], ai[2], br[2], bim[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
          const C a = xmul<D>(S[m * LDSLD + wr * 32 + bi * 16 + l16], d);
          ar[bi] = a.x; ai[bi] = a.y;
        }
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const C b = S[m * LDSLD + wc * 32 + bj * 16 + l16];
          br[bj] = b.x; bim[bj] = b.y;
        }
        acc3_step<C, D>(d3, ar, ai, br, bim);
      }
    }
    acc3_finish<C, D>(d3, dl);
  }
  __syncthreads();  // S (L_ij) no longer needed
  C* Pii = fac + tile_index(i, i) * TILE_ELEMS;
  if (j == 0) {
    for (int e = threadIdx.x; e < TILE_ELEMS; e += 256) {
      const int c = e >> 6, r = e & 63;
      const double2 b = shifted_entry<D>(g, coef, lamn, M, i * TILE + r, i * TILE + c);
      S[c * LDSLD + r] = cmk<C>((R)b.x, (R)b.y);
    }
  } else {
    for (int e = threadIdx.x; e < TILE_ELEMS; e += 256) S[(e >> 6) * LDSLD + (e & 63)] = Pii[e];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = wr * 32 + bi * 16 + mma<C>::row(lane, e);
          const int c = wc * 32 + bj * 16 + l16;
          S[c * LDSLD + r] = csub(S[c * LDSLD + r], cmk<C>(dl.re[bi][bj][e], dl.im[bi][bj][e]));
        }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TILE_ELEMS; e += 256) Pii[e] = S[(e >> 6) * LDSLD + (e & 63)];
  __syncthreads();  // smem is reused by the next item
  };
  auto run = [&](int item) {
    const int slot = find_slot(map, item);
    const int fm = map.fam[slot];
    const int per = set->T[fm] - 1 - j;
    const int lb = item - map.start[slot];
    const int n = lb / per, i = j + 1 + lb % per;
    if (n == 0 && set->dual[fm]) body(slot, fm, n, i, std::true_type{});
    else body(slot, fm, n, i, std::false_type{});
  };
  const int lbr = xcd_remap(blockIdx.x, gridDim.x);
  if constexpr (P) {
    const int total = map.start[map.cnt];
    for (int base = 0; base + lbr < total; base += gridDim.x) run(base + lbr);
  } else {
    run(lbr);
  }
}

// Items of column j: diag -> nb per family with T > j; panel -> nb (T - 1 - j) per family.
static ItemMap column_map(const BlockSet& hs, int j, bool panel) {
  ItemMap m;
  m.cnt = 0;
  m.start[0] = 0;
  for (int k = 0; k < hs.count; ++k) {
    const int per = panel ? hs.T[k] - 1 - j : (hs.T[k] > j ? 1 : 0);
    if (per <= 0) continue;
    m.fam[m.cnt] = k;
    m.fac[m.cnt] = hs.fac[k];
    m.start[m.cnt + 1] = m.start[m.cnt] + hs.nb[k] * per;
    ++m.cnt;
  }
  return m;
}

template <typename C>
static int factorize_t(const BlockSet& hs, const BlockSet* ds, int grid_cap, hipStream_t st) {
  int Tmax = 0;
  for (int k = 0; k < hs.count; ++k) Tmax = std::max(Tmax, hs.T[k]);
  for (int j = 0; j < Tmax; ++j) {
    const ItemMap md = column_map(hs, j, false);
    if (md.total() > 0) {
      if (grid_cap > 0 && grid_cap < md.total())
        k_ldlt_diag<C, true><<<grid_cap, 256, 0, st>>>(ds, md, j);
      else
        k_ldlt_diag<C, false><<<md.total(), 256, 0, st>>>(ds, md, j);
      RFDE_HIP(hipGetLastError());
    }
    const ItemMap mp = column_map(hs, j, true);
    if (mp.total() > 0) {
      if (grid_cap > 0 && grid_cap < mp.total())
        k_ldlt_panel<C, true><<<grid_cap, 256, 0, st>>>(ds, mp, j);
      else
        k_ldlt_panel<C, false><<<mp.total(), 256, 0, st>>>(ds, mp, j);
      RFDE_HIP(hipGetLastError());
    }
  }
  return RFDE_OK;
}

int launch_factorize_set(const BlockSet& hs, const BlockSet* ds, int bits, int grid_cap,
                         hipStream_t st) {
  if (hs.count < 1 || hs.count > MAX_BATCH) return RFDE_EINVAL;
  if (bits == 32) return factorize_t<float2>(hs, ds, grid_cap, st);
  return factorize_t<double2>(hs, ds, grid_cap, st);
}

static BlockSet plan_set(const Plan& p) {
  BlockSet hs{};
  hs.count = 1;
  set_family(hs, 0, p);
  return hs;
}

int launch_factorize(Plan& p) {
  return launch_factorize_set(plan_set(p), p.set, p.opts.precond_bits, 0, p.stream);
}

// ------------------------------------------------------------------------------------------
// Triangular solves: z = L^{-T} D^{-1} L^{-1} b for every block n (one workgroup per block).
// Forward (row-oriented): y_i = Linv_ii (b_i - sum_{k<i} L_ik y_k).
// Backward (column-oriented): x_k = Linv_kk^T (y'_k - sum_{i>k} L_ik^T x_i), y' = D^{-1} y.
// Each wave streams one quarter (16 columns) of every tile; lane = tile row.
template <typename C> __device__ __forceinline__ C shfl_xor_c(C v, int m) {
  return cmk<C>(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}
template <typename C> __device__ __forceinline__ C wave_sum(C v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = cadd(v, shfl_xor_c(v, m));
  return v;
}

// Input/output frequency-domain arrays of the families of a trsv launch (by value).
struct ZIO {
  const void* in[MAX_BATCH];
  void* out[MAX_BATCH];
};

// Items: the blocks n of every family (one workgroup each).
template <typename C, int TMAX, bool P>
__global__ void __launch_bounds__(256) k_trsv(const BlockSet* __restrict__ set, ItemMap map,
                                              ZIO io) {
  using R = typename mma<C>::R;
  __shared__ C xs[TMAX * TILE];
  __shared__ C red[4][TILE];
  __shared__ C tb[TILE];
  auto body = [&](int slot, int fm, int n, auto dtag) {
  constexpr bool D = decltype(dtag)::value;
  const int M = set->M[fm], T = set->T[fm];
  const C* fac = (const C*)map.fac[slot] + (size_t)n * lower_tiles(T) * TILE_ELEMS;
  const C* zin = (const C*)io.in[fm];
  C* zout = (C*)io.out[fm];
  const size_t nyq = (size_t)(set->nfreq[fm] - 1) * M;  // dual block: level N_t/2 of z
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int Mp = T * TILE;
  for (int r = t; r < Mp; r += 256) {
    C v = cmk<C>((R)0, (R)0);
    if (r < M) {
      if constexpr (D) v = cmk<C>(zin[r].x, zin[nyq + r].x);  // both right-hand sides are real
      else v = zin[(size_t)n * M + r];
    }
    xs[r] = v;
  }
  __syncthreads();
  // forward.  The off-diagonal tiles of tile row i are contiguous (tile index i(i+1)/2 + k), so
  // two consecutive tiles are fetched together to keep 32 loads per lane in flight.
  for (int i = 0; i < T; ++i) {
    C acc = cmk<C>((R)0, (R)0), acc1 = cmk<C>((R)0, (R)0);
    const C* Lrow = fac + tile_index(i, 0) * TILE_ELEMS + (16 * w) * TILE + lane;
    int k = 0;
    for (; k + 1 < i; k += 2) {
      const C* L0 = Lrow + (size_t)k * TILE_ELEMS;
      C a0[16], a1[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        a0[cc] = L0[cc * TILE];
        a1[cc] = L0[TILE_ELEMS + cc * TILE];
      }
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        acc = cadd(acc, xmul<D>(a0[cc], xs[k * TILE + 16 * w + cc]));
        acc1 = cadd(acc1, xmul<D>(a1[cc], xs[(k + 1) * TILE + 16 * w + cc]));
      }
    }
    if (k < i) {
      const C* L0 = Lrow + (size_t)k * TILE_ELEMS;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc = cadd(acc, xmul<D>(L0[cc * TILE], xs[k * TILE + 16 * w + cc]));
    }
    acc = cadd(acc, acc1);
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
      const C s = cadd(cadd(red[0][lane], red[1][lane]), cadd(red[2][lane], red[3][lane]));
      tb[lane] = csub(xs[i * TILE + lane], s);
    }
    __syncthreads();
    const C* Dii = fac + tile_index(i, i) * TILE_ELEMS;
    C acc2 = cmk<C>((R)0, (R)0);
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int c = 16 * w + cc;
      if (lane > c) acc2 = cadd(acc2, xmul<D>(Dii[c * TILE + lane], tb[c]));
    }
    red[w][lane] = acc2;
    __syncthreads();
    if (w == 0) {
      const C s = cadd(cadd(red[0][lane], red[1][lane]), cadd(red[2][lane], red[3][lane]));
      xs[i * TILE + lane] = cadd(tb[lane], s);
    }
    __syncthreads();
  }
  // diagonal
  for (int r = t; r < Mp; r += 256) {
    const C* Dkk = fac + tile_index(r >> 6, r >> 6) * TILE_ELEMS;
    xs[r] = xmul<D>(xs[r], xinv<D>(Dkk[(r & 63) * (TILE + 1)]));
  }
  __syncthreads();
  // backward
  for (int k = T - 1; k >= 0; --k) {
    C acc[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc[cc] = cmk<C>((R)0, (R)0);
    int i = k + 1;
    for (; i + 1 < T; i += 2) {
      const C* L0 = fac + tile_index(i, k) * TILE_ELEMS + (16 * w) * TILE + lane;
      const C* L1 = fac + tile_index(i + 1, k) * TILE_ELEMS + (16 * w) * TILE + lane;
      C a0[16], a1[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        a0[cc] = L0[cc * TILE];
        a1[cc] = L1[cc * TILE];
      }
      const C x0 = xs[i * TILE + lane], x1 = xs[(i + 1) * TILE + lane];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc)
        acc[cc] = cadd(acc[cc], cadd(xmul<D>(a0[cc], x0), xmul<D>(a1[cc], x1)));
    }
    if (i < T) {
      const C* L0 = fac + tile_index(i, k) * TILE_ELEMS + (16 * w) * TILE + lane;
      const C x0 = xs[i * TILE + lane];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc[cc] = cadd(acc[cc], xmul<D>(L0[cc * TILE], x0));
    }
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const C s = wave_sum(acc[cc]);
      if (lane == cc) tb[16 * w + cc] = csub(xs[k * TILE + 16 * w + cc], s);
    }
    __syncthreads();
    const C* Dkk = fac + tile_index(k, k) * TILE_ELEMS;
    const C tr = tb[lane];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int c = 16 * w + cc;
      C pterm = cmk<C>((R)0, (R)0);
      if (lane > c) pterm = xmul<D>(Dkk[c * TILE + lane], tr);
      else if (lane == c) pterm = tr;
      acc[cc] = wave_sum(pterm);
    }
#pragma unroll
    for (int cc = 0; cc < 16; ++cc)
      if (lane == cc) xs[k * TILE + 16 * w + cc] = acc[cc];
    __syncthreads();
  }
  for (int r = t; r < M; r += 256) {
    if constexpr (D) {
      zout[r] = cmk<C>(xs[r].x, (R)0);
      zout[nyq + r] = cmk<C>(xs[r].y, (R)0);
    } else {
      zout[(size_t)n * M + r] = xs[r];
    }
  }
  __syncthreads();  // xs is reused by the next item
  };
  auto run = [&](int item) {
    const int slot = find_slot(map, item);
    const int fm = map.fam[slot];
    if (set->live[fm] && *set->live[fm] == 0) return;  // uniform across the workgroup
    const int n = item - map.start[slot];
    if (n == 0 && set->dual[fm]) body(slot, fm, n, std::true_type{});
    else body(slot, fm, n, std::false_type{});
  };
  if constexpr (P) {
    for (int item = blockIdx.x; item < map.start[map.cnt]; item += gridDim.x) run(item);
  } else {
    run(blockIdx.x);
  }
}

int launch_trsv_set(const BlockSet& hs, const BlockSet* ds, const void* const* zin,
                    void* const* zout, int bits, int grid_cap, hipStream_t st) {
  if (hs.count < 1 || hs.count > MAX_BATCH) return RFDE_EINVAL;
  ItemMap m;
  m.cnt = 0;
  m.start[0] = 0;
  ZIO io{};
  for (int k = 0; k < hs.count; ++k) {
    if (hs.T[k] > 64) return RFDE_EINVAL;
    io.in[k] = zin[k];
    io.out[k] = zout[k];
    if (!zin[k] || !zout[k]) continue;  // family skipped in this launch
    m.fam[m.cnt] = k;
    m.fac[m.cnt] = hs.fac[k];
    m.start[m.cnt + 1] = m.start[m.cnt] + hs.nb[k];
    ++m.cnt;
  }
  if (m.total() == 0) return RFDE_OK;
  const bool persist = grid_cap > 0 && grid_cap < m.total();
  const int grid = persist ? grid_cap : m.total();
  if (bits == 32) {
    if (persist) k_trsv<float2, 64, true><<<grid, 256, 0, st>>>(ds, m, io);
    else k_trsv<float2, 64, false><<<grid, 256, 0, st>>>(ds, m, io);
  } else {
    if (persist) k_trsv<double2, 64, true><<<grid, 256, 0, st>>>(ds, m, io);
    else k_trsv<double2, 64, false><<<grid, 256, 0, st>>>(ds, m, io);
  }
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

int launch_trsv(const Plan& p, const void* zin, void* zout) {
  const BlockSet hs = plan_set(p);
  return launch_trsv_set(hs, p.set, &zin, &zout, p.opts.precond_bits, p.trsv_cap, p.stream);
}

// Export frequency block `index` as a dense row-major Mp x Mp matrix: strict lower = L,
// diagonal = D.  comp < 0: a complex block; comp = 0 / 1: the .x / .y part of the dual block.
template <typename C>
__global__ void k_export_factor(const C* __restrict__ fac, C* __restrict__ out, int T, int comp) {
  const int Mp = T * TILE;
  const size_t total = (size_t)Mp * Mp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int R = (int)(e / Mp), Cc = (int)(e % Mp);
    const int i = R >> 6, j = Cc >> 6, r = R & 63, c = Cc & 63;
    C val;
    val.x = 0; val.y = 0;
    if (i > j) val = fac[tile_index(i, j) * TILE_ELEMS + c * TILE + r];
    else if (i == j && r > c) val = fac[tile_index(i, i) * TILE_ELEMS + r * TILE + c];  // L^T store
    else if (i == j && r == c) val = fac[tile_index(i, i) * TILE_ELEMS + c * (TILE + 1)];
    if (comp >= 0) {
      val.x = comp == 0 ? val.x : val.y;
      val.y = 0;
    }
    out[e] = val;
  }
}

int launch_export_factor(const Plan& p, int index, void* dst) {
  const size_t sys = lower_tiles(p.T) * TILE_ELEMS;
  const size_t total = (size_t)p.Mp * p.Mp;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 16384);
  // frequency -> storage block (the dual block 0 holds frequencies 0 and N_t/2)
  int blk = index, comp = -1;
  if (p.dual) {
    if (index == 0) comp = 0;
    else if (index == p.nf - 1) { blk = 0; comp = 1; }
  }
  if (p.opts.precond_bits == 32)
    k_export_factor<float2><<<blocks, 256, 0, p.stream>>>((const float2*)p.factors + blk * sys,
                                                          (float2*)dst, p.T, comp);
  else
    k_export_factor<double2><<<blocks, 256, 0, p.stream>>>((const double2*)p.factors + blk * sys,
                                                           (double2*)dst, p.T, comp);
  RFDE_HIP(hipGetLastError());
  return RFDE_OK;
}

}  // namespace rfde
