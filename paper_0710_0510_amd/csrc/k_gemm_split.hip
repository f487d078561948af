// d-split packed-FP64 GEMM over GF(p^k), k = 3 or 4, on gfx950 MFMA: the
// chunking of Section 6 (Y = X^(d+1), d = 1) applied to field elements.
// Every element a = a_lo + Y a_hi (Y = X^2) is packed as two binary64 values
// at q = 2^17 (chunks of 2 coefficients, eq. (1); for k = 3 the high chunk
// has one coefficient), so q^3 < 2^53 leaves room for the 3 digits of a
// chunk product and the accumulator bias.  Three exact FP64 contractions
//   S_0 = sum a_lo b_lo,  S_2 = sum a_hi b_hi,
//   S_K = sum (a_lo + a_hi)(b_lo + b_hi)
// give the chunk-pair sums; the middle one is S_1 = S_K - S_0 - S_2 (one
// Karatsuba step), taken digit by digit mod p, so three MFMAs per k-group
// stand for the four products of chunks.  S_K has the largest digits, up to
// 8 (p-1)^2 per k for k = 4 (4 (p-1)^2 for k = 3); while K times that stays
// below q (eq. (2) for these chunks) -- K <= 4095 for GF(3^4), against 7
// products per block when all 4 coefficients share q = 2^7 -- the K loop has
// no block boundary.  Longer K is cut into blocks; at a boundary every
// accumulator is replaced by its digits mod p (REDQ_3 with the Q_d
// correction), re-packed at q, so later blocks add to digits below p.
//
// Epilogue per output element: REDQ_3 of each sum (Alg. 2, with Q_d's
// correction) gives 3 digits mod p; digit j of S_u is the coefficient of
// X^(2u+j) of the product polynomial, overlapping digits are added mod p, and
// the 2k-1 coefficients are reduced mod P by the L and H tables taken at a q
// divisible by p (Q_d is then the identity, and Thm. 3's tables reduce a
// plain coefficient vector).
//
// Loading follows k_gemm_direct.hip: a shared permutation of k and a
// renumbering of each wave's output columns make every lane's operand bytes
// contiguous; wave tile 16TM x 16TN, workgroup WGM x WGN waves, no LDS for
// operands.  Edge waves load whole words under per-lane predicates (rows,
// columns and k out of range read as zero, a partial word byte by byte).

#include "fqt_packed.h"

namespace fqt {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KE, int TM, int TN, int WGM, int WGN>
struct ST {
  static constexpr int WM = 16 * TM, WN = 16 * TN;
  static constexpr int BM = WGM * WM, BN = WGN * WN;
  static constexpr int BW = TN * KE / 4;  // words of one lane's B row segment
  static_assert((TN * KE) % 4 == 0, "B row segments are whole words");
  static_assert(WGM * WGN == 4, "four waves per workgroup");
  static_assert(KE == 3 || KE == 4, "d-split pairs coefficients of k = 3 or 4");
};

// The chunks of element e of a word run as integers at q = 2^17: low chunk
// c_0 + q c_1, high chunk c_2 (+ q c_3).
template <int KE, int NWD>
__device__ __forceinline__ void split_words(const uint32_t (&raw)[NWD], int e, uint32_t s17,
                                            uint32_t& lo, uint32_t& hi) {
  const int o = e * KE;
  lo = add_byte(byte_shl(raw[(o + 1) >> 2], (o + 1) & 3, s17), raw[o >> 2], o & 3);
  if constexpr (KE == 4)
    hi = add_byte(byte_shl(raw[(o + 3) >> 2], (o + 3) & 3, s17), raw[(o + 2) >> 2], (o + 2) & 3);
  else
    hi = (raw[(o + 2) >> 2] >> (8 * ((o + 2) & 3))) & 0xffu;
}

// Words of a run whose first vb bytes are valid; the rest read as zero.
// Whole words load as words, a partial one byte by byte; nothing at or past
// byte vb is touched.
template <int NW>
__device__ __forceinline__ void load_valid(const uint8_t* src, int vb, uint32_t (&w)[NW]) {
  const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
#pragma unroll
  for (int x = 0; x < NW; ++x) {
    uint32_t v = 0;
    if (4 * x + 4 <= vb) {
      v = s32[x];
    } else if (4 * x < vb) {
      v = src[4 * x];
      if (4 * x + 1 < vb) v |= (uint32_t)src[4 * x + 1] << 8;
      if (4 * x + 2 < vb) v |= (uint32_t)src[4 * x + 2] << 16;
    }
    w[x] = v;
  }
}

// Digits mod p of a biased chunk-pair sum 2^52 + sum_j D_j q^j (D_j < q,
// q = 2^b): Thm. 2's residues u_j, then d_j = (u_j - q u_{j+1}) mod p.
__device__ __forceinline__ void split_digits(double acc, uint32_t b, const FieldArgs& fa,
                                             uint32_t (&d)[3]) {
  uint32_t t[3];
  redq_residues_biased<3>(acc, b, fa, t);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const uint32_t x = t[j] & 0xffu;
    d[j] = x >= fa.p ? x - fa.p : x;
  }
  d[0] = mod_p_small(d[0] + fa.c * d[1], fa);
  d[1] = mod_p_small(d[1] + fa.c * d[2], fa);
}

// Block boundary: the sum restarts from its digits mod p (each below p, so
// the next block's digit bound is (p-1) + n_q w (p-1)^2 < q).
__device__ __forceinline__ double split_reseed(double acc, uint32_t b, const FieldArgs& fa) {
  uint32_t d[3];
  split_digits(acc, b, fa, d);
  const uint64_t v = (uint64_t)d[0] | ((uint64_t)d[1] << b) | ((uint64_t)d[2] << (2 * b));
  return __longlong_as_double((long long)(bits64(kTwo52) | v));
}

template <int KE, int TM, int TN, int WGM, int WGN>
__device__ __forceinline__ void split_tile(const GemmArgs& g, int tile_m, int tile_n,
                                           const PackedParams& pp,
                                           const uint32_t* __restrict__ Ls,
                                           const uint32_t* __restrict__ Hs) {
  using T = ST<KE, TM, TN, WGM, WGN>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, grp = lane >> 4;
  const int64_t wm0 = (int64_t)tile_m * T::BM + (wave / WGN) * T::WM;
  const int64_t wn0 = (int64_t)tile_n * T::BN + (wave % WGN) * T::WN;
  if (wm0 >= g.M || wn0 >= g.N) return;  // no barrier below
  const bool inner = pp.aligned != 0 && wm0 + T::WM <= g.M && wn0 + T::WN <= g.N;
  const uint32_t s17 = pp.b;
  const int64_t nks = (g.K + 15) / 16, nfull = g.K / 16;
  const uint32_t blk = pp.nq_groups / 4;  // 16-k steps per block, 0: one block
  const FieldArgs& fa = pp.fa;

  const v4d bias = {kTwo52, kTwo52, kTwo52, kTwo52};
  v4d acc[3][TM][TN];  // S_0, S_K, S_2
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[u][i][j] = bias;

  const uint8_t* pa = g.A + ((wm0 + c) * g.lda + 4 * grp) * KE;
  const uint8_t* pb = g.B + ((int64_t)(4 * grp) * g.ldb + wn0 + TN * c) * KE;
  const int64_t a_istep = 16 * g.lda * KE, b_gstep = g.ldb * KE, b_sstep = 16 * g.ldb * KE;

  // one K-step of raw operand bytes: A rows wm0+16i+c at k = 16s+4g..+3,
  // B rows 16s+4g+gk at columns wn0+TN*c..+TN-1
  auto load_step = [&](int64_t s, uint32_t (&ra)[TM][KE], uint32_t (&rb)[4][T::BW]) {
    if (inner && s < nfull) {
      const uint8_t* a0 = pa + s * 16 * KE;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a0 + i * a_istep);
#pragma unroll
        for (int w = 0; w < KE; ++w) ra[i][w] = src[w];
      }
      const uint8_t* b0 = pb + s * b_sstep;
#pragma unroll
      for (int gk = 0; gk < 4; ++gk) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(b0 + gk * b_gstep);
#pragma unroll
        for (int w = 0; w < T::BW; ++w) rb[gk][w] = src[w];
      }
      return;
    }
    const int64_t k0 = 16 * s + 4 * grp;
    const int nka = (int)min<int64_t>(max<int64_t>(g.K - k0, 0), 4);  // valid k of the group
    if (pp.aligned) {
      // predicated word loads: every run starts on a word boundary
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int64_t row = wm0 + 16 * i + c;
        const int vb = row < g.M ? nka * KE : 0;
        load_valid<KE>(g.A + (row * g.lda + k0) * KE, vb, ra[i]);
      }
      const int64_t col0 = wn0 + TN * c;
      const int nvc = (int)min<int64_t>(max<int64_t>(g.N - col0, 0), TN);
#pragma unroll
      for (int gk = 0; gk < 4; ++gk) {
        const int vb = gk < nka ? nvc * KE : 0;
        load_valid<T::BW>(g.B + ((k0 + gk) * g.ldb + col0) * KE, vb, rb[gk]);
      }
      return;
    }
    // unaligned rows: bounds-checked byte gathers
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int w = 0; w < KE; ++w) ra[i][w] = 0;
      const int64_t row = wm0 + 16 * i + c;
      if (row < g.M) {
        const uint8_t* src = g.A + (row * g.lda + k0) * KE;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (e < nka)
#pragma unroll
            for (int cc = 0; cc < KE; ++cc) {
              const int pos = e * KE + cc;
              ra[i][pos >> 2] |= (uint32_t)src[pos] << (8 * (pos & 3));
            }
      }
    }
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) {
#pragma unroll
      for (int w = 0; w < T::BW; ++w) rb[gk][w] = 0;
      if (gk < nka) {
        const uint8_t* src = g.B + (k0 + gk) * g.ldb * KE;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int64_t col = wn0 + TN * c + j;
          if (col < g.N)
#pragma unroll
            for (int cc = 0; cc < KE; ++cc) {
              const int pos = j * KE + cc;
              rb[gk][pos >> 2] |= (uint32_t)src[col * KE + cc] << (8 * (pos & 3));
            }
        }
      }
    }
  };
  auto compute_step = [&](const uint32_t (&ra)[TM][KE], const uint32_t (&rb)[4][T::BW]) {
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) {
      double alo[TM], ahi[TM], asum[TM], blo[TN], bhi[TN], bsum[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        uint32_t lo, hi;
        split_words<KE, KE>(ra[i], gk, s17, lo, hi);
        alo[i] = (double)lo;
        ahi[i] = (double)hi;
        asum[i] = (double)(lo + hi);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        uint32_t lo, hi;
        split_words<KE, T::BW>(rb[gk], j, s17, lo, hi);
        blo[j] = (double)lo;
        bhi[j] = (double)hi;
        bsum[j] = (double)(lo + hi);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[0][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(alo[i], blo[j], acc[0][i][j], 0, 0, 0);
          acc[1][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(asum[i], bsum[j], acc[1][i][j], 0, 0, 0);
          acc[2][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ahi[i], bhi[j], acc[2][i][j], 0, 0, 0);
        }
    }
  };
  uint32_t bcnt = 0;
  auto boundary = [&]() {
    if (blk && ++bcnt == blk) {
      bcnt = 0;
#pragma unroll
      for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][i][j][v] = split_reseed(acc[u][i][j][v], s17, fa);
    }
  };
  // two stages: the next K-step loads while this one runs on the matrix cores
  uint32_t ra0[TM][KE], rb0[4][T::BW], ra1[TM][KE], rb1[4][T::BW];
  if (nks > 0) load_step(0, ra0, rb0);
  for (int64_t s = 0; s < nks; s += 2) {
    if (s + 1 < nks) load_step(s + 1, ra1, rb1);
    compute_step(ra0, rb0);
    boundary();
    if (s + 1 >= nks) break;
    if (s + 2 < nks) load_step(s + 2, ra0, rb0);
    compute_step(ra1, rb1);
    boundary();
  }

  // Epilogue: digits of S_0, S_1 = S_K - S_0 - S_2, S_2 -> coefficients
  // c_0..c_{2k-2} -> L + H.
  const bool c_words = ((((uintptr_t)g.C) & 3) == 0) && (((g.ldc * KE) & 3) == 0);
  const int64_t col0 = wn0 + TN * c;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = wm0 + 16 * i + grp + 4 * v;
      uint32_t e[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        uint32_t d0[3], dk[3], d2[3];
        split_digits(acc[0][i][j][v], s17, fa, d0);
        split_digits(acc[1][i][j][v], s17, fa, dk);
        split_digits(acc[2][i][j][v], s17, fa, d2);
        uint32_t cc[2 * KE - 1];
#pragma unroll
        for (int n = 0; n < 2 * KE - 1; ++n) cc[n] = 0;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          if (jj < 2 * KE - 1) cc[jj] += d0[jj];
          if (4 + jj < 2 * KE - 1) cc[4 + jj] += d2[jj];
          // S_1 digit: dk - d0 - d2 mod p, every term below p
          if (2 + jj < 2 * KE - 1)
            cc[2 + jj] += mod_p_small(dk[jj] + 2 * fa.p - d0[jj] - d2[jj], fa);
        }
#pragma unroll
        for (int n = 0; n < 2 * KE - 1; ++n) cc[n] = cc[n] >= fa.p ? cc[n] - fa.p : cc[n];
        e[j] = lh_combine<KE>(cc, pp, Ls, Hs);
      }
      if (row >= g.M) continue;
      uint8_t* dst = g.C + (row * g.ldc + col0) * KE;
      if (c_words && col0 + TN <= g.N) {
        uint32_t w[T::BW];
#pragma unroll
        for (int x = 0; x < T::BW; ++x) w[x] = 0;
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int cb = 0; cb < KE; ++cb) {
            const int pos = j * KE + cb;
            w[pos >> 2] |= ((e[j] >> (8 * cb)) & 0xffu) << (8 * (pos & 3));
          }
        uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
        for (int x = 0; x < T::BW; ++x) d32[x] = w[x];
      } else {
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (col0 + j < g.N) store_elem<KE>(dst + j * KE, e[j]);
      }
    }
}

template <int KE, int TM, int TN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_split_kernel(GemmArgs g, PackedParams pp, int tiles_n,
                                                         int ntiles) {
  extern __shared__ uint32_t tabs[];
  uint32_t* Ls = tabs;
  uint32_t* Hs = tabs + (1 << pp.tbl_log2);
  load_tables(pp, Ls, Hs);
  __syncthreads();
  const int tile = xcd_tile((int)blockIdx.x, ntiles / tiles_n, tiles_n);
  split_tile<KE, TM, TN, WGM, WGN>(g, tile / tiles_n, tile % tiles_n, pp, Ls, Hs);
}

template <int KE, int TM, int TN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_split_batched_kernel(
    const GemmArgs* __restrict__ descs, const TileItem* __restrict__ items, int32_t n_items,
    uint32_t* counter, PackedParams pp) {
  __shared__ int32_t cur;
  extern __shared__ uint32_t tabs[];
  uint32_t* Ls = tabs;
  uint32_t* Hs = tabs + (1 << pp.tbl_log2);
  load_tables(pp, Ls, Hs);
  for (;;) {
    if (threadIdx.x == 0) cur = (int32_t)atomicAdd(&counter[0], 1u);
    __syncthreads();
    const int32_t it = cur;
    __syncthreads();
    if (it >= n_items) break;
    const TileItem ti = items[it];
    const GemmArgs g = descs[ti.gemm];
    split_tile<KE, TM, TN, WGM, WGN>(g, ti.tm, ti.tn, pp, Ls, Hs);
  }
  // The last workgroup to leave resets the queue for the next launch.
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
  }
}

template <int KE, int TM, int TN, int WGM, int WGN>
static hipError_t split_one(const GemmArgs& g, const PackedParams& pp, hipStream_t s) {
  using T = ST<KE, TM, TN, WGM, WGN>;
  const int tiles_m = (int)((g.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((g.N + T::BN - 1) / T::BN);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_split_kernel<KE, TM, TN, WGM, WGN>), dim3(ntiles), dim3(256), dyn, s,
                     g, pp, tiles_n, ntiles);
  return hipGetLastError();
}

template <int KE, int TM, int TN, int WGM, int WGN>
static hipError_t split_batched(const GemmArgs* descs, const TileItem* items, int32_t n_items,
                                uint32_t* counter, int grid, const PackedParams& pp,
                                hipStream_t s) {
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_split_batched_kernel<KE, TM, TN, WGM, WGN>), dim3(grid), dim3(256),
                     dyn, s, descs, items, n_items, counter, pp);
  return hipGetLastError();
}

template <int KE, int TM, int TN, int WGM, int WGN>
static int split_occ(uint32_t tbl_log2) {
  int blocks = 0;
  const size_t dyn = 2u * (1u << tbl_log2) * sizeof(uint32_t);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_split_batched_kernel<KE, TM, TN, WGM, WGN>, 256, dyn) !=
      hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

// tile ids (shapes in packed_tile_shape): kFirstSplitTile = 2 x 2 waves of
// 16 x 64 (32 x 128), the next one 4 x 1 waves of 16 x 64 (64 x 64)
#define FQT_SPLIT_DISPATCH(F, RET_BAD, ...)                                          \
  switch (k * 100 + tile) {                                                          \
    case 300 + kFirstSplitTile: return F<3, 1, 4, 2, 2>(__VA_ARGS__);               \
    case 300 + kFirstSplitTile + 1: return F<3, 1, 4, 4, 1>(__VA_ARGS__);           \
    case 400 + kFirstSplitTile: return F<4, 1, 4, 2, 2>(__VA_ARGS__);               \
    case 400 + kFirstSplitTile + 1: return F<4, 1, 4, 4, 1>(__VA_ARGS__);           \
    default: return RET_BAD;                                                         \
  }

hipError_t launch_gemm_split(int k, int tile, const GemmArgs& g, const PackedParams& pp,
                             hipStream_t s) {
  FQT_SPLIT_DISPATCH(split_one, hipErrorInvalidValue, g, pp, s)
}

hipError_t launch_gemm_split_batched(int k, int tile, const GemmArgs* descs,
                                     const TileItem* items, int32_t n_items, uint32_t* counter,
                                     int grid, const PackedParams& pp, hipStream_t s) {
  FQT_SPLIT_DISPATCH(split_batched, hipErrorInvalidValue, descs, items, n_items, counter, grid,
                     pp, s)
}

int split_batched_occupancy(int k, int tile, uint32_t tbl_log2) {
  FQT_SPLIT_DISPATCH(split_occ, 1, tbl_log2)
}

}  // namespace fqt
