// Packed-FP64 GEMM over GF(p^k) on gfx950 MFMA (the FQT path).
//
// Alg. 4 (fast dot product over GF(p^k) via FQT) for every entry of C:
//   1. DQT of each operand element at q = 2^b (Section 2: shifts), fused into
//      the global->LDS loader: k coefficient bytes -> one exact binary64.
//   2. The dot products as one dense FP64 contraction on the matrix cores
//      (v_mfma_f64_16x16x4f64); exact while eq. (2) holds, i.e. at most n_q
//      products per K-block with q > n_q k (p-1)^2 and q^(2k-1) < 2^53.
//   3. REDQ residues u_0..u_{2k-2} of each block (Alg. 4 steps 3-7, Thm. 2).
//   4. Two table lookups L[u_0..u_{k-1}] + H[u_{k-1}..u_{2k-2}] (Thm. 3) and
//      one coefficient-wise addition mod p.
//
// Several K-blocks (delayed reduction, Section 6) carry a per-element state
// between blocks: modes 0/1/2 of BlockLanes in fqt_packed.h.
//
// Layout: workgroup = 256 threads = 2 x 2 waves; wave tile 16TM x 16TN made of
// TM x TN MFMA blocks of 16 x 16; workgroup tile BM x BN = 32TM x 32TN;
// K-tiles of BK (16 or 32) elements, double-buffered in LDS as packed doubles.
// MFMA 16x16x4 f64 operand layout (per lane l of the wave):
//   A: row l%16, k l/16;  B: k l/16, column l%16;
//   D: element v in 0..3 at row l/16 + 4v, column l%16 (checked on gfx950).

#include "fqt_packed.h"

namespace fqt {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KE, int TM, int TN, int BK_>
struct PT {
  static constexpr int BM = 32 * TM;
  static constexpr int BN = 32 * TN;
  static constexpr int BK = BK_;
  // Row strides in doubles chosen so that the 32 lanes of one ds_read_b64 of
  // an MFMA operand hit distinct LDS banks.
  static constexpr int SA = BK == 32 ? BK + 2 : BK + 1;
  static constexpr int SB = BN + 16;
  static constexpr int ND = 2 * KE - 1;
  static constexpr int NW = (ND + 1) / 2;  // 16-bit-lane words per output element
  static constexpr int NCA = BM * BK / 4;  // A chunks: 4 consecutive k of one row
  static constexpr int NCB = BK * BN / 4;  // B chunks: 4 consecutive n of one k-row
  static constexpr int RA = NCA / 256;
  static constexpr int RB = NCB / 256;
  static constexpr int LDS_A = BM * SA;
  static constexpr int LDS_B = BK * SB;
  static_assert(NCA % 256 == 0 && NCB % 256 == 0, "every thread loads whole chunks");
};

// Raw bytes of a 4-element chunk (4*KE bytes) from a row segment starting at
// element (row, col) with ld elements per row; missing elements read as 0.
template <int KE>
__device__ __forceinline__ void load_chunk(const uint8_t* base, int64_t row, int64_t col,
                                           int64_t nrows, int64_t ncols, int64_t ld,
                                           bool aligned, uint32_t (&raw)[KE]) {
  if (aligned && row < nrows && col + 3 < ncols) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(base + (row * ld + col) * KE);
#pragma unroll
    for (int j = 0; j < KE; ++j) raw[j] = src[j];
    return;
  }
#pragma unroll
  for (int j = 0; j < KE; ++j) raw[j] = 0;
  if (row >= nrows) return;
  const uint8_t* src = base + row * ld * KE;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (col + e < ncols) {
#pragma unroll
      for (int c = 0; c < KE; ++c) {
        const int j = e * KE + c;
        raw[j >> 2] |= (uint32_t)src[(col + e) * KE + c] << (8 * (j & 3));
      }
    }
  }
}

template <int KE, int TM, int TN, int BK, int MODE>
__device__ __forceinline__ void packed_tile(const GemmArgs& g, int tile_m, int tile_n,
                                            const PackedParams& pp, double* __restrict__ As,
                                            double* __restrict__ Bs,
                                            const uint32_t* __restrict__ Ls,
                                            const uint32_t* __restrict__ Hs) {
  using T = PT<KE, TM, TN, BK>;
  constexpr bool MULTI = MODE != 0;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * 16 * TM;
  const int wn0 = (wave & 1) * 16 * TN;
  const int64_t m0 = (int64_t)tile_m * T::BM;
  const int64_t n0 = (int64_t)tile_n * T::BN;
  const bool aligned = pp.aligned != 0;
  // Several K-blocks: q is the largest power of two eq. (2) admits, fixed at
  // compile time so that digit windows become constant bit-field extracts.
  const uint32_t b = MODE ? multi_block_b<KE>() : pp.b;
  const DqtShifts sh(b);
  // Interior tiles (and full K-tiles) load without bounds checks.
  const bool interior = aligned && m0 + T::BM <= g.M && n0 + T::BN <= g.N;
  // Padded K-blocks: blk_real products in blk_slots = 4 * nq_groups MFMA
  // slots, the last slots of a block zero (blk_slots divides BK).
  const bool padded = MULTI && pp.blk_real != 4 * pp.nq_groups;

  // every block starts from 2^52 (centred packing: plus q/2 in every digit)
  const double bz = pp.centered ? pp.cbias : kTwo52;
  const v4d bias = {bz, bz, bz, bz};
  v4d acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = bias;

  BlockLanes<KE, MODE> st[MULTI ? TM : 1][MULTI ? TN : 1][4];
  if constexpr (MULTI) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) st[i][j][v].clear();
  }

  // Fixed chunk geometry of this thread: A chunk r covers row arow + r*(1024/BK),
  // k = 4*akc..4*akc+3 of the K-tile; B chunk r covers k-row bkr + r*(1024/BN),
  // n = 4*bnc..4*bnc+3.
  const int arow = tid / (T::BK / 4), akc = tid % (T::BK / 4);
  const int bkr = tid / (T::BN / 4), bnc = tid % (T::BN / 4);
  constexpr int ARS = 1024 / T::BK, BRS = 1024 / T::BN;
  const uint8_t* pa = g.A + ((m0 + arow) * g.lda + 4 * akc) * KE;
  const uint8_t* pb = g.B + ((int64_t)bkr * g.ldb + n0 + 4 * bnc) * KE;
  const int64_t a_rstep = (int64_t)ARS * g.lda * KE;  // bytes between chunk rows
  const int64_t b_rstep = (int64_t)BRS * g.ldb * KE;
  const int64_t b_kstep = (int64_t)T::BK * g.ldb * KE;  // bytes per K-tile

  uint32_t ra[T::RA][KE];
  uint32_t rb[T::RB][KE];

  // Padded mode: this thread's A chunk starts at slot offset 4*akc of the
  // K-tile, i.e. block a_blk of the tile, offset a_off in it; its B rows sit
  // at slot offsets bkr + r*BRS.
  const uint32_t slots = 4 * pp.nq_groups, real = pp.blk_real;
  const uint32_t a_blk = padded ? (4u * akc) / slots : 0u, a_off = padded ? (4u * akc) % slots : 0u;
  const int a_cnt = padded ? (int)min(4u, real - a_off) : 4;
  auto gload_padded = [&](int64_t kt) {
    const int64_t blk0 = kt * (T::BK / slots);  // first block of this K-tile
    const int64_t ka = (blk0 + a_blk) * real + a_off;
#pragma unroll
    for (int r = 0; r < T::RA; ++r) {
      const int64_t row = m0 + arow + r * ARS;
#pragma unroll
      for (int j = 0; j < KE; ++j) ra[r][j] = 0;
      if (row < g.M) {
        const uint8_t* src = g.A + row * g.lda * KE;
        for (int e = 0; e < a_cnt; ++e) {
          if (ka + e >= g.K) break;
#pragma unroll
          for (int c = 0; c < KE; ++c) {
            const int jb = e * KE + c;
            ra[r][jb >> 2] |= (uint32_t)src[(ka + e) * KE + c] << (8 * (jb & 3));
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < T::RB; ++r) {
      const uint32_t sl = (uint32_t)(bkr + r * BRS);
      const uint32_t off = sl % slots;
      const int64_t krow = (blk0 + sl / slots) * real + off;
      if (off < real) {
        load_chunk<KE>(g.B, krow, n0 + 4 * bnc, g.K, g.N, g.ldb, aligned, rb[r]);
      } else {
#pragma unroll
        for (int j = 0; j < KE; ++j) rb[r][j] = 0;
      }
    }
  };

  auto gload = [&](int64_t k0) {
    if (padded) {
      gload_padded(k0 / T::BK);
      return;
    }
    if (interior && k0 + T::BK <= g.K) {
      const uint8_t* a0 = pa + k0 * KE;
      const uint8_t* b0 = pb + (k0 / T::BK) * b_kstep;
#pragma unroll
      for (int r = 0; r < T::RA; ++r) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a0 + r * a_rstep);
#pragma unroll
        for (int j = 0; j < KE; ++j) ra[r][j] = src[j];
      }
#pragma unroll
      for (int r = 0; r < T::RB; ++r) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(b0 + r * b_rstep);
#pragma unroll
        for (int j = 0; j < KE; ++j) rb[r][j] = src[j];
      }
      return;
    }
#pragma unroll
    for (int r = 0; r < T::RA; ++r)
      load_chunk<KE>(g.A, m0 + arow + r * ARS, k0 + 4 * akc, g.M, g.K, g.lda, aligned, ra[r]);
#pragma unroll
    for (int r = 0; r < T::RB; ++r)
      load_chunk<KE>(g.B, k0 + bkr + r * BRS, n0 + 4 * bnc, g.K, g.N, g.ldb, aligned, rb[r]);
  };

  auto lstore = [&](int buf) {
    double* as = As + buf * T::LDS_A;
    double* bs = Bs + buf * T::LDS_B;
#pragma unroll
    for (int r = 0; r < T::RA; ++r) {
      double v[4];
      dqt_chunk<KE>(ra[r], sh, pp, v);
#pragma unroll
      for (int e = 0; e < 4; ++e) as[(arow + r * ARS) * T::SA + 4 * akc + e] = v[e];
    }
#pragma unroll
    for (int r = 0; r < T::RB; ++r) {
      double v[4];
      dqt_chunk<KE>(rb[r], sh, pp, v);
#pragma unroll
      for (int e = 0; e < 4; ++e) bs[(bkr + r * BRS) * T::SB + 4 * bnc + e] = v[e];
    }
  };

  uint32_t nbound = 0, nblk = 1;  // blocks seeded so far (the centred correction counts them)
  uint32_t nadd = 0;              // blocks in the lane state since its last fold
  auto boundary = [&]() {
    if constexpr (MULTI) {
      ++nblk;
      ++nadd;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) st[i][j][v].add(acc[i][j][v], pp.fa);
          acc[i][j] = bias;
        }
      // fold the sums mod p before another block could overflow them
      if (pp.fold_blocks && ++nbound == pp.fold_blocks) {
        nbound = 0;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) st[i][j][v].fold(pp.fa, nadd);
        nadd = 0;
      }
    }
  };

  // K-tiles cover K products, or ceil(K / real) padded blocks of `slots`.
  const int64_t kslots = padded ? (g.K + real - 1) / real * slots : g.K;
  const int64_t nkt = (kslots + T::BK - 1) / T::BK;
  uint32_t gcnt = 0;
  if (nkt > 0) {
    gload(0);
    lstore(0);
    __syncthreads();
  }
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nkt) gload((kt + 1) * T::BK);
    const double* as = As + buf * T::LDS_A;
    const double* bs = Bs + buf * T::LDS_B;
#pragma unroll
    for (int gk = 0; gk < T::BK / 4; ++gk) {
      double a[TM], bb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = as[(wm0 + 16 * i + (lane & 15)) * T::SA + 4 * gk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bb[j] = bs[(4 * gk + (lane >> 4)) * T::SB + wn0 + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
      if constexpr (MULTI) {
        if (++gcnt == pp.nq_groups) {
          boundary();
          gcnt = 0;
        }
      }
    }
    if (kt + 1 < nkt) lstore(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: final residues, L + H (Thm. 3), store k bytes per element.
  const uint32_t corr = pp.centered ? centred_correction<KE>(pp.c0neg, nblk, pp.fa) : 0u;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        uint32_t u[T::ND];
        st[MULTI ? i : 0][MULTI ? j : 0][v].residues(acc[i][j][v], b, pp, u, nadd);
        uint32_t e = lh_combine<KE>(u, pp, Ls, Hs);
        if (pp.centered) e = add_bytes_mod_p(e, corr, pp.fa);
        const int64_t row = m0 + wm0 + 16 * i + (lane >> 4) + 4 * v;
        const int64_t col = n0 + wn0 + 16 * j + (lane & 15);
        if (row < g.M && col < g.N) store_elem<KE>(g.C + (row * g.ldc + col) * KE, e);
      }
}

template <int KE, int TM, int TN, int BK, int MODE>
__global__ __launch_bounds__(256) void gemm_packed_kernel(GemmArgs g, PackedParams pp,
                                                          int tiles_n, int ntiles) {
  using T = PT<KE, TM, TN, BK>;
  __shared__ double As[2 * T::LDS_A];
  __shared__ double Bs[2 * T::LDS_B];
  extern __shared__ uint32_t tabs[];
  uint32_t* Ls = tabs;
  uint32_t* Hs = tabs + (1 << pp.tbl_log2);
  load_tables(pp, Ls, Hs);
  __syncthreads();
  const int tile = xcd_tile((int)blockIdx.x, ntiles / tiles_n, tiles_n);
  packed_tile<KE, TM, TN, BK, MODE>(g, tile / tiles_n, tile % tiles_n, pp, As, Bs, Ls, Hs);
}

template <int KE, int TM, int TN, int BK, int MODE>
__global__ __launch_bounds__(256) void gemm_packed_batched_kernel(
    const GemmArgs* __restrict__ descs, const TileItem* __restrict__ items, int32_t n_items,
    uint32_t* counter, PackedParams pp) {
  using T = PT<KE, TM, TN, BK>;
  __shared__ double As[2 * T::LDS_A];
  __shared__ double Bs[2 * T::LDS_B];
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
    packed_tile<KE, TM, TN, BK, MODE>(g, ti.tm, ti.tn, pp, As, Bs, Ls, Hs);
  }
  // The last workgroup to leave resets the queue for the next launch (every
  // workgroup has made its final counter[0] increment before counter[1]).
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
  }
}

template <int KE, int TM, int TN, int BK, int MODE>
static hipError_t launch_one(const GemmArgs& g, const PackedParams& pp, hipStream_t s) {
  using T = PT<KE, TM, TN, BK>;
  const int tiles_m = (int)((g.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((g.N + T::BN - 1) / T::BN);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_packed_kernel<KE, TM, TN, BK, MODE>), dim3(ntiles), dim3(256), dyn,
                     s, g, pp, tiles_n, ntiles);
  return hipGetLastError();
}

template <int KE, int TM, int TN, int BK, int MODE>
static hipError_t launch_batched(const GemmArgs* descs, const TileItem* items, int32_t n_items,
                                 uint32_t* counter, int grid, const PackedParams& pp,
                                 hipStream_t s) {
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_packed_batched_kernel<KE, TM, TN, BK, MODE>), dim3(grid), dim3(256),
                     dyn, s, descs, items, n_items, counter, pp);
  return hipGetLastError();
}

template <int KE, int TM, int TN, int BK, int MODE>
static int occupancy(uint32_t tbl_log2) {
  int blocks = 0;
  const size_t dyn = 2u * (1u << tbl_log2) * sizeof(uint32_t);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_packed_batched_kernel<KE, TM, TN, BK, MODE>, 256, dyn) !=
      hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

// Dispatch over (k, tile id, multi-block); the tile list is FQT_PACKED_TILES.
// (digit-sum boundaries only where 2b <= 24: the host never asks for others)
#define FQT_TILE_CASE(ID, TM, TN, BK)                                    \
  case ID:                                                                \
    if constexpr (MODE != 2 || digit_sums_fit<KE>())                      \
      return FN<KE, TM, TN, BK, MODE>(ARGS);                              \
    else                                                                  \
      return FAIL;

template <int KE, int MODE>
static hipError_t dispatch_one(int tile, const GemmArgs& g, const PackedParams& pp,
                               hipStream_t s) {
#define FN launch_one
#define ARGS g, pp, s
#define FAIL hipErrorInvalidValue
  switch (tile) { FQT_PACKED_TILES(FQT_TILE_CASE) default: return hipErrorInvalidValue; }
#undef FN
#undef ARGS
#undef FAIL
}

template <int KE, int MODE>
static hipError_t dispatch_batched(int tile, const GemmArgs* descs, const TileItem* items,
                                   int32_t n_items, uint32_t* counter, int grid,
                                   const PackedParams& pp, hipStream_t s) {
#define FN launch_batched
#define ARGS descs, items, n_items, counter, grid, pp, s
#define FAIL hipErrorInvalidValue
  switch (tile) { FQT_PACKED_TILES(FQT_TILE_CASE) default: return hipErrorInvalidValue; }
#undef FN
#undef ARGS
#undef FAIL
}

template <int KE, int MODE>
static int dispatch_occupancy(int tile, uint32_t tbl_log2) {
#define FN occupancy
#define ARGS tbl_log2
#define FAIL 1
  switch (tile) { FQT_PACKED_TILES(FQT_TILE_CASE) default: return 1; }
#undef FN
#undef ARGS
#undef FAIL
}
#undef FQT_TILE_CASE

#define FQT_MODE_DISPATCH(F, KE, ...)                                         \
  switch (mode) {                                                             \
    case 0: return F<KE, 0>(__VA_ARGS__);                                     \
    case 1: return F<KE, 1>(__VA_ARGS__);                                     \
    case 2: return F<KE, 2>(__VA_ARGS__);                                     \
    default: break;                                                           \
  }
#define FQT_K_DISPATCH(F, ...)                                                \
  switch (k) {                                                                \
    case 1: FQT_MODE_DISPATCH(F, 1, __VA_ARGS__) break;                       \
    case 2: FQT_MODE_DISPATCH(F, 2, __VA_ARGS__) break;                       \
    case 3: FQT_MODE_DISPATCH(F, 3, __VA_ARGS__) break;                       \
    case 4: FQT_MODE_DISPATCH(F, 4, __VA_ARGS__) break;                       \
    default: break;                                                           \
  }

hipError_t launch_gemm_packed(int k, int tile, int mode, const GemmArgs& g,
                              const PackedParams& pp, hipStream_t s) {
  FQT_K_DISPATCH(dispatch_one, tile, g, pp, s)
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_packed_batched(int k, int tile, int mode, const GemmArgs* descs,
                                      const TileItem* items, int32_t n_items, uint32_t* counter,
                                      int grid, const PackedParams& pp, hipStream_t s) {
  FQT_K_DISPATCH(dispatch_batched, tile, descs, items, n_items, counter, grid, pp, s)
  return hipErrorInvalidValue;
}

// Occupancy of the batched kernel (workgroups per CU) for the persistent grid.
int packed_batched_occupancy(int k, int tile, int mode, uint32_t tbl_log2) {
  FQT_K_DISPATCH(dispatch_occupancy, tile, tbl_log2)
  return 1;
}

}  // namespace fqt
