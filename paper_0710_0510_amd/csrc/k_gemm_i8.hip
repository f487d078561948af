// Coefficient-wise INT8 GEMM over GF(p^k) on gfx950 MFMA (v_mfma_i32_16x16x64_i8).
//
// This is the delayed-reduction alternative of Section 6 applied to field
// elements: products of coefficients are accumulated without reduction in
// INT32 while n_d (p-1)^2 < 2^31 (eq. (3) with an unsigned representation),
// then reduced once.
//
// The reduction modulo the defining polynomial P is folded into B: the map
// a -> a*b on GF(p^k) = GF(p)[X]/(P) is GF(p)-linear with matrix rows
// (X^i b mod P), i < k.  Writing A' for A's bytes read as an M x (Kk) matrix
// (column l*k + i holds coefficient i of A[m][l]) and
//     B'[(l,i)][(n,s)] = coefficient s of X^i * B[l][n] mod P,
// one plain integer product C' = A' B' (M x Nk) gives, after a final mod p,
// exactly the coefficient bytes of C = AB in C's own layout.
//
// expand_b_kernel writes B' transposed (Nk rows of Kk bytes, zero padded to a
// multiple of 128 columns) so that both MFMA operands are 16 contiguous bytes
// per lane.  gemm_i8_kernel: workgroup = 2 x WGN waves (WGN = 2 or 4), wave
// tile 16TM x 16TN, K-tiles of 128 or 256 bytes double-buffered in LDS;
// operand layout of
// 16x16x64 i8: lane l supplies row l%16, bytes k = 16(l/16)..16(l/16)+15 of a
// 64-deep step (A and B use the same k order, so any order shared by both is
// correct); result element v of lane l sits at row 4(l/16)+v, column l%16.
// Tile ids 1..3 and 7..10 run expand_b_kernel and gemm_i8_kernel; ids 4..6 run
// gemm_i8f_kernel, which builds B'^T tile by tile in LDS instead.

#include "fqt_internal.h"

namespace fqt {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---- B -> B'^T expansion ------------------------------------------------------
//
// Row n*k + s of B'^T holds, at columns l*k .. l*k + k-1, coefficient s of
// X^i * B[l][n] mod P for i = 0..k-1: k bytes of the element's multiplication
// matrix, read from a table indexed like L and H (mt, stride mt_stride(k)).
// A workgroup expands a block of kExpandL = 128 (l) x kExpandN = 16 (n)
// elements: it stages the block's B bytes in LDS (rows l), then every thread
// writes whole runs of E consecutive elements (16 bytes; 12 for k = 3) of
// one output row, so consecutive threads store consecutive pieces of a row
// (128 k contiguous bytes per row and block; with 32 x 64 blocks, 32 k bytes
// per row, the 4096^3 GF(5^3) step took 755 us instead of 708 us).  Columns at
// or beyond KKpad (the padded row length) are not written; elements l >= K
// expand to zeros.

template <int KE>
struct EXP {
  static constexpr int L = kExpandL, NB = kExpandN;
  static constexpr int RB = NB * KE;               // B bytes of one block row
  static constexpr int RS = RB + 4;                // LDS row stride (bytes)
  static constexpr int E = KE == 3 ? 4 : 16 / KE;  // elements per output run
  static constexpr int RUN = E * KE;               // bytes per output run
  static constexpr int NRUN = L / E;               // runs per block row of B'^T
  static constexpr int MTS = (int)mt_stride(KE);
};

__device__ __forceinline__ void load_mt(const uint8_t* __restrict__ mt, uint32_t tbl_log2,
                                        uint32_t mts, uint8_t* __restrict__ lds) {
  const int words = (int)(((size_t)1 << tbl_log2) * mts / 4);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(mt);
  uint32_t* dst = reinterpret_cast<uint32_t*>(lds);
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

template <int KE>
__device__ __forceinline__ void expand_block(const uint8_t* __restrict__ B, int64_t ldb, int64_t K,
                                             int64_t N, const uint8_t* __restrict__ mts,
                                             uint32_t cb, uint32_t tmask, uint8_t* __restrict__ Bt,
                                             int64_t ldbt, int64_t KKpad, int64_t l0, int64_t n0,
                                             uint8_t* __restrict__ tile) {
  using X = EXP<KE>;
  // the block's B bytes, zero beyond row K and column N
  const bool al = ((((uintptr_t)B) | (uintptr_t)(ldb * KE)) & 3) == 0;
  const int64_t rowbytes = N * KE;
  for (int e = threadIdx.x; e < X::L * (X::RB / 4); e += blockDim.x) {
    const int r = e / (X::RB / 4), c4 = (e % (X::RB / 4)) * 4;
    const int64_t l = l0 + r, col = n0 * KE + c4;
    uint32_t w = 0;
    if (l < K) {
      const uint8_t* src = B + l * ldb * KE + col;
      if (al && col + 4 <= rowbytes) {
        w = *reinterpret_cast<const uint32_t*>(src);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (col + j < rowbytes) w |= (uint32_t)src[j] << (8 * j);
      }
    }
    *reinterpret_cast<uint32_t*>(tile + r * X::RS + c4) = w;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < X::NB * X::NRUN; t += blockDim.x) {
    const int n = t / X::NRUN, run = t % X::NRUN;
    const int64_t col0 = (l0 + run * X::E) * KE;  // first byte column of the run
    if (n0 + n >= N || col0 >= KKpad) continue;
    uint32_t ent[X::E][X::MTS / 4];
#pragma unroll
    for (int e = 0; e < X::E; ++e) {
      const uint8_t* eb = tile + (run * X::E + e) * X::RS + n * KE;
      uint32_t idx = 0;
#pragma unroll
      for (int j = 0; j < KE; ++j) idx |= (uint32_t)eb[j] << (cb * j);
      const uint32_t* m = reinterpret_cast<const uint32_t*>(mts + (size_t)(idx & tmask) * X::MTS);
#pragma unroll
      for (int w = 0; w < X::MTS / 4; ++w) ent[e][w] = m[w];
    }
#pragma unroll
    for (int s = 0; s < KE; ++s) {
      uint32_t out[X::RUN / 4];
#pragma unroll
      for (int w = 0; w < X::RUN / 4; ++w) out[w] = 0;
#pragma unroll
      for (int e = 0; e < X::E; ++e)
#pragma unroll
        for (int i = 0; i < KE; ++i) {
          const int src = s * KE + i, pos = e * KE + i;
          const uint32_t byte = (ent[e][src >> 2] >> (8 * (src & 3))) & 0xffu;
          out[pos >> 2] |= byte << (8 * (pos & 3));
        }
      uint8_t* dst = Bt + ((n0 + n) * KE + s) * ldbt + col0;
      if constexpr (X::RUN == 16) {
        // 16-byte runs never straddle the 128-byte padding
        *reinterpret_cast<uint4*>(dst) = make_uint4(out[0], out[1], out[2], out[3]);
      } else {
#pragma unroll
        for (int w = 0; w < X::RUN / 4; ++w)
          if (col0 + 4 * w < KKpad) reinterpret_cast<uint32_t*>(dst)[w] = out[w];
      }
    }
  }
}

template <int KE>
__global__ __launch_bounds__(256) void expand_b_kernel(const uint8_t* __restrict__ B, int64_t ldb,
                                                       int64_t K, int64_t N,
                                                       const uint8_t* __restrict__ mt,
                                                       uint32_t cb, uint32_t tbl_log2,
                                                       uint8_t* __restrict__ Bt, int64_t ldbt,
                                                       int64_t KKpad) {
  using X = EXP<KE>;
  __shared__ __align__(16) uint8_t tile[X::L * X::RS];
  extern __shared__ __align__(16) uint8_t mts[];
  load_mt(mt, tbl_log2, X::MTS, mts);
  expand_block<KE>(B, ldb, K, N, mts, cb, (1u << tbl_log2) - 1u, Bt, ldbt, KKpad,
                   (int64_t)blockIdx.x * X::L, (int64_t)blockIdx.y * X::NB, tile);
}

// Batched expansion: one workgroup per (product, 64 x 64 block) item.
template <int KE>
__global__ __launch_bounds__(256) void expand_b_batched_kernel(const I8Batch* __restrict__ gs,
                                                               const ExpandItem* __restrict__ items,
                                                               const uint8_t* __restrict__ mt,
                                                               uint32_t cb, uint32_t tbl_log2) {
  using X = EXP<KE>;
  __shared__ __align__(16) uint8_t tile[X::L * X::RS];
  extern __shared__ __align__(16) uint8_t mts[];
  load_mt(mt, tbl_log2, X::MTS, mts);
  const ExpandItem it = items[blockIdx.x];
  const I8Batch g = gs[it.gemm];
  expand_block<KE>(g.B, g.ldb, g.K, g.N, mts, cb, (1u << tbl_log2) - 1u,
                   const_cast<uint8_t*>(g.a.Bt), g.a.ldbt, g.a.KKpad, (int64_t)it.lb * X::L,
                   (int64_t)it.nb * X::NB, tile);
}

template <int KE>
static hipError_t launch_expand(const uint8_t* B, int64_t ldb, int64_t K, int64_t N,
                                const uint8_t* mt, uint32_t cb, uint32_t tbl_log2, uint8_t* Bt,
                                int64_t ldbt, int64_t KKpad, hipStream_t s) {
  using X = EXP<KE>;
  const int64_t lcols = (KKpad + KE - 1) / KE;  // elements covering the padded row
  const dim3 grid((unsigned)((lcols + X::L - 1) / X::L), (unsigned)((N + X::NB - 1) / X::NB));
  const size_t dyn = ((size_t)1 << tbl_log2) * X::MTS;
  hipLaunchKernelGGL(expand_b_kernel<KE>, grid, dim3(256), dyn, s, B, ldb, K, N, mt, cb, tbl_log2,
                     Bt, ldbt, KKpad);
  return hipGetLastError();
}

hipError_t launch_expand_b(int k, const uint8_t* B, int64_t ldb, int64_t K, int64_t N,
                           const uint8_t* mt, uint32_t cb, uint32_t tbl_log2, uint8_t* Bt,
                           int64_t ldbt, int64_t KKpad, hipStream_t s) {
  if (N == 0 || KKpad == 0) return hipSuccess;
  switch (k) {
    case 1: return launch_expand<1>(B, ldb, K, N, mt, cb, tbl_log2, Bt, ldbt, KKpad, s);
    case 2: return launch_expand<2>(B, ldb, K, N, mt, cb, tbl_log2, Bt, ldbt, KKpad, s);
    case 3: return launch_expand<3>(B, ldb, K, N, mt, cb, tbl_log2, Bt, ldbt, KKpad, s);
    case 4: return launch_expand<4>(B, ldb, K, N, mt, cb, tbl_log2, Bt, ldbt, KKpad, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- the INT8 GEMM --------------------------------------------------------------

// Workgroup = 2 x WGN waves (wave tile 16TM x 16TN): 4 waves, or 8 for the
// 128 x 256 and 256 x 256 tiles that halve the L2 traffic per output of
// large products.
template <int TM, int TN, int WGN = 2, int BK = 128>
struct I8T {
  static constexpr int NT = 128 * WGN;     // threads
  static constexpr int BM = 32 * TM, BN = 16 * TN * WGN;
  static constexpr int BKK = BK;           // bytes of K per tile (128 or 256)
  static constexpr int S = BKK + 16;       // LDS row stride (bytes): conflict-free b128 reads
  static constexpr int CA = BM * BKK / 16;  // 16-byte chunks of A per tile
  static constexpr int CB = BN * BKK / 16;
  static constexpr int RA = CA / NT, RB = CB / NT;
  static_assert(CA % NT == 0 && CB % NT == 0, "whole chunks per thread");
};

// exact x mod p for 0 <= x < 2^31 through binary64
__device__ __forceinline__ uint32_t mod_p_i32(int32_t x, uint32_t p, double inv_p) {
  const double xd = (double)x;
  const int32_t t = (int32_t)__builtin_floor(xd * inv_p);
  int32_t r = x - t * (int32_t)p;
  r += r < 0 ? (int32_t)p : 0;
  r -= r >= (int32_t)p ? (int32_t)p : 0;
  return (uint32_t)r;
}

// 16 bytes of row `row` starting at byte column `col` of a matrix with `ld`
// bytes per row and `rows` x `cols` valid bytes; missing bytes read as 0.
// align: 16 or 4 when every row start and every 16-byte column offset is
// aligned that far, else 1.
__device__ __forceinline__ uint4 load16(const uint8_t* base, int64_t ld, int64_t row, int64_t col,
                                        int64_t rows, int64_t cols, uint32_t align) {
  if (row < rows && col + 15 < cols) {
    const uint8_t* src = base + row * ld + col;
    if (align >= 16) return *reinterpret_cast<const uint4*>(src);
    if (align >= 4) {
      const uint32_t* w = reinterpret_cast<const uint32_t*>(src);
      return make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
  uint32_t w[4] = {0, 0, 0, 0};
  if (row < rows) {
    const uint8_t* src = base + row * ld;
    for (int j = 0; j < 16; ++j)
      if (col + j < cols) w[j >> 2] |= (uint32_t)src[col + j] << (8 * (j & 3));
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

template <int TM, int TN, int WGN, int BK>
__device__ __forceinline__ void i8_tile(
    const I8Args& a, int64_t m0, int64_t n0,
    uint8_t (*As)[I8T<TM, TN, WGN, BK>::BM * I8T<TM, TN, WGN, BK>::S],
    uint8_t (*Bs)[I8T<TM, TN, WGN, BK>::BN * I8T<TM, TN, WGN, BK>::S]) {
  using T = I8T<TM, TN, WGN, BK>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * 16 * TM, wn0 = (wave % WGN) * 16 * TN;
  // chunk r: row crow + r NT/CPR, bytes ccol..ccol+15 (CPR chunks per row)
  constexpr int CPR = T::BKK / 16, RSTEP = T::NT / CPR;
  const int crow = tid / CPR, ccol = (tid % CPR) * 16;

  v4i acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (v4i){0, 0, 0, 0};

  uint4 ra[T::RA], rb[T::RB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < T::RA; ++r)
      ra[r] = load16(a.A, a.lda, m0 + crow + RSTEP * r, k0 + ccol, a.M, a.KK, a.a_vec);
#pragma unroll
    for (int r = 0; r < T::RB; ++r)
      rb[r] = load16(a.Bt, a.ldbt, n0 + crow + RSTEP * r, k0 + ccol, a.NN, a.KKpad, 16u);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < T::RA; ++r)
      *reinterpret_cast<uint4*>(&As[buf][(crow + RSTEP * r) * T::S + ccol]) = ra[r];
#pragma unroll
    for (int r = 0; r < T::RB; ++r)
      *reinterpret_cast<uint4*>(&Bs[buf][(crow + RSTEP * r) * T::S + ccol]) = rb[r];
  };

  const int64_t nkt = (a.KK + T::BKK - 1) / T::BKK;
  if (nkt > 0) {
    gload(0);
    lstore(0);
    __syncthreads();
  }
  uint32_t since_red = 0;
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nkt) gload((kt + 1) * T::BKK);
#pragma unroll
    for (int ks = 0; ks < T::BKK / 64; ++ks) {
      v4i av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        av[i] = *reinterpret_cast<const v4i*>(
            &As[buf][(wm0 + 16 * i + (lane & 15)) * T::S + 64 * ks + 16 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bv[j] = *reinterpret_cast<const v4i*>(
            &Bs[buf][(wn0 + 16 * j + (lane & 15)) * T::S + 64 * ks + 16 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    // delayed reduction: reduce before the INT32 sums could reach 2^31
    if (a.red_tiles && ++since_red == a.red_tiles) {
      since_red = 0;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] = (int)mod_p_i32(acc[i][j][v], a.p, a.inv_p);
    }
    if (kt + 1 < nkt) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm0 + 16 * i + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn0 + 16 * j + (lane & 15);
        if (row < a.M && col < a.NN)
          a.C[row * a.ldc + col] = (uint8_t)mod_p_i32(acc[i][j][v], a.p, a.inv_p);
      }
}

template <int TM, int TN, int WGN, int BK>
__global__ __launch_bounds__(128 * WGN) void gemm_i8_kernel(I8Args a, int tiles_n,
                                                                       int ntiles) {
  using T = I8T<TM, TN, WGN, BK>;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][T::BM * T::S];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][T::BN * T::S];
  int tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
  i8_tile<TM, TN, WGN, BK>(a, (int64_t)(tile / tiles_n) * T::BM, (int64_t)(tile % tiles_n) * T::BN,
                       As, Bs);
}

// Persistent INT8 kernel over the tiles of a whole batch (atomic queue, the
// last workgroup out resets it for the next launch).
template <int TM, int TN, int WGN, int BK>
__global__ __launch_bounds__(128 * WGN) void gemm_i8_batched_kernel(
    const I8Batch* __restrict__ gs, const TileItem* __restrict__ items, int32_t n_items,
    uint32_t* counter) {
  using T = I8T<TM, TN, WGN, BK>;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][T::BM * T::S];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][T::BN * T::S];
  __shared__ int32_t cur;
  for (;;) {
    if (threadIdx.x == 0) cur = (int32_t)atomicAdd(&counter[0], 1u);
    __syncthreads();
    const int32_t it = cur;
    __syncthreads();
    if (it >= n_items) break;
    const TileItem ti = items[it];
    const I8Args a = gs[ti.gemm].a;
    i8_tile<TM, TN, WGN, BK>(a, (int64_t)ti.tm * T::BM, (int64_t)ti.tn * T::BN, As, Bs);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
  }
}

template <int TM, int TN, int WGN, int BK>
static hipError_t launch_i8(const I8Args& a, hipStream_t s) {
  using T = I8T<TM, TN, WGN, BK>;
  const int tiles_m = (int)((a.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((a.NN + T::BN - 1) / T::BN);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_i8_kernel<TM, TN, WGN, BK>), dim3(ntiles), dim3(T::NT), 0, s, a, tiles_n,
                     ntiles);
  return hipGetLastError();
}

template <int TM, int TN, int WGN, int BK>
static hipError_t launch_i8_batched(const I8Batch* gs, const TileItem* items, int32_t n,
                                    uint32_t* counter, int grid, hipStream_t s) {
  hipLaunchKernelGGL((gemm_i8_batched_kernel<TM, TN, WGN, BK>), dim3(grid),
                     dim3(I8T<TM, TN, WGN, BK>::NT), 0, s, gs, items, n, counter);
  return hipGetLastError();
}

template <int TM, int TN, int WGN, int BK>
static int occ_i8() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_i8_batched_kernel<TM, TN, WGN, BK>, I8T<TM, TN, WGN, BK>::NT,
          0) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

// INT8 tile ids of the two-kernel path: X(id, TM, TN, WGN, BK)
#define FQT_I8_TILES(X)                                                                  \
  X(1, 2, 2, 2, 128) X(2, 4, 4, 2, 128) X(3, 2, 4, 2, 128) X(7, 8, 4, 4, 128)            \
  X(8, 4, 4, 4, 128) X(9, 2, 2, 2, 256) X(10, 2, 4, 2, 256)

int i8_batched_occupancy(int tile) {
  switch (tile) {
#define FQT_I8_OCC(ID, TM, TN, WGN, BK) \
  case ID: return occ_i8<TM, TN, WGN, BK>();
    FQT_I8_TILES(FQT_I8_OCC)
#undef FQT_I8_OCC
    default: return 1;
  }
}

int i8_tile_m(int tile) {
  switch (tile) {
#define FQT_I8_BM(ID, TM, TN, WGN, BK) \
  case ID: return I8T<TM, TN, WGN, BK>::BM;
    FQT_I8_TILES(FQT_I8_BM)
#undef FQT_I8_BM
    default: return 0;
  }
}

int i8_tile_k(int tile) {
  switch (tile) {
#define FQT_I8_BK(ID, TM, TN, WGN, BK) \
  case ID: return BK;
    FQT_I8_TILES(FQT_I8_BK)
#undef FQT_I8_BK
    default: return 128;
  }
}

int i8_tile_n(int tile) {
  switch (tile) {
#define FQT_I8_BN(ID, TM, TN, WGN, BK) \
  case ID: return I8T<TM, TN, WGN, BK>::BN;
    FQT_I8_TILES(FQT_I8_BN)
#undef FQT_I8_BN
    default: return 0;
  }
}

hipError_t launch_gemm_i8_batched(int tile, const I8Batch* gs, const TileItem* items,
                                  int32_t n_items, uint32_t* counter, int grid, hipStream_t s) {
  switch (tile) {
#define FQT_I8_BATCHED(ID, TM, TN, WGN, BK) \
  case ID: return launch_i8_batched<TM, TN, WGN, BK>(gs, items, n_items, counter, grid, s);
    FQT_I8_TILES(FQT_I8_BATCHED)
#undef FQT_I8_BATCHED
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_expand_b_batched(int k, const I8Batch* gs, const ExpandItem* items,
                                   int32_t n_items, const uint8_t* mt, uint32_t cb,
                                   uint32_t tbl_log2, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const size_t dyn = ((size_t)1 << tbl_log2) * mt_stride((uint32_t)k);
  switch (k) {
#define FQT_EXP_CASE(KE)                                                                   \
  case KE:                                                                                 \
    hipLaunchKernelGGL(expand_b_batched_kernel<KE>, dim3(n_items), dim3(256), dyn, s, gs, \
                       items, mt, cb, tbl_log2);                                           \
    break;
    FQT_EXP_CASE(1) FQT_EXP_CASE(2) FQT_EXP_CASE(3) FQT_EXP_CASE(4)
#undef FQT_EXP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_i8(int tile, const I8Args& a, hipStream_t s) {
  switch (tile) {
#define FQT_I8_ONE(ID, TM, TN, WGN, BK) \
  case ID: return launch_i8<TM, TN, WGN, BK>(a, s);
    FQT_I8_TILES(FQT_I8_ONE)
#undef FQT_I8_ONE
    default: return hipErrorInvalidValue;
  }
}

// ---- INT8 GEMM with B'^T built in LDS (tile ids 4..6) -----------------------------
//
// The same product C' = A' B' without B' in HBM: every K-tile of BKE elements
// of l stages the raw bytes of its BKE x BNE block of B in LDS (coalesced
// words, rows l), then expands each element through the multiplication-matrix
// table (also in LDS) into the k rows (n, s) of the B'^T operand tile.  One
// kernel per product; HBM sees A, B and C only.  A K-tile is 128 bytes of A'
// (192 for k = 3, so that it holds whole elements); an output tile spans
// BNE = floor(BN / k) elements of N, BNE k columns of C' (for k = 3 the
// remaining B'^T rows stay zero and their columns are not stored).

template <int KE, int TM, int TN>
struct I8F {
  static constexpr int BM = 32 * TM, BN = 32 * TN;
  static constexpr int BKK = KE == 3 ? 192 : 128;  // bytes of A' per K-tile
  static constexpr int BKE = BKK / KE;              // elements of l per K-tile
  static constexpr int BNE = BN / KE;               // elements of n per output tile
  static constexpr int S = BKK + 16;                // operand row stride in LDS (bytes)
  static constexpr int CPR = BKK / 16;              // 16-byte chunks per A' row
  static constexpr int RA = BM * CPR / 256;         // A chunks per thread
  static constexpr int RW = (BNE * KE + 3) / 4;     // words of one raw B row segment
  static constexpr int RS = 4 * RW + 4;             // raw row stride in LDS (bytes)
  static constexpr int NRW = (BKE * RW + 255) / 256;
  static constexpr int E = KE == 3 ? 4 : 16 / KE;   // elements per expansion run
  static constexpr int RUN = E * KE;                // bytes per run
  static constexpr int NRUN = BKE / E;              // runs per B'^T row of a K-tile
  static constexpr int MTS = (int)mt_stride(KE);
  static constexpr size_t LDS = (size_t)2 * (BM + BN) * S + (size_t)BKE * RS;
  static_assert((BM * CPR) % 256 == 0 && BKE % E == 0 && BKK % 64 == 0, "tile shape");
};

// Table index of one element: coefficient j in bits [cb j, cb (j+1)).
template <int KE>
__device__ __forceinline__ uint32_t elem_index(const uint8_t* eb, uint32_t cb) {
  if constexpr (KE == 4) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(eb);
    return (w & 0xffu) | ((w >> 8) & 0xffu) << cb | ((w >> 16) & 0xffu) << (2 * cb) |
           (w >> 24) << (3 * cb);
  } else if constexpr (KE == 2) {
    const uint32_t w = *reinterpret_cast<const uint16_t*>(eb);
    return (w & 0xffu) | (w >> 8) << cb;
  } else {
    uint32_t idx = 0;
#pragma unroll
    for (int j = 0; j < KE; ++j) idx |= (uint32_t)eb[j] << (cb * j);
    return idx;
  }
}

template <int KE, int TM, int TN>
__device__ __forceinline__ void i8f_tile(const I8Batch& g, const uint8_t* __restrict__ mts,
                                         uint32_t cb, uint32_t tmask, int64_t m0, int64_t ne0,
                                         uint8_t (*As)[I8F<KE, TM, TN>::BM * I8F<KE, TM, TN>::S],
                                         uint8_t (*Bs)[I8F<KE, TM, TN>::BN * I8F<KE, TM, TN>::S],
                                         uint8_t* __restrict__ Rs) {
  using T = I8F<KE, TM, TN>;
  const I8Args& a = g.a;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 16 * TM, wn0 = (wave & 1) * 16 * TN;
  const int64_t rowbytes = g.N * KE, ldb = g.ldb * KE;
  const bool bal = ((((uintptr_t)g.B) | (uintptr_t)ldb) & 3) == 0;

  v4i acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (v4i){0, 0, 0, 0};

  uint4 ra[T::RA];
  uint32_t rw[T::NRW];
  auto gload = [&](int64_t kt) {
    const int64_t k0 = kt * T::BKK, l0 = kt * T::BKE;
#pragma unroll
    for (int r = 0; r < T::RA; ++r) {
      const int c = tid + 256 * r;
      ra[r] = load16(a.A, a.lda, m0 + c / T::CPR, k0 + (c % T::CPR) * 16, a.M, a.KK, a.a_vec);
    }
#pragma unroll
    for (int r = 0; r < T::NRW; ++r) {
      const int w = tid + 256 * r;
      const int64_t l = l0 + w / T::RW, col = ne0 * KE + 4 * (w % T::RW);
      uint32_t v = 0;
      if (w < T::BKE * T::RW && l < g.K) {
        const uint8_t* src = g.B + l * ldb + col;
        if (bal && col + 4 <= rowbytes) {
          v = *reinterpret_cast<const uint32_t*>(src);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (col + j < rowbytes) v |= (uint32_t)src[j] << (8 * j);
        }
      }
      rw[r] = v;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < T::RA; ++r) {
      const int c = tid + 256 * r;
      *reinterpret_cast<uint4*>(&As[buf][(c / T::CPR) * T::S + (c % T::CPR) * 16]) = ra[r];
    }
#pragma unroll
    for (int r = 0; r < T::NRW; ++r) {
      const int w = tid + 256 * r;
      if (w < T::BKE * T::RW)
        *reinterpret_cast<uint32_t*>(&Rs[(w / T::RW) * T::RS + 4 * (w % T::RW)]) = rw[r];
    }
  };
  // B'^T rows n k + s, columns e k + i of one run: coefficient s of X^i b
  auto expand = [&](int buf) {
    for (int t = tid; t < T::BNE * T::NRUN; t += 256) {
      const int n = t / T::NRUN, run = t % T::NRUN;
      uint32_t ent[T::E][T::MTS / 4];
#pragma unroll
      for (int e = 0; e < T::E; ++e) {
        const uint32_t idx = elem_index<KE>(Rs + (run * T::E + e) * T::RS + n * KE, cb);
        const uint32_t* m = reinterpret_cast<const uint32_t*>(mts + (size_t)(idx & tmask) * T::MTS);
#pragma unroll
        for (int w = 0; w < T::MTS / 4; ++w) ent[e][w] = m[w];
      }
#pragma unroll
      for (int s = 0; s < KE; ++s) {
        uint32_t out[(T::RUN + 3) / 4];
#pragma unroll
        for (int w = 0; w < (T::RUN + 3) / 4; ++w) out[w] = 0;
#pragma unroll
        for (int e = 0; e < T::E; ++e)
#pragma unroll
          for (int i = 0; i < KE; ++i) {
            const int src = s * KE + i, pos = e * KE + i;
            const uint32_t byte = (ent[e][src >> 2] >> (8 * (src & 3))) & 0xffu;
            out[pos >> 2] |= byte << (8 * (pos & 3));
          }
        uint8_t* dst = &Bs[buf][(n * KE + s) * T::S + run * T::RUN];
        if constexpr (T::RUN == 16) {
          *reinterpret_cast<uint4*>(dst) = make_uint4(out[0], out[1], out[2], out[3]);
        } else {
#pragma unroll
          for (int w = 0; w < T::RUN / 4; ++w) reinterpret_cast<uint32_t*>(dst)[w] = out[w];
        }
      }
    }
  };

  const int64_t nkt = (a.KK + T::BKK - 1) / T::BKK;
  if (nkt > 0) {
    gload(0);
    lstore(0);
    __syncthreads();
    expand(0);
    __syncthreads();
  }
  uint32_t since_red = 0;
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
    for (int ks = 0; ks < T::BKK / 64; ++ks) {
      v4i av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        av[i] = *reinterpret_cast<const v4i*>(
            &As[buf][(wm0 + 16 * i + (lane & 15)) * T::S + 64 * ks + 16 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bv[j] = *reinterpret_cast<const v4i*>(
            &Bs[buf][(wn0 + 16 * j + (lane & 15)) * T::S + 64 * ks + 16 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (a.red_tiles && ++since_red == a.red_tiles) {
      since_red = 0;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] = (int)mod_p_i32(acc[i][j][v], a.p, a.inv_p);
    }
    if (kt + 1 < nkt) {
      lstore(buf ^ 1);
      __syncthreads();
      expand(buf ^ 1);
    }
    __syncthreads();
  }

  const int64_t c0 = ne0 * KE;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm0 + 16 * i + 4 * (lane >> 4) + v;
        const int c = wn0 + 16 * j + (lane & 15);
        if (row < a.M && c < T::BNE * KE && c0 + c < a.NN)
          a.C[row * a.ldc + c0 + c] = (uint8_t)mod_p_i32(acc[i][j][v], a.p, a.inv_p);
      }
}

// Table to LDS and the B'^T rows no element expands into (k = 3) zeroed.
template <int KE, int TM, int TN>
__device__ __forceinline__ void i8f_setup(const uint8_t* __restrict__ mt, uint32_t tbl_log2,
                                          uint8_t* __restrict__ mts,
                                          uint8_t (*Bs)[I8F<KE, TM, TN>::BN * I8F<KE, TM, TN>::S]) {
  using T = I8F<KE, TM, TN>;
  load_mt(mt, tbl_log2, T::MTS, mts);
  constexpr int tail = (T::BN - T::BNE * KE) * T::S / 4;  // words per buffer
  if constexpr (tail > 0) {
    for (int w = threadIdx.x; w < 2 * tail; w += blockDim.x) {
      const int b = w / tail, o = w % tail;
      reinterpret_cast<uint32_t*>(&Bs[b][T::BNE * KE * T::S])[o] = 0;
    }
  }
}

template <int KE, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_i8f_kernel(I8Batch g, const uint8_t* __restrict__ mt,
                                                       uint32_t cb, uint32_t tbl_log2,
                                                       int tiles_n, int ntiles) {
  using T = I8F<KE, TM, TN>;
  __shared__ __align__(16) uint8_t As[2][T::BM * T::S];
  __shared__ __align__(16) uint8_t Bs[2][T::BN * T::S];
  __shared__ __align__(16) uint8_t Rs[T::BKE * T::RS];
  extern __shared__ __align__(16) uint8_t mts[];
  i8f_setup<KE, TM, TN>(mt, tbl_log2, mts, Bs);
  int tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
  i8f_tile<KE, TM, TN>(g, mts, cb, (1u << tbl_log2) - 1u, (int64_t)(tile / tiles_n) * T::BM,
                       (int64_t)(tile % tiles_n) * T::BNE, As, Bs, Rs);
}

// Persistent version over the tiles of a batch (atomic queue; the last
// workgroup out resets it for the next launch).
template <int KE, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_i8f_batched_kernel(const I8Batch* __restrict__ gs,
                                                               const TileItem* __restrict__ items,
                                                               int32_t n_items, uint32_t* counter,
                                                               const uint8_t* __restrict__ mt,
                                                               uint32_t cb, uint32_t tbl_log2) {
  using T = I8F<KE, TM, TN>;
  __shared__ __align__(16) uint8_t As[2][T::BM * T::S];
  __shared__ __align__(16) uint8_t Bs[2][T::BN * T::S];
  __shared__ __align__(16) uint8_t Rs[T::BKE * T::RS];
  extern __shared__ __align__(16) uint8_t mts[];
  __shared__ int32_t cur;
  i8f_setup<KE, TM, TN>(mt, tbl_log2, mts, Bs);
  for (;;) {
    if (threadIdx.x == 0) cur = (int32_t)atomicAdd(&counter[0], 1u);
    __syncthreads();
    const int32_t it = cur;
    __syncthreads();
    if (it >= n_items) break;
    const TileItem ti = items[it];
    i8f_tile<KE, TM, TN>(gs[ti.gemm], mts, cb, (1u << tbl_log2) - 1u, (int64_t)ti.tm * T::BM,
                         (int64_t)ti.tn * T::BNE, As, Bs, Rs);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
  }
}

// tile id -> (TM, TN); FN is a template taking <KE, TM, TN>
#define FQT_I8F_DISPATCH(tile, k, FN, ...)                            \
  switch ((tile) * 8 + (k)) {                                         \
    case 4 * 8 + 1: return FN<1, 2, 2>(__VA_ARGS__);                  \
    case 4 * 8 + 2: return FN<2, 2, 2>(__VA_ARGS__);                  \
    case 4 * 8 + 3: return FN<3, 2, 2>(__VA_ARGS__);                  \
    case 4 * 8 + 4: return FN<4, 2, 2>(__VA_ARGS__);                  \
    case 5 * 8 + 1: return FN<1, 4, 4>(__VA_ARGS__);                  \
    case 5 * 8 + 2: return FN<2, 4, 4>(__VA_ARGS__);                  \
    case 5 * 8 + 3: return FN<3, 4, 4>(__VA_ARGS__);                  \
    case 5 * 8 + 4: return FN<4, 4, 4>(__VA_ARGS__);                  \
    case 6 * 8 + 1: return FN<1, 2, 4>(__VA_ARGS__);                  \
    case 6 * 8 + 2: return FN<2, 2, 4>(__VA_ARGS__);                  \
    case 6 * 8 + 3: return FN<3, 2, 4>(__VA_ARGS__);                  \
    case 6 * 8 + 4: return FN<4, 2, 4>(__VA_ARGS__);                  \
    default: break;                                                   \
  }

template <int KE, int TM, int TN>
static size_t i8f_lds_of() { return I8F<KE, TM, TN>::LDS + 16; }
template <int KE, int TM, int TN>
static int i8f_bne_of() { return I8F<KE, TM, TN>::BNE; }
template <int KE, int TM, int TN>
static int i8f_bm_of() { return I8F<KE, TM, TN>::BM; }

size_t i8f_static_lds(int tile, int k) {
  FQT_I8F_DISPATCH(tile, k, i8f_lds_of)
  return 0;
}

int i8f_tile_n(int tile, int k) {
  FQT_I8F_DISPATCH(tile, k, i8f_bne_of)
  return 0;
}

int i8f_tile_m(int tile) { return tile == 5 ? 128 : 64; }

int i8f_k_bytes(int k) { return k == 3 ? 192 : 128; }

template <int KE, int TM, int TN>
static hipError_t launch_i8f(const I8Batch& g, const uint8_t* mt, uint32_t cb, uint32_t tbl_log2,
                             hipStream_t s) {
  using T = I8F<KE, TM, TN>;
  const int tiles_m = (int)((g.a.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((g.N + T::BNE - 1) / T::BNE);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  const size_t dyn = ((size_t)1 << tbl_log2) * T::MTS;
  hipLaunchKernelGGL((gemm_i8f_kernel<KE, TM, TN>), dim3(ntiles), dim3(256), dyn, s, g, mt, cb,
                     tbl_log2, tiles_n, ntiles);
  return hipGetLastError();
}

hipError_t launch_gemm_i8f(int tile, int k, const I8Batch& g, const uint8_t* mt, uint32_t cb,
                           uint32_t tbl_log2, hipStream_t s) {
  FQT_I8F_DISPATCH(tile, k, launch_i8f, g, mt, cb, tbl_log2, s)
  return hipErrorInvalidValue;
}

template <int KE, int TM, int TN>
static hipError_t launch_i8f_batched(const I8Batch* gs, const TileItem* items, int32_t n,
                                     uint32_t* counter, int grid, const uint8_t* mt, uint32_t cb,
                                     uint32_t tbl_log2, hipStream_t s) {
  const size_t dyn = ((size_t)1 << tbl_log2) * I8F<KE, TM, TN>::MTS;
  hipLaunchKernelGGL((gemm_i8f_batched_kernel<KE, TM, TN>), dim3(grid), dim3(256), dyn, s, gs,
                     items, n, counter, mt, cb, tbl_log2);
  return hipGetLastError();
}

hipError_t launch_gemm_i8f_batched(int tile, int k, const I8Batch* gs, const TileItem* items,
                                   int32_t n_items, uint32_t* counter, int grid,
                                   const uint8_t* mt, uint32_t cb, uint32_t tbl_log2,
                                   hipStream_t s) {
  FQT_I8F_DISPATCH(tile, k, launch_i8f_batched, gs, items, n_items, counter, grid, mt, cb,
                   tbl_log2, s)
  return hipErrorInvalidValue;
}

template <int KE, int TM, int TN>
static int occ_i8f(uint32_t tbl_log2) {
  int blocks = 0;
  const size_t dyn = ((size_t)1 << tbl_log2) * I8F<KE, TM, TN>::MTS;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_i8f_batched_kernel<KE, TM, TN>, 256, dyn) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

int i8f_batched_occupancy(int tile, int k, uint32_t tbl_log2) {
  FQT_I8F_DISPATCH(tile, k, occ_i8f, tbl_log2)
  return 1;
}

#undef FQT_I8F_DISPATCH

}  // namespace fqt
