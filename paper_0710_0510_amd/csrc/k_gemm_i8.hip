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
// per lane.  gemm_i8_kernel: workgroup = 2 x 2 waves, wave tile 16TM x 16TN,
// K-tiles of 128 bytes double-buffered in LDS; operand layout of
// 16x16x64 i8: lane l supplies row l%16, bytes k = 16(l/16)..16(l/16)+15 of a
// 64-deep step (A and B use the same k order, so any order shared by both is
// correct); result element v of lane l sits at row 4(l/16)+v, column l%16.

#include "fqt_internal.h"

namespace fqt {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---- B -> B'^T expansion ------------------------------------------------------

// Expand the 32 (l) x 32 (n) block of B at (l0, n0): output row n*k+s holds,
// at column l*k+i, coefficient s of X^i * B[l][n] mod P.
template <int KE>
__device__ __forceinline__ void expand_block(const uint8_t* __restrict__ B, int64_t ldb, int64_t K,
                                             int64_t N, uint32_t p, const PlainFieldArgs& pf,
                                             uint8_t* __restrict__ Bt, int64_t ldbt, int64_t l0,
                                             int64_t n0, uint8_t (*tile)[32 * KE + 4]) {
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int ll = e >> 5, nl = e & 31;  // consecutive threads -> consecutive n (coalesced)
    const int64_t l = l0 + ll, n = n0 + nl;
    uint32_t c[KE];
#pragma unroll
    for (int s = 0; s < KE; ++s) c[s] = 0;
    if (l < K && n < N) {
      const uint8_t* src = B + (l * ldb + n) * KE;
#pragma unroll
      for (int s = 0; s < KE; ++s) c[s] = src[s];
    }
    // row i of the multiplication matrix: X^i * b mod P, by repeated X-shifts
#pragma unroll
    for (int i = 0; i < KE; ++i) {
#pragma unroll
      for (int s = 0; s < KE; ++s) tile[nl * KE + s][ll * KE + i] = (uint8_t)c[s];
      // c <- X*c mod P: shift up, then X^k = -sum P_low[s] X^s
      const uint32_t top = c[KE - 1];
#pragma unroll
      for (int s = KE - 1; s > 0; --s) c[s] = (c[s - 1] + top * (p - pf.P_low[s])) % p;
      c[0] = (top * (p - pf.P_low[0])) % p;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * KE * 32 * KE; e += 256) {
    const int r = e / (32 * KE), cc = e % (32 * KE);
    const int64_t orow = n0 * KE + r;
    if (orow < N * KE) Bt[orow * ldbt + l0 * KE + cc] = tile[r][cc];
  }
}

template <int KE>
__global__ __launch_bounds__(256) void expand_b_kernel(const uint8_t* __restrict__ B, int64_t ldb,
                                                       int64_t K, int64_t N, uint32_t p,
                                                       PlainFieldArgs pf,
                                                       uint8_t* __restrict__ Bt, int64_t ldbt) {
  __shared__ uint8_t tile[32 * KE][32 * KE + 4];
  expand_block<KE>(B, ldb, K, N, p, pf, Bt, ldbt, (int64_t)blockIdx.x * 32,
                   (int64_t)blockIdx.y * 32, tile);
}

// Batched expansion: one workgroup per (product, 32 x 32 block) item.
template <int KE>
__global__ __launch_bounds__(256) void expand_b_batched_kernel(const I8Batch* __restrict__ gs,
                                                               const ExpandItem* __restrict__ items,
                                                               uint32_t p, PlainFieldArgs pf) {
  __shared__ uint8_t tile[32 * KE][32 * KE + 4];
  const ExpandItem it = items[blockIdx.x];
  const I8Batch g = gs[it.gemm];
  expand_block<KE>(g.B, g.ldb, g.K, g.N, p, pf, const_cast<uint8_t*>(g.a.Bt), g.a.ldbt,
                   (int64_t)it.lb * 32, (int64_t)it.nb * 32, tile);
}

template <int KE>
static hipError_t launch_expand(const uint8_t* B, int64_t ldb, int64_t K, int64_t N, uint32_t p,
                                const PlainFieldArgs& pf, uint8_t* Bt, int64_t ldbt,
                                int64_t Kpad, hipStream_t s) {
  const dim3 grid((unsigned)(Kpad / 32), (unsigned)((N + 31) / 32));
  hipLaunchKernelGGL(expand_b_kernel<KE>, grid, dim3(256), 0, s, B, ldb, K, N, p, pf, Bt, ldbt);
  return hipGetLastError();
}

hipError_t launch_expand_b(int k, const uint8_t* B, int64_t ldb, int64_t K, int64_t N,
                           uint32_t p, const PlainFieldArgs& pf, uint8_t* Bt, int64_t ldbt,
                           int64_t Kpad, hipStream_t s) {
  if (K == 0 || N == 0) return hipSuccess;
  switch (k) {
    case 1: return launch_expand<1>(B, ldb, K, N, p, pf, Bt, ldbt, Kpad, s);
    case 2: return launch_expand<2>(B, ldb, K, N, p, pf, Bt, ldbt, Kpad, s);
    case 3: return launch_expand<3>(B, ldb, K, N, p, pf, Bt, ldbt, Kpad, s);
    case 4: return launch_expand<4>(B, ldb, K, N, p, pf, Bt, ldbt, Kpad, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- the INT8 GEMM --------------------------------------------------------------

template <int TM, int TN>
struct I8T {
  static constexpr int BM = 32 * TM, BN = 32 * TN;
  static constexpr int BKK = 128;          // bytes of K per tile
  static constexpr int S = BKK + 16;       // LDS row stride (bytes): conflict-free b128 reads
  static constexpr int CA = BM * BKK / 16;  // 16-byte chunks of A per tile
  static constexpr int CB = BN * BKK / 16;
  static constexpr int RA = CA / 256, RB = CB / 256;
  static_assert(CA % 256 == 0 && CB % 256 == 0, "whole chunks per thread");
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

template <int TM, int TN>
__device__ __forceinline__ void i8_tile(const I8Args& a, int64_t m0, int64_t n0,
                                        uint8_t (*As)[I8T<TM, TN>::BM * I8T<TM, TN>::S],
                                        uint8_t (*Bs)[I8T<TM, TN>::BN * I8T<TM, TN>::S]) {
  using T = I8T<TM, TN>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 16 * TM, wn0 = (wave & 1) * 16 * TN;
  const int crow = tid >> 3, ccol = (tid & 7) * 16;  // chunk r: row crow + 32r, bytes ccol..+15

  v4i acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (v4i){0, 0, 0, 0};

  uint4 ra[T::RA], rb[T::RB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < T::RA; ++r)
      ra[r] = load16(a.A, a.lda, m0 + crow + 32 * r, k0 + ccol, a.M, a.KK, a.a_vec);
#pragma unroll
    for (int r = 0; r < T::RB; ++r)
      rb[r] = load16(a.Bt, a.ldbt, n0 + crow + 32 * r, k0 + ccol, a.NN, a.KKpad, 16u);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < T::RA; ++r)
      *reinterpret_cast<uint4*>(&As[buf][(crow + 32 * r) * T::S + ccol]) = ra[r];
#pragma unroll
    for (int r = 0; r < T::RB; ++r)
      *reinterpret_cast<uint4*>(&Bs[buf][(crow + 32 * r) * T::S + ccol]) = rb[r];
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

template <int TM, int TN>
__global__ __launch_bounds__(256) void gemm_i8_kernel(I8Args a, int tiles_n, int ntiles) {
  using T = I8T<TM, TN>;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][T::BM * T::S];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][T::BN * T::S];
  int tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
  i8_tile<TM, TN>(a, (int64_t)(tile / tiles_n) * T::BM, (int64_t)(tile % tiles_n) * T::BN, As, Bs);
}

// Persistent INT8 kernel over the tiles of a whole batch (atomic queue, the
// last workgroup out resets it for the next launch).
template <int TM, int TN>
__global__ __launch_bounds__(256) void gemm_i8_batched_kernel(const I8Batch* __restrict__ gs,
                                                              const TileItem* __restrict__ items,
                                                              int32_t n_items, uint32_t* counter) {
  using T = I8T<TM, TN>;
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
    i8_tile<TM, TN>(a, (int64_t)ti.tm * T::BM, (int64_t)ti.tn * T::BN, As, Bs);
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

template <int TM, int TN>
static hipError_t launch_i8(const I8Args& a, hipStream_t s) {
  using T = I8T<TM, TN>;
  const int tiles_m = (int)((a.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((a.NN + T::BN - 1) / T::BN);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_i8_kernel<TM, TN>), dim3(ntiles), dim3(256), 0, s, a, tiles_n, ntiles);
  return hipGetLastError();
}

template <int TM, int TN>
static hipError_t launch_i8_batched(const I8Batch* gs, const TileItem* items, int32_t n,
                                    uint32_t* counter, int grid, hipStream_t s) {
  hipLaunchKernelGGL((gemm_i8_batched_kernel<TM, TN>), dim3(grid), dim3(256), 0, s, gs, items, n,
                     counter);
  return hipGetLastError();
}

template <int TM, int TN>
static int occ_i8() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_i8_batched_kernel<TM, TN>, 256, 0) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

int i8_batched_occupancy(int tile) {
  switch (tile) {
    case 1: return occ_i8<2, 2>();
    case 2: return occ_i8<4, 4>();
    case 3: return occ_i8<2, 4>();
    default: return 1;
  }
}

hipError_t launch_gemm_i8_batched(int tile, const I8Batch* gs, const TileItem* items,
                                  int32_t n_items, uint32_t* counter, int grid, hipStream_t s) {
  switch (tile) {
    case 1: return launch_i8_batched<2, 2>(gs, items, n_items, counter, grid, s);
    case 2: return launch_i8_batched<4, 4>(gs, items, n_items, counter, grid, s);
    case 3: return launch_i8_batched<2, 4>(gs, items, n_items, counter, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_expand_b_batched(int k, const I8Batch* gs, const ExpandItem* items,
                                   int32_t n_items, uint32_t p, const PlainFieldArgs& pf,
                                   hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  switch (k) {
    case 1: hipLaunchKernelGGL(expand_b_batched_kernel<1>, dim3(n_items), dim3(256), 0, s, gs, items, p, pf); break;
    case 2: hipLaunchKernelGGL(expand_b_batched_kernel<2>, dim3(n_items), dim3(256), 0, s, gs, items, p, pf); break;
    case 3: hipLaunchKernelGGL(expand_b_batched_kernel<3>, dim3(n_items), dim3(256), 0, s, gs, items, p, pf); break;
    case 4: hipLaunchKernelGGL(expand_b_batched_kernel<4>, dim3(n_items), dim3(256), 0, s, gs, items, p, pf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_i8(int tile, const I8Args& a, hipStream_t s) {
  switch (tile) {
    case 1: return launch_i8<2, 2>(a, s);
    case 2: return launch_i8<4, 4>(a, s);
    case 3: return launch_i8<2, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fqt
