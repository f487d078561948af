// Coefficient-wise INT8 GEMM over GF(p^4) for batches of small uneven
// products (INT8 tile id 11): one workgroup per column strip of 16 output
// elements of one product, sweeping all of its rows.
//
// Same product as k_gemm_i8.hip, C' = A' B' over int8 with INT32
// accumulation and one final reduction mod p (eq. (3)'s delayed reduction),
// the reduction mod P folded into B: B'[(l, i)][(n, s)] = coefficient s of
// X^i B[l][n] mod P.  What changes is where B' lives: for each K-tile the
// workgroup expands the strip's B elements through the multiplication-matrix
// table into LDS once, and every row of the product (up to 256 at a time)
// multiplies against that copy.  B' never reaches HBM, and the expansion
// costs one table read per B element per 256 rows.
//
// Layout.  A K-tile is 64 elements of K (256 bytes of A' and of a B' row).
// LDS row (s, n) holds coefficient s of X^i B[l][n] mod P at byte 4 l + i.
// MFMA v_mfma_i32_16x16x64_i8: lane l supplies row l%16 and bytes
// 16 (l/16) .. + 15 of a 64-byte k-step for both operands; result element v
// of lane l sits at row 4 (l/16) + v, column l%16.  Column block j of the
// MFMAs is coefficient s = j and column c is element n0 + c, so one lane ends
// holding all 4 coefficients of one output element: one word store.
// Rows: chunks of 32 (two MFMA row blocks); wave w takes chunks w and w + 4
// of each group of 256 rows, chunks past M are skipped.
// Operands come through buffer resources bounded by their last byte: rows of
// A past M read 0, B rows past K read 0 (element 0 expands to zeros), so only
// outputs that are never stored see anything else.

#include "fqt_direct.h"  // buffer-resource loads

namespace fqt {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int kCsK = 64;              // elements of K per K-tile
constexpr int kCsRow = 4 * kCsK + 16;  // LDS bytes per B' row (padding: conflict-free reads)
constexpr int kCsN = 16;              // output elements per strip

struct CsItem {
  int32_t gemm, nc, pad0, pad1;  // product, strip (elements 16 nc .. 16 nc + 15)
};

// x mod p for 0 <= x < 2^25 (small accumulators)
__device__ __forceinline__ uint32_t cs_mod_small(int32_t x, uint32_t magic, uint32_t p) {
  const uint32_t q = __umulhi((uint32_t)x, magic);
  return (uint32_t)(x - __mul24((int32_t)q, (int32_t)p));
}

// exact x mod p for 0 <= x < 2^31 through binary64
__device__ __forceinline__ uint32_t cs_mod_big(int32_t x, uint32_t p, double inv_p) {
  const int32_t t = (int32_t)__builtin_floor((double)x * inv_p);
  int32_t r = x - t * (int32_t)p;
  r += r < 0 ? (int32_t)p : 0;
  r -= r >= (int32_t)p ? (int32_t)p : 0;
  return (uint32_t)r;
}

struct CsParams {
  uint32_t p, cb, tmask, magic;
  uint32_t red_tiles;  // K-tiles between reductions mod p (0: never)
  double inv_p;
};

// One strip: C[0 .. M)[n0 .. n0 + 16) of product g.  SMALL: every final
// accumulator stays below 2^25, so the epilogue takes the cheap reduction
// (a compile-time choice: a run-time one branches around every accumulator).
template <bool SMALL>
__device__ __forceinline__ void cs_strip(const GemmArgs& g, int64_t n0, const CsParams& cp,
                                         const uint8_t* __restrict__ mts,
                                         uint8_t (*Bs)[64 * kCsRow]) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, grp = lane >> 4;
  const int64_t K = g.K;
  const uint32_t extA = K ? (uint32_t)(((g.M - 1) * g.lda + K) * 4) : 0u;
  const uint32_t extB = K ? (uint32_t)(((K - 1) * g.ldb + g.N) * 4) : 0u;
  const auto rsa = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.A), (short)0,
                                                     (int)extA, kBufferWord3);
  const auto rsb = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.B), (short)0,
                                                     (int)extB, kBufferWord3);
  const int64_t nkt = K > 0 ? (K + kCsK - 1) / kCsK : 0;
  // B elements this thread expands per K-tile: l = tid / 16 + 16 r, n = tid % 16
  const int bl = tid >> 4, bn = tid & 15;
  auto clamp_off = [](int64_t off) { return (int32_t)(off < (1 << 30) ? off : (1 << 30)); };
  const int32_t vob = clamp_off(((int64_t)bl * g.ldb + n0 + bn) * 4);
  const int32_t lstep = (int32_t)(16 * g.ldb * 4);  // bytes between this thread's rows

  for (int64_t rg = 0; rg < g.M; rg += 256) {  // row groups of 256
    // this wave's chunks of 32 rows: rg + 32 w and rg + 32 (w + 4)
    const int64_t r0 = rg + 32 * wave, r1 = rg + 32 * (wave + 4);
    const bool c0 = r0 < g.M, c1 = r1 < g.M;
    int32_t voa[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        voa[h][rb] = clamp_off(((h ? r1 : r0) + 16 * rb + c) * g.lda * 4 + 16 * grp);
    v4i acc[2][2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[h][rb][j] = (v4i){0, 0, 0, 0};

    uint32_t rbw[4];  // raw B elements of the next K-tile
    auto bload = [&](int64_t kt) {
      const int32_t so = (int32_t)(kt * kCsK * g.ldb * 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        uint32_t w[1];
        buf_load<1>(rsb, vob + r * lstep, so, w);
        rbw[r] = w[0];
      }
    };
    // element (l, n) -> LDS rows (s, n), bytes 4 l .. 4 l + 3: row s of its
    // multiplication matrix (coefficient s of X^i b for i = 0..3)
    auto expand = [&](int buf) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t w = rbw[r];
        const uint32_t idx = ((w & 0xffu) | ((w >> 8) & 0xffu) << cp.cb |
                              ((w >> 16) & 0xffu) << (2 * cp.cb) | (w >> 24) << (3 * cp.cb)) &
                             cp.tmask;
        const uint4 m = *reinterpret_cast<const uint4*>(mts + (size_t)idx * 16);
        const int l = bl + 16 * r;
        uint8_t* dst = &Bs[buf][bn * kCsRow + 4 * l];
        *reinterpret_cast<uint32_t*>(dst + 0 * 16 * kCsRow) = m.x;
        *reinterpret_cast<uint32_t*>(dst + 1 * 16 * kCsRow) = m.y;
        *reinterpret_cast<uint32_t*>(dst + 2 * 16 * kCsRow) = m.z;
        *reinterpret_cast<uint32_t*>(dst + 3 * 16 * kCsRow) = m.w;
      }
    };

    // A' operands, a ring of four 64-byte k-steps per chunk and row block,
    // refilled three k-steps ahead (across K-tiles)
    uint32_t ra[4][2][2][4];
    auto aload = [&](int st, int64_t kt, int ks) {
      const int32_t sa = (int32_t)(kt * kCsK * 4 + 64 * ks);  // past the bound: zeros
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (h ? c1 : c0) {
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) buf_load<4>(rsa, voa[h][rb], sa, ra[st][h][rb]);
        }
    };
    if (nkt > 0) {
      bload(0);
      aload(0, 0, 0);
      aload(1, 0, 1);
      aload(2, 0, 2);
      expand(0);
    }
    __syncthreads();
    uint32_t since_red = 0;
    for (int64_t kt = 0; kt < nkt; ++kt) {
      const int buf = (int)(kt & 1);
      if (kt + 1 < nkt) bload(kt + 1);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        if (ks == 0) aload(3, kt, 3);
        else aload(ks - 1, kt + 1, ks - 1);
        v4i bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bv[j] = *reinterpret_cast<const v4i*>(
              &Bs[buf][(16 * j + c) * kCsRow + 64 * ks + 16 * grp]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!(h ? c1 : c0)) continue;
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            const v4i av = (v4i){(int)ra[ks][h][rb][0], (int)ra[ks][h][rb][1],
                                 (int)ra[ks][h][rb][2], (int)ra[ks][h][rb][3]};
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[h][rb][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv[j], acc[h][rb][j], 0,
                                                                     0, 0);
          }
        }
      }
      // delayed reduction: reduce before the INT32 sums could reach 2^31
      if (cp.red_tiles && ++since_red == cp.red_tiles) {
        since_red = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                acc[h][rb][j][v] = (int)cs_mod_big(acc[h][rb][j][v], cp.p, cp.inv_p);
      }
      if (kt + 1 < nkt) expand(buf ^ 1);
      __syncthreads();
    }

    // epilogue: lane (c, grp) holds the 4 coefficients of C[row][n0 + c]
    const int64_t col = n0 + c;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!(h ? c1 : c0)) continue;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = (h ? r1 : r0) + 16 * rb + 4 * grp + v;
          uint32_t e = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int32_t x = acc[h][rb][j][v];
            const uint32_t m = SMALL ? cs_mod_small(x, cp.magic, cp.p)
                                     : cs_mod_big(x, cp.p, cp.inv_p);
            e |= m << (8 * j);
          }
          if (row < g.M && col < g.N) store_elem<4>(g.C + (row * g.ldc + col) * 4, e);
        }
    }
  }
}

// Strips of workgroup w: items[wg_begin[w] .. wg_begin[w + 1]), in order.
template <bool SMALL>
__global__ __launch_bounds__(256) void gemm_i8cs_batched_kernel(
    const GemmArgs* __restrict__ descs, const CsItem* __restrict__ items,
    const int32_t* __restrict__ wg_begin, const uint8_t* __restrict__ mt, uint32_t tbl_log2,
    CsParams cp) {
  __shared__ __align__(16) uint8_t Bs[2][64 * kCsRow];
  extern __shared__ __align__(16) uint8_t mts[];
  {
    const int words = (int)(((size_t)1 << tbl_log2) * 16 / 4);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(mt);
    uint32_t* dst = reinterpret_cast<uint32_t*>(mts);
    for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int32_t beg = wg_begin[blockIdx.x], end = wg_begin[blockIdx.x + 1];
  for (int32_t it = beg; it < end; ++it) {
    const CsItem ci = items[it];
    const GemmArgs g = descs[__builtin_amdgcn_readfirstlane(ci.gemm)];
    cs_strip<SMALL>(g, (int64_t)__builtin_amdgcn_readfirstlane(ci.nc) * kCsN, cp, mts, Bs);
    __syncthreads();  // the next strip's first expansion reuses buffer 0
  }
}

}  // namespace

size_t i8cs_lds_bytes(uint32_t tbl_log2) {
  return (size_t)2 * 64 * kCsRow + ((size_t)1 << tbl_log2) * 16;
}

int i8cs_occupancy(uint32_t tbl_log2) {
  int blocks = 0;
  const size_t dyn = ((size_t)1 << tbl_log2) * 16;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_i8cs_batched_kernel<true>, 256, dyn) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

hipError_t launch_gemm_i8cs_batched(const GemmArgs* descs, const int32_t* items_raw,
                                    const int32_t* wg_begin, int grid, const uint8_t* mt,
                                    uint32_t tbl_log2, uint32_t p, uint32_t cb,
                                    uint32_t red_tiles, uint32_t small, hipStream_t s) {
  CsParams cp;
  cp.p = p;
  cp.cb = cb;
  cp.tmask = (1u << tbl_log2) - 1u;
  cp.magic = (uint32_t)(((1ull << 32) + p - 1) / p);
  cp.red_tiles = red_tiles;
  cp.inv_p = 1.0 / (double)p;
  const size_t dyn = ((size_t)1 << tbl_log2) * 16;
  if (small)
    hipLaunchKernelGGL(gemm_i8cs_batched_kernel<true>, dim3(grid), dim3(256), dyn, s, descs,
                       reinterpret_cast<const CsItem*>(items_raw), wg_begin, mt, tbl_log2, cp);
  else
    hipLaunchKernelGGL(gemm_i8cs_batched_kernel<false>, dim3(grid), dim3(256), dyn, s, descs,
                       reinterpret_cast<const CsItem*>(items_raw), wg_begin, mt, tbl_log2, cp);
  return hipGetLastError();
}

}  // namespace fqt
