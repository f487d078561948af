// Packed-FP64 GEMM over GF(p^4) for batches of small uneven products: one
// persistent launch in which every wave pulls 32 x 32 output tiles of any
// product from a queue and computes each one alone (packed tile id 15).
//
// Alg. 4 for every entry, as in k_gemm_f64.hip, with three choices made for
// products whose sides are a few dozen to a few hundred elements:
//  * No LDS for operands and no barrier: a wave loads its operands straight
//    into registers and converts them itself, so a tile costs only its own
//    work and edge tiles of every size need no shared staging.
//  * K-blocks of 4 NQG products with NQG fixed at compile time, so the block
//    steps sit at known places in a branch-free MFMA stream.  Lane group
//    g = l/16 takes k = 4 NQG s + NQG g + gk at MFMA step gk of block s:
//    the NQG consecutive elements of its A row segment, and NQG rows of B.
//    Summation order is free because every partial sum is an exact integer.
//  * Operands come through buffer resources bounded by the operand's last
//    byte: reads past it return 0 without a fault.  Rows of A at or past M
//    and columns of B at or past N only feed outputs that are never
//    stored; k at or past K inside the last block must be zero on one side,
//    so those B rows take an offset past the bound.
// On gfx950 every VALU instruction takes issue cycles from the SIMD that
// runs the FP64 MFMAs (measured: about 4 cycles per instruction beside 64
// per v_mfma_f64_16x16x4f64, with one or two waves per SIMD), so the kernel
// counts instructions: the DQT is one byte dot product (the element's
// index, as the byte offset of its entry), a clamp and an LDS read of the
// packed value from a table of the p^4 <= 81 elements' values built at
// launch by wave_dqt (a byte permutation for centring, two byte dot
// products, a shift-add and a conversion); a block step is two masks and
// two 64-bit adds per accumulator (digit sums), and the next block starts
// by passing the bias as the MFMA addend, so no accumulator is re-seeded.
//
// Epilogue: the digit sums D_j of all blocks give mu_j = D_j mod p, the
// coefficients of sum_l A_l B_l in GF(p)[X] (Alg. 2's mu, every block's
// digits read as bit fields since q = 2^7); Thm. 3's tables built for
// q = 0 mod p (Q_d the identity) reduce them modulo P.  Centred packing
// shifts every digit of every block by q/2: n_blocks * (q/2) mod p comes off
// every digit sum before its reduction.
//
// Work order, fixed on the host: products are dealt to the 8 XCDs (workgroup
// i runs on XCD i % 8 and each XCD has its own L2), longest first onto the
// lightest; the tiles of an XCD's products are dealt to its waves the same
// way.  A wave walks its own list: no queue atomics, and the operand loads
// of its next tile are in flight while the current tile's epilogue runs.

#include "fqt_direct.h"  // buffer-resource loads

namespace fqt {

namespace {

constexpr int kWaveKE = 4;           // bytes (coefficients) per element
constexpr int32_t kFarOffset = 1 << 30;  // past every operand bound (extents < 2^30)

template <int NQG>
struct WStage {
  uint32_t a[2][NQG];  // A rows m0 + 16 i + c, k = 4 NQG s + NQG g .. + NQG - 1
  uint32_t b[NQG][2];  // B rows 4 NQG s + NQG g + gk, columns n0 + 2c, n0 + 2c + 1
};

// mu = x mod p for x < 2^24 (p >= 2): floor(x/p) from one high multiply,
// the remainder from one 24-bit multiply-add
__device__ __forceinline__ uint32_t mod_p_24(uint32_t x, const FieldArgs& fa) {
  const uint32_t qq = __umulhi(x, fa.mod_magic);
  return (uint32_t)((int32_t)x + __mul24((int32_t)qq, -(int32_t)fa.p));
}

// DQT of one element (4 coefficient bytes in a word) at q = 2^7: a byte
// permutation to the offset form (c + h) mod p (the identity without
// centring), c0 + q c1 and c2 + q c3 as byte dot products, the offset
// -h (1 + q + q^2 + q^3) in the first one's addend, one shift-add.
__device__ __forceinline__ double wave_dqt(uint32_t w, const PackedParams& pp) {
  const uint32_t x = perm_b32(pp.lut_hi, pp.lut_lo, w);
  const uint32_t lo = __builtin_amdgcn_udot4(x, 0x00008001u, (uint32_t)pp.dqt_off, false);
  const uint32_t hi = __builtin_amdgcn_udot4(x, 0x80010000u, 0u, false);
  return (double)(int32_t)(lo + (hi << 14));
}

// The DQT by table: the element's index sum_j c_j p^j selects its packed
// value, built at launch from wave_dqt itself.  One byte dot product with
// the weights 8, 8p, 8p^2, 8p^3 (bytes for p <= 3) gives the entry's byte
// offset, clamped into the table.
struct DqtTable {
  const double* v;   // LDS, p^4 values
  uint32_t weights;  // bytes 8, 8p, 8p^2, 8p^3
  uint32_t last;     // byte offset of the last entry, 8 (p^4 - 1)
  __device__ __forceinline__ double operator()(uint32_t w) const {
    const uint32_t o = __builtin_amdgcn_udot4(w, weights, 0u, false);
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(v) +
                                            (o < last ? o : last));
  }
};

// Field element of the digit sums held in (E, T), q = 2^7, tables for
// q = 0 mod p.  kE and kO are the tile's constants for the even and the odd
// fields: in every field the non-negative offset that takes the centred
// shift off modulo p, and in kO also minus the 2^52 bits of the blocks added
// since the last fold (each field stays below 2^14: the host keeps room for
// the offset when it sets the folds).
__device__ __forceinline__ uint32_t digit_sums_elem(const BlockLanes<kWaveKE, 2>& st,
                                                    uint64_t kE, uint64_t kO,
                                                    const PackedParams& pp,
                                                    const uint32_t* __restrict__ Ls,
                                                    const uint32_t* __restrict__ Hs) {
  using BL = BlockLanes<kWaveKE, 2>;
  constexpr int ND = 2 * kWaveKE - 1;
  const uint64_t E = st.E + kE;
  const uint64_t O = st.T - st.E + kO;
  uint32_t il = 0, ih = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const uint32_t mu = mod_p_24(BL::field((d & 1) ? O : E, d), pp.fa);
    if (d < kWaveKE) il |= mu << (pp.fa.cb * d);
    if (d >= kWaveKE - 1) ih |= mu << (pp.fa.cb * (d - kWaveKE + 1));
  }
  const uint32_t tmask = (1u << pp.tbl_log2) - 1u;
  return add_bytes_mod_p(Ls[il & tmask], Hs[ih & tmask], pp.fa);
}

// Load context of one item: operand resources and this lane's offsets.
template <int NQG>
struct WCtx {
  __amdgpu_buffer_rsrc_t rsa, rsb;
  int32_t voa[2], vob[NQG];
  int64_t nb;     // K-blocks, at least 1 (K = 0: one block of zeros)
  int64_t K;
  int64_t bstep;  // bytes of B per block of K
};

template <int NQG>
__device__ __forceinline__ void make_ctx(const GemmArgs& g, int tm, int tn, WCtx<NQG>& x) {
  constexpr int KE = kWaveKE, KB = 4 * NQG;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, grp = lane >> 4;
  const int64_t m0 = (int64_t)tm * 32, n0 = (int64_t)tn * 32;
  // operand bounds: the last byte of A (M x K of lda) and of B (K x N of ldb)
  const uint32_t extA = g.K ? (uint32_t)(((g.M - 1) * g.lda + g.K) * KE) : 0u;
  const uint32_t extB = g.K ? (uint32_t)(((g.K - 1) * g.ldb + g.N) * KE) : 0u;
  x.rsa = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.A), (short)0, (int)extA,
                                            kBufferWord3);
  x.rsb = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.B), (short)0, (int)extB,
                                            kBufferWord3);
  auto clamp_off = [](int64_t off) { return (int32_t)(off < kFarOffset ? off : kFarOffset); };
#pragma unroll
  for (int i = 0; i < 2; ++i) x.voa[i] = clamp_off(((m0 + 16 * i + c) * g.lda + NQG * grp) * KE);
#pragma unroll
  for (int gk = 0; gk < NQG; ++gk)
    x.vob[gk] = clamp_off(((int64_t)(NQG * grp + gk) * g.ldb + n0 + 2 * c) * KE);
  x.K = g.K;
  x.nb = g.K > 0 ? (g.K + KB - 1) / KB : 1;
  x.bstep = (int64_t)KB * g.ldb * KE;
}

// Block s of an item into a stage: A segments, and B rows with k at or past
// K read as zero (the same loads for every block, no branch).
template <int NQG>
__device__ __forceinline__ void load_block(const WCtx<NQG>& x, int64_t s, WStage<NQG>& st) {
  constexpr int KE = kWaveKE, KB = 4 * NQG;
  const int grp = (threadIdx.x & 63) >> 4;
  const int32_t sa = (int32_t)(s * KB * KE), sb = (int32_t)(s * x.bstep);
  // k left in this block, in 32 bits (K < 2^30); may be <= 0
  int32_t krem = (int32_t)x.K - (int32_t)s * KB;
  krem = krem < KB ? krem : KB;
#pragma unroll
  for (int i = 0; i < 2; ++i) buf_load<NQG>(x.rsa, x.voa[i], sa, st.a[i]);
#pragma unroll
  for (int gk = 0; gk < NQG; ++gk)
    buf_load<2>(x.rsb, NQG * grp + gk < krem ? x.vob[gk] : kFarOffset, sb, st.b[gk]);
}

// One wave's list of items, in order.  The operand loads run two K-blocks
// ahead of the MFMAs across item boundaries, so the next item's first blocks
// arrive while the current item's epilogue runs.
template <int NQG>
__device__ __forceinline__ void wave_items(const GemmArgs* __restrict__ descs,
                                           const TileItem* __restrict__ items, int32_t beg,
                                           int32_t end, const PackedParams& pp,
                                           const uint32_t* __restrict__ Ls,
                                           const uint32_t* __restrict__ Hs, const DqtTable dq) {
  constexpr int KE = kWaveKE, TM = 2, TN = 2;
  static_assert(multi_block_b<KE>() == 7, "q = 2^7 for k = 4");
  using St = WStage<NQG>;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, grp = lane >> 4;

  auto item_args = [&](int32_t it, GemmArgs& g, int& tm, int& tn) {
    const TileItem ti = items[it];
    g = descs[__builtin_amdgcn_readfirstlane(ti.gemm)];
    tm = __builtin_amdgcn_readfirstlane(ti.tm);
    tn = __builtin_amdgcn_readfirstlane(ti.tn);
  };

  // load cursor: item lit, its next block lblk
  int32_t lit = beg;
  int64_t lblk = 0;
  WCtx<NQG> lc;
  {
    GemmArgs g;
    int tm, tn;
    item_args(lit, g, tm, tn);
    make_ctx<NQG>(g, tm, tn, lc);
  }
  auto load_next = [&](St& x) {
    if (lit < end) {
      load_block<NQG>(lc, lblk, x);
      if (++lblk == lc.nb) {
        lblk = 0;
        if (++lit < end) {
          GemmArgs g;
          int tm, tn;
          item_args(lit, g, tm, tn);
          make_ctx<NQG>(g, tm, tn, lc);
        }
      }
    }
  };

  auto convert = [&](const St& x, double (&av)[TM][NQG], double (&bv)[NQG][TN]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int e = 0; e < NQG; ++e) av[i][e] = dq(x.a[i][e]);
#pragma unroll
    for (int gk = 0; gk < NQG; ++gk)
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[gk][j] = dq(x.b[gk][j]);
  };

  const double bz = pp.centered ? pp.cbias : kTwo52;
  const v4d bias = {bz, bz, bz, bz};
  BlockLanes<KE, 2> st[TM][TN][4];
  auto clear_state = [&]() {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) st[i][j][v].clear();
  };
  clear_state();
  uint32_t nblk = 0, nadd = 0, nbound = 0;

  // compute cursor: item cit (arguments cg, ctm, ctn), block cblk of cnb
  int32_t cit = beg;
  int64_t cblk = 0;
  GemmArgs cg;
  int ctm, ctn;
  item_args(cit, cg, ctm, ctn);
  int64_t cnb = cg.K > 0 ? (cg.K + 4 * NQG - 1) / (4 * NQG) : 1;

  St stg[2];
  load_next(stg[0]);
  load_next(stg[1]);
  bool done = false;
  while (!done) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (done) break;
      double av[TM][NQG], bv[NQG][TN];
      convert(stg[u], av, bv);
      load_next(stg[u]);
      v4d acc[TM][TN];
      // a block starts from the bias, passed as the first MFMA's addend
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][0], bv[0][j], bias, 0, 0, 0);
#pragma unroll
      for (int gk = 1; gk < NQG; ++gk)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][gk], bv[gk][j], acc[i][j], 0, 0, 0);
      // block step: the block's digits into the digit sums
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) st[i][j][v].add(acc[i][j][v], pp.fa);
      ++nblk;
      ++nadd;
      if (++cblk < cnb) {
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
        continue;
      }
      // last block of the item: mu_j = D_j mod p with the centred shift
      // nblk (q/2) taken off every digit sum, L + H at q = 0 mod p, k bytes
      // per element
      uint64_t kE = 0, kO = (uint64_t)0 - (uint64_t)nadd * BlockLanes<KE, 2>::XB;
      if (pp.centered) {
        const uint32_t p = pp.fa.p;
        const uint32_t cc = (p - (nblk % p) * pp.dshift % p) % p;
#pragma unroll
        for (int d = 0; d < 2 * KE - 1; ++d) {
          if (d & 1) kO += (uint64_t)cc << (7 * d);
          else kE += (uint64_t)cc << (7 * d);
        }
      }
      // C through a buffer resource bounded by its last element: rows at or
      // past M lie past the bound, and columns at or past N take an offset
      // past it, so every store is issued and none needs a branch
      const int64_t m0 = (int64_t)ctm * 32, n0 = (int64_t)ctn * 32;
      const uint32_t extC = (uint32_t)(((cg.M - 1) * cg.ldc + cg.N) * KE);
      const auto rsc =
          __builtin_amdgcn_make_buffer_rsrc(cg.C, (short)0, (int)extC, kBufferWord3);
      const int32_t rstep = (int32_t)(4 * cg.ldc * KE);  // four rows
      int32_t cbase[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int64_t col = n0 + 2 * c + j;
        cbase[j] = col < cg.N ? (int32_t)(((m0 + grp) * cg.ldc + col) * KE) : kFarOffset;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const uint32_t e = digit_sums_elem(st[i][j][v], kE, kO, pp, Ls, Hs);
            __builtin_amdgcn_raw_buffer_store_b32(e, rsc, cbase[j] + (4 * i + v) * rstep, 0, 0);
          }
      clear_state();
      nblk = nadd = nbound = 0;
      cblk = 0;
      if (++cit >= end) {
        done = true;
      } else {
        item_args(cit, cg, ctm, ctn);
        cnb = cg.K > 0 ? (cg.K + 4 * NQG - 1) / (4 * NQG) : 1;
      }
    }
  }
}

// Items of wave w: items[wave_begin[w] .. wave_begin[w + 1]), in order.
// Three waves per SIMD; with NQG = 4 (p = 2) two, whose registers hold the
// larger stages without spilling.
template <int NQG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NQG == 4 ? 2 : 3))) void gemm_wave_batched_kernel(
    const GemmArgs* __restrict__ descs, const TileItem* __restrict__ items,
    const int32_t* __restrict__ wave_begin, PackedParams pp) {
  extern __shared__ uint32_t tabs[];
  __shared__ double dqt_tab[kWaveDqtEntries];
  uint32_t* Ls = tabs;
  uint32_t* Hs = tabs + (1 << pp.tbl_log2);
  load_tables(pp, Ls, Hs);
  const uint32_t p = pp.fa.p;
  const uint32_t ne = p * p * p * p;  // at most kWaveDqtEntries (checked on the host)
  for (uint32_t t = threadIdx.x; t < ne && t < (uint32_t)kWaveDqtEntries; t += blockDim.x) {
    uint32_t x = t, wd = 0;
#pragma unroll
    for (int j = 0; j < kWaveKE; ++j) {
      wd |= (x % p) << (8 * j);
      x /= p;
    }
    dqt_tab[t] = wave_dqt(wd, pp);
  }
  __syncthreads();
  DqtTable dq;
  dq.v = dqt_tab;
  dq.weights = 8u * (1u | (p << 8) | (p * p << 16) | (p * p * p << 24));  // 8 p^3 <= 216
  dq.last = 8u * ((ne < (uint32_t)kWaveDqtEntries ? ne : (uint32_t)kWaveDqtEntries) - 1u);
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  const int32_t beg = wave_begin[w], end = wave_begin[w + 1];
  if (beg < end) wave_items<NQG>(descs, items, beg, end, pp, Ls, Hs, dq);
}

template <int NQG>
hipError_t launch_wave(const GemmArgs* descs, const TileItem* items, const int32_t* wave_begin,
                       int grid, const PackedParams& pp, hipStream_t s) {
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL(gemm_wave_batched_kernel<NQG>, dim3(grid), dim3(256), dyn, s, descs, items,
                     wave_begin, pp);
  return hipGetLastError();
}

template <int NQG>
int occupancy_wave(uint32_t tbl_log2) {
  int blocks = 0;
  const size_t dyn = 2u * (1u << tbl_log2) * sizeof(uint32_t);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)gemm_wave_batched_kernel<NQG>, 256, dyn) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace

hipError_t launch_gemm_wave_batched(int nqg, const GemmArgs* descs, const TileItem* items,
                                    const int32_t* wave_begin, int grid, const PackedParams& pp,
                                    hipStream_t s) {
  switch (nqg) {
    case 1: return launch_wave<1>(descs, items, wave_begin, grid, pp, s);
    case 2: return launch_wave<2>(descs, items, wave_begin, grid, pp, s);
    case 3: return launch_wave<3>(descs, items, wave_begin, grid, pp, s);
    case 4: return launch_wave<4>(descs, items, wave_begin, grid, pp, s);
    default: return hipErrorInvalidValue;
  }
}

int wave_batched_occupancy(int nqg, uint32_t tbl_log2) {
  switch (nqg) {
    case 1: return occupancy_wave<1>(tbl_log2);
    case 2: return occupancy_wave<2>(tbl_log2);
    case 3: return occupancy_wave<3>(tbl_log2);
    case 4: return occupancy_wave<4>(tbl_log2);
    default: return 1;
  }
}

}  // namespace fqt
