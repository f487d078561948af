// Register-direct packed-FP64 GEMM tile over GF(p^k) on gfx950 MFMA: the same
// Alg. 4 pipeline as k_gemm_f64.hip (DQT on load, exact FP64 contraction,
// REDQ + L/H tables), with no LDS staging of the operands and no barrier in
// the K loop.  Every wave loads its MFMA operands straight from global memory.
//
// Why that is possible: the contraction is exact, so any order of the
// products over k, and any numbering of a wave's output columns, gives the
// same integers.  We pick both so that every lane's operands are contiguous:
//   * K-step s = 16 consecutive k; lane group g = l/16 of the wave takes
//     k = 16s + 4g + gk at MFMA step gk (0..3), i.e. the 4 consecutive
//     elements 16s + 4g .. 16s + 4g + 3 of its A row over the 4 steps;
//   * MFMA block j (0..TN-1) of the wave's column strip holds output column
//     wn0 + TN*c + j at MFMA column c = l%16, so lane l reads the TN
//     consecutive elements wn0 + TN*c .. + TN-1 of one B row, and holds the
//     same TN consecutive outputs of one row at the end.
// For k = 2 and TN = 4 every operand load is 8 bytes per lane, and 16 lanes
// read one 128-byte run of a B row.
//
// Workgroup = 4 or 8 waves = SP waves side by side x SK waves splitting the
// K-steps (SK = 1, 2, 4); with 8 waves every SIMD runs two, so one wave's
// DQT and loads issue while the other's MFMAs occupy the matrix core.  With SK > 1 the waves of one output tile run
// through disjoint K ranges and combine their (single-block, biased)
// accumulators in LDS at the end: partial sums r_w are exact integers and
// 2^52 + sum r_w stays exact while the total obeys eq. (2).  Accumulator
// element v of MFMA row-block i (output rows 16i + l/16 + 4v) is owned by
// split-K wave (4i + v) % SK, which adds the others' partials and finishes
// those outputs.
//
// MFMA 16x16x4 f64 lane layout: A row l%16, k l/16; B k l/16, column l%16;
// D element v at row l/16 + 4v, column l%16.
//
// Operands are either k coefficient bytes per element (DQT by shifts on load)
// or, with LOG, one 16-bit discrete-log code per element (Alg. 4: the packed
// value comes from a table lookup, and L and H return codes that are added
// with the Zech table).
#pragma once

#include <type_traits>

#include "fqt_packed.h"

namespace fqt {

typedef double v4d __attribute__((ext_vector_type(4)));

// Tile geometry; EB = bytes per operand element.
template <int EB, int TM, int TN, int SK, int NWV>
struct DT {
  static constexpr int SP = NWV / SK;          // waves side by side
  static constexpr int WGM = SP >= 2 ? 2 : 1;  // ... as WGM x WGN wave tiles
  static constexpr int WGN = SP / WGM;
  static constexpr int WM = 16 * TM, WN = 16 * TN;
  static constexpr int BM = WM * WGM, BN = WN * WGN;
  static constexpr int BW = TN * EB / 4;  // words of one lane's B row segment
  // LDS doubles for combining split-K partial accumulators
  static constexpr int RED = SK > 1 ? SP * TM * TN * (SK - 1) * 256 : 1;
  static_assert((TN * EB) % 4 == 0, "B row segments are whole words");
  static_assert((NWV == 4 || NWV == 8) && (SK == 1 || SK == 2 || SK == 4) && SP <= 4,
                "4 or 8 waves: up to 4 side by side, up to 4 splitting K");
};

// Raw operand bytes of one K-step of one lane (EB bytes per element).
template <int EB, int TM, int TN>
struct DStage {
  uint32_t a[TM][EB];          // A rows wm0+16i+c, k = 16s+4g .. +3
  uint32_t b[4][TN * EB / 4];  // B rows 16s+4g+gk, columns wn0+TN*c .. +TN-1
};

// Operand words through a buffer resource: voff is the lane's byte offset,
// soff a wave-uniform one (the K-step advance), both below 2^31.
template <int NW>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t r, int32_t voff, int32_t soff,
                                         uint32_t (&out)[NW]) {
  if constexpr (NW == 1) {
    out[0] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  } else if constexpr (NW == 2) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    out[0] = v[0];
    out[1] = v[1];
  } else if constexpr (NW == 3) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
  } else {
    static_assert(NW == 4, "1 to 4 words");
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    out[3] = v[3];
  }
}

// gfx9 buffer resource word 3 (raw, untyped 32-bit data)
constexpr int kBufferWord3 = 0x00020000;

// BUF: interior K-steps load through buffer resources with the K-step in
// the scalar offset, so no per-load address arithmetic; needs both operand
// extents below 2^31 bytes (checked on the host).
template <int KE, int TM, int TN, int SK, int NWV, int MODE, int PD, bool LOG = false,
          bool BUF = false>
__device__ __forceinline__ void direct_tile(const GemmArgs& g, int tile_m, int tile_n,
                                            const PackedParams& pp, double* __restrict__ red,
                                            const uint32_t* __restrict__ Ls,
                                            const uint32_t* __restrict__ Hs,
                                            const uint32_t* __restrict__ pks = nullptr,
                                            const uint16_t* __restrict__ Zs = nullptr) {
  constexpr int EB = LOG ? 2 : KE;  // bytes per operand element: a code or k coefficients
  using T = DT<EB, TM, TN, SK, NWV>;
  using St = DStage<EB, TM, TN>;
  constexpr bool MULTI = MODE != 0;
  static_assert(!(MULTI && SK > 1), "split-K waves combine single-block accumulators");
  const int lane = threadIdx.x & 63;
  // BUF: the wave index as a scalar, so the K range and the scalar offsets
  // derived from it are wave-uniform for the compiler too
  const int wave = BUF ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : threadIdx.x >> 6;
  const int sw = wave % T::SP, kw = wave / T::SP;
  const int c = lane & 15, grp = lane >> 4;
  const int64_t wm0 = (int64_t)tile_m * T::BM + (sw / T::WGN) * T::WM;
  const int64_t wn0 = (int64_t)tile_n * T::BN + (sw % T::WGN) * T::WN;
  const uint32_t b = MODE ? multi_block_b<KE>() : pp.b;
  const DqtShifts sh(b);
  const bool inner = pp.aligned != 0 && wm0 + T::WM <= g.M && wn0 + T::WN <= g.N;

  const int64_t nks = (g.K + 15) / 16;  // K-steps
  const int64_t nfull = g.K / 16;       // K-steps without a ragged end
  const int64_t s_begin = nks * kw / SK, s_end = nks * (kw + 1) / SK;

  const v4d bias = {kTwo52, kTwo52, kTwo52, kTwo52};
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
  uint32_t gcnt = 0, nbound = 0, nadd = 0;  // nadd: blocks in the lane state since its last fold

  // Byte pointers of this lane's first K-step.
  const uint8_t* pa = g.A + ((wm0 + c) * g.lda + 4 * grp) * EB;
  const uint8_t* pb = g.B + ((int64_t)(4 * grp) * g.ldb + wn0 + TN * c) * EB;
  const int64_t a_istep = 16 * g.lda * EB;  // next MFMA row-block
  const int64_t b_gstep = g.ldb * EB;       // next B row
  const int64_t b_sstep = 16 * g.ldb * EB;  // next K-step

  int32_t voa[TM], vob[4];
  if constexpr (BUF) {
#pragma unroll
    for (int i = 0; i < TM; ++i) voa[i] = (int32_t)((pa - g.A) + i * a_istep);
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) vob[gk] = (int32_t)((pb - g.B) + gk * b_gstep);
  }
  auto load_fast = [&](St& x, int64_t s) {
    if constexpr (BUF) {
      const auto rsa = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.A), (short)0,
                                                         0x7fffffff, kBufferWord3);
      const auto rsb = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(g.B), (short)0,
                                                         0x7fffffff, kBufferWord3);
      const int32_t sa = (int32_t)(s * 16 * EB), sb = (int32_t)(s * b_sstep);
#pragma unroll
      for (int i = 0; i < TM; ++i) buf_load<EB>(rsa, voa[i], sa, x.a[i]);
#pragma unroll
      for (int gk = 0; gk < 4; ++gk) buf_load<T::BW>(rsb, vob[gk], sb, x.b[gk]);
      return;
    }
    const uint8_t* a0 = pa + s * 16 * EB;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(a0 + i * a_istep);
#pragma unroll
      for (int w = 0; w < EB; ++w) x.a[i][w] = src[w];
    }
    const uint8_t* b0 = pb + s * b_sstep;
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(b0 + gk * b_gstep);
#pragma unroll
      for (int w = 0; w < T::BW; ++w) x.b[gk][w] = src[w];
    }
  };
  // Bounds-checked byte gathers: rows >= M, columns >= N and k >= K read 0.
  auto load_slow = [&](St& x, int64_t s) {
    if constexpr (LOG) {
      // codes: an absent element must read as zero, whose code is not 0
      // (code 0 is g^0 = 1); 0xffff is above every code and reads as zero
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int64_t row = wm0 + 16 * i + c;
        const uint8_t* src = g.A + row * g.lda * 2;
#pragma unroll
        for (int w = 0; w < 2; ++w) x.a[i][w] = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t k = 16 * s + 4 * grp + e;
          uint32_t v = 0xffffu;
          if (row < g.M && k < g.K) v = (uint32_t)src[2 * k] | ((uint32_t)src[2 * k + 1] << 8);
          x.a[i][e >> 1] |= v << (16 * (e & 1));
        }
      }
#pragma unroll
      for (int gk = 0; gk < 4; ++gk) {
        const int64_t krow = 16 * s + 4 * grp + gk;
        const uint8_t* src = g.B + krow * g.ldb * 2;
#pragma unroll
        for (int w = 0; w < T::BW; ++w) x.b[gk][w] = 0;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int64_t col = wn0 + TN * c + j;
          uint32_t v = 0xffffu;
          if (krow < g.K && col < g.N) v = (uint32_t)src[2 * col] | ((uint32_t)src[2 * col + 1] << 8);
          x.b[gk][j >> 1] |= v << (16 * (j & 1));
        }
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int w = 0; w < EB; ++w) x.a[i][w] = 0;
      const int64_t row = wm0 + 16 * i + c;
      if (row < g.M) {
        const uint8_t* src = g.A + row * g.lda * EB;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t k = 16 * s + 4 * grp + e;
          if (k < g.K) {
#pragma unroll
            for (int cc = 0; cc < EB; ++cc) {
              const int pos = e * EB + cc;
              x.a[i][pos >> 2] |= (uint32_t)src[k * EB + cc] << (8 * (pos & 3));
            }
          }
        }
      }
    }
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) {
#pragma unroll
      for (int w = 0; w < T::BW; ++w) x.b[gk][w] = 0;
      const int64_t krow = 16 * s + 4 * grp + gk;
      if (krow < g.K) {
        const uint8_t* src = g.B + krow * g.ldb * EB;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int64_t col = wn0 + TN * c + j;
          if (col < g.N) {
#pragma unroll
            for (int cc = 0; cc < EB; ++cc) {
              const int pos = j * EB + cc;
              x.b[gk][pos >> 2] |= (uint32_t)src[col * EB + cc] << (8 * (pos & 3));
            }
          }
        }
      }
    }
  };

  auto boundary = [&]() {
    if constexpr (MULTI) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) st[i][j][v].add(acc[i][j][v], pp.fa);
          acc[i][j] = bias;
        }
      ++nadd;
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

  // One K-step on the matrix cores from a loaded stage.
  auto convert = [&](const St& x, double (&av)[TM][4], double (&bv)[4][TN]) {
    if constexpr (LOG) {
      // Alg. 4's tabulated conversion: a code's packed value from one lookup
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int gk = 0; gk < 4; ++gk) av[i][gk] = log_elem(x.a[i], gk, pp.zero_code, pks);
#pragma unroll
      for (int gk = 0; gk < 4; ++gk)
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[gk][j] = log_elem(x.b[gk], j, pp.zero_code, pks);
    } else {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int gk = 0; gk < 4; ++gk) av[i][gk] = packed_elem<KE, KE>(x.a[i], gk, sh);
#pragma unroll
      for (int gk = 0; gk < 4; ++gk)
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[gk][j] = packed_elem<KE, T::BW>(x.b[gk], j, sh);
    }
  };
  auto mfma_step = [&](const double (&av)[TM][4], const double (&bv)[4][TN]) {
#pragma unroll
    for (int gk = 0; gk < 4; ++gk) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][gk], bv[gk][j], acc[i][j], 0, 0, 0);
      if constexpr (MULTI) {
        if (++gcnt == pp.nq_groups) {
          boundary();
          gcnt = 0;
        }
      }
    }
  };

  // K-steps [s0, s1) with PD stages in flight.  Refills past the end reload
  // step s1 - 1 (its data goes unused) so that the loop body has no
  // data-dependent branch.
  auto kloop = [&](auto fast_tag, int64_t s0, int64_t s1) {
    constexpr bool FAST = decltype(fast_tag)::value;
    if (s0 >= s1) return;
    St stg[PD];
    auto load = [&](St& x, int64_t s) {
      s = s < s1 ? s : s1 - 1;
      if constexpr (FAST) load_fast(x, s);
      else load_slow(x, s);
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) load(stg[u], s0 + u);
    int64_t s = s0;
    for (; s + PD <= s1; s += PD) {
#pragma unroll
      for (int u = 0; u < PD; ++u) {
        double av[TM][4], bv[4][TN];
        convert(stg[u], av, bv);
        load(stg[u], s + u + PD);
        mfma_step(av, bv);
      }
    }
    // fewer than PD steps left, already loaded in stages 0 .. rest-1
    const int rest = (int)(s1 - s);
#pragma unroll
    for (int u = 0; u < PD - 1; ++u) {
      if (u < rest) {
        double av[TM][4], bv[4][TN];
        convert(stg[u], av, bv);
        mfma_step(av, bv);
      }
    }
  };
  if (inner) {
    const int64_t mid = s_end < nfull ? s_end : (nfull > s_begin ? nfull : s_begin);
    kloop(std::true_type{}, s_begin, mid);
    kloop(std::false_type{}, mid, s_end);  // the ragged last K-step, if this wave has it
  } else {
    kloop(std::false_type{}, s_begin, s_end);
  }

  // Split-K: hand the accumulator rows this wave does not own to their owner.
  if constexpr (SK > 1) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int own = (4 * i + v) % SK;
        if (own != kw) {
          const int slot = (kw - own + SK) % SK - 1;
#pragma unroll
          for (int j = 0; j < TN; ++j)
            red[(((((sw * TM + i) * 4 + v) * (SK - 1) + slot) * TN) + j) * 64 + lane] =
                acc[i][j][v] - kTwo52;
        }
      }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if ((4 * i + v) % SK == kw) {
#pragma unroll
          for (int slot = 0; slot < SK - 1; ++slot)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j][v] += red[(((((sw * TM + i) * 4 + v) * (SK - 1) + slot) * TN) + j) * 64 + lane];
        }
      }
  }

  // Epilogue: residues, L + H (Thm. 3), TN consecutive outputs per lane.
  const bool c_words = ((((uintptr_t)g.C) & 3) == 0) && (((g.ldc * EB) & 3) == 0);
  const int64_t col0 = wn0 + TN * c;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (SK > 1 && (4 * i + v) % SK != kw) continue;
      uint32_t e[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        uint32_t u[2 * KE - 1];
        st[MULTI ? i : 0][MULTI ? j : 0][v].residues(acc[i][j][v], b, pp, u, nadd);
        e[j] = LOG ? lh_log<KE>(u, pp, Ls, Hs, Zs) : lh_combine<KE>(u, pp, Ls, Hs);
      }
      const int64_t row = wm0 + 16 * i + grp + 4 * v;
      if (row >= g.M) continue;
      uint8_t* dst = g.C + (row * g.ldc + col0) * EB;
      if (c_words && col0 + TN <= g.N) {
        uint32_t w[T::BW];
#pragma unroll
        for (int x = 0; x < T::BW; ++x) w[x] = 0;
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int cc = 0; cc < EB; ++cc) {
            const int pos = j * EB + cc;
            w[pos >> 2] |= ((e[j] >> (8 * cc)) & 0xffu) << (8 * (pos & 3));
          }
        uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
        for (int x = 0; x < T::BW; ++x) d32[x] = w[x];
      } else {
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (col0 + j < g.N) store_elem<EB>(dst + j * EB, e[j]);
      }
    }
  }
}

template <int KE, int TM, int TN, int SK, int NWV, int MODE, int PD, bool LOG = false,
          bool BUF = false>
__global__ __launch_bounds__(64 * NWV) void gemm_direct_kernel(GemmArgs g, PackedParams pp,
                                                          int tiles_n, int ntiles) {
  using T = DT<LOG ? 2 : KE, TM, TN, SK, NWV>;
  __shared__ double red[T::RED];
  extern __shared__ uint32_t tabs[];
  uint32_t* Ls = tabs;
  uint32_t* Hs = tabs + (1 << pp.tbl_log2);
  load_tables(pp, Ls, Hs);
  uint32_t* pks = nullptr;
  uint16_t* Zs = nullptr;
  if constexpr (LOG) log_lds_tables(pp, tabs, &pks, &Zs);
  __syncthreads();
  const int tile = xcd_tile((int)blockIdx.x, ntiles / tiles_n, tiles_n);
  direct_tile<KE, TM, TN, SK, NWV, MODE, PD, LOG, BUF>(g, tile / tiles_n, tile % tiles_n, pp, red,
                                                       Ls, Hs, pks, Zs);
}

template <int KE, int TM, int TN, int SK, int NWV, int MODE, int PD, bool LOG = false,
          bool BUF = false>
__global__ __launch_bounds__(64 * NWV) void gemm_direct_batched_kernel(
    const GemmArgs* __restrict__ descs, const TileItem* __restrict__ items, int32_t n_items,
    uint32_t* counter, PackedParams pp) {
  using T = DT<LOG ? 2 : KE, TM, TN, SK, NWV>;
  __shared__ double red[T::RED];
  __shared__ int32_t cur;
  extern __shared__ uint32_t tabs[];
  uint32_t* Ls = tabs;
  uint32_t* Hs = tabs + (1 << pp.tbl_log2);
  load_tables(pp, Ls, Hs);
  uint32_t* pks = nullptr;
  uint16_t* Zs = nullptr;
  if constexpr (LOG) log_lds_tables(pp, tabs, &pks, &Zs);
  for (;;) {
    // the barriers also separate one tile's LDS reduction from the next
    if (threadIdx.x == 0) cur = (int32_t)atomicAdd(&counter[0], 1u);
    __syncthreads();
    const int32_t it = cur;
    __syncthreads();
    if (it >= n_items) break;
    const TileItem ti = items[it];
    const GemmArgs g = descs[ti.gemm];
    direct_tile<KE, TM, TN, SK, NWV, MODE, PD, LOG, BUF>(g, ti.tm, ti.tn, pp, red, Ls, Hs, pks,
                                                         Zs);
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

}  // namespace fqt
