// Device pieces shared by the two packed-FP64 GEMM kernel families (LDS-staged
// in k_gemm_f64.hip, register-direct in k_gemm_direct.hip): operand bytes ->
// packed doubles, the per-element state carried across K-blocks, and the
// final REDQ + table step of Alg. 4.
//
// K-block state (Section 6 delays the reduction while eq. (2) holds; how the
// blocks combine is a reading of Thm. 2): the residue vector u of a block is
// linear in its digits modulo p, and L + H is linear in u, so blocks are
// summed before the tables are applied once.
//   MODE 0: one block (K <= n_q); the biased accumulator is the whole state.
//   MODE 1: REDQ residues u'_i < 2p of every block summed in 16-bit lanes,
//           two residues per word (digit 2w low, 2w+1 high).
//   MODE 2: digit sums.  With q = 2^b the digits of a block are bit fields of
//           its accumulator; the bits of its even digits are added into E,
//           those of its odd digits form O, so every field has b spare bits
//           above it and sums below q^2 never carry (needs 2b <= 24).  O is
//           not kept: T, the plain sum of the accumulators' bit patterns, is
//           (odd + even digit bits) + n * bits(2^52), so O = T - E - n bits(2^52)
//           with n the blocks added since the last fold (one mask-and-add less
//           per block).  At the end Horner's rule mod p gives
//           u_i = sum_{j>=i} D_j q^(j-i) mod p.
// Lanes and fields are folded mod p every fold_blocks boundaries, before they
// could overflow.  In modes 1 and 2, q is the largest power of two eq. (2)
// admits and is fixed at compile time.
#pragma once

#include "fqt_internal.h"

namespace fqt {

// q = 2^b of the multi-block modes.
template <int KE>
constexpr uint32_t multi_block_b() {
  return 52u / (2u * KE - 1u);
}

// Digit-sum boundaries (mode 2) need fields of 2b <= 24 bits.
template <int KE>
constexpr bool digit_sums_fit() {
  return 2 * multi_block_b<KE>() <= 24;
}

constexpr uint64_t digit_mask(int nd, uint32_t b, int parity) {
  uint64_t m = 0;
  for (int d = parity; d < nd; d += 2) m |= ((1ull << b) - 1) << (b * d);
  return m;
}

// Byte-select forms of a shift and an add (gfx9 SDWA: an operand can be one
// zero-extended byte of a register), so that a coefficient byte enters the
// DQT sum without a separate extract instruction.
#define FQT_SDWA_BYTE(S)                                                            \
  __device__ __forceinline__ uint32_t byte_shl_##S(uint32_t w, uint32_t s) {      \
    uint32_t r;                                                                     \
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD "        \
        "src0_sel:DWORD src1_sel:BYTE_" #S                                          \
        : "=v"(r)                                                                   \
        : "v"(s), "v"(w));                                                          \
    return r;                                                                       \
  }                                                                                 \
  __device__ __forceinline__ uint32_t add_byte_##S(uint32_t v, uint32_t w) {      \
    uint32_t r;                                                                     \
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD "            \
        "src0_sel:DWORD src1_sel:BYTE_" #S                                          \
        : "=v"(r)                                                                   \
        : "v"(v), "v"(w));                                                          \
    return r;                                                                       \
  }
FQT_SDWA_BYTE(0)
FQT_SDWA_BYTE(1)
FQT_SDWA_BYTE(2)
FQT_SDWA_BYTE(3)
#undef FQT_SDWA_BYTE

// byte `sel` (a constant after unrolling) of w, shifted left by s
__device__ __forceinline__ uint32_t byte_shl(uint32_t w, int sel, uint32_t s) {
  switch (sel) {
    case 0: return byte_shl_0(w, s);
    case 1: return byte_shl_1(w, s);
    case 2: return byte_shl_2(w, s);
    default: return byte_shl_3(w, s);
  }
}
// v + byte `sel` of w
__device__ __forceinline__ uint32_t add_byte(uint32_t v, uint32_t w, int sel) {
  switch (sel) {
    case 0: return add_byte_0(v, w);
    case 1: return add_byte_1(v, w);
    case 2: return add_byte_2(v, w);
    default: return add_byte_3(v, w);
  }
}

// Shift amounts j*b of the DQT at q = 2^b (Section 2: multiplication by q^j
// is a shift), j < 4.
struct DqtShifts {
  uint32_t s[4];
  __device__ __forceinline__ explicit DqtShifts(uint32_t b) : s{0u, b, 2u * b, 3u * b} {}
};

// DQT of element e of a little-endian run of NWD words holding consecutive
// KE-byte elements, straight to binary64: sum_j c_j << (j*b), exact since the
// host keeps it below 2^32.  KE - 1 byte-select shifts and adds (KE = 1: one
// extract) and one conversion; elements that straddle words need no realign.
template <int KE, int NWD>
__device__ __forceinline__ uint32_t dqt_u32(const uint32_t (&raw)[NWD], int e,
                                            const DqtShifts& sh) {
  const int o = e * KE;
  if constexpr (KE == 1) {
    return (raw[o >> 2] >> (8 * (o & 3))) & 0xffu;
  } else {
    uint32_t v = add_byte(byte_shl(raw[(o + 1) >> 2], (o + 1) & 3, sh.s[1]), raw[o >> 2], o & 3);
#pragma unroll
    for (int j = 2; j < KE; ++j) v += byte_shl(raw[(o + j) >> 2], (o + j) & 3, sh.s[j]);
    return v;
  }
}

template <int KE, int NWD>
__device__ __forceinline__ double packed_elem(const uint32_t (&raw)[NWD], int e,
                                              const DqtShifts& sh) {
  return (double)dqt_u32<KE, NWD>(raw, e, sh);
}

// Centred packing: coefficients c > h = (p-1)/2 stand for c - p, so the
// packed value is sum_j c_j q^j - p sum_j [c_j > h] q^j, a signed integer
// below 2^31 in magnitude.  gt holds the bytes [c > h] of raw (centred_flags).
__device__ __forceinline__ uint32_t centred_flags(uint32_t w, uint32_t hmask) {
  return ((w + hmask) >> 7) & 0x01010101u;  // hmask = (0x7f - h) in every byte; c < 128
}

template <int KE, int NWD>
__device__ __forceinline__ double packed_elem_centred(const uint32_t (&raw)[NWD],
                                                      const uint32_t (&gt)[NWD], int e,
                                                      const DqtShifts& sh, uint32_t p) {
  const int32_t v = (int32_t)dqt_u32<KE, NWD>(raw, e, sh) - (int32_t)(p * dqt_u32<KE, NWD>(gt, e, sh));
  return (double)v;
}

// DQT of a chunk of 4 consecutive elements (KE raw words) into 4 binary64
// values, the form the LDS-staged loaders store.  Every VALU instruction here
// costs issue cycles of the SIMD that runs the FP64 MFMAs (they do not
// overlap on gfx950), so the conversion takes the shortest route the field
// admits:
//  * centred, p <= 8 (kDqtLut): one byte permutation per word maps every
//    coefficient c to its offset form (c + h) mod p = c' + h, c' in [-h, h];
//    the packed offset form minus h (1 + q + ... + q^(k-1)) is sum c'_j q^j.
//  * k = 4, q <= 2^7 (kDqtDot4): an element is one word; two byte dot
//    products give c0 + q c1 and c2 + q c3, one shift-add joins them (the
//    offset above rides in the first dot product's addend).
//  * otherwise the byte-select shifts of dqt_u32, or the flag arithmetic of
//    packed_elem_centred for centred fields with p > 8.
template <int KE>
__device__ __forceinline__ void dqt_chunk(uint32_t (&raw)[KE], const DqtShifts& sh,
                                          const PackedParams& pp, double (&out)[4]) {
  if (pp.centered && !(pp.dqt_flags & kDqtLut)) {
    const uint32_t hmask = (0x7fu - (pp.fa.p - 1) / 2) * 0x01010101u;
    uint32_t gt[KE];
#pragma unroll
    for (int w = 0; w < KE; ++w) gt[w] = centred_flags(raw[w], hmask);
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = packed_elem_centred<KE, KE>(raw, gt, e, sh, pp.fa.p);
    return;
  }
  if (pp.dqt_flags & kDqtLut) {
#pragma unroll
    for (int w = 0; w < KE; ++w) raw[w] = perm_b32(pp.lut_hi, pp.lut_lo, raw[w]);
  }
  if constexpr (KE == 4) {
    if (pp.dqt_flags & kDqtDot4) {
      const uint32_t q = 1u << sh.s[1];
      const uint32_t wlo = 1u | (q << 8), whi = (1u << 16) | (q << 24);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t lo = __builtin_amdgcn_udot4(raw[e], wlo, (uint32_t)pp.dqt_off, false);
        const uint32_t hi = __builtin_amdgcn_udot4(raw[e], whi, 0u, false);
        out[e] = (double)(int32_t)(lo + (hi << sh.s[2]));
      }
      return;
    }
  }
  if (pp.dqt_flags & kDqtLut) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      out[e] = (double)(int32_t)(dqt_u32<KE, KE>(raw, e, sh) + (uint32_t)pp.dqt_off);
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) out[e] = packed_elem<KE, KE>(raw, e, sh);
}

// Centred packing's final correction: n_blocks times the constant -(L + H)
// of the shift's residues, every coefficient scaled mod p.
template <int KE>
__device__ __forceinline__ uint32_t centred_correction(uint32_t c0neg, uint32_t nblocks,
                                                       const FieldArgs& fa) {
  const uint32_t n = nblocks % fa.p;
  uint32_t w = 0;
#pragma unroll
  for (int i = 0; i < KE; ++i) w |= mod_p_small(((c0neg >> (8 * i)) & 0xffu) * n, fa) << (8 * i);
  return w;
}

template <int KE, int MODE>
struct BlockLanes {
  static constexpr int ND = 2 * KE - 1;
  static constexpr int NW = KE;  // 16-bit lane words, (ND + 1) / 2
  static constexpr uint32_t BQ = MODE ? multi_block_b<KE>() : 0u;
  static constexpr uint64_t EM = MODE == 2 ? digit_mask(ND, BQ, 0) : 0;
  static constexpr uint64_t XB = 0x4330000000000000ull;  // bits of 2^52, one per block

  uint64_t E, T;   // MODE 2: even digit fields; sum of the blocks' bit patterns
  uint32_t W[NW];  // MODE 1

  __device__ __forceinline__ void clear() {
    E = T = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) W[w] = 0;
  }

  // digit field d of a gapped sum: bits [d*b, d*b + 2b)
  static __device__ __forceinline__ uint32_t field(uint64_t x, int d) {
    return (uint32_t)(x >> (BQ * d)) & (uint32_t)((1ull << (2 * BQ)) - 1);
  }

  // REDQ residues of a block as lane words.
  static __device__ __forceinline__ void residue_words(double acc, const FieldArgs& fa,
                                                       uint32_t (&wd)[NW]) {
    uint32_t t[ND];
    redq_residues_biased<ND>(acc, BQ, fa, t);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t lo = t[2 * w];
      const uint32_t hi = (2 * w + 1 < ND) ? t[2 * w + 1] : 0u;
      wd[w] = perm_b32(hi, lo, 0x0c040c00u);
    }
  }

  // A block boundary: take the block's contribution out of its accumulator.
  __device__ __forceinline__ void add(double acc, const FieldArgs& fa) {
    if constexpr (MODE == 2) {
      const uint64_t rb = bits64(acc);
      E += rb & EM;
      T += rb;
    } else if constexpr (MODE == 1) {
      uint32_t wd[NW];
      residue_words(acc, fa, wd);
#pragma unroll
      for (int w = 0; w < NW; ++w) W[w] += wd[w];
    }
  }

  // Reduce every lane or field mod p; nadd = blocks added since the last fold.
  __device__ __forceinline__ void fold(const FieldArgs& fa, uint32_t nadd) {
    if constexpr (MODE == 2) {
      const uint64_t O = T - E - (uint64_t)nadd * XB;
      uint64_t e = 0, o = 0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const uint64_t r = mod_p_small(field((d & 1) ? O : E, d), fa);
        if (d & 1) o |= r << (BQ * d);
        else e |= r << (BQ * d);
      }
      E = e;
      T = e + o;  // no block bits: the count starts again
    } else if constexpr (MODE == 1) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t x = W[w];
        W[w] = mod_p_small(x & 0xffffu, fa) | (mod_p_small(x >> 16, fa) << 16);
      }
    }
  }

  // Final residues u_0..u_{2k-2} in [0, p) of all blocks, the last block
  // still in its accumulator; nadd = blocks added since the last fold.  b is
  // q's exponent for MODE 0.
  __device__ __forceinline__ void residues(double acc, uint32_t b, const PackedParams& pp,
                                           uint32_t (&u)[ND], uint32_t nadd = 0) const {
    const FieldArgs& fa = pp.fa;
    if constexpr (MODE == 2) {
      const uint64_t rb = bits64(acc);
      const uint64_t e = E + (rb & EM);
      const uint64_t o = T + rb - e - (uint64_t)(nadd + 1) * XB;
      u[ND - 1] = mod_p_small(field(((ND - 1) & 1) ? o : e, ND - 1), fa);
#pragma unroll
      for (int d = ND - 2; d >= 0; --d)
        u[d] = mod_p_small(field((d & 1) ? o : e, d) + pp.qmod * u[d + 1], fa);
    } else if constexpr (MODE == 1) {
      uint32_t wd[NW];
      residue_words(acc, fa, wd);
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t tot = W[w] + wd[w];
        u[2 * w] = mod_p_small(tot & 0xffffu, fa);
        if (2 * w + 1 < ND) u[2 * w + 1] = mod_p_small(tot >> 16, fa);
      }
    } else {
      uint32_t t[ND];
      redq_residues_biased<ND>(acc, b, fa, t);
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const uint32_t x = t[d] & 0xffu;
        u[d] = x >= fa.p ? x - fa.p : x;
      }
    }
  }
};

// Thm. 3: the field element of residues u as L[u_0..u_{k-1}] + H[u_{k-1}..u_{2k-2}]
// (binary table index, Section 5.3), one coefficient per byte.
template <int KE>
__device__ __forceinline__ uint32_t lh_combine(const uint32_t (&u)[2 * KE - 1],
                                               const PackedParams& pp,
                                               const uint32_t* __restrict__ Ls,
                                               const uint32_t* __restrict__ Hs) {
  uint32_t il = 0, ih = 0;
#pragma unroll
  for (int d = 0; d < KE; ++d) {
    il |= u[d] << (pp.fa.cb * d);
    ih |= u[KE - 1 + d] << (pp.fa.cb * d);
  }
  const uint32_t tmask = (1u << pp.tbl_log2) - 1u;  // keeps lookups inside the tables
  return add_bytes_mod_p(Ls[il & tmask], Hs[ih & tmask], pp.fa);
}

// ---- discrete-log operands (Alg. 4) ------------------------------------------
// A code e < m = p^k - 1 stands for g^e, the code m for zero; larger codes
// read as zero.

// Packed value of code e of a run of 16-bit codes: one table lookup
// (Alg. 4's tabulated conversion to the evaluation at q).  Every packed value
// of an element is below p q^(k-1) < 2^32 under eq. (2), so the table holds
// 32-bit integers.
template <int NWD>
__device__ __forceinline__ double log_elem(const uint32_t (&raw)[NWD], int e, uint32_t zero,
                                           const uint32_t* __restrict__ pks) {
  const uint32_t code = (raw[e >> 1] >> (16 * (e & 1))) & 0xffffu;
  return (double)pks[min(code, zero)];
}

// Field addition of codes a, b in [0, m]: zero is the identity, otherwise
// g^a + g^b = g^a (1 + g^(b-a)) = g^(a + Z[b-a]), zero where Z gives m.
__device__ __forceinline__ uint32_t zech_add(uint32_t a, uint32_t b, uint32_t m,
                                             const uint16_t* __restrict__ Zs) {
  const int32_t dd = (int32_t)b - (int32_t)a;
  const uint32_t d = (uint32_t)(dd < 0 ? dd + (int32_t)m : dd);  // in [0, m]
  const uint32_t z = Zs[d];
  const uint32_t s = a + z;
  uint32_t r = z >= m ? m : (s >= m ? s - m : s);
  r = a >= m ? b : r;
  return b >= m ? a : r;
}

// Alg. 4's last steps on codes: L and H looked up by the binary indices of
// (u_0..u_{k-1}) and (u_{k-1}..u_{2k-2}) (Thm. 3's tables, holding codes),
// then R = H + L by the Zech table.
template <int KE>
__device__ __forceinline__ uint32_t lh_log(const uint32_t (&u)[2 * KE - 1],
                                           const PackedParams& pp,
                                           const uint32_t* __restrict__ Ls,
                                           const uint32_t* __restrict__ Hs,
                                           const uint16_t* __restrict__ Zs) {
  uint32_t il = 0, ih = 0;
#pragma unroll
  for (int d = 0; d < KE; ++d) {
    il |= u[d] << (pp.fa.cb * d);
    ih |= u[KE - 1 + d] << (pp.fa.cb * d);
  }
  const uint32_t tmask = (1u << pp.tbl_log2) - 1u;
  return zech_add(Hs[ih & tmask], Ls[il & tmask], pp.zero_code, Zs);
}

// Bytes of dynamic LDS the log kernels need: L, H, the packed values, the
// Zech table.
__host__ __device__ inline size_t log_lds_bytes(uint32_t tbl_log2, uint32_t zero_code) {
  const size_t n = (size_t)1 << tbl_log2, e = (size_t)zero_code + 1;
  return (2 * n + e) * 4 + (e * 2 + 3) / 4 * 4;
}

// Copy the packed values and the Zech table into LDS after L and H.
__device__ __forceinline__ void log_lds_tables(const PackedParams& pp, uint32_t* tabs,
                                               uint32_t** pks, uint16_t** Zs) {
  const int n = 1 << pp.tbl_log2, e = (int)pp.zero_code + 1;
  uint32_t* pk = tabs + 2 * n;
  uint16_t* z = reinterpret_cast<uint16_t*>(pk + e);
  for (int i = threadIdx.x; i < e; i += blockDim.x) {
    pk[i] = pp.pk[i];
    z[i] = pp.Z[i];
  }
  *pks = pk;
  *Zs = z;
}

// Workgroup -> output tile.  Workgroups reach the 8 XCDs round-robin
// (workgroup i runs on XCD i % 8), and every XCD has its own L2; each XCD is
// handed one rectangular block of the tile grid (2 x 4 or 4 x 2 blocks), so it
// reads one band of A rows and one band of B columns instead of all of B.
// Grids that do not split that way fall back to contiguous runs of tiles.
__device__ __forceinline__ int xcd_tile(int bid, int tiles_m, int tiles_n) {
  const int ntiles = tiles_m * tiles_n;
  if (ntiles & 7) return bid;
  const int x = bid & 7, r = bid >> 3;  // XCD, rank within the XCD
  int gm, gn;
  if (tiles_m % 2 == 0 && tiles_n % 4 == 0) {
    gm = 2;
    gn = 4;
  } else if (tiles_m % 4 == 0 && tiles_n % 2 == 0) {
    gm = 4;
    gn = 2;
  } else {
    return x * (ntiles >> 3) + r;
  }
  const int bm = tiles_m / gm, bn = tiles_n / gn;  // block of bm x bn tiles
  return ((x / gn) * bm + r / bn) * tiles_n + (x % gn) * bn + r % bn;
}

__device__ __forceinline__ void load_tables(const PackedParams& pp, uint32_t* Ls, uint32_t* Hs) {
  const int n = 1 << pp.tbl_log2;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    Ls[i] = pp.L[i];
    Hs[i] = pp.H[i];
  }
}

}  // namespace fqt
