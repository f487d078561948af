// Device helpers shared by the FQT kernels (gfx950, wave64).
//
// Numerical conventions
// ---------------------
// * A packed value is an exact integer r < 2^52 held in binary64.  The GEMM
//   accumulators are seeded with 2^52 ("biased"): acc = 2^52 + r lies in
//   [2^52, 2^53), where consecutive doubles differ by exactly 1, so every
//   partial sum and every FMA stays exact, and the low 52 bits of the bit
//   pattern of acc ARE r.  No float->int conversion is needed.
// * REDQ (Alg. 2 / Alg. 4 steps 3-7) needs rop = floor(r/p).  We take
//       t = fma(r, RN(1/p), 2^52 - 1/2),
//   whose low 52 bits hold rop' in {rop-1, rop} (two's complement for -1):
//   |r*RN(1/p) - r/p| <= r/p * 2^-53 < 1/(2p) for r < 2^52, so the value
//   rounded to the integer grid is floor(r/p) or floor(r/p) - 1 (p >= 3;
//   for p = 2 the reciprocal is exact).  For rop = 0 and rop' = -1 the sum
//   falls just below 2^52 and rounds to 2^52 - 1/2, whose mantissa bits are
//   all ones, i.e. -1 modulo 2^52.
//   With rop' the residues u'_i = floor(r/q^i) - p*floor(rop'/q^i) satisfy
//   u'_i in {u_i, u_i + p} subset [0, 2p) and u'_i == u_i (mod p), where
//   u_i are Thm. 2's residues; one conditional subtraction gives u_i.
// * Residues are computed modulo 2^24 with 24-bit multiply-adds and only
//   their low byte is kept (u'_i < 2p <= 254).  The low byte depends only on
//   bits [b*i, b*i+8) of r and rop', which the host keeps below bit 52
//   (b*(2k-2) + 8 <= 52), so the exponent bits above never leak in.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fqt {

constexpr double kTwo52 = 4503599627370496.0;  // 2^52

__device__ __forceinline__ uint64_t bits64(double x) {
  return (uint64_t)__double_as_longlong(x);
}

// v_perm_b32: result byte j = byte sel_j of the 8-byte value {hi:lo};
// selector 0x0c yields a zero byte.
__device__ __forceinline__ uint32_t perm_b32(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Field parameters passed by value to kernels (built on the host).
struct FieldArgs {
  uint32_t p;          // characteristic, 2 <= p <= 127
  uint32_t cb;         // ceil(log2 p): bits per residue in a table index
  uint32_t negp24;     // 2^24 - p: mad24 by it subtracts p*x modulo 2^24
  uint32_t mod_magic;  // ceil(2^32 / p): floor(x/p) = umulhi(x, magic), x < 2^25
  uint32_t sub_magic;  // (0x80 - p) in every byte
  uint32_t c;          // (-q) mod p, the off-diagonal of Q_d (Section 5.1)
  double inv_p;        // RN(1/p)
};

// x mod p for x < 2^25.
__device__ __forceinline__ uint32_t mod_p_small(uint32_t x, const FieldArgs& fa) {
  const uint32_t qq = __umulhi(x, fa.mod_magic);
  return x - qq * fa.p;
}

// Coefficient-wise sum of two field elements held one coefficient per byte,
// every byte in [0, p), reduced back into [0, p).  p <= 127, so byte sums
// stay below 2p <= 254 and nothing carries between bytes.
__device__ __forceinline__ uint32_t add_bytes_mod_p(uint32_t a, uint32_t b, const FieldArgs& fa) {
  const uint32_t s = a + b;
  const uint32_t t = (s + fa.sub_magic) & 0x80808080u;  // bit 7 set where byte >= p
  return s - (t >> 7) * fa.p;
}

// REDQ residues of a biased accumulator acc = 2^52 + r (r < 2^52), q = 2^b.
// t[i]'s low byte is u'_i in [0, 2p), congruent to floor(r/q^i) mod p.
template <int ND>
__device__ __forceinline__ void redq_residues_biased(double acc, uint32_t b,
                                                     const FieldArgs& fa,
                                                     uint32_t (&t)[ND]) {
  const uint64_t rb = bits64(acc);
  const uint64_t ob = bits64(__builtin_fma(acc - kTwo52, fa.inv_p, kTwo52 - 0.5));
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const uint32_t s = b * (uint32_t)i;
    const uint32_t rw = (uint32_t)(rb >> s);
    const uint32_t ow = (uint32_t)(ob >> s);
    t[i] = __umul24(ow, fa.negp24) + rw;
  }
}

// Store k coefficient bytes (held in the low k bytes of e) at dst.
template <int KE>
__device__ __forceinline__ void store_elem(uint8_t* dst, uint32_t e) {
  if constexpr (KE == 1) {
    dst[0] = (uint8_t)e;
  } else if constexpr (KE == 2) {
    *reinterpret_cast<uint16_t*>(dst) = (uint16_t)e;
  } else if constexpr (KE == 3) {
    dst[0] = (uint8_t)e;
    dst[1] = (uint8_t)(e >> 8);
    dst[2] = (uint8_t)(e >> 16);
  } else {
    *reinterpret_cast<uint32_t*>(dst) = e;
  }
}

// Load k coefficient bytes of one element into the low bytes of a word.
template <int KE>
__device__ __forceinline__ uint32_t load_elem(const uint8_t* src) {
  if constexpr (KE == 1) {
    return src[0];
  } else if constexpr (KE == 2) {
    return (uint32_t)src[0] | ((uint32_t)src[1] << 8);
  } else if constexpr (KE == 3) {
    return (uint32_t)src[0] | ((uint32_t)src[1] << 8) | ((uint32_t)src[2] << 16);
  } else {
    return (uint32_t)src[0] | ((uint32_t)src[1] << 8) | ((uint32_t)src[2] << 16) |
           ((uint32_t)src[3] << 24);
  }
}

}  // namespace fqt
