// Streaming transforms of the Q-adic path on gfx950:
//   * DQT pack (Section 2, eq. (1); Alg. 1 step 1): k coefficient bytes ->
//     one exact binary64 evaluation at q (shifts for q = 2^b, an exact FP64
//     Horner evaluation otherwise).
//   * REDQ unpack (Alg. 2; Alg. 4 steps 3-10): one floor division by p gives
//     rop; u_i = floor(r/q^i) - p floor(rop/q^i) for every digit (Thm. 2);
//     then either the Q_d correction mu_i = u_i + c u_{i+1} mod p (c = -q mod
//     p, Section 5.1) for polynomial output, or L[u_0..u_{k-1}] +
//     H[u_{k-1}..u_{2k-2}] (Thm. 3) for field output.
//   * Alg. 1 for a batch of independent polynomial products: pack, one FP64
//     product, REDQ + Q_d.
// These kernels are bound by HBM bandwidth.  With q = 2^b and word-aligned
// buffers (pack, unpack; Alg. 1 also needs every intermediate below 2^32)
// each thread takes four consecutive items straight from whole words;
// otherwise every workgroup stages its input and output bytes through LDS so
// that global accesses are whole dwords.

#include "fqt_internal.h"

namespace fqt {

constexpr int kTB = 256;  // threads per workgroup, items per workgroup

// Copy len bytes g[off, off+len) into LDS (bytes at or beyond total read 0).
__device__ __forceinline__ void stage_in(uint8_t* lds, const uint8_t* g, size_t off, size_t len,
                                         size_t total) {
  const bool al = (((uintptr_t)(g + off)) & 3) == 0;
  if (al) {
    const size_t nd = len >> 2;
    const uint32_t* gs = reinterpret_cast<const uint32_t*>(g + off);
    uint32_t* ls = reinterpret_cast<uint32_t*>(lds);
    for (size_t i = threadIdx.x; i < nd; i += blockDim.x) {
      if (off + 4 * i + 3 < total) {
        ls[i] = gs[i];
      } else {
        uint32_t w = 0;
        for (int j = 0; j < 4; ++j)
          if (off + 4 * i + j < total) w |= (uint32_t)g[off + 4 * i + j] << (8 * j);
        ls[i] = w;
      }
    }
    for (size_t i = 4 * nd + threadIdx.x; i < len; i += blockDim.x)
      lds[i] = off + i < total ? g[off + i] : 0;
  } else {
    for (size_t i = threadIdx.x; i < len; i += blockDim.x) lds[i] = off + i < total ? g[off + i] : 0;
  }
}

// Copy len bytes from LDS to g[off, off+len), never writing at or past total.
__device__ __forceinline__ void stage_out(uint8_t* g, const uint8_t* lds, size_t off, size_t len,
                                          size_t total) {
  const size_t lim = off + len < total ? len : (off < total ? total - off : 0);
  const bool al = (((uintptr_t)(g + off)) & 3) == 0;
  if (al) {
    const size_t nd = lim >> 2;
    uint32_t* gs = reinterpret_cast<uint32_t*>(g + off);
    const uint32_t* ls = reinterpret_cast<const uint32_t*>(lds);
    for (size_t i = threadIdx.x; i < nd; i += blockDim.x) gs[i] = ls[i];
    for (size_t i = 4 * nd + threadIdx.x; i < lim; i += blockDim.x) g[off + i] = lds[i];
  } else {
    for (size_t i = threadIdx.x; i < lim; i += blockDim.x) g[off + i] = lds[i];
  }
}

// 16-byte staging (batched products, REDQ unpack): whole uint4 transfers where the
// global range is 16-byte aligned, the dword/byte copies above otherwise.
__device__ __forceinline__ void stage_in16(uint8_t* lds, const uint8_t* g, size_t off,
                                           size_t len, size_t total) {
  if ((((uintptr_t)(g + off)) & 15) != 0 || (len & 15) != 0) {
    stage_in(lds, g, off, len, total);
    return;
  }
  const size_t nc = len >> 4;
  for (size_t i = threadIdx.x; i < nc; i += blockDim.x) {
    uint4 v;
    if (off + 16 * i + 15 < total) {
      v = reinterpret_cast<const uint4*>(g + off)[i];
    } else {
      uint32_t w[4] = {0, 0, 0, 0};
      for (int j = 0; j < 16; ++j)
        if (off + 16 * i + j < total) w[j >> 2] |= (uint32_t)g[off + 16 * i + j] << (8 * (j & 3));
      v = make_uint4(w[0], w[1], w[2], w[3]);
    }
    reinterpret_cast<uint4*>(lds)[i] = v;
  }
}

__device__ __forceinline__ void stage_out16(uint8_t* g, const uint8_t* lds, size_t off,
                                            size_t len, size_t total) {
  if ((((uintptr_t)(g + off)) & 15) != 0 || (len & 15) != 0) {
    stage_out(g, lds, off, len, total);
    return;
  }
  const size_t lim = off + len < total ? len : (off < total ? total - off : 0);
  const size_t nc = lim >> 4;
  for (size_t i = threadIdx.x; i < nc; i += blockDim.x)
    reinterpret_cast<uint4*>(g + off)[i] = reinterpret_cast<const uint4*>(lds)[i];
  for (size_t i = 16 * nc + threadIdx.x; i < lim; i += blockDim.x) g[off + i] = lds[i];
}

// Exact floor(x / d) for x < 2^53, d >= 2: binary64 estimate, then one
// correction from the exact remainder (the estimate is off by at most 1).
__device__ __forceinline__ uint64_t floor_div53(uint64_t x, uint64_t d, double inv_d) {
  uint64_t t = (uint64_t)__builtin_floor((double)x * inv_d);
  const int64_t e = (int64_t)(x - t * d);
  if (e < 0) t -= 1;
  else if (e >= (int64_t)d) t += 1;
  return t;
}

// Evaluation at q of the k coefficients at src (Alg. 1 step 1).
__device__ __forceinline__ double dqt_eval(const uint8_t* src, int k, int pow2, uint32_t b,
                                           double qd) {
  if (pow2) {
    uint64_t v = 0;
    for (int j = k - 1; j >= 0; --j) v = (v << b) | src[j];
    return (double)v;
  }
  double v = 0.0;
  for (int j = k - 1; j >= 0; --j) v = __builtin_fma(v, qd, (double)src[j]);
  return v;
}

// ---- pack ------------------------------------------------------------------

__global__ __launch_bounds__(kTB) void pack_kernel(const uint8_t* __restrict__ coeffs, size_t n,
                                                   int k, int pow2, uint32_t b, double qd,
                                                   double* __restrict__ out) {
  __shared__ uint8_t buf[kTB * 16];
  const size_t base = (size_t)blockIdx.x * kTB;
  stage_in(buf, coeffs, base * k, (size_t)kTB * k, n * k);
  __syncthreads();
  const size_t i = base + threadIdx.x;
  if (i < n) out[i] = dqt_eval(buf + threadIdx.x * k, k, pow2, b, qd);
}

// DQT pack for q = 2^b from word-aligned coefficient bytes: thread t packs
// elements 4t .. 4t+3 from K whole words and writes their four binary64
// values, with no LDS.  Each value is sum_j c_j 2^(b j) built by exact FP64
// multiply-adds (every partial sum is an integer below 2^53).
template <int K>
__global__ __launch_bounds__(kTB) void pack_w_kernel(const uint8_t* __restrict__ coeffs, size_t n,
                                                     uint32_t b, double* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * kTB + threadIdx.x;
  const size_t i0 = 4 * t;
  if (i0 >= n) return;
  const int nv = n - i0 < 4 ? (int)(n - i0) : 4;
  uint32_t w[K];
  if (nv == 4) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(coeffs + i0 * K);
#pragma unroll
    for (int j = 0; j < K; ++j) w[j] = src[j];
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) w[j] = 0;
    for (int j = 0; j < nv * K; ++j) w[j >> 2] |= (uint32_t)coeffs[i0 * K + j] << (8 * (j & 3));
  }
  double qj[K];
#pragma unroll
  for (int j = 0; j < K; ++j) qj[j] = __builtin_ldexp(1.0, (int)(b * j));
  double v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double x = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int pos = e * K + j;
      x = __builtin_fma((double)((w[pos >> 2] >> (8 * (pos & 3))) & 0xffu), qj[j], x);
    }
    v[e] = x;
  }
  if (nv == 4) {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[i0 + e] = v[e];
  } else {
    for (int e = 0; e < nv; ++e) out[i0 + e] = v[e];
  }
}

hipError_t launch_pack(int k, uint64_t q, int pow2, uint32_t b, const uint8_t* coeffs, size_t n,
                       double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (pow2 && ((uintptr_t)coeffs & 3) == 0 && ((uintptr_t)out & 7) == 0) {
    const size_t gw = ((n + 3) / 4 + kTB - 1) / kTB;
    switch (k) {
#define FQT_PK_CASE(K)                                                                      \
  case K:                                                                                   \
    hipLaunchKernelGGL(pack_w_kernel<K>, dim3((unsigned)gw), dim3(kTB), 0, s, coeffs, n, b, out); \
    return hipGetLastError();
      FQT_PK_CASE(1) FQT_PK_CASE(2) FQT_PK_CASE(3) FQT_PK_CASE(4)  // fields have k <= 4
#undef FQT_PK_CASE
      default: break;
    }
  }
  const size_t grid = (n + kTB - 1) / kTB;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)grid), dim3(kTB), 0, s, coeffs, n, k, pow2, b,
                     (double)q, out);
  return hipGetLastError();
}

// ---- REDQ ------------------------------------------------------------------

struct RedqArgs {
  uint64_t q;
  double inv_q;
  double inv_p;
  uint32_t p, b, pow2, c;  // c = (-q) mod p
  uint32_t mod_magic;
  uint32_t pm24;  // 2^24 - p: x - p y modulo 2^24 as x + pm24 y
};

// Residues u_0..u_{nd-1} of Alg. 2 for r < 2^53 (binary64 input, WIDE = 0)
// or r < 2^64 (uint64 input, WIDE = 1).  Every u_i is exact in [0, p).
template <bool WIDE>
__device__ __forceinline__ void redq_residues(uint64_t r, int nd, const RedqArgs& ra,
                                              uint32_t* u) {
  const uint64_t p = ra.p;
  uint64_t rop = WIDE ? r / p : floor_div53(r, p, ra.inv_p);  // Alg. 2, first step
  uint64_t x = r, y = rop;
  for (int i = 0; i < nd; ++i) {
    u[i] = (uint32_t)(x - p * y);  // floor(r/q^i) - p floor(rop/q^i)
    if (ra.pow2) {
      x >>= ra.b;
      y >>= ra.b;
    } else if (WIDE) {
      x /= ra.q;  // Lemma 2: floor(floor(r/q^i)/q) = floor(r/q^(i+1))
      y /= ra.q;
    } else {
      x = floor_div53(x, ra.q, ra.inv_q);
      y = floor_div53(y, ra.q, ra.inv_q);
    }
  }
}

__device__ __forceinline__ uint32_t modp(uint32_t x, const RedqArgs& ra) {
  return x - __umulhi(x, ra.mod_magic) * ra.p;
}

template <bool WIDE>
__global__ __launch_bounds__(kTB) void unpack_kernel(const void* __restrict__ in, size_t n,
                                                     int k, int nd, int mode, RedqArgs ra,
                                                     FieldArgs fa, const uint32_t* __restrict__ L,
                                                     const uint32_t* __restrict__ H,
                                                     uint8_t* __restrict__ out) {
  // four values per thread, 4 kTB per workgroup; outputs staged in LDS and
  // written as 16-byte runs
  __shared__ __align__(16) uint8_t buf[4 * kTB * 16];
  const size_t base = (size_t)blockIdx.x * (4 * kTB);
  const int ob = mode == 0 ? nd : k;  // output bytes per value
  for (int j = 0; j < 4; ++j) {
    const int t = threadIdx.x + j * kTB;
    const size_t i = base + t;
    if (i >= n) break;
    uint64_t r;
    if (WIDE) r = reinterpret_cast<const uint64_t*>(in)[i];
    else r = (uint64_t)reinterpret_cast<const double*>(in)[i];
    uint32_t u[16];
    const int nr = mode == 0 ? nd : 2 * k - 1;
    redq_residues<WIDE>(r, nr, ra, u);
    uint8_t* dst = buf + t * ob;
    if (mode == 0) {
      // Q_d: mu_{nd-1} = u_{nd-1}; mu_i = u_i - q u_{i+1} = u_i + c u_{i+1} mod p.
      for (int d = 0; d < nd - 1; ++d) dst[d] = (uint8_t)modp(u[d] + ra.c * u[d + 1], ra);
      dst[nd - 1] = (uint8_t)u[nd - 1];
    } else {
      uint32_t il = 0, ih = 0;
      for (int d = 0; d < k; ++d) {
        il |= u[d] << (fa.cb * d);
        ih |= u[k - 1 + d] << (fa.cb * d);
      }
      const uint32_t tmask = (1u << (fa.cb * k)) - 1u;  // keeps lookups inside the tables
      const uint32_t e = add_bytes_mod_p(L[il & tmask], H[ih & tmask], fa);
      for (int d = 0; d < k; ++d) dst[d] = (uint8_t)(e >> (8 * d));
    }
  }
  __syncthreads();
  stage_out16(out, buf, base * ob, (size_t)(4 * kTB) * ob, n * ob);
}

static RedqArgs make_redq(uint64_t q, int pow2, uint32_t b, const FieldArgs& fa) {
  RedqArgs ra;
  ra.q = q;
  ra.inv_q = 1.0 / (double)q;
  ra.inv_p = fa.inv_p;
  ra.p = fa.p;
  ra.b = b;
  ra.pow2 = (uint32_t)pow2;
  ra.c = (uint32_t)((fa.p - (q % fa.p)) % fa.p);
  ra.mod_magic = fa.mod_magic;
  ra.pm24 = (1u << 24) - fa.p;
  return ra;
}

// The integer value of a binary64 holding an integer below 2^53, as words.
__device__ __forceinline__ uint64_t f64_to_u64(double v) {
  const double hi = __builtin_trunc(v * 0x1p-32);
  const uint32_t lo = (uint32_t)__builtin_fma(hi, -0x1p32, v);
  return ((uint64_t)(uint32_t)hi << 32) | lo;
}

// REDQ unpack for q = 2^b and binary64 input, NR residues per value known at
// compile time, word-aligned output.  Thread t unpacks values 4t .. 4t+3
// (two 16-byte loads) and writes their 4 OB output bytes as OB whole words,
// with no LDS.  rop = floor(r/p) from a binary64 estimate and one exact
// correction (fma); u_i = floor(r/q^i) - p floor(rop/q^i) lies in [0, p), so
// its low 24 bits, from the low words of the two shifted values and one
// 24-bit multiply-add, are the residue itself.  POLY: Q_d correction, NR = OB
// digits.  FIELD: L + H (Thm. 3) on NR = 2k-1 residues, OB = k bytes.
template <int NR, int OB, bool FIELD>
__global__ __launch_bounds__(kTB) void unpack_w_kernel(const double* __restrict__ in, size_t n,
                                                       RedqArgs ra, FieldArgs fa,
                                                       const uint32_t* __restrict__ L,
                                                       const uint32_t* __restrict__ H,
                                                       uint8_t* __restrict__ out) {
  constexpr int K = (NR + 1) / 2;  // FIELD: the extension degree
  const size_t t = (size_t)blockIdx.x * kTB + threadIdx.x;
  const size_t i0 = 4 * t;
  if (i0 >= n) return;
  const int nv = n - i0 < 4 ? (int)(n - i0) : 4;
  double v[4];
  if (nv == 4) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = in[i0 + e];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = e < nv ? in[i0 + e] : 0.0;
  }
  const uint32_t p = ra.p, b = ra.b, pm = ra.pm24;
  const double pd = (double)p;
  uint32_t o[OB];
#pragma unroll
  for (int w = 0; w < OB; ++w) o[w] = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    // Alg. 2's first step: rop = floor(r / p)
    double td = __builtin_floor(v[e] * ra.inv_p);
    const double rem = __builtin_fma(-pd, td, v[e]);  // exact: |rem| < 2p
    td += rem < 0.0 ? -1.0 : (rem >= pd ? 1.0 : 0.0);
    uint64_t x = f64_to_u64(v[e]), y = f64_to_u64(td);
    uint32_t u[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      u[i] = ((uint32_t)x + __umul24((uint32_t)y, pm)) & 0xffffffu;
      x >>= b;  // one digit at a time: b < 64, and digits past the value read 0
      y >>= b;
    }
    if constexpr (!FIELD) {
      // Q_d: mu_i = u_i + c u_{i+1} mod p, the top digit as it is
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        uint32_t mu = u[d];
        if (d < NR - 1) {
          const uint32_t x = u[d] + __umul24(ra.c, u[d + 1]);
          mu = (x + __umul24(__umulhi(x, ra.mod_magic), pm)) & 0xffffffu;
        }
        const int pos = e * OB + d;
        o[pos >> 2] |= mu << (8 * (pos & 3));
      }
    } else {
      uint32_t il = 0, ih = 0;
#pragma unroll
      for (int d = 0; d < K; ++d) {
        il |= u[d] << (fa.cb * d);
        ih |= u[K - 1 + d] << (fa.cb * d);
      }
      const uint32_t tmask = (1u << (fa.cb * K)) - 1u;  // keeps lookups inside the tables
      const uint32_t x = add_bytes_mod_p(L[il & tmask], H[ih & tmask], fa);
#pragma unroll
      for (int d = 0; d < OB; ++d) {
        const int pos = e * OB + d;
        o[pos >> 2] |= ((x >> (8 * d)) & 0xffu) << (8 * (pos & 3));
      }
    }
  }
  if (nv == 4) {
    uint32_t* dst = reinterpret_cast<uint32_t*>(out + i0 * OB);
#pragma unroll
    for (int w = 0; w < OB; ++w) dst[w] = o[w];
  } else {
    for (int j = 0; j < nv * OB; ++j) out[i0 * OB + j] = (uint8_t)(o[j >> 2] >> (8 * (j & 3)));
  }
}

template <int NR, int OB, bool FIELD>
static hipError_t launch_unpack_w(const double* in, size_t n, const RedqArgs& ra,
                                  const FieldArgs& fa, const uint32_t* L, const uint32_t* H,
                                  uint8_t* out, hipStream_t s) {
  const size_t grid = ((n + 3) / 4 + kTB - 1) / kTB;
  hipLaunchKernelGGL((unpack_w_kernel<NR, OB, FIELD>), dim3((unsigned)grid), dim3(kTB), 0, s, in,
                     n, ra, fa, L, H, out);
  return hipGetLastError();
}

hipError_t launch_unpack_f64(int k, uint32_t nd, int mode, uint64_t q, int pow2, uint32_t b,
                             const FieldArgs& fa, const uint32_t* L, const uint32_t* H,
                             const double* in, size_t n, uint8_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (pow2 && ((uintptr_t)out & 3) == 0 && ((uintptr_t)in & 7) == 0) {
    const RedqArgs ra = make_redq(q, pow2, b, fa);
    if (mode == 0) {
      switch (nd) {
#define FQT_UP_CASE(D) \
  case D: return launch_unpack_w<D, D, false>(in, n, ra, fa, L, H, out, s);
        FQT_UP_CASE(1) FQT_UP_CASE(2) FQT_UP_CASE(3) FQT_UP_CASE(4) FQT_UP_CASE(5)
        FQT_UP_CASE(6) FQT_UP_CASE(7) FQT_UP_CASE(8) FQT_UP_CASE(9) FQT_UP_CASE(10)
        FQT_UP_CASE(11) FQT_UP_CASE(12) FQT_UP_CASE(13) FQT_UP_CASE(14) FQT_UP_CASE(15)
#undef FQT_UP_CASE
        default: break;
      }
    } else {
      switch (k) {
#define FQT_UF_CASE(K) \
  case K: return launch_unpack_w<2 * K - 1, K, true>(in, n, ra, fa, L, H, out, s);
        FQT_UF_CASE(1) FQT_UF_CASE(2) FQT_UF_CASE(3) FQT_UF_CASE(4)  // fields have k <= 4
#undef FQT_UF_CASE
        default: break;
      }
    }
  }
  const size_t grid = (n + 4 * kTB - 1) / (4 * kTB);
  hipLaunchKernelGGL(unpack_kernel<false>, dim3((unsigned)grid), dim3(kTB), 0, s,
                     (const void*)in, n, k, (int)nd, mode, make_redq(q, pow2, b, fa), fa, L, H,
                     out);
  return hipGetLastError();
}

hipError_t launch_unpack_u64(int k, uint32_t nd, int mode, uint64_t q, int pow2, uint32_t b,
                             const FieldArgs& fa, const uint32_t* L, const uint32_t* H,
                             const uint64_t* in, size_t n, uint8_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t grid = (n + 4 * kTB - 1) / (4 * kTB);
  hipLaunchKernelGGL(unpack_kernel<true>, dim3((unsigned)grid), dim3(kTB), 0, s,
                     (const void*)in, n, k, (int)nd, mode, make_redq(q, pow2, b, fa), fa, L, H,
                     out);
  return hipGetLastError();
}

// ---- Alg. 1 on a batch of polynomial pairs -----------------------------------

// K coefficients per operand known at compile time; every workgroup takes
// kPM = 4 kTB pairs (each thread four), so the HBM transfers are 16-byte
// runs and the digit loops unroll.
constexpr int kPM = 4 * kTB;

template <int K>
__global__ __launch_bounds__(kTB) void polymul_k_kernel(const uint8_t* __restrict__ a,
                                                        const uint8_t* __restrict__ bb,
                                                        size_t n, RedqArgs ra,
                                                        uint8_t* __restrict__ c) {
  constexpr int ND = 2 * K - 1;
  __shared__ __align__(16) uint8_t sa[kPM * K];
  __shared__ __align__(16) uint8_t sb[kPM * K];
  __shared__ __align__(16) uint8_t sc[kPM * ND];
  const size_t base = (size_t)blockIdx.x * kPM;
  stage_in16(sa, a, base * K, (size_t)kPM * K, n * K);
  stage_in16(sb, bb, base * K, (size_t)kPM * K, n * K);
  __syncthreads();
  const double qd = (double)ra.q;
#pragma unroll
  for (int j = 0; j < kPM / kTB; ++j) {
    const int t = threadIdx.x + j * kTB;
    if (base + t < n) {
      const double va = dqt_eval(sa + t * K, K, ra.pow2, ra.b, qd);
      const double vb = dqt_eval(sb + t * K, K, ra.pow2, ra.b, qd);
      const double r = va * vb;  // Alg. 1 step 2: exact, r < q^(2k-1) < 2^53
      uint32_t u[ND];
      redq_residues<false>((uint64_t)r, ND, ra, u);
      uint8_t* dst = sc + t * ND;
#pragma unroll
      for (int d = 0; d < ND - 1; ++d) dst[d] = (uint8_t)modp(u[d] + ra.c * u[d + 1], ra);
      dst[ND - 1] = (uint8_t)u[ND - 1];
    }
  }
  __syncthreads();
  stage_out16(c, sc, base * ND, (size_t)kPM * ND, n * ND);
}

// Alg. 1 when every intermediate fits in 32 bits (q = 2^b, (2K-1) b <= 32,
// so r < q^(2K-1) <= 2^32), with 4-byte aligned operands and output.  No
// LDS: thread t multiplies the four pairs 4t .. 4t+3, whose operand bytes
// are K whole words of each input and whose digits are 2K-1 whole words of
// the output, so a wave reads and writes contiguous runs.  The product is
// the FP64 one of Alg. 1; rop = floor(r/p) comes from a binary64 estimate
// and one correction, the u_i of Thm. 2 from 32-bit shifts.  The last
// thread of a batch that is not a multiple of four goes byte by byte.
template <int K>
__global__ __launch_bounds__(kTB) void polymul_w32_kernel(const uint8_t* __restrict__ a,
                                                          const uint8_t* __restrict__ bb,
                                                          size_t n, RedqArgs ra,
                                                          uint8_t* __restrict__ c) {
  constexpr int ND = 2 * K - 1;
  const size_t t = (size_t)blockIdx.x * kTB + threadIdx.x;
  const size_t i0 = 4 * t;  // first pair of this thread
  if (i0 >= n) return;
  const int np = n - i0 < 4 ? (int)(n - i0) : 4;
  uint32_t wa[K], wb[K];
  if (np == 4) {
    const uint32_t* sa = reinterpret_cast<const uint32_t*>(a + i0 * K);
    const uint32_t* sb = reinterpret_cast<const uint32_t*>(bb + i0 * K);
#pragma unroll
    for (int w = 0; w < K; ++w) {
      wa[w] = sa[w];
      wb[w] = sb[w];
    }
  } else {
#pragma unroll
    for (int w = 0; w < K; ++w) wa[w] = wb[w] = 0;
    for (int j = 0; j < np * K; ++j) {
      wa[j >> 2] |= (uint32_t)a[i0 * K + j] << (8 * (j & 3));
      wb[j >> 2] |= (uint32_t)bb[i0 * K + j] << (8 * (j & 3));
    }
  }
  const uint32_t p = ra.p, b = ra.b;
  uint32_t o[ND];
#pragma unroll
  for (int w = 0; w < ND; ++w) o[w] = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    // DQT of both operands (Alg. 1 step 1)
    uint32_t va = 0, vb = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int pos = e * K + j;
      va |= ((wa[pos >> 2] >> (8 * (pos & 3))) & 0xffu) << (b * j);
      vb |= ((wb[pos >> 2] >> (8 * (pos & 3))) & 0xffu) << (b * j);
    }
    // step 2: the exact FP64 product, below 2^32
    const uint32_t r = (uint32_t)((double)va * (double)vb);
    // Alg. 2: rop = floor(r / p), then u_i = floor(r/q^i) - p floor(rop/q^i).
    // Every such difference is small (the remainder in [-p, 2p), each u_i
    // and each reduction mod p in [0, p)), so it is taken modulo 2^24 with
    // one 24-bit multiply-add by pm = 2^24 - p.
    const uint32_t pm = ra.pm24;
    uint32_t rop = (uint32_t)((double)r * ra.inv_p);
    const int32_t rem = __builtin_amdgcn_sbfe((int32_t)(r + __umul24(rop, pm)), 0, 24);
    rop = rem < 0 ? rop - 1 : (rem >= (int32_t)p ? rop + 1 : rop);
    uint32_t u[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) u[i] = ((r >> (b * i)) + __umul24(rop >> (b * i), pm)) & 0xffffffu;
    // Q_d: mu_i = u_i + c u_{i+1} mod p, the top digit as it is
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      uint32_t mu = u[d];
      if (d < ND - 1) {
        const uint32_t x = u[d] + __umul24(ra.c, u[d + 1]);
        mu = (x + __umul24(__umulhi(x, ra.mod_magic), pm)) & 0xffffffu;
      }
      const int pos = e * ND + d;
      o[pos >> 2] |= mu << (8 * (pos & 3));
    }
  }
  if (np == 4) {
    uint32_t* dst = reinterpret_cast<uint32_t*>(c + i0 * ND);
#pragma unroll
    for (int w = 0; w < ND; ++w) dst[w] = o[w];
  } else {
    for (int j = 0; j < np * ND; ++j) c[i0 * ND + j] = (uint8_t)(o[j >> 2] >> (8 * (j & 3)));
  }
}

hipError_t launch_polymul(int k, uint64_t q, int pow2, uint32_t b, const FieldArgs& fa,
                          const uint8_t* a, const uint8_t* bb, size_t n, uint8_t* c,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  const RedqArgs ra = make_redq(q, pow2, b, fa);
  const bool words = ((((uintptr_t)a) | ((uintptr_t)bb) | ((uintptr_t)c)) & 3) == 0;
  // k <= 5 always: eq. (2) needs q > k, so b >= 3 once k >= 4, and 11 b > 32
  if (pow2 && (uint32_t)(2 * k - 1) * b <= 32 && words && k <= 5) {
    const size_t gw = ((n + 3) / 4 + kTB - 1) / kTB;
    switch (k) {
#define FQT_PW_CASE(K)                                                                    \
  case K:                                                                                 \
    hipLaunchKernelGGL(polymul_w32_kernel<K>, dim3((unsigned)gw), dim3(kTB), 0, s, a, bb, n, \
                       ra, c);                                                            \
    return hipGetLastError();
      FQT_PW_CASE(1) FQT_PW_CASE(2) FQT_PW_CASE(3) FQT_PW_CASE(4) FQT_PW_CASE(5)
#undef FQT_PW_CASE
      default: break;
    }
  }
  const size_t gk = (n + kPM - 1) / kPM;
  switch (k) {
#define FQT_PM_CASE(K)                                                                   \
  case K:                                                                                \
    hipLaunchKernelGGL(polymul_k_kernel<K>, dim3((unsigned)gk), dim3(kTB), 0, s, a, bb, n, \
                       ra, c);                                                           \
    return hipGetLastError();
    FQT_PM_CASE(1) FQT_PM_CASE(2) FQT_PM_CASE(3) FQT_PM_CASE(4)
    FQT_PM_CASE(5) FQT_PM_CASE(6) FQT_PM_CASE(7) FQT_PM_CASE(8)
#undef FQT_PM_CASE
    default: return hipErrorInvalidValue;  // k is checked on the host (1..8)
  }
}

}  // namespace fqt
