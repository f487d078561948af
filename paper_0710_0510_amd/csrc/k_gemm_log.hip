// GF(p^k) GEMM on discrete-log codes (Section 7, Alg. 4) on gfx950, and the
// element-wise kernels of the log representation.
//
// A code e < m = p^k - 1 stands for g^e, the code m for zero (codes above m
// read as zero).  The GEMM runs Alg. 4 per output: the packed value of every
// operand code is one lookup in a table of evaluations at q (held in LDS),
// the packed products are contracted exactly on the FP64 MFMA, REDQ gives the
// residues u, Thm. 3's L and H tables return codes, and R = H + L is the
// field addition of codes through the Zech table Z[n] = log(1 + g^n).  The
// register-direct tiles of fqt_direct.h carry it with 2-byte operands; their
// K-block handling (one block, REDQ residue lanes or digit sums) is the one
// of the coefficient form, since blocks add before L and H.

#include "fqt_direct.h"

namespace fqt {

template <int KE, int TM, int TN, int SK, int NWV, int MODE>
static hipError_t log_one(const GemmArgs& g, const PackedParams& pp, hipStream_t s) {
  using T = DT<2, TM, TN, SK, NWV>;
  const int tiles_m = (int)((g.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((g.N + T::BN - 1) / T::BN);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  const size_t dyn = log_lds_bytes(pp.tbl_log2, pp.zero_code);
  hipLaunchKernelGGL((gemm_direct_kernel<KE, TM, TN, SK, NWV, MODE, kDirectStages, true>),
                     dim3(ntiles), dim3(64 * NWV), dyn, s, g, pp, tiles_n, ntiles);
  return hipGetLastError();
}

#define FQT_LOG_CASE(ID, TM, TN, SK, NWV, MULTI_OK)                                \
  case ID:                                                                          \
    if constexpr ((MODE == 0 || MULTI_OK) && (MODE != 2 || digit_sums_fit<KE>()))   \
      return log_one<KE, TM, TN, SK, NWV, MODE>(g, pp, s);                          \
    else                                                                            \
      return hipErrorInvalidValue;

template <int KE, int MODE>
static hipError_t log_dispatch(int tile, const GemmArgs& g, const PackedParams& pp,
                               hipStream_t s) {
  switch (tile) { FQT_LOG_TILES(FQT_LOG_CASE) default: return hipErrorInvalidValue; }
}
#undef FQT_LOG_CASE

hipError_t launch_gemm_log(int k, int tile, int mode, const GemmArgs& g, const PackedParams& pp,
                           hipStream_t s) {
#define FQT_LOG_MODES(KE)                                                  \
  switch (mode) {                                                          \
    case 0: return log_dispatch<KE, 0>(tile, g, pp, s);                    \
    case 1: return log_dispatch<KE, 1>(tile, g, pp, s);                    \
    case 2: return log_dispatch<KE, 2>(tile, g, pp, s);                    \
    default: return hipErrorInvalidValue;                                  \
  }
  switch (k) {
    case 1: FQT_LOG_MODES(1)
    case 2: FQT_LOG_MODES(2)
    case 3: FQT_LOG_MODES(3)
    case 4: FQT_LOG_MODES(4)
    default: return hipErrorInvalidValue;
  }
#undef FQT_LOG_MODES
}

bool log_tile_fits(int tile, uint32_t tbl_log2, uint32_t zero_code) {
  const size_t dyn = log_lds_bytes(tbl_log2, zero_code);
  size_t red = 0;
#define FQT_LOG_RED(ID, TM, TN, SK, NWV, MULTI_OK) \
  if (tile == ID) red = sizeof(double) * DT<2, TM, TN, SK, NWV>::RED;
  FQT_LOG_TILES(FQT_LOG_RED)
#undef FQT_LOG_RED
  return red + dyn + 64 <= 160 * 1024;
}

// ---- element-wise kernels ------------------------------------------------------

// Coefficient form -> code: the binary index sum c_i 2^(cb i) (Section 5.3)
// looks up the code; indices with a coefficient >= p hold the zero code.
__global__ __launch_bounds__(256) void to_log_kernel(int k, uint32_t cb, const uint8_t* __restrict__ x,
                                                     int64_t n, const uint16_t* __restrict__ logt,
                                                     uint16_t* __restrict__ codes) {
  const uint32_t cmask = (1u << cb) - 1u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t idx = 0;
    for (int j = 0; j < k; ++j) idx |= ((uint32_t)x[i * k + j] & cmask) << (cb * j);
    codes[i] = logt[idx];
  }
}

// Code -> coefficient form: k bytes of the word expw[code].
__global__ __launch_bounds__(256) void from_log_kernel(int k, const uint16_t* __restrict__ codes,
                                                       int64_t n, uint32_t zero,
                                                       const uint32_t* __restrict__ expw,
                                                       uint8_t* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t w = expw[min((uint32_t)codes[i], zero)];
    for (int j = 0; j < k; ++j) x[i * k + j] = (uint8_t)(w >> (8 * j));
  }
}

// c = a + b on codes through the Zech table.
__global__ __launch_bounds__(256) void log_add_kernel(const uint16_t* __restrict__ a,
                                                      const uint16_t* __restrict__ b, int64_t n,
                                                      uint32_t zero, const uint16_t* __restrict__ Z,
                                                      uint16_t* c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = min((uint32_t)a[i], zero), y = min((uint32_t)b[i], zero);
    c[i] = (uint16_t)zech_add(x, y, zero, Z);
  }
}

static dim3 ew_grid(int64_t n) {
  const int64_t blocks = (n + 255) / 256;
  return dim3((unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192));
}

hipError_t launch_to_log(int k, uint32_t cb, const uint8_t* coeffs, int64_t n,
                         const uint16_t* logt, uint16_t* codes, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_log_kernel, ew_grid(n), dim3(256), 0, s, k, cb, coeffs, n, logt, codes);
  return hipGetLastError();
}

hipError_t launch_from_log(int k, const uint16_t* codes, int64_t n, uint32_t zero_code,
                           const uint32_t* expw, uint8_t* coeffs, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(from_log_kernel, ew_grid(n), dim3(256), 0, s, k, codes, n, zero_code, expw,
                     coeffs);
  return hipGetLastError();
}

hipError_t launch_log_add(const uint16_t* a, const uint16_t* b, int64_t n, uint32_t zero_code,
                          const uint16_t* Z, uint16_t* c, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(log_add_kernel, ew_grid(n), dim3(256), 0, s, a, b, n, zero_code, Z, c);
  return hipGetLastError();
}

}  // namespace fqt
