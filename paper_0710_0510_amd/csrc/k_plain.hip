// Plain comparator GEMM over GF(p^k): the classical method that the FQT is
// measured against.  Every product of two elements is a schoolbook
// polynomial product whose 2k-1 coefficients are reduced mod p, then divided
// by the defining polynomial P, then added into the accumulator mod p.  No
// packing, no matrix cores, no delayed reduction.  Operand tiles are staged
// through LDS so that the comparison measures arithmetic, not memory.

#include "fqt_internal.h"

namespace fqt {

template <int KE>
__global__ __launch_bounds__(256) void gemm_plain_kernel(GemmArgs g, FieldArgs fa,
                                                         PlainFieldArgs pf) {
  constexpr int T = 16;
  __shared__ uint32_t As[T][T + 1];
  __shared__ uint32_t Bs[T][T + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t row = (int64_t)blockIdx.y * T + ty;
  const int64_t col = (int64_t)blockIdx.x * T + tx;
  uint32_t acc[KE];
#pragma unroll
  for (int s = 0; s < KE; ++s) acc[s] = 0;
  for (int64_t k0 = 0; k0 < g.K; k0 += T) {
    const int64_t ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (row < g.M && ka < g.K) ? load_elem<KE>(g.A + (row * g.lda + ka) * KE) : 0u;
    Bs[ty][tx] = (kb < g.K && col < g.N) ? load_elem<KE>(g.B + (kb * g.ldb + col) * KE) : 0u;
    __syncthreads();
    for (int l = 0; l < T; ++l) {
      const uint32_t x = As[ty][l], y = Bs[l][tx];
      uint32_t c[2 * KE - 1];
#pragma unroll
      for (int t = 0; t < 2 * KE - 1; ++t) c[t] = 0;
#pragma unroll
      for (int i = 0; i < KE; ++i)
#pragma unroll
        for (int j = 0; j < KE; ++j) c[i + j] += ((x >> (8 * i)) & 0xffu) * ((y >> (8 * j)) & 0xffu);
#pragma unroll
      for (int t = 0; t < 2 * KE - 1; ++t) c[t] = mod_p_small(c[t], fa);
      // long division by the monic P: X^k = -sum P_low[i] X^i
#pragma unroll
      for (int t = 2 * KE - 2; t >= KE; --t) {
        const uint32_t lead = c[t];
#pragma unroll
        for (int i = 0; i < KE; ++i)
          c[t - KE + i] = mod_p_small(c[t - KE + i] + lead * (fa.p - pf.P_low[i]), fa);
      }
#pragma unroll
      for (int s = 0; s < KE; ++s) acc[s] = mod_p_small(acc[s] + c[s], fa);
    }
    __syncthreads();
  }
  if (row < g.M && col < g.N) {
    uint32_t e = 0;
#pragma unroll
    for (int s = 0; s < KE; ++s) e |= acc[s] << (8 * s);
    store_elem<KE>(g.C + (row * g.ldc + col) * KE, e);
  }
}

hipError_t launch_gemm_plain(int k, const GemmArgs& g, const FieldArgs& fa,
                             const uint32_t* P_low, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  PlainFieldArgs pf{};
  for (int i = 0; i < k && i < 4; ++i) pf.P_low[i] = P_low[i] % fa.p;
  const dim3 grid((unsigned)((g.N + 15) / 16), (unsigned)((g.M + 15) / 16));
  switch (k) {
    case 1: hipLaunchKernelGGL(gemm_plain_kernel<1>, grid, dim3(256), 0, s, g, fa, pf); break;
    case 2: hipLaunchKernelGGL(gemm_plain_kernel<2>, grid, dim3(256), 0, s, g, fa, pf); break;
    case 3: hipLaunchKernelGGL(gemm_plain_kernel<3>, grid, dim3(256), 0, s, g, fa, pf); break;
    case 4: hipLaunchKernelGGL(gemm_plain_kernel<4>, grid, dim3(256), 0, s, g, fa, pf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fqt
