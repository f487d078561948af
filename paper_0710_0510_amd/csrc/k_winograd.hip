// Block additions of Winograd's recursion over GF(p^k): Z = X + Y or X - Y,
// coefficient-wise mod p, on row-strided matrices of k-byte elements.
// HBM-bound.  Each thread takes V consecutive bytes of one row; V = 16 or 4
// when every row start is aligned to V, and then works on 32-bit words, four
// coefficients at once (p <= 127: byte sums stay below 2p and never carry).

#include <algorithm>

#include "fqt_internal.h"

namespace fqt {

// x + y (sub: x - y) mod p in every byte of a word, bytes in [0, p).
__device__ __forceinline__ uint32_t addsub_word(uint32_t x, uint32_t y, uint32_t p4, uint32_t magic,
                                                uint32_t p, int sub) {
  const uint32_t yy = sub ? p4 - y : y;  // p - y per byte, in [1, p]: no borrow
  const uint32_t s = x + yy;
  const uint32_t t = (s + magic) & 0x80808080u;  // bit 7 set where the byte is >= p
  return s - (t >> 7) * p;
}

template <int V>
__global__ __launch_bounds__(256) void mat_addsub_kernel(const uint8_t* __restrict__ X, int64_t ldx,
                                                         const uint8_t* __restrict__ Y, int64_t ldy,
                                                         uint8_t* __restrict__ Z, int64_t ldz,
                                                         int64_t rows, int64_t rowbytes, uint32_t p,
                                                         int sub) {
  const int64_t per_row = (rowbytes + V - 1) / V;
  const int64_t total = rows * per_row;
  const uint32_t p4 = p * 0x01010101u, magic = (0x80u - p) * 0x01010101u;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / per_row, c0 = (t - r * per_row) * V;
    const uint8_t* x = X + r * ldx + c0;
    const uint8_t* y = Y + r * ldy + c0;
    uint8_t* z = Z + r * ldz + c0;
    if constexpr (V == 16) {
      if (c0 + 16 <= rowbytes) {
        const uint4 a = *reinterpret_cast<const uint4*>(x);
        const uint4 b = *reinterpret_cast<const uint4*>(y);
        uint4 o;
        o.x = addsub_word(a.x, b.x, p4, magic, p, sub);
        o.y = addsub_word(a.y, b.y, p4, magic, p, sub);
        o.z = addsub_word(a.z, b.z, p4, magic, p, sub);
        o.w = addsub_word(a.w, b.w, p4, magic, p, sub);
        *reinterpret_cast<uint4*>(z) = o;
        continue;
      }
    } else if constexpr (V == 4) {
      if (c0 + 4 <= rowbytes) {
        *reinterpret_cast<uint32_t*>(z) =
            addsub_word(*reinterpret_cast<const uint32_t*>(x),
                        *reinterpret_cast<const uint32_t*>(y), p4, magic, p, sub);
        continue;
      }
    }
    // ragged end of a row (or V = 1): byte by byte
    for (int j = 0; j < V && c0 + j < rowbytes; ++j) {
      const uint32_t yv = y[j];
      const uint32_t v = x[j] + (sub ? p - yv : yv);  // p - 0 = p: x + p reduces to x
      z[j] = (uint8_t)(v >= p ? v - p : v);
    }
  }
}

hipError_t launch_mat_addsub(int k, uint32_t p, const uint8_t* X, int64_t ldx, const uint8_t* Y,
                             int64_t ldy, uint8_t* Z, int64_t ldz, int64_t rows, int64_t cols,
                             bool sub, hipStream_t s) {
  const int64_t rowbytes = cols * k, bx = ldx * k, by = ldy * k, bz = ldz * k;
  if (rows == 0 || rowbytes == 0) return hipSuccess;
  const uintptr_t bits = (uintptr_t)X | (uintptr_t)Y | (uintptr_t)Z | (uintptr_t)bx |
                         (uintptr_t)by | (uintptr_t)bz;
  const int V = (bits & 15) == 0 ? 16 : (bits & 3) == 0 ? 4 : 1;
  const int64_t total = rows * ((rowbytes + V - 1) / V);
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 16384);
  switch (V) {
    case 16:
      hipLaunchKernelGGL(mat_addsub_kernel<16>, dim3(blocks), dim3(256), 0, s, X, bx, Y, by, Z, bz,
                         rows, rowbytes, p, sub ? 1 : 0);
      break;
    case 4:
      hipLaunchKernelGGL(mat_addsub_kernel<4>, dim3(blocks), dim3(256), 0, s, X, bx, Y, by, Z, bz,
                         rows, rowbytes, p, sub ? 1 : 0);
      break;
    default:
      hipLaunchKernelGGL(mat_addsub_kernel<1>, dim3(blocks), dim3(256), 0, s, X, bx, Y, by, Z, bz,
                         rows, rowbytes, p, sub ? 1 : 0);
  }
  return hipGetLastError();
}

}  // namespace fqt
