// d-FQT products of long polynomials over GF(p) on gfx950 (Section 6), and
// the classical product with delayed reduction it is compared with.
//
// d-FQT: a polynomial of len coefficients is split into nch = ceil(len/(d+1))
// chunks of d+1 coefficients, each packed at q = 2^b into one binary64 (DQT,
// eq. (1)).  The product is the convolution S_t = sum_i P_i Q_{t-i} of the
// packed chunks (t = 0..2nch-2), accumulated exactly in FP64 in blocks of at
// most n_q products (eq. (2) with k = d+1); each block leaves its 2d+1 digits
// in the per-element state of fqt_packed.h (one block: REDQ_{2d+1} of the
// biased accumulator; several: residue lanes or digit sums), which yields
// Thm. 2's residues u_i of S_t; the Q_d correction turns them into the digits
// mod p.  Digit j of S_t is the coefficient of X^(t(d+1)+j); consecutive S_t
// overlap in d digits, which are added mod p.
//
// One wave per product, four per workgroup.  The packed chunks of both
// operands sit in LDS, sized at launch for the longest operand, so short
// operands leave room for more workgroups per CU.  Lane l accumulates S_t for the four consecutive
// t = t0 + 4l .. t0 + 4l + 3 over a chunk index i that runs in step across
// the wave (so P_i is one broadcast read), keeping Q_{t-i} .. Q_{t+3-i} as a
// sliding window (one more read per i); out-of-range chunks read as zero,
// which only adds zero products to a block.  Passes t0 = 0, 256, ... cover
// t = 0..2nch-1 (the last t has no products of its own and only receives the
// overlapping digits of the one before).  The digits that overlap into t come
// from t-1: the same lane for r > 0, the previous lane (a shuffle) for r = 0,
// lane 63 of the previous pass for the first lane.
// Pairs of uneven lengths (la, lb) run the same convolution over nca and
// ncb chunks, every wave taking its share of the pairs (dfqt_batched_kernel).

#include "fqt_packed.h"

#include <map>
#include <mutex>

namespace fqt {

// DQT of one chunk from its coefficient bytes (those at or past len read as
// zero): sum_j c_j 2^(b j) < 2^52, exact in binary64; centred chunks take
// c - p for c > (p-1)/2 (a signed sum, as exact).
template <int KE, bool CEN>
__device__ __forceinline__ double dfqt_chunk(const uint32_t (&c)[KE], int first, int len,
                                             uint32_t b, int32_t p, int32_t h) {
  // sums of (possibly negative) c_j 2^(b j) in two's complement mod 2^64;
  // the true value is below 2^52 in magnitude
  uint64_t v = 0;
#pragma unroll
  for (int j = 0; j < KE; ++j) {
    int32_t cx = first + j < len ? (int32_t)c[j] : 0;
    if constexpr (CEN) cx -= cx > h ? p : 0;
    v += (uint64_t)(int64_t)cx << (b * j);
  }
  return (double)(int64_t)v;
}

// DQT of the chunks of one operand of len coefficients into X[0 .. nch).  The
// lanes of one wave split the chunks, two per lane and step; every byte is
// read at an index clamped into the operand, so the loads carry no branch
// and all of a step's loads are in flight together.
template <int KE, bool CEN>
__device__ __forceinline__ void dfqt_pack(const uint8_t* __restrict__ x, int len, int nch,
                                          uint32_t b, const PackedParams& pp,
                                          double* __restrict__ X, int lane) {
  const int32_t p = (int32_t)pp.fa.p, h = (p - 1) / 2;
  for (int i = lane; i < nch; i += 128) {
    const int i2 = i + 64;
    uint32_t c0[KE], c1[KE];
#pragma unroll
    for (int j = 0; j < KE; ++j) {
      c0[j] = x[min(i * KE + j, len - 1)];
      c1[j] = x[min(i2 * KE + j, len - 1)];
    }
    X[i] = dfqt_chunk<KE, CEN>(c0, i * KE, len, b, p, h);
    if (i2 < nch) X[i2] = dfqt_chunk<KE, CEN>(c1, i2 * KE, len, b, p, h);
  }
}

// The product of one pair by one wave from its packed chunks P (nca) and Q
// (ncb) in LDS: S_t = sum_i P_i Q_{t-i} for t = 0 .. nca + ncb - 2, blocks of
// nq products, digits mod p, overlap-add into the nc = la + lb - 1 output
// coefficients.  Q[-1] and Q[ncb] hold zero: a window read clamps its index
// into [-1, ncb] instead of branching.
template <int KE, int MODE, bool CEN>
__device__ __forceinline__ void dfqt_convolve(const double* __restrict__ P, int nca,
                                              const double* __restrict__ Q, int ncb, int nc,
                                              uint8_t* __restrict__ pc, uint32_t nq, uint32_t b,
                                              const PackedParams& pp, int lane) {
  constexpr int ND = 2 * KE - 1;
  constexpr bool MULTI = MODE != 0;
  const int nt = nca + ncb;  // t = 0 .. nca + ncb - 1
  // every block starts from 2^52 (centred: plus q/2 in every digit)
  const double bz = CEN ? pp.cbias : kTwo52;
  uint32_t carry[KE > 1 ? KE - 1 : 1];
#pragma unroll
  for (int j = 0; j < KE - 1; ++j) carry[j] = 0;
  for (int t0 = 0; t0 < nt; t0 += 256) {
    const int tb = t0 + 4 * lane;
    double acc[4];
    BlockLanes<KE, MODE> st[MULTI ? 4 : 1];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = bz;
    if constexpr (MULTI) {
#pragma unroll
      for (int r = 0; r < 4; ++r) st[r].clear();
    }
    const int ilo = max(0, t0 - (ncb - 1)), ihi = min(nca - 1, t0 + 255);
    auto qat = [&](int j) { return Q[min(max(j, -1), ncb)]; };
    double qw[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) qw[r] = qat(tb + r - ilo);
    uint32_t cnt = 0, nbound = 0, nblk = 1;  // blocks of this pass (the centred shift counts them)
    uint32_t nadd = 0;                       // blocks in the lane state since its last fold
    // one chunk index i: P_i times the window, the block step when a block
    // is full, the window slid one chunk down Q (qn = Q_{t-i-1})
    auto step = [&](double pi, double qn) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = __builtin_fma(pi, qw[r], acc[r]);
      if constexpr (MULTI) {
        if (++cnt == nq) {
          cnt = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            st[r].add(acc[r], pp.fa);
            acc[r] = bz;
          }
          ++nblk;
          ++nadd;
          if (pp.fold_blocks && ++nbound == pp.fold_blocks) {
            nbound = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) st[r].fold(pp.fa, nadd);
            nadd = 0;
          }
        }
      }
      qw[3] = qw[2];
      qw[2] = qw[1];
      qw[1] = qw[0];
      qw[0] = qn;
    };
    // four chunk indices per round, their P and Q reads issued together
    int i = ilo;
    for (; i + 3 <= ihi; i += 4) {
      const double p0 = P[i], p1 = P[i + 1], p2 = P[i + 2], p3 = P[i + 3];
      const int j = tb - i - 1;
      const double n0 = qat(j), n1 = qat(j - 1), n2 = qat(j - 2), n3 = qat(j - 3);
      step(p0, n0);
      step(p1, n1);
      step(p2, n2);
      step(p3, n3);
    }
    for (; i <= ihi; ++i) step(P[i], qat(tb - i - 1));

    // Thm. 2's residues u_i, then Alg. 2's second part (the Q_d correction of
    // Section 5.1): digit i mod p is (u_i - q u_{i+1}) mod p, the top one u_2d
    // centred: every digit carries q/2 per block, taken off mod p
    const uint32_t shift = CEN ? (pp.fa.p - (nblk % pp.fa.p) * pp.c0neg % pp.fa.p) % pp.fa.p : 0u;
    uint32_t u[4][ND];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      st[MULTI ? r : 0].residues(acc[r], b, pp, u[r], nadd);
#pragma unroll
      for (int i = 0; i < ND - 1; ++i) u[r][i] = mod_p_small(u[r][i] + pp.fa.c * u[r][i + 1], pp.fa);
      if constexpr (CEN) {
#pragma unroll
        for (int i = 0; i < ND; ++i) u[r][i] = mod_p_small(u[r][i] + shift, pp.fa);
      }
    }
    // digits d+1..2d of S_{tb-1}: previous lane's last t, or the carried ones
    uint32_t prev[KE > 1 ? KE - 1 : 1];
#pragma unroll
    for (int j = 0; j < KE - 1; ++j) {
      const uint32_t up = (uint32_t)__shfl_up((int)u[3][KE + j], 1, 64);
      prev[j] = lane == 0 ? carry[j] : up;
      carry[j] = (uint32_t)__shfl((int)u[3][KE + j], 63, 64);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = tb + r;
      if (t >= nt) break;
#pragma unroll
      for (int j = 0; j < KE; ++j) {
        const int n = t * KE + j;
        if (n >= nc) break;
        uint32_t v = u[r][j];
        if (j < KE - 1) v += r ? u[r - 1][KE + j] : prev[j];
        pc[n] = (uint8_t)(v >= pp.fa.p ? v - pp.fa.p : v);
      }
    }
  }
}

// One wave per product, four per workgroup, every pair of len coefficients.
template <int KE, int MODE, bool CEN>
__global__ __launch_bounds__(256) void dfqt_kernel(DfqtArgs g) {
  extern __shared__ double dsh[];  // 4 waves x (P, zero, Q, zero): 2 cap + 2 chunks
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t prod = (int64_t)blockIdx.x * 4 + w;
  const bool live = prod < g.count;  // idle waves still reach every barrier
  double* P = dsh + (size_t)w * (2 * g.cap + 2);
  double* Q = P + g.cap + 1;
  const uint32_t b = MODE ? multi_block_b<KE>() : g.lg2q;
  const int len = g.len, nch = g.nch;
  const uint8_t* pa = g.a + (live ? prod : 0) * len;
  const uint8_t* pb = g.b + (live ? prod : 0) * len;
  uint8_t* pc = g.c + (live ? prod : 0) * (int64_t)(2 * len - 1);
  if (live) {
    dfqt_pack<KE, CEN>(pa, len, nch, b, g.pp, P, lane);
    dfqt_pack<KE, CEN>(pb, len, nch, b, g.pp, Q, lane);
    if (lane == 0) Q[-1] = Q[nch] = 0.0;
  }
  __syncthreads();
  if (!live) return;  // no barrier below
  dfqt_convolve<KE, MODE, CEN>(P, nch, Q, nch, 2 * len - 1, pc, g.nq, b, g.pp, lane);
}

// Uneven batch: the host orders the pairs longest first and wave w of W
// takes, in round r, pair r W + w (r even) or r W + W - 1 - w (r odd), so
// the cost is spread evenly without a shared queue (one atomic counter
// hammered by every wave of 8 XCDs costs more than short pairs do).  Each
// pair is computed alone in the wave's LDS region: pack both operands, a
// wave-wide fence, the convolution; the next pair's descriptor is read
// while the current one runs.
template <int KE, int MODE, bool CEN>
__global__ __launch_bounds__(256) void dfqt_batched_kernel(DfqtBatchArgs g) {
  extern __shared__ double dsh[];  // 4 waves x (P, zero, Q, zero): 2 cap + 2 chunks
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  const int W = (int)gridDim.x * 4;
  double* P = dsh + (size_t)(w & 3) * (2 * g.cap + 2);
  double* Q = P + g.cap + 1;
  const uint32_t b = MODE ? multi_block_b<KE>() : g.lg2q;
  auto pick = [&](int r) -> int64_t {
    const int64_t it = (int64_t)r * W + ((r & 1) ? W - 1 - w : w);
    return it < g.count ? it : -1;
  };
  int64_t it = pick(0);
  PolyDesc d{};
  if (it >= 0) d = g.descs[g.order ? g.order[it] : it];
  for (int r = 0; it >= 0; ++r) {
    const int64_t nx = pick(r + 1);
    PolyDesc dn{};
    if (nx >= 0) dn = g.descs[g.order ? g.order[nx] : nx];
    const int la = __builtin_amdgcn_readfirstlane((int)d.la);
    const int lb = __builtin_amdgcn_readfirstlane((int)d.lb);
    if (la > 0 && lb > 0) {
      const int nca = (la + KE - 1) / KE, ncb = (lb + KE - 1) / KE;
      // the previous pair's reads of P and Q are done before they are rewritten
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      dfqt_pack<KE, CEN>(d.a, la, nca, b, g.pp, P, lane);
      dfqt_pack<KE, CEN>(d.b, lb, ncb, b, g.pp, Q, lane);
      if (lane == 0) Q[-1] = Q[ncb] = 0.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      dfqt_convolve<KE, MODE, CEN>(P, nca, Q, ncb, la + lb - 1, d.c, g.nq, b, g.pp, lane);
    }
    it = nx;
    d = dn;
  }
}

// Classical product, delayed reduction (eq. (3)): c_n = sum_i a_i b_{n-i} in
// INT32, reduced mod p once, or every n_d products when len (p-1)^2 would
// overflow.  Same wave layout as the d-FQT kernel, on coefficients.
__global__ __launch_bounds__(256) void polymul_delayed_kernel(DelayedArgs g) {
  __shared__ uint8_t sh[4][2][kDelayedMaxLen];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t prod = (int64_t)blockIdx.x * 4 + w;
  const bool live = prod < g.count;
  uint8_t* A = sh[w][0];
  uint8_t* B = sh[w][1];
  const int len = g.len;
  const uint8_t* pa = g.a + (live ? prod : 0) * len;
  const uint8_t* pb = g.b + (live ? prod : 0) * len;
  uint8_t* pc = g.c + (live ? prod : 0) * (int64_t)(2 * len - 1);
  if (live)
    for (int i = lane; i < len; i += 64) {
      A[i] = pa[i];
      B[i] = pb[i];
    }
  __syncthreads();
  if (!live) return;
  const int nout = 2 * len - 1;
  for (int n0 = 0; n0 < nout; n0 += 256) {
    const int nb = n0 + 4 * lane;
    uint32_t acc[4] = {0, 0, 0, 0};
    const int ilo = max(0, n0 - (len - 1)), ihi = min(len - 1, n0 + 255);
    uint32_t bw[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = nb + r - ilo;
      bw[r] = (j >= 0 && j < len) ? B[j] : 0u;
    }
    uint32_t cnt = 0;
    for (int i = ilo; i <= ihi; ++i) {
      const uint32_t ai = A[i];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += ai * bw[r];
      if (g.nd && ++cnt == g.nd) {
        cnt = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] %= g.p;
      }
      bw[3] = bw[2];
      bw[2] = bw[1];
      bw[1] = bw[0];
      const int j = nb - i - 1;
      bw[0] = (j >= 0 && j < len) ? B[j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (nb + r < nout) pc[nb + r] = (uint8_t)(acc[r] % g.p);
  }
}

// LDS of one workgroup: four waves, two operands of cap chunks each and the
// two zero chunks around the second
static size_t dfqt_lds_bytes(int32_t cap) {
  return (size_t)4 * (2 * (size_t)cap + 2) * sizeof(double);
}

template <int KE, bool CEN>
static hipError_t dfqt_k(int mode, const DfqtArgs& g, hipStream_t s) {
  if (g.cap < g.nch || g.cap > kDfqtMaxChunks) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.count + 3) / 4));
  const size_t lds = dfqt_lds_bytes(g.cap);
  switch (mode) {
    case 0: hipLaunchKernelGGL((dfqt_kernel<KE, 0, CEN>), grid, dim3(256), lds, s, g); break;
    case 1: hipLaunchKernelGGL((dfqt_kernel<KE, 1, CEN>), grid, dim3(256), lds, s, g); break;
    case 2:
      if constexpr (digit_sums_fit<KE>()) {
        hipLaunchKernelGGL((dfqt_kernel<KE, 2, CEN>), grid, dim3(256), lds, s, g);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KE>
static hipError_t dfqt_k(int mode, const DfqtArgs& g, hipStream_t s) {
  return g.pp.centered ? dfqt_k<KE, true>(mode, g, s) : dfqt_k<KE, false>(mode, g, s);
}

template <int KE, bool CEN>
static hipError_t dfqt_bk(int mode, const DfqtBatchArgs& g, int grid, hipStream_t s) {
  if (g.cap < 1 || g.cap > kDfqtMaxChunks) return hipErrorInvalidValue;
  const size_t lds = dfqt_lds_bytes(g.cap);
  switch (mode) {
    case 0: hipLaunchKernelGGL((dfqt_batched_kernel<KE, 0, CEN>), grid, dim3(256), lds, s, g); break;
    case 1: hipLaunchKernelGGL((dfqt_batched_kernel<KE, 1, CEN>), grid, dim3(256), lds, s, g); break;
    case 2:
      if constexpr (digit_sums_fit<KE>()) {
        hipLaunchKernelGGL((dfqt_batched_kernel<KE, 2, CEN>), grid, dim3(256), lds, s, g);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KE>
static hipError_t dfqt_bk(int mode, const DfqtBatchArgs& g, int grid, hipStream_t s) {
  return g.pp.centered ? dfqt_bk<KE, true>(mode, g, grid, s)
                       : dfqt_bk<KE, false>(mode, g, grid, s);
}

hipError_t launch_dfqt(int ke, int mode, const DfqtArgs& g, hipStream_t s) {
  if (g.count == 0) return hipSuccess;
  switch (ke) {
    case 1: return dfqt_k<1>(mode, g, s);
    case 2: return dfqt_k<2>(mode, g, s);
    case 3: return dfqt_k<3>(mode, g, s);
    case 4: return dfqt_k<4>(mode, g, s);
    case 5: return dfqt_k<5>(mode, g, s);
    case 6: return dfqt_k<6>(mode, g, s);
    case 7: return dfqt_k<7>(mode, g, s);
    case 8: return dfqt_k<8>(mode, g, s);
    default: return hipErrorInvalidValue;
  }
}

template <int KE, int MODE, bool CEN>
static int dfqt_occ(int32_t cap) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks, (const void*)dfqt_batched_kernel<KE, MODE, CEN>, 256,
          dfqt_lds_bytes(cap)) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

template <int KE, bool CEN>
static int dfqt_occ(int mode, int32_t cap) {
  switch (mode) {
    case 0: return dfqt_occ<KE, 0, CEN>(cap);
    case 1: return dfqt_occ<KE, 1, CEN>(cap);
    case 2:
      if constexpr (digit_sums_fit<KE>()) return dfqt_occ<KE, 2, CEN>(cap);
      return 1;
    default: return 1;
  }
}

template <int KE>
static int dfqt_occ(int mode, bool centered, int32_t cap) {
  return centered ? dfqt_occ<KE, true>(mode, cap) : dfqt_occ<KE, false>(mode, cap);
}

int dfqt_batched_occupancy(int ke, int mode, bool centered, int32_t cap) {
  switch (ke) {
    case 1: return dfqt_occ<1>(mode, centered, cap);
    case 2: return dfqt_occ<2>(mode, centered, cap);
    case 3: return dfqt_occ<3>(mode, centered, cap);
    case 4: return dfqt_occ<4>(mode, centered, cap);
    case 5: return dfqt_occ<5>(mode, centered, cap);
    case 6: return dfqt_occ<6>(mode, centered, cap);
    case 7: return dfqt_occ<7>(mode, centered, cap);
    case 8: return dfqt_occ<8>(mode, centered, cap);
    default: return 1;
  }
}

hipError_t launch_dfqt_batched(int ke, int mode, const DfqtBatchArgs& g, int grid,
                               hipStream_t s) {
  switch (ke) {
    case 1: return dfqt_bk<1>(mode, g, grid, s);
    case 2: return dfqt_bk<2>(mode, g, grid, s);
    case 3: return dfqt_bk<3>(mode, g, grid, s);
    case 4: return dfqt_bk<4>(mode, g, grid, s);
    case 5: return dfqt_bk<5>(mode, g, grid, s);
    case 6: return dfqt_bk<6>(mode, g, grid, s);
    case 7: return dfqt_bk<7>(mode, g, grid, s);
    case 8: return dfqt_bk<8>(mode, g, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- the batch without allocation ---------------------------------------------
// One scratch array per GPU (kept until the process ends): the descriptors
// in schedule order.  Calls that overlap on one GPU share it and race.
static __device__ __align__(256) uint8_t scratch[kDfqtNoAllocScratch];

// The device address of the current GPU's copy of `scratch`, looked up once
// per device with that device current (the array's name in host code is a
// host-side stand-in, never passed to a kernel).
static hipError_t noalloc_scratch(uint8_t** out) {
  static std::mutex mu;
  static std::map<int, uint8_t*> ptrs;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it == ptrs.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = ptrs.emplace(dev, static_cast<uint8_t*>(p)).first;
  }
  *out = it->second;
  return hipSuccess;
}

hipError_t launch_dfqt_batched_noalloc(int ke, int mode, DfqtBatchArgs g,
                                       const PolyDesc* host_descs, int grid, hipStream_t s) {
  if (g.count < 0 || (size_t)g.count > kDfqtNoAllocMaxPairs) return hipErrorInvalidValue;
  uint8_t* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return e;
  PolyDesc* descs = reinterpret_cast<PolyDesc*>(base);
  if (g.count == 0) return hipSuccess;
  e = hipMemcpyAsync(descs, host_descs, sizeof(PolyDesc) * (size_t)g.count,
                     hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  g.descs = descs;
  g.order = nullptr;  // the descriptors are in schedule order
  return launch_dfqt_batched(ke, mode, g, grid, s);
}

hipError_t launch_polymul_delayed(const DelayedArgs& g, hipStream_t s) {
  if (g.count == 0) return hipSuccess;
  hipLaunchKernelGGL(polymul_delayed_kernel, dim3((unsigned)((g.count + 3) / 4)), dim3(256), 0, s,
                     g);
  return hipGetLastError();
}

}  // namespace fqt
