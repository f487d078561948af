// Register-direct packed-FP64 GEMM over GF(p^k), coefficient form: the
// kernels of fqt_direct.h instantiated for the tile ids of FQT_DIRECT_TILES,
// single launches and persistent batches.

#include "fqt_direct.h"

namespace fqt {

// ---- dispatch ----------------------------------------------------------------

template <int KE, int TM, int TN, int SK, int NWV, int MODE, bool BUF>
static hipError_t direct_one(const GemmArgs& g, const PackedParams& pp, hipStream_t s) {
  using T = DT<KE, TM, TN, SK, NWV>;
  const int tiles_m = (int)((g.M + T::BM - 1) / T::BM);
  const int tiles_n = (int)((g.N + T::BN - 1) / T::BN);
  const int ntiles = tiles_m * tiles_n;
  if (ntiles == 0) return hipSuccess;
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_direct_kernel<KE, TM, TN, SK, NWV, MODE, kDirectStages, false, BUF>),
                     dim3(ntiles), dim3(64 * NWV), dyn, s, g, pp, tiles_n, ntiles);
  return hipGetLastError();
}

template <int KE, int TM, int TN, int SK, int NWV, int MODE, bool BUF>
static hipError_t direct_batched(const GemmArgs* descs, const TileItem* items, int32_t n_items,
                                 uint32_t* counter, int grid, const PackedParams& pp,
                                 hipStream_t s) {
  const size_t dyn = 2u * (1u << pp.tbl_log2) * sizeof(uint32_t);
  hipLaunchKernelGGL(
      (gemm_direct_batched_kernel<KE, TM, TN, SK, NWV, MODE, kDirectStages, false, BUF>), dim3(grid),
      dim3(64 * NWV), dyn, s, descs, items, n_items, counter, pp);
  return hipGetLastError();
}

template <int KE, int TM, int TN, int SK, int NWV, int MODE, bool BUF>
static int direct_occupancy(uint32_t tbl_log2) {
  int blocks = 0;
  const size_t dyn = 2u * (1u << tbl_log2) * sizeof(uint32_t);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &blocks,
          (const void*)gemm_direct_batched_kernel<KE, TM, TN, SK, NWV, MODE, kDirectStages, false, BUF>,
          64 * NWV, dyn) != hipSuccess)
    blocks = 1;
  return blocks > 0 ? blocks : 1;
}

// Only the (tile, mode) pairs the host can ask for are instantiated: several
// K-blocks only on MULTI_OK tiles, digit sums only where 2b <= 24.
#define FQT_DIRECT_CASE(ID, TM, TN, SK, NWV, MULTI_OK)                       \
  case ID:                                                                    \
    if constexpr ((MODE == 0 || MULTI_OK) && (MODE != 2 || digit_sums_fit<KE>())) \
      return FN<KE, TM, TN, SK, NWV, MODE, direct_tile_buffered(ID)>(ARGS);   \
    else                                                                      \
      return FAIL;

template <int KE, int MODE>
static hipError_t direct_dispatch_one(int tile, const GemmArgs& g, const PackedParams& pp,
                                      hipStream_t s) {
#define FN direct_one
#define ARGS g, pp, s
#define FAIL hipErrorInvalidValue
  switch (tile) { FQT_DIRECT_TILES(FQT_DIRECT_CASE) default: return hipErrorInvalidValue; }
#undef FN
#undef ARGS
#undef FAIL
}

template <int KE, int MODE>
static hipError_t direct_dispatch_batched(int tile, const GemmArgs* descs, const TileItem* items,
                                          int32_t n_items, uint32_t* counter, int grid,
                                          const PackedParams& pp, hipStream_t s) {
#define FN direct_batched
#define ARGS descs, items, n_items, counter, grid, pp, s
#define FAIL hipErrorInvalidValue
  switch (tile) { FQT_DIRECT_TILES(FQT_DIRECT_CASE) default: return hipErrorInvalidValue; }
#undef FN
#undef ARGS
#undef FAIL
}

template <int KE, int MODE>
static int direct_dispatch_occupancy(int tile, uint32_t tbl_log2) {
#define FN direct_occupancy
#define ARGS tbl_log2
#define FAIL 1
  switch (tile) { FQT_DIRECT_TILES(FQT_DIRECT_CASE) default: return 1; }
#undef FN
#undef ARGS
#undef FAIL
}
#undef FQT_DIRECT_CASE

#define FQT_DIRECT_MODE_DISPATCH(F, KE, FAILV, ...)                           \
  switch (mode) {                                                             \
    case 0: return F<KE, 0>(__VA_ARGS__);                                     \
    case 1: return F<KE, 1>(__VA_ARGS__);                                     \
    case 2: return F<KE, 2>(__VA_ARGS__);                                     \
    default: return FAILV;                                                    \
  }
#define FQT_DIRECT_K_DISPATCH(F, FAILV, ...)                                  \
  switch (k) {                                                                \
    case 1: FQT_DIRECT_MODE_DISPATCH(F, 1, FAILV, __VA_ARGS__)                \
    case 2: FQT_DIRECT_MODE_DISPATCH(F, 2, FAILV, __VA_ARGS__)                \
    case 3: FQT_DIRECT_MODE_DISPATCH(F, 3, FAILV, __VA_ARGS__)                \
    case 4: FQT_DIRECT_MODE_DISPATCH(F, 4, FAILV, __VA_ARGS__)                \
    default: return FAILV;                                                    \
  }

hipError_t launch_gemm_direct(int k, int tile, int mode, const GemmArgs& g,
                              const PackedParams& pp, hipStream_t s) {
  FQT_DIRECT_K_DISPATCH(direct_dispatch_one, hipErrorInvalidValue, tile, g, pp, s)
}

hipError_t launch_gemm_direct_batched(int k, int tile, int mode, const GemmArgs* descs,
                                      const TileItem* items, int32_t n_items, uint32_t* counter,
                                      int grid, const PackedParams& pp, hipStream_t s) {
  FQT_DIRECT_K_DISPATCH(direct_dispatch_batched, hipErrorInvalidValue, tile, descs, items,
                        n_items, counter, grid, pp, s)
}

int direct_batched_occupancy(int k, int tile, int mode, uint32_t tbl_log2) {
  FQT_DIRECT_K_DISPATCH(direct_dispatch_occupancy, 1, tile, tbl_log2)
}

}  // namespace fqt
