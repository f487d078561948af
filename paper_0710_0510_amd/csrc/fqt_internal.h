// Internal declarations shared by the host API (fqt_api.cpp) and the kernel
// translation units.  Not installed; the public interface is include/fqt.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fqt_device.h"

namespace fqt {

// One GEMM problem; ld* in elements.
struct GemmArgs {
  const uint8_t* A;
  const uint8_t* B;
  uint8_t* C;
  int64_t M, N, K, lda, ldb, ldc;
};

// PackedParams::dqt_flags
constexpr uint32_t kDqtLut = 1u, kDqtDot4 = 2u;

// Parameters of the packed-FP64 path (Alg. 4 with K-blocks, eq. (2)).
struct PackedParams {
  uint32_t b;          // q = 2^b
  uint32_t nq_groups;  // K-block = 4*nq_groups products (MFMA k-groups of 4)
  uint32_t tbl_log2;   // each table has 2^tbl_log2 entries (k*cb)
  uint32_t aligned;    // rows of A and B start on 4-byte boundaries
  uint32_t fold_blocks;  // block boundaries between folds of the lanes mod p (0: never)
  uint32_t qmask;      // q - 1
  uint32_t qmod;       // q mod p
  uint32_t blk_real;   // products per K-block (< 4*nq_groups: padded blocks)
  uint32_t centered;   // centred packing (staged tiles): digits shifted by q/2
  uint32_t c0neg;      // centred: -(L + H of the shift's residues), one word
                       // (d-FQT: (q/2) mod p, the shift of every digit of a block)
  uint32_t dshift;     // centred, wave tile: (q/2) mod p, taken off every digit sum
  double cbias;        // centred: 2^52 + sum_{i<2k-1} (q/2) q^i, every block's seed
  // DQT of the LDS-staged loaders (fqt_packed.h dqt_chunk):
  uint32_t dqt_flags;  // kDqtLut: centred bytes through the perm table below (p <= 8);
                       // kDqtDot4: k = 4 and q <= 2^7, two byte dot products per element
  uint32_t lut_lo, lut_hi;  // byte c -> (c + h) mod p for c = 0..7, h = (p-1)/2
  int32_t dqt_off;     // -h (1 + q + ... + q^(k-1)): offset form back to centred values
  FieldArgs fa;
  const uint32_t* L;   // device tables of Thm. 3 (binary index, Section 5.3)
  const uint32_t* H;
  // discrete-log operands (Alg. 4): packed value of every code at q, Zech
  // logarithms, and the code of zero m = p^k - 1 (L and H then hold codes)
  const uint32_t* pk;  // m + 1 entries, pk[m] = 0 (each below 2^32 under eq. (2))
  const uint16_t* Z;   // m + 1 entries, Z[n] = log(1 + g^n) (m where 1 + g^n = 0)
  uint32_t zero_code;
};

// d-FQT product of long polynomials (k_dfqt.hip): count pairs of len
// coefficients, chunks of d+1 = KE coefficients packed at q = 2^lg2q.
struct DfqtArgs {
  const uint8_t* a;
  const uint8_t* b;
  uint8_t* c;            // count x (2 len - 1)
  int64_t count;
  int32_t len, nch;      // coefficients, chunks per operand
  uint32_t nq, lg2q;     // products per block; q = 2^lg2q
  PackedParams pp;       // fa, qmod and fold_blocks are used
  int32_t cap;           // LDS chunks per operand and wave (>= nch): sizes the launch's LDS
};

// One pair of an uneven polynomial batch: c (la + lb - 1 coefficients) =
// a (la) * b (lb); the layout of the public fqt_poly_desc.
struct PolyDesc {
  int64_t la, lb;
  const uint8_t* a;
  const uint8_t* b;
  uint8_t* c;
};

// d-FQT over an uneven batch: the pairs in the order order[0 .. count)
// (longest first; null: descs is already in that order), dealt to the
// waves of the grid in a fixed snake order.
struct DfqtBatchArgs {
  const PolyDesc* descs;
  const int32_t* order;
  int32_t count;
  uint32_t nq, lg2q;  // products per block; q = 2^lg2q
  PackedParams pp;    // fa, qmod, fold_blocks, centring as DfqtArgs
  int32_t cap;        // LDS chunks per operand and wave (>= every nca, ncb)
};

// Classical product with delayed reduction (eq. (3)), the comparator.
struct DelayedArgs {
  const uint8_t* a;
  const uint8_t* b;
  uint8_t* c;
  int64_t count;
  int32_t len;
  uint32_t p, nd;        // nd: products between reductions (0: once at the end)
};

// Low coefficients of the monic defining polynomial (k <= 4), each < p.
struct PlainFieldArgs {
  uint32_t P_low[4];
};

// Arguments of the INT8 GEMM C' = A' B' (see k_gemm_i8.hip); strides in bytes.
struct I8Args {
  const uint8_t* A;   // A' = A's bytes, M x KK
  int64_t lda;
  const uint8_t* Bt;  // B'^T, NN x KKpad (zero beyond KK)
  int64_t ldbt;
  uint8_t* C;         // C' = C's bytes, M x NN
  int64_t ldc;
  int64_t M, NN, KK, KKpad;
  uint32_t p;
  uint32_t red_tiles;  // K-tiles between reductions mod p (0: never needed)
  uint32_t a_vec;      // alignment of A' rows and 16-byte columns: 16, 4 or 1
  uint32_t pad;
  double inv_p;
};

// One product of an INT8 batch: the GEMM arguments plus its source B.
struct I8Batch {
  I8Args a;
  const uint8_t* B;
  int64_t ldb, K, N;  // B is K x N elements, ldb elements per row
};

// Bytes per entry of the INT8 path's multiplication-matrix table (k^2 bytes
// padded to 4 or 16).
__host__ __device__ constexpr uint32_t mt_stride(uint32_t k) { return k <= 2 ? 4u : 16u; }

// One 32 (K) x 64 (N) block of the B -> B'^T expansion of a batch.
struct ExpandItem {
  int32_t gemm, lb, nb, pad;
};

// Tile work item of the persistent batched kernel.
struct TileItem {
  int32_t gemm;    // index into the descriptor array
  int32_t tm, tn;  // tile coordinates
  int32_t pad;
};

// Tile configurations of the packed path, ids 1..kPackedTiles.
// LDS-staged kernels (k_gemm_f64.hip), WG of 256 threads = 2x2 waves:
// X(id, TM, TN, BK): wave tile 16TM x 16TN, workgroup tile 32TM x 32TN,
// K-tiles of BK elements.
#define FQT_PACKED_TILES(X) \
  X(1, 1, 1, 32) X(2, 2, 2, 32) X(3, 2, 4, 16) X(4, 4, 4, 16) X(5, 2, 1, 32) X(6, 1, 2, 32)
constexpr int kStagedTiles = 6;
// Register-direct kernels (k_gemm_direct.hip), WG of NWV waves = NWV/SK waves
// side by side x SK waves splitting K: X(id, TM, TN, SK, NWV, MULTI_OK);
// MULTI_OK = 0 tiles take single-block problems only (their per-element block
// state would not fit in registers).
#define FQT_DIRECT_TILES(X)                                                     \
  X(7, 4, 4, 4, 4, 0) X(8, 2, 4, 2, 4, 0) X(9, 4, 4, 1, 4, 0) X(10, 2, 4, 1, 4, 0) \
  X(11, 1, 4, 1, 4, 1) X(12, 2, 4, 4, 8, 0)
// Tiles whose interior loads go through buffer resources (32-bit offsets:
// both operands' extents below 2^31 bytes; measured faster for 8 waves).
constexpr bool direct_tile_buffered(int id) { return id == 12; }
// d-split kernels (k_gemm_split.hip), k = 3 or 4, wave tile 16 x 64:
// id kFirstSplitTile = 2 x 2 waves, kFirstSplitTile + 1 = 4 x 1 waves.
constexpr int kFirstSplitTile = 13, kLastSplitTile = 14;
// Wave-persistent tile for batches over GF(p^4) (k_gemm_wave.hip): every wave
// computes 32 x 32 outputs alone, K-blocks fixed at compile time.
constexpr int kWaveTile = 15;
constexpr int kPackedTiles = 15;
#ifndef FQT_DIRECT_STAGES
#define FQT_DIRECT_STAGES 2
#endif
constexpr int kDirectStages = FQT_DIRECT_STAGES;  // K-steps in flight per wave
inline bool is_direct_tile(int id) { return id > kStagedTiles && id < kFirstSplitTile; }
inline bool is_split_tile(int id) { return id >= kFirstSplitTile && id <= kLastSplitTile; }
inline bool direct_tile_multi_ok(int id) { return id == 11; }
// Workgroup tile (rows x columns of C) of every tile id.
inline void packed_tile_shape(int id, int* bm, int* bn) {
  //                                     1   2    3    4   5   6   7   8    9   10   11  12  13  14  15
  static const int m[kPackedTiles] = {32, 64, 64, 128, 64, 32, 64, 64, 128, 64, 32, 64, 32, 64, 32};
  static const int n[kPackedTiles] = {32, 64, 128, 128, 32, 64, 64, 64, 128, 128, 128, 64, 128,
                                      64, 32};
  *bm = m[id - 1];
  *bn = n[id - 1];
}

// ---- launchers (each returns the launch's hipError_t) ----------------------

hipError_t launch_pack(int k, uint64_t q, int pow2, uint32_t b, const uint8_t* coeffs,
                       size_t n, double* out, hipStream_t s);

// mode 0 = POLY, 1 = FIELD.  For FIELD, L/H are device tables.
hipError_t launch_unpack_f64(int k, uint32_t nd, int mode, uint64_t q, int pow2, uint32_t b,
                             const FieldArgs& fa, const uint32_t* L, const uint32_t* H,
                             const double* in, size_t n, uint8_t* out, hipStream_t s);
hipError_t launch_unpack_u64(int k, uint32_t nd, int mode, uint64_t q, int pow2, uint32_t b,
                             const FieldArgs& fa, const uint32_t* L, const uint32_t* H,
                             const uint64_t* in, size_t n, uint8_t* out, hipStream_t s);

hipError_t launch_polymul(int k, uint64_t q, int pow2, uint32_t b, const FieldArgs& fa,
                          const uint8_t* a, const uint8_t* bb, size_t n, uint8_t* c,
                          hipStream_t s);

hipError_t launch_gemm_packed(int k, int tile, int mode, const GemmArgs& g,
                              const PackedParams& pp, hipStream_t s);

hipError_t launch_gemm_packed_batched(int k, int tile, int mode, const GemmArgs* descs,
                                      const TileItem* items, int32_t n_items,
                                      uint32_t* counter, int grid, const PackedParams& pp,
                                      hipStream_t s);

int packed_batched_occupancy(int k, int tile, int mode, uint32_t tbl_log2);

// Register-direct packed kernels (tile ids > kStagedTiles).
hipError_t launch_gemm_direct(int k, int tile, int mode, const GemmArgs& g,
                              const PackedParams& pp, hipStream_t s);
hipError_t launch_gemm_direct_batched(int k, int tile, int mode, const GemmArgs* descs,
                                      const TileItem* items, int32_t n_items,
                                      uint32_t* counter, int grid, const PackedParams& pp,
                                      hipStream_t s);
int direct_batched_occupancy(int k, int tile, int mode, uint32_t tbl_log2);

// Discrete-log operands (k_gemm_log.hip): register-direct tiles on 16-bit
// codes, X(id, TM, TN, SK, NWV, MULTI_OK) as in FQT_DIRECT_TILES.
#define FQT_LOG_TILES(X) X(7, 4, 4, 4, 4, 0) X(9, 4, 4, 1, 4, 0) X(11, 1, 4, 1, 4, 1)
inline bool is_log_tile(int id) { return id == 7 || id == 9 || id == 11; }
hipError_t launch_gemm_log(int k, int tile, int mode, const GemmArgs& g, const PackedParams& pp,
                           hipStream_t s);
// Whether a log tile's split-K buffer and tables fit one workgroup's LDS.
bool log_tile_fits(int tile, uint32_t tbl_log2, uint32_t zero_code);
hipError_t launch_to_log(int k, uint32_t cb, const uint8_t* coeffs, int64_t n,
                         const uint16_t* logt, uint16_t* codes, hipStream_t s);
hipError_t launch_from_log(int k, const uint16_t* codes, int64_t n, uint32_t zero_code,
                           const uint32_t* expw, uint8_t* coeffs, hipStream_t s);
hipError_t launch_log_add(const uint16_t* a, const uint16_t* b, int64_t n, uint32_t zero_code,
                          const uint16_t* Z, uint16_t* c, hipStream_t s);

// Winograd's block additions (k_winograd.hip): Z = X +/- Y coefficient-wise
// mod p on rows x cols elements of k bytes; ld* in elements.
hipError_t launch_mat_addsub(int k, uint32_t p, const uint8_t* X, int64_t ldx, const uint8_t* Y,
                             int64_t ldy, uint8_t* Z, int64_t ldz, int64_t rows, int64_t cols,
                             bool sub, hipStream_t s);

// Wave-persistent batched kernel (tile kWaveTile, k = 4, q = 2^7): blocks of
// 4 nqg products (nqg 1..4), items = 32 x 32 wave tiles; wave w of the grid
// (workgroup w / 4) computes items[wave_begin[w] .. wave_begin[w + 1]).
hipError_t launch_gemm_wave_batched(int nqg, const GemmArgs* descs, const TileItem* items,
                                    const int32_t* wave_begin, int grid, const PackedParams& pp,
                                    hipStream_t s);
int wave_batched_occupancy(int nqg, uint32_t tbl_log2);
constexpr int kWaveMaxNqg = 4;
// Its DQT reads the packed value of each element of GF(p^4) from a table of
// p^4 entries in LDS: p = 2 or 3, the only p whose n_q at q = 2^7 reaches 4.
constexpr int kWaveDqtEntries = 81;

// d-split kernels (tile ids kFirstSplitTile..kLastSplitTile, k = 3 or 4).
hipError_t launch_gemm_split(int k, int tile, const GemmArgs& g, const PackedParams& pp,
                             hipStream_t s);
hipError_t launch_gemm_split_batched(int k, int tile, const GemmArgs* descs,
                                     const TileItem* items, int32_t n_items, uint32_t* counter,
                                     int grid, const PackedParams& pp, hipStream_t s);
int split_batched_occupancy(int k, int tile, uint32_t tbl_log2);

// INT8 path, tile ids 1..3, 7..10: B -> B'^T expansion in HBM, then the INT8
// MFMA GEMM; ids 4..6: one kernel that expands each K-tile of B in LDS.
constexpr int kInt8Tiles = 11;
// INT8 id 11 (k_gemm_i8cs.hip, k = 4): one workgroup per strip of 16 output
// elements of a product, B' of each K-tile built in LDS once for all rows;
// items = (product, strip) int32 pairs padded to 4 words, workgroup w takes
// items[wg_begin[w] .. wg_begin[w + 1]).
constexpr uint32_t kInt8StripTile = 11;
hipError_t launch_gemm_i8cs_batched(const GemmArgs* descs, const int32_t* items_raw,
                                    const int32_t* wg_begin, int grid, const uint8_t* mt,
                                    uint32_t tbl_log2, uint32_t p, uint32_t cb,
                                    uint32_t red_tiles, uint32_t small, hipStream_t s);
int i8cs_occupancy(uint32_t tbl_log2);
// Block of the B -> B'^T expansion: kExpandL elements of K x kExpandN of N.
constexpr int kExpandL = 128, kExpandN = 16;
constexpr bool i8_fused_tile(uint32_t tile) { return tile >= 4 && tile <= 6; }
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one gfx950 CU
hipError_t launch_expand_b(int k, const uint8_t* B, int64_t ldb, int64_t K, int64_t N,
                           const uint8_t* mt, uint32_t cb, uint32_t tbl_log2, uint8_t* Bt,
                           int64_t ldbt, int64_t Kpad, hipStream_t s);
hipError_t launch_gemm_i8(int tile, const I8Args& a, hipStream_t s);
hipError_t launch_expand_b_batched(int k, const I8Batch* gs, const ExpandItem* items,
                                   int32_t n_items, const uint8_t* mt, uint32_t cb,
                                   uint32_t tbl_log2, hipStream_t s);
hipError_t launch_gemm_i8_batched(int tile, const I8Batch* gs, const TileItem* items,
                                  int32_t n_items, uint32_t* counter, int grid, hipStream_t s);
int i8_batched_occupancy(int tile);
int i8_tile_m(int tile);  // output tile of the two-kernel ids: rows of C'
int i8_tile_n(int tile);  // ... and columns of C' (bytes)
int i8_tile_k(int tile);  // ... and bytes of K per K-tile (128 or 256)
// Fused tiles (ids 4..6): bytes of K per K-tile, elements of N per output
// tile, rows of M per output tile, and static LDS bytes (the dynamic part is
// the multiplication-matrix table, 2^tbl_log2 entries of mt_stride(k)).
int i8f_k_bytes(int k);
int i8f_tile_n(int tile, int k);
int i8f_tile_m(int tile);
size_t i8f_static_lds(int tile, int k);
hipError_t launch_gemm_i8f(int tile, int k, const I8Batch& g, const uint8_t* mt, uint32_t cb,
                           uint32_t tbl_log2, hipStream_t s);
hipError_t launch_gemm_i8f_batched(int tile, int k, const I8Batch* gs, const TileItem* items,
                                   int32_t n_items, uint32_t* counter, int grid,
                                   const uint8_t* mt, uint32_t cb, uint32_t tbl_log2,
                                   hipStream_t s);
int i8f_batched_occupancy(int tile, int k, uint32_t tbl_log2);

// d-FQT (ke = d + 1 in 1..8, mode 0/1/2 as in fqt_packed.h) and its comparator.
hipError_t launch_dfqt(int ke, int mode, const DfqtArgs& g, hipStream_t s);
hipError_t launch_polymul_delayed(const DelayedArgs& g, hipStream_t s);
hipError_t launch_dfqt_batched(int ke, int mode, const DfqtBatchArgs& g, int grid,
                               hipStream_t s);
// Workgroups of the batched d-FQT kernel that fit on one CU with LDS for
// `cap` chunks per operand and wave.
int dfqt_batched_occupancy(int ke, int mode, bool centered, int32_t cap);
constexpr int kDfqtMaxChunks = 1024;  // chunks of one operand (in LDS)

// The d-FQT batch variant that allocates nothing keeps its descriptors in
// one static device array of this many bytes per GPU: at most
// kDfqtNoAllocMaxPairs descriptors.
constexpr size_t kDfqtNoAllocMaxPairs = 16384;
constexpr size_t kDfqtNoAllocScratch = kDfqtNoAllocMaxPairs * sizeof(PolyDesc);
// Copies `host_descs` (g.count descriptors, already in schedule order) into
// the current GPU's scratch array on stream s and launches the batch on
// them; g.descs and g.order are ignored.
hipError_t launch_dfqt_batched_noalloc(int ke, int mode, DfqtBatchArgs g,
                                       const PolyDesc* host_descs, int grid, hipStream_t s);
constexpr int kDelayedMaxLen = 8192;  // coefficients of one operand (in LDS)

// Plain comparator: schoolbook with % p and division by P per product.
hipError_t launch_gemm_plain(int k, const GemmArgs& g, const FieldArgs& fa,
                             const uint32_t* P_low, hipStream_t s);

}  // namespace fqt
