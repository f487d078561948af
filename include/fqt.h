/*
 * fqt.h -- C ABI of the Q-adic transform (FQT) library for MI355X (gfx950).
 *
 * Method: J.-G. Dumas, "Q-adic Transform Revisited" (arXiv 0710.0510).
 *   - DQT packing (Section 2, eq. (1)): a polynomial sum_i a_i X^i over GF(p)
 *     with k coefficients is evaluated at an integer q and held as an exact
 *     integer inside an IEEE binary64 number.
 *   - Exact floating-point products / dot products / GEMM on the packed values
 *     (Alg. 1 step 2, Alg. 4 step 2), exact while eq. (2) holds:
 *         q > n_q * k * (p-1)^2   and   (2k-1) * log2(q) < 53,
 *     n_q being the number of products accumulated before a reduction.
 *   - The inverse transform REDQ (Section 4, Alg. 2): one floor division by p
 *     gives every residue u_i = floor(r/q^i) - p*floor(floor(r/p)/q^i) in
 *     [0, p) (Thm. 2); the corrections mu_i = u_i - q*u_{i+1} mod p are either
 *     applied directly (the matrix Q_d of Section 5.1) or folded, together with
 *     the reduction modulo the defining polynomial, into the two tables L and
 *     H of Alg. 4 (Thm. 3), indexed in binary (Section 5.3).
 *
 * Data format (all entry points):
 *   - A field element or a polynomial operand is k consecutive uint8 bytes,
 *     byte i holding the coefficient of X^i, every byte in [0, p).  Outputs
 *     are canonical: every coefficient in [0, p), degree below k (fields) or
 *     below 2k-1 (polynomial products).
 *   - Matrices are row-major; leading dimensions count ELEMENTS (not bytes).
 *   - Buffers named "device" are device pointers (hipMalloc / torch CUDA
 *     tensors) on the current HIP device.  The caller allocates and frees
 *     every data buffer; the library never frees them and never keeps them.
 *   - Input bytes must lie in [0, p).  This is a documented precondition of
 *     the device paths (checked by the tests, not by the kernels).
 *
 * Errors and asynchrony:
 *   - Every call returns an fqt_status.  All argument and exactness checks run
 *     on the host before anything is launched, so every error code except
 *     FQT_ERR_DEVICE is reported without touching a GPU.
 *   - Launches are asynchronous on the caller's stream (NULL = default
 *     stream).  A device failure shows up as FQT_ERR_DEVICE from the call that
 *     observed it.
 *   - Ordering: the library keeps device state per field and device (tables,
 *     INT8 and Winograd workspaces, batch plans with their queue counters)
 *     and, for the polynomial batches, per process and device.  Calls that
 *     share such state must be ordered on the device: issue them on one
 *     stream, or make a second stream wait for the first.  Calls on one
 *     field that overlap in time on two streams may race and write wrong
 *     bytes; different fields never share state.
 *   - Batch plans: a batched call builds a plan the first time it sees a
 *     descriptor list and replays it later.  At most 32 plans are kept per
 *     field (and 32 polynomial-batch plans per process); building one more
 *     destroys the least recently used after waiting for the device to go
 *     idle.  fqt_field_destroy waits likewise and releases everything.
 *   - fqt_last_error() returns a thread-local, human-readable message for the
 *     last failing call of the calling thread.
 *   - Nothing throws across this ABI.
 */
#ifndef FQT_H
#define FQT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* fqt_stream_t; /* same type as hipStream_t */

typedef enum {
  FQT_OK = 0,
  FQT_ERR_INVALID_ARG = 1, /* null pointer, negative size, bad leading
                              dimension, overlapping input/output buffers */
  FQT_ERR_BOUNDS = 2,      /* eq. (2) violated for the requested q / n_q */
  FQT_ERR_NOT_PRIME = 3,   /* p is not prime */
  FQT_ERR_REDUCIBLE = 4,   /* the defining polynomial is reducible */
  FQT_ERR_UNSUPPORTED = 5, /* parameters outside what the kernels handle */
  FQT_ERR_DEVICE = 6,      /* a HIP runtime call failed */
  FQT_ERR_OOM = 7          /* host or device allocation failed */
} fqt_status;

typedef enum {
  FQT_PATH_AUTO = 0,       /* the autotuner's (or the default) choice */
  FQT_PATH_PACKED_F64 = 1, /* q-adic packed FP64 MFMA + REDQ (the FQT) */
  FQT_PATH_INT8 = 2,       /* coefficient-wise INT8 MFMA, INT32 accumulation,
                              delayed reduction (Section 6, eq. (3)) */
  FQT_PATH_PLAIN = 3,      /* comparator: schoolbook product with % p and
                              division by P for every product, no packing */
  FQT_PATH_INT_RANGE_ = 0x7fffffff /* not a path: gives the type the range of
                              int, so any int a caller passes is a value of it
                              (and refused as FQT_ERR_INVALID_ARG) */
} fqt_path;

typedef enum {
  FQT_UNPACK_POLY = 0,  /* ndigits coefficients mod p (Alg. 2 + Q_d) */
  FQT_UNPACK_FIELD = 1, /* k coefficients mod p and mod P (Alg. 4 L + H) */
  FQT_UNPACK_INT_RANGE_ = 0x7fffffff /* not a mode: int range, as fqt_path */
} fqt_unpack_mode;

typedef struct fqt_field_s* fqt_field; /* opaque, immutable after creation */

/* One product of a batch: C (M x N) = A (M x K) * B (K x N) over the field.
 * Pointers are device pointers; ld* count elements. */
typedef struct {
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  const uint8_t* A;
  const uint8_t* B;
  uint8_t* C;
} fqt_gemm_desc;

/* Tuning knobs of the GEMM paths; zero fields mean "library default". */
typedef struct {
  uint32_t log2q;  /* packed path: q = 2^log2q; 0 = largest allowed by eq.(2) */
  uint32_t n_q;    /* packed path: products per K-block before a REDQ; 0 = the
                      largest eq. (2) allows for q */
  uint32_t tile;   /* kernel tile configuration id (see fqt_tile_count); 0 =
                      default for the shape.  Packed path: ids 1..6 stage
                      operands through LDS; ids 7..12 load them straight
                      into MFMA registers (all but 11 need K <= n_q and
                      return FQT_ERR_UNSUPPORTED otherwise; these ids never
                      pad a K-block: n_q is rounded down to a multiple of
                      4; id 12 also needs each operand's extent, rows x ld
                      x k bytes, below 2^31, else FQT_ERR_UNSUPPORTED).
                      Ids 13 and 14 (k = 3 or 4 only, else
                      FQT_ERR_UNSUPPORTED) split every element into two
                      chunks of 2 coefficients (Section 6's chunking with
                      d = 1) packed at q = 2^17 and contract three
                      chunk-pair sums (three MFMAs per k-group); one block
                      holds n_q <= (2^17 - 1) / (w (p-1)^2) products, w = 8
                      for k = 4 and 4 for k = 3 (4095 for GF(3^4)); longer
                      K runs in blocks of a multiple of 16 products.  They
                      accept log2q 0 or 17 only (FQT_ERR_INVALID_ARG) and
                      ignore boundary.
                      Id 15 (k = 4 only, else FQT_ERR_UNSUPPORTED) is made
                      for batches of small products: every wave computes a
                      32 x 32 output tile alone, K-blocks of 4, 8, 12 or 16
                      products (the largest multiple of 4 up to n_q and
                      16), q = 2^7 (log2q 0 or 7), digit-sum block steps
                      (boundary 0 or 2), centred packing for p = 3, 5, 7;
                      other settings, A, B or C not 4-byte aligned, an
                      operand extent ((rows - 1) ld + cols) k of 2^30 bytes
                      or more, or (M + 32) ldc k of 2^30 bytes or more give
                      FQT_ERR_UNSUPPORTED.  A single product runs as a batch
                      of one.
                      INT8 path, id 11 (k = 4 only): one workgroup per strip
                      of 16 output elements sweeping all rows, B' of each
                      K-tile built once in LDS; A and B 4-byte aligned,
                      operand extents and 256 rows of A or B below 2^30
                      bytes, else FQT_ERR_UNSUPPORTED.
                      INT8 path: ids 1..3 and 7..10 expand B into B' (k x k
                      multiplication matrices) in a device workspace, then
                      run the INT8 GEMM (C' tiles 64 x 64, 128 x 128,
                      64 x 128, 256 x 256, 128 x 256, 64 x 64, 64 x 128
                      bytes; 7 and 8 with 8 waves, 9 and 10 with K-tiles of
                      256 bytes); ids 4..6 build B' K-tile by K-tile
                      in LDS inside the GEMM (no workspace) and return
                      FQT_ERR_UNSUPPORTED when their operand tiles and the
                      table (2^(k ceil(log2 p)) entries of k^2 bytes padded
                      to 4 or 16) exceed the 160 KiB LDS of a CU.  All INT8
                      ids give identical bytes. */
  uint32_t boundary; /* packed path, K > n_q: step at each K-block boundary.
                        0 = default (2 when q <= 2^12, else 1); 1 = REDQ
                        residues of the block (Alg. 2,
                        first part); 2 = the block's q-adic digits (Alg. 1's
                        radix conversion, bit fields for q = 2^b) with the
                        reduction mod p delayed to the end (Section 6).  Both
                        give identical bytes. */
  uint32_t centered; /* packed path, LDS-staged tiles 1..6 and 15, odd p: 1 packs
                        centred coefficients (c > (p-1)/2 taken as c - p, the
                        residues Section 6 names for delayed reduction) with
                        q/2 added to every digit of a block, so a block holds
                        n_q <= (q/2 - 1) / (k ((p-1)/2)^2) products, about
                        twice the eq. (2) bound; the same bytes come out.
                        FQT_ERR_UNSUPPORTED for p = 2 or other tiles. */
} fqt_gemm_opts;

/* ---- field handle (Section 7: GF(p^k) = GF(p)[X]/(P)) ------------------- */

/* Create GF(p^k) with defining polynomial P = X^k + sum_{i<k} P_low[i] X^i.
 *   p      prime, 2 <= p <= 127 (FQT_ERR_NOT_PRIME / FQT_ERR_UNSUPPORTED)
 *   k      1 <= k <= 4 (FQT_ERR_UNSUPPORTED); k == 1 is the prime field
 *   P_low  host array of k values in [0, p); for k == 1 may be NULL (P = X)
 *   out    receives the handle; destroy with fqt_field_destroy.
 * P must be irreducible (FQT_ERR_REDUCIBLE).  The L/H tables of Thm. 3 must
 * fit the binary indexing of Section 5.3 with at most 4096 entries each
 * (k * ceil(log2 p) <= 12), else FQT_ERR_UNSUPPORTED.  Needs no GPU: device
 * copies of the tables are made on first use on each device. */
fqt_status fqt_field_create(uint32_t p, uint32_t k, const uint32_t* P_low,
                            fqt_field* out);
void fqt_field_destroy(fqt_field f);

/* Host copy of the L and H tables of Alg. 4 / Thm. 3 for radix q.
 *   L, H   host arrays of at least *n_entries uint32 each (may be NULL to
 *          query the size); entry index = sum_i u_i << (i*ceil(log2 p)),
 *          u_0 least significant (Section 5.3).  An entry holds k
 *          coefficients, coefficient s in byte s.  Index tuples with some
 *          u_i >= p are unused and hold 0.
 *   For L the tuple is (u_0..u_{k-1}); for H it is (u_{k-1}..u_{2k-2}). */
fqt_status fqt_field_tables(fqt_field f, uint64_t q, uint32_t* L, uint32_t* H,
                            size_t* n_entries);

/* ---- parameters (Thm. 1, eq. (2), m = 53) -------------------------------- */

/* Choose q for a block of n_q products (n_q >= 1).
 *   pow2_q    nonzero: q is the LARGEST power of two with q^(2k-1) < 2^53
 *             (so digit extraction is a shift, Section 2); zero: the largest
 *             integer q with q^(2k-1) < 2^53.
 *   carry_in  nonzero: the bound is q > n_q*k*(p-1)^2 + (p-1), which also
 *             admits a reduced value re-entering the accumulator.
 *   q_out     receives q (may be NULL)
 *   nq_max_out receives the largest n_q that q admits (may be NULL)
 * Returns FQT_ERR_BOUNDS if no q satisfies eq. (2) for n_q. */
fqt_status fqt_params(uint32_t p, uint32_t k, uint64_t n_q, int pow2_q,
                      int carry_in, uint64_t* q_out, uint64_t* nq_max_out);

/* ---- DQT: pack (Alg. 1 step 1, Section 2) -------------------------------- */

/* packed[i] = sum_j coeffs[i*k + j] * q^j as an exact binary64.
 *   coeffs  device, n*k bytes;  packed  device, n doubles.
 *   q       2 <= q; the largest packed value (p-1) sum_{j<k} q^j at most
 *           2^53 and q^k at most 2^70 (FQT_ERR_BOUNDS otherwise).  Powers of
 *           two use shifts; other q use an exact FP64 Horner evaluation.
 *   With q a power of two, coeffs 4-byte and packed 8-byte aligned, each
 *   thread packs four elements from whole words (the faster kernel); other
 *   calls stage bytes through LDS.  Results are the same either way. */
fqt_status fqt_pack(fqt_field f, uint64_t q, const uint8_t* coeffs, size_t n,
                    double* packed, fqt_stream_t s);

/* ---- inverse transform: REDQ (Alg. 2; Alg. 4 steps 3-10) ----------------- */

/* packed[i] = sum_{j<ndigits} d_j q^j with 0 <= d_j < q (an exact integer
 * below 2^53; the caller guarantees the digit bound, eq. (2)).
 *   POLY:  out holds n*ndigits bytes, out[i*ndigits + j] = d_j mod p
 *          (REDQ residues u_j, then the Q_d correction).
 *   FIELD: ndigits <= 2k-1; out holds n*k bytes, the element
 *          sum_j (d_j mod p) X^j reduced modulo P (REDQ residues, then the
 *          L and H tables of Thm. 3 and one addition in the field).
 *   q      2 <= q, q^ndigits <= 2^53 (FQT_ERR_BOUNDS), ndigits in [1, 15]
 *          (FQT_ERR_UNSUPPORTED otherwise).
 *   With q a power of two and out 4-byte aligned, each thread unpacks four
 *   values and writes whole words, with the digit count fixed at compile
 *   time (the faster kernel); other calls stage bytes through LDS. */
fqt_status fqt_unpack_redq(fqt_field f, uint64_t q, const double* packed,
                           size_t n, uint32_t ndigits, fqt_unpack_mode mode,
                           uint8_t* out, fqt_stream_t s);

/* Same with packed values held as uint64, for values beyond binary64's exact
 * range (the paper's Example 2 is one).  Any value below 2^64 is accepted;
 * q^(ndigits-1) must be below 2^64 (FQT_ERR_BOUNDS).  The top digit is then
 * floor(r / q^(ndigits-1)), whatever its size. */
fqt_status fqt_unpack_redq_u64(fqt_field f, uint64_t q, const uint64_t* packed,
                               size_t n, uint32_t ndigits,
                               fqt_unpack_mode mode, uint8_t* out,
                               fqt_stream_t s);

/* ---- Alg. 1: batch of independent polynomial products over GF(p) -------- */

/* c[i] = a[i] * b[i] in GF(p)[X] for i < n: pack at q, one FP64 product,
 * REDQ and the Q_d correction.
 *   a, b  device, n*k bytes;  c  device, n*(2k-1) bytes.
 *   q     must satisfy eq. (2) with n_q = 1 (FQT_ERR_BOUNDS), any q >= 2;
 *         powers of two use the shift path.  1 <= k <= 8.
 *   With q = 2^b, (2k-1) b <= 32 and a, b, c 4-byte aligned, every
 *   intermediate fits 32 bits and each thread multiplies four pairs from
 *   whole words (the faster kernel); other calls stage bytes through LDS. */
fqt_status fqt_polymul_batch(uint32_t p, uint32_t k, uint64_t q,
                             const uint8_t* a, const uint8_t* b, size_t n,
                             uint8_t* c, fqt_stream_t s);

/* ---- d-FQT: long polynomials over GF(p) (Section 6) --------------------- */

/* c[i] = a[i] * b[i] in GF(p)[X] for i < count, each operand len
 * coefficients (degree len - 1): the d-FQT of Section 6.  Every operand is
 * split into ceil(len/(d+1)) chunks of d+1 coefficients (a polynomial in
 * Y = X^(d+1)), each chunk packed at q = 2^log2q into one binary64 (DQT,
 * eq. (1)); the packed chunks are convolved exactly in FP64, in blocks of at
 * most n_q products, each block reduced by REDQ_{2d+1} (or, with q <= 2^12,
 * by summing its q-adic digit fields); the 2d+1 digits of every packed
 * product are the coefficients of X^(t(d+1)+j), and overlapping digits of
 * consecutive ones are added mod p.
 *   a, b   device, count*len bytes, every byte in [0, p);
 *   c      device, count*(2 len - 1) bytes; must not overlap a or b.
 *   p      prime <= 127; d in [0, 7]; 1 <= len <= 1024 (d+1)
 *          (FQT_ERR_UNSUPPORTED beyond).
 *   log2q  0 = the largest q with q^(2d+1) < 2^53 ((2d+1) log2q <= 52);
 *          smaller q only while one block holds every product of a chunk
 *          pair sum (n_q >= ceil(len/(d+1))), else FQT_ERR_UNSUPPORTED.
 *   n_q    products per block; 0 = the largest eq. (2) allows,
 *          q > n_q (d+1)(p-1)^2 (FQT_ERR_BOUNDS when q cannot hold one).
 *   boundary  as fqt_gemm_opts.boundary (0 default, 1 REDQ residues,
 *          2 digit sums, q <= 2^12); identical bytes.
 *   centered  0 or 1 (else FQT_ERR_INVALID_ARG); 1, for odd p only
 *          (FQT_ERR_UNSUPPORTED for p = 2): coefficients above (p-1)/2
 *          enter the chunks as c - p (the centred residues Section 6 names
 *          for delayed reduction) and every block's digits are shifted by
 *          q/2, so n_q may reach (q/2 - 1) / ((d+1) ((p-1)/2)^2), about twice
 *          eq. (2)'s bound (3 instead of 1 for p = 3, d = 4); identical
 *          bytes. */
fqt_status fqt_polymul_dfqt(uint32_t p, uint32_t d, uint32_t log2q, uint32_t n_q,
                            uint32_t boundary, uint32_t centered, const uint8_t* a,
                            const uint8_t* b, int64_t count, int64_t len, uint8_t* c,
                            fqt_stream_t s);

/* One pair of an uneven polynomial batch (device pointers): c = a * b in
 * GF(p)[X], a of la coefficients, b of lb, c of la + lb - 1 (nothing is
 * written when la or lb is 0). */
typedef struct {
  int64_t la, lb;
  const uint8_t* a;
  const uint8_t* b;
  uint8_t* c;
} fqt_poly_desc;

/* The d-FQT of Section 6 (as fqt_polymul_dfqt, same p, d, log2q, n_q,
 * boundary and centered, with the same errors) on a batch of pairs of
 * uneven lengths, in ONE persistent launch: the pairs, ordered longest
 * first, are dealt to the waves in a fixed snake order and every wave
 * multiplies each of its pairs alone.  n_q and the
 * block steps are chosen for the batch's longest chunk-pair sum.
 *   descs  host array of count descriptors; every byte of a, b in [0, p);
 *          la, lb >= 0 (FQT_ERR_INVALID_ARG if negative), at most
 *          1024 (d+1) each (FQT_ERR_UNSUPPORTED beyond); c must not overlap
 *          its own a or b (FQT_ERR_INVALID_ARG).
 * The first call with a given descriptor list builds a plan (pair order,
 * device descriptors) and captures the launch in a hipGraph; later calls
 * with the same list replay it, on whatever stream s is given. */
fqt_status fqt_polymul_dfqt_batched(uint32_t p, uint32_t d, uint32_t log2q, uint32_t n_q,
                                    uint32_t boundary, uint32_t centered, int64_t count,
                                    const fqt_poly_desc* descs, fqt_stream_t s);

/* fqt_polymul_dfqt_batched for callers that cannot allocate device memory
 * (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc): the same arguments, checks, errors and output bytes, but no
 * plan and no graph; it calls no hipMalloc, hipFree or other allocating
 * routine.  Each call copies the descriptors, in schedule order, into a
 * static device array of this library (640 KiB, one per GPU, held until the
 * process ends) on stream s and launches the batch on them.  At most 16384 pairs with output per call
 * (FQT_ERR_UNSUPPORTED beyond).  Every call on one GPU uses that GPU's one
 * array: calls that overlap in time on one GPU (two streams, two threads)
 * race and may write wrong bytes; calls ordered on one stream do not. */
fqt_status fqt_polymul_dfqt_batched_noalloc(uint32_t p, uint32_t d, uint32_t log2q,
                                            uint32_t n_q, uint32_t boundary, uint32_t centered,
                                            int64_t count, const fqt_poly_desc* descs,
                                            fqt_stream_t s);

/* Time the d-FQT of an uneven batch for every chunk length d + 1 = 1..8,
 * for odd p both chunk representations, and both block-boundary modes
 * (digit sums where q <= 2^12, REDQ residues); q and n_q are the largest
 * eq. (2) admits for each.  Every candidate's output must be byte-identical
 * to the first admissible one's (else FQT_ERR_DEVICE).  Writes the fastest
 * (d, centered, boundary), each pointer may be NULL.  cache_path (NULL:
 * none) is a JSON-lines file read first and appended to. */
fqt_status fqt_autotune_polymul(uint32_t p, int64_t count, const fqt_poly_desc* descs,
                                const char* cache_path, uint32_t* d, uint32_t* centered,
                                uint32_t* boundary, fqt_stream_t s);

/* The comparator of Section 6: the classical product with delayed reduction
 * (eq. (3)): every coefficient accumulated in 32-bit integers and reduced
 * mod p once (or every n_d products if len (p-1)^2 could overflow).
 *   Same buffers as fqt_polymul_dfqt; p prime <= 127; 1 <= len <= 8192. */
fqt_status fqt_polymul_delayed(uint32_t p, const uint8_t* a, const uint8_t* b,
                               int64_t count, int64_t len, uint8_t* c,
                               fqt_stream_t s);

/* ---- GEMM over GF(p^k) (Alg. 4 for every entry, Section 7) -------------- */

/* C = A * B over the field; A is M x K, B is K x N, C is M x N elements.
 *   lda >= K, ldb >= N, ldc >= N (elements).  M, N, K >= 0; K == 0 writes
 *   zeros.  C must not overlap A or B.
 *   path  FQT_PATH_PACKED_F64: packed FP64 MFMA with q = 2^b and K-blocks of
 *         n_q products, REDQ residues at every block boundary, L/H at the end.
 *         FQT_PATH_INT8: INT8 MFMA on coefficient planes, INT32 accumulation.
 *         FQT_PATH_PLAIN: per-product schoolbook comparator.
 *         FQT_PATH_AUTO: the autotuned choice for this field and shape.
 * The library may keep a device workspace per field and device. */
fqt_status fqt_gemm_gfpk(fqt_field f, fqt_path path, int64_t M, int64_t N,
                         int64_t K, const uint8_t* A, int64_t lda,
                         const uint8_t* B, int64_t ldb, uint8_t* C,
                         int64_t ldc, fqt_stream_t s);

/* fqt_gemm_gfpk with explicit tuning knobs (NULL opts = defaults).  Returns
 * FQT_ERR_BOUNDS when opts ask for a q / n_q that breaks eq. (2). */
fqt_status fqt_gemm_gfpk_ex(fqt_field f, fqt_path path,
                            const fqt_gemm_opts* opts, int64_t M, int64_t N,
                            int64_t K, const uint8_t* A, int64_t lda,
                            const uint8_t* B, int64_t ldb, uint8_t* C,
                            int64_t ldc, fqt_stream_t s);

/* Batch of independent GEMMs of uneven sizes in ONE persistent launch.
 *   descs  host array of count descriptors (device data pointers).
 * The first call with a given descriptor list builds a plan (tiles sorted by
 * cost, uploaded to the device) and captures it in a hipGraph; later calls
 * with an identical list replay the graph on whatever stream s is given
 * (replays of one plan must not overlap on two streams: they share its queue
 * counter and, on FQT_PATH_INT8, the field's B' workspace).  FQT_PATH_PLAIN
 * runs one launch per product (the comparator). */
fqt_status fqt_gemm_gfpk_batched(fqt_field f, fqt_path path, int64_t count,
                                 const fqt_gemm_desc* descs, fqt_stream_t s);

/* Same with tuning knobs (NULL = defaults / autotuned). */
fqt_status fqt_gemm_gfpk_batched_ex(fqt_field f, fqt_path path,
                                    const fqt_gemm_opts* opts, int64_t count,
                                    const fqt_gemm_desc* descs,
                                    fqt_stream_t s);

/* ---- Winograd's product over GF(p^k) (the paper's Fig. 3 setting) ------ */

/* C = A * B over the field with `levels` levels (0..6, else
 * FQT_ERR_INVALID_ARG) of Winograd's variant of Strassen's recursion: per
 * level seven block products, run as fqt_gemm_gfpk_ex(path, opts) calls,
 * and fifteen block additions coefficient-wise mod p.  Odd dimensions are
 * peeled (last row, last column, and the last k as a rank-one product added
 * in); blocks below 2 in any dimension go straight to the path.  Same
 * buffers, layout and validation as fqt_gemm_gfpk_ex; the result is the same
 * bytes.  The library keeps device temporaries per field and device, about
 * (4hd + 4dw + 7hw) k bytes per level for blocks of h x d, d x w, h x w
 * elements (h = M/2, d = K/2, w = N/2 at the first level): calls on one
 * field must not overlap in time on one device.  FQT_ERR_OOM if they cannot
 * be allocated. */
fqt_status fqt_gemm_winograd(fqt_field f, fqt_path path, const fqt_gemm_opts* opts,
                             uint32_t levels, int64_t M, int64_t N, int64_t K,
                             const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb,
                             uint8_t* C, int64_t ldc, fqt_stream_t s);

/* ---- discrete-log representation (Section 7, Alg. 4) -------------------- */

/* Alg. 4 takes field elements as exponents of a generator g.  A code is a
 * uint16: e in [0, m-1] stands for g^e, m = p^k - 1 stands for zero, and
 * every entry point below reads codes above m as zero.  g is the first
 * element of multiplicative order m in base-p order (element index
 * sum_i c_i p^i), a choice the paper leaves open.  All buffers are device
 * pointers; calls are asynchronous on stream s.  Tables are built on first
 * use on each device (a few KB, held by the field). */

/* Host query: the generator's base-p index and the code of zero (m).
 * Either pointer may be NULL. */
fqt_status fqt_log_info(fqt_field f, uint32_t* generator_index, uint32_t* zero_code);

/* codes[i] = log of the element held in coeffs[k*i .. k*i + k-1] (one
 * coefficient per byte, each in [0, p); an element with a byte >= p is read
 * as zero).  n >= 0 elements; the buffers must not overlap
 * (FQT_ERR_INVALID_ARG). */
fqt_status fqt_to_log(fqt_field f, const uint8_t* coeffs, int64_t n, uint16_t* codes,
                      fqt_stream_t s);

/* coeffs[k*i ..] = the coefficients of the element with code codes[i]. */
fqt_status fqt_from_log(fqt_field f, const uint16_t* codes, int64_t n, uint8_t* coeffs,
                        fqt_stream_t s);

/* c[i] = a[i] + b[i] in the field, on codes, through the Zech table
 * Z[n] = log(1 + g^n): g^a + g^b = g^(a + Z[b-a]) (Alg. 4's last step).
 * c may equal a or b; any other overlap is FQT_ERR_INVALID_ARG. */
fqt_status fqt_log_add(fqt_field f, const uint16_t* a, const uint16_t* b, int64_t n,
                       uint16_t* c, fqt_stream_t s);

/* C = A * B over the field on codes (Alg. 4 for every entry): each operand
 * code becomes its element's evaluation at q by one table lookup, the
 * packed products are contracted exactly on the FP64 MFMA in K-blocks of
 * n_q (eq. (2)), REDQ gives the residues u, Thm. 3's L and H tables return
 * codes and R = H + L by the Zech table.  A is M x K, B is K x N, C is
 * M x N codes, ld* in elements (lda >= K, ldb >= N, ldc >= N); C must not
 * overlap A or B; K == 0 writes the zero code.  opts as for the packed
 * path; tile 0 (default), 7, 9 or 11 (else FQT_ERR_UNSUPPORTED); 7 and 9
 * take one K-block, 11 several; a tile whose split-K buffer and tables do
 * not fit LDS is FQT_ERR_UNSUPPORTED. */
fqt_status fqt_gemm_log(fqt_field f, const fqt_gemm_opts* opts, int64_t M, int64_t N,
                        int64_t K, const uint16_t* A, int64_t lda, const uint16_t* B,
                        int64_t ldb, uint16_t* C, int64_t ldc, fqt_stream_t s);

/* ---- autotuner ----------------------------------------------------------- */

/* Time every admissible (path, q, n_q, tile) candidate on the given problem
 * (a single GEMM when count == 1, else a batch), require byte-identical
 * outputs across candidates (FQT_ERR_DEVICE with a message otherwise), and
 * remember the fastest for FQT_PATH_AUTO on this field and shape class.
 *   only        FQT_PATH_AUTO: candidates of every path; FQT_PATH_PACKED_F64 or
 *               FQT_PATH_INT8: that path's candidates only (the tuned entry
 *               is then stored for that path, and for AUTO only if none is).
 *   cache_path  JSON-lines file (may be NULL): an entry with the same key is
 *               reused without timing; a new winner is appended.
 * The winner is written to best_path / best (may be NULL).  The C buffers of
 * the descriptors are overwritten.  Timing uses HIP events on stream s. */
fqt_status fqt_autotune(fqt_field f, fqt_path only, int64_t count,
                        const fqt_gemm_desc* descs, const char* cache_path,
                        fqt_path* best_path, fqt_gemm_opts* best, fqt_stream_t s);

/* Number of tile configurations of a path (ids 1..count). */
uint32_t fqt_tile_count(fqt_path path);

/* ---- diagnostics ---------------------------------------------------------- */

const char* fqt_last_error(void);
const char* fqt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FQT_H */
