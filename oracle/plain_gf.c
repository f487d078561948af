/* Plain schoolbook arithmetic over GF(p)[X] and GF(p^k), threaded with OpenMP.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY: the multi-core CPU comparator that
 * the benchmark times beside the GPU path, and a second, independent oracle
 * that the CPU tests check against the Python one.  It shares no code, table
 * or constant with the HIP library.
 *
 * Every field product is the textbook one (the classical method the paper
 * measures the Q-adic transform against, Section 1 and Section 7):
 * multiply the two coefficient polynomials, reduce every coefficient mod p,
 * divide by the monic defining polynomial P = X^k + sum_i P_low[i] X^i, and
 * add the remainder into the accumulator mod p.  No packing and no delayed
 * reduction.  Elements are k consecutive bytes in [0, p); matrices are
 * row-major with leading dimensions counted in elements.
 *
 * Every entry point returns 0, or -1 for arguments outside 2 <= p <= 251,
 * 1 <= k <= 8, negative sizes or null pointers with nonzero sizes.
 */
#include <omp.h>
#include <stddef.h>
#include <stdint.h>

#define GF_KMAX 8

typedef struct {
  int p, k;
  int negP[GF_KMAX]; /* -P_low[i] mod p: X^k = sum_i negP[i] X^i in GF(p)[X]/(P) */
} gf_field;

static int gf_setup(gf_field* f, int p, int k, const uint8_t* P_low) {
  if (p < 2 || p > 251 || k < 1 || k > GF_KMAX || !P_low) return -1;
  f->p = p;
  f->k = k;
  for (int i = 0; i < k; ++i) f->negP[i] = (p - (int)(P_low[i] % p)) % p;
  return 0;
}

/* acc += a * b in GF(p^k): product in GF(p)[X], coefficients mod p, then
 * the top coefficients folded down with X^k = -P_low (schoolbook division). */
static void gf_mul_add(const gf_field* f, const uint8_t* a, const uint8_t* b, int* acc) {
  const int p = f->p, k = f->k;
  int prod[2 * GF_KMAX - 1];
  for (int t = 0; t < 2 * k - 1; ++t) prod[t] = 0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) prod[i + j] += (int)a[i] * (int)b[j];
  for (int t = 0; t < 2 * k - 1; ++t) prod[t] %= p;
  for (int t = 2 * k - 2; t >= k; --t) {
    const int c = prod[t];
    if (c)
      for (int i = 0; i < k; ++i) prod[t - k + i] = (prod[t - k + i] + c * f->negP[i]) % p;
  }
  for (int s = 0; s < k; ++s) acc[s] = (acc[s] + prod[s]) % p;
}

static void gf_gemm_rows(const gf_field* f, int64_t r0, int64_t r1, int64_t N, int64_t K,
                         const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb,
                         uint8_t* C, int64_t ldc) {
  const int k = f->k;
  for (int64_t i = r0; i < r1; ++i)
    for (int64_t j = 0; j < N; ++j) {
      int acc[GF_KMAX] = {0};
      for (int64_t l = 0; l < K; ++l)
        gf_mul_add(f, A + (i * lda + l) * k, B + (l * ldb + j) * k, acc);
      for (int s = 0; s < k; ++s) C[(i * ldc + j) * k + s] = (uint8_t)acc[s];
    }
}

/* Threads the last call ran on (the count a timing should report). */
static int gf_last_threads = 1;

int gf_plain_threads(void) { return gf_last_threads; }

/* C (M x N) = A (M x K) * B (K x N) over GF(p^k); rows of C split over
 * `threads` OpenMP threads (0: the OpenMP default). */
int gf_plain_gemm(int p, int k, const uint8_t* P_low, int64_t M, int64_t N, int64_t K,
                  const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb, uint8_t* C,
                  int64_t ldc, int threads) {
  gf_field f;
  if (gf_setup(&f, p, k, P_low) || M < 0 || N < 0 || K < 0) return -1;
  if (M == 0 || N == 0) return 0;
  if (!C || (K && (!A || !B))) return -1;
  int used = 1;
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i) gf_gemm_rows(&f, i, i + 1, N, K, A, lda, B, ldb, C, ldc);
  }
  gf_last_threads = used;
  return 0;
}

/* A batch of independent products (dense, ld = row length); products split
 * over the threads, largest first in the caller's order. */
int gf_plain_gemm_batched(int p, int k, const uint8_t* P_low, int64_t count, const int64_t* mnk,
                          const uint8_t* const* As, const uint8_t* const* Bs, uint8_t* const* Cs,
                          int threads) {
  gf_field f;
  if (gf_setup(&f, p, k, P_low) || count < 0 || (count && (!mnk || !As || !Bs || !Cs)))
    return -1;
  for (int64_t g = 0; g < count; ++g)
    if (mnk[3 * g] < 0 || mnk[3 * g + 1] < 0 || mnk[3 * g + 2] < 0) return -1;
  int used = 1;
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
    for (int64_t g = 0; g < count; ++g) {
      const int64_t M = mnk[3 * g], N = mnk[3 * g + 1], K = mnk[3 * g + 2];
      gf_gemm_rows(&f, 0, M, N, K, As[g], K, Bs[g], N, Cs[g], N);
    }
  }
  gf_last_threads = used;
  return 0;
}

/* c[r] = a[r] * b[r] in GF(p)[X] for n pairs of k coefficients (2k - 1 out). */
int gf_plain_polymul(int p, int k, int64_t n, const uint8_t* a, const uint8_t* b, uint8_t* c,
                     int threads) {
  if (p < 2 || p > 251 || k < 1 || k > GF_KMAX || n < 0 || (n && (!a || !b || !c))) return -1;
  int used = 1;
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
      int prod[2 * GF_KMAX - 1] = {0};
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) prod[i + j] += (int)a[r * k + i] * (int)b[r * k + j];
      for (int t = 0; t < 2 * k - 1; ++t) c[r * (2 * k - 1) + t] = (uint8_t)(prod[t] % p);
    }
  }
  gf_last_threads = used;
  return 0;
}
