// Host side of the FQT library: the C ABI declared in include/fqt.h.
//
// Everything that can be checked is checked here, synchronously, before any
// launch: field validity (Section 7: p prime, P monic irreducible), the
// exactness conditions of Thm. 1 / eq. (2), pointer and size sanity.  Tables
// of Thm. 3 are built here from their definitions and copied to each device
// on first use.

#include "fqt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cinttypes>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "fqt_internal.h"
#include "plan_cache.h"

using namespace fqt;

namespace {

thread_local std::string g_last_error;

fqt_status fail(fqt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

fqt_status ok() { return FQT_OK; }

fqt_status hip_fail(hipError_t e, const char* what) {
  return fail(FQT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define FQT_HIP(call)                                 \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t d = 2; d * d <= n; ++d)
    if (n % d == 0) return false;
  return true;
}

uint32_t ceil_log2(uint32_t x) {  // smallest c with 2^c >= x
  uint32_t c = 0;
  while ((1u << c) < x) ++c;
  return c;
}

// a^e computed in 128-bit with saturation at 2^64 (returns false on overflow)
bool pow_u64(uint64_t a, uint32_t e, uint64_t* out) {
  unsigned __int128 v = 1;
  for (uint32_t i = 0; i < e; ++i) {
    v *= a;
    if (v > (unsigned __int128)UINT64_MAX) return false;
  }
  *out = (uint64_t)v;
  return true;
}

// q^e <= 2^m, exactly.
bool pow_at_most(uint64_t q, uint32_t e, uint32_t m) {
  unsigned __int128 v = 1, lim = (unsigned __int128)1 << m;
  for (uint32_t i = 0; i < e; ++i) {
    v *= q;
    if (v > lim) return false;
  }
  return true;
}

// q^e < 2^m, exactly.
bool pow_below(uint64_t q, uint32_t e, uint32_t m) {
  unsigned __int128 v = 1, lim = (unsigned __int128)1 << m;
  for (uint32_t i = 0; i < e; ++i) {
    v *= q;
    if (v >= lim) return false;
  }
  return true;
}

// ---- polynomial helpers over GF(p) (host) --------------------------------

// Remainder of c (length n) modulo the monic D = X^d + sum D_low[i] X^i.
std::vector<uint32_t> poly_mod(std::vector<uint32_t> c, const uint32_t* D_low, uint32_t d,
                               uint32_t p) {
  for (int64_t t = (int64_t)c.size() - 1; t >= (int64_t)d; --t) {
    const uint32_t lead = c[t] % p;
    c[t] = 0;
    if (!lead) continue;
    for (uint32_t i = 0; i < d; ++i)
      c[t - d + i] = (c[t - d + i] + lead * (p - D_low[i] % p)) % p;
  }
  c.resize(d, 0);
  return c;
}

bool irreducible(const uint32_t* P_low, uint32_t k, uint32_t p) {
  std::vector<uint32_t> P(P_low, P_low + k);
  P.push_back(1);
  for (uint32_t d = 1; d <= k / 2; ++d) {
    std::vector<uint32_t> D(d, 0);
    uint64_t count = 1;
    for (uint32_t i = 0; i < d; ++i) count *= p;
    for (uint64_t idx = 0; idx < count; ++idx) {
      uint64_t t = idx;
      for (uint32_t i = 0; i < d; ++i) {
        D[i] = (uint32_t)(t % p);
        t /= p;
      }
      auto r = poly_mod(P, D.data(), d, p);
      bool zero = true;
      for (uint32_t x : r) zero = zero && x == 0;
      if (zero) return false;
    }
  }
  return true;
}

struct DevTables {
  uint32_t* L = nullptr;
  uint32_t* H = nullptr;
};

// Calls on one device copy their work into a plan once per descriptor list:
// device copies of the descriptors, the schedule, the captured graph.  The
// plan owns them; its destructor waits for the device (a replay may still be
// in flight) and releases them.
struct BatchPlan {
  BatchPlan() = default;
  BatchPlan(const BatchPlan&) = delete;
  BatchPlan& operator=(const BatchPlan&) = delete;
  ~BatchPlan();
  GemmArgs* d_descs = nullptr;
  TileItem* d_items = nullptr;
  uint32_t* d_counter = nullptr;
  int32_t n_items = 0;
  int grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
  int32_t* d_wbeg = nullptr;  // tile kWaveTile: first item of every wave
  // INT8 plans only
  I8Batch* d_i8 = nullptr;
  ExpandItem* d_exp = nullptr;
  bool shares_ws = false;  // its graph reads the field's batch workspace of B'
};

// Runs `fn` with `device` current, then restores the caller's device.
template <class Fn>
void on_device(int device, Fn fn) {
  int cur = -1;
  const bool sw = device >= 0 && hipGetDevice(&cur) == hipSuccess && cur != device;
  if (sw) hipSetDevice(device);
  fn();
  if (sw) hipSetDevice(cur);
}

BatchPlan::~BatchPlan() {
  on_device(device, [&] {
    if (exec) hipDeviceSynchronize();
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    hipFree(d_descs);
    hipFree(d_items);
    hipFree(d_counter);
    hipFree(d_wbeg);
    hipFree(d_i8);
    hipFree(d_exp);
  });
}

// Plans kept per field; the least recently used beyond this are destroyed.
constexpr size_t kMaxPlans = 32;

struct Workspace {
  uint8_t* ptr = nullptr;
  size_t bytes = 0;
};

struct TuneEntry {
  fqt_path path;
  fqt_gemm_opts opts;
};

// Discrete-log representation (Alg. 4).  Codes e < m = p^k - 1 stand for
// g^e; m codes zero.
struct LogHost {
  bool built = false;
  uint32_t gen = 0;                // base-p index sum c_i p^i of the generator
  uint32_t m = 0;                  // p^k - 1
  std::vector<uint32_t> expw;      // code -> coefficient word (byte i = c_i), m + 1 entries
  std::vector<uint16_t> logt;      // binary index (Section 5.3) -> code
  std::vector<uint16_t> zech;      // Z[n] = log(1 + g^n), m + 1 entries (Z[m] = m)
};

struct DevLogBase {  // per device
  uint32_t* expw = nullptr;
  uint16_t* logt = nullptr;
  uint16_t* zech = nullptr;
};

struct DevLogQ {  // per device and q = 2^b
  uint32_t* pk = nullptr;  // evaluation at q of every code's element, pk[m] = 0
  uint32_t* L = nullptr;  // Thm. 3's tables, holding codes
  uint32_t* H = nullptr;
};

}  // namespace

struct fqt_field_s {
  uint32_t p = 0, k = 0, cb = 0, tbl_log2 = 0;
  uint32_t P_low[4] = {0, 0, 0, 0};
  std::mutex mu;
  std::map<uint32_t, std::pair<std::vector<uint32_t>, std::vector<uint32_t>>> host_tables;
  std::map<std::pair<int, uint32_t>, DevTables> dev_tables;
  fqt_detail::PlanCache<BatchPlan> plans{kMaxPlans};
  std::map<int, hipStream_t> cap_stream;  // per device: where plans are captured
  std::map<int, Workspace> bws;  // per device: B' of batched INT8 plans, shared by all
  std::map<std::string, TuneEntry> tuned;
  std::map<int, Workspace> ws;  // per device: B' of the INT8 path
  std::map<int, Workspace> wg_ws;  // per device: temporaries of Winograd's recursion
  std::map<int, uint8_t*> dev_mt;  // per device: multiplication-matrix table
  LogHost lg;
  std::map<int, DevLogBase> dev_logb;
  std::map<std::pair<int, uint32_t>, DevLogQ> dev_logq;  // (device, b)
};

namespace {

// The stream the plans of `f` on device `dev` are captured on: one per field
// and device, created on first use (f->mu is held).
hipError_t capture_stream(fqt_field f, int dev, hipStream_t* out) {
  auto it = f->cap_stream.find(dev);
  if (it == f->cap_stream.end()) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    it = f->cap_stream.emplace(dev, st).first;
  }
  *out = it->second;
  return hipSuccess;
}

FieldArgs field_args(const fqt_field_s* f, uint64_t q) {
  FieldArgs fa{};
  fa.p = f->p;
  fa.cb = f->cb;
  fa.negp24 = (1u << 24) - f->p;
  fa.mod_magic = (uint32_t)(((1ull << 32) + f->p - 1) / f->p);
  fa.sub_magic = 0x01010101u * (0x80u - f->p);
  fa.c = (uint32_t)((f->p - (uint32_t)(q % f->p)) % f->p);
  fa.inv_p = 1.0 / (double)f->p;
  return fa;
}

// Thm. 3: L over (u_0..u_{k-1}) and H over (u_{k-1}..u_{2k-2}).
void build_tables(const fqt_field_s* f, uint64_t q, std::vector<uint32_t>& L,
                  std::vector<uint32_t>& H) {
  const uint32_t p = f->p, k = f->k, cb = f->cb;
  const uint32_t qm = (uint32_t)(q % p);
  const size_t n = (size_t)1 << (k * cb);
  L.assign(n, 0);
  H.assign(n, 0);
  std::vector<uint32_t> w(k);
  uint64_t count = 1;
  for (uint32_t i = 0; i < k; ++i) count *= p;
  for (uint64_t idx = 0; idx < count; ++idx) {
    uint64_t t = idx;
    size_t bin = 0;
    for (uint32_t i = 0; i < k; ++i) {
      w[i] = (uint32_t)(t % p);
      t /= p;
      bin |= (size_t)w[i] << (cb * i);
    }
    // corrected digit: (w_i - q w_{i+1}) mod p
    auto corr = [&](uint32_t i) { return (w[i] + (p - qm) * w[i + 1]) % p; };
    // L: sum_{i <= k-2} corr(i) X^i
    uint32_t le = 0;
    for (uint32_t i = 0; i + 1 < k; ++i) le |= corr(i) << (8 * i);
    L[bin] = le;
    // H: w_{k-1} X^{2k-2} + sum_{t<k-1} corr(t) X^{k-1+t}, reduced mod P
    std::vector<uint32_t> poly(2 * k - 1, 0);
    poly[2 * k - 2] = w[k - 1];
    for (uint32_t i = 0; i + 1 < k; ++i) poly[k - 1 + i] = corr(i);
    auto red = poly_mod(poly, f->P_low, k, p);
    uint32_t he = 0;
    for (uint32_t i = 0; i < k; ++i) he |= red[i] << (8 * i);
    H[bin] = he;
  }
}

const std::pair<std::vector<uint32_t>, std::vector<uint32_t>>& host_tables(fqt_field_s* f,
                                                                          uint64_t q) {
  const uint32_t key = (uint32_t)(q % f->p);
  auto it = f->host_tables.find(key);
  if (it == f->host_tables.end()) {
    std::vector<uint32_t> L, H;
    build_tables(f, q, L, H);
    it = f->host_tables.emplace(key, std::make_pair(std::move(L), std::move(H))).first;
  }
  return it->second;
}

fqt_status device_tables(fqt_field_s* f, uint64_t q, DevTables* out) {
  std::lock_guard<std::mutex> lk(f->mu);
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  const auto key = std::make_pair(dev, (uint32_t)(q % f->p));
  auto it = f->dev_tables.find(key);
  if (it != f->dev_tables.end()) {
    *out = it->second;
    return ok();
  }
  const auto& ht = host_tables(f, q);
  const size_t bytes = ht.first.size() * sizeof(uint32_t);
  DevTables dt;
  FQT_HIP(hipMalloc(&dt.L, bytes));
  FQT_HIP(hipMalloc(&dt.H, bytes));
  FQT_HIP(hipMemcpy(dt.L, ht.first.data(), bytes, hipMemcpyHostToDevice));
  FQT_HIP(hipMemcpy(dt.H, ht.second.data(), bytes, hipMemcpyHostToDevice));
  f->dev_tables[key] = dt;
  *out = dt;
  return ok();
}

// Multiplication-matrix table of the INT8 path: for every binary index
// idx = sum_j c_j << (cb j) of an element b (Section 5.3's indexing), entry
// idx holds at byte s*k + i coefficient s of X^i * b mod P (the matrix of
// a -> a*b, transposed), mt_stride(k) bytes per entry; indices with a digit
// >= p hold zeros.

fqt_status device_mt(fqt_field_s* f, uint8_t** out) {
  std::lock_guard<std::mutex> lk(f->mu);
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  auto it = f->dev_mt.find(dev);
  if (it != f->dev_mt.end()) {
    *out = it->second;
    return ok();
  }
  const uint32_t k = f->k, p = f->p, cb = f->cb, stride = mt_stride(k);
  const size_t n = (size_t)1 << f->tbl_log2;
  std::vector<uint8_t> mt(n * stride, 0);
  for (size_t idx = 0; idx < n; ++idx) {
    std::vector<uint32_t> b(k);
    bool valid = true;
    for (uint32_t j = 0; j < k; ++j) {
      b[j] = (uint32_t)(idx >> (cb * j)) & ((1u << cb) - 1);
      valid = valid && b[j] < p;
    }
    if (!valid) continue;
    std::vector<uint32_t> row = b;  // X^i * b mod P, i = 0, 1, ...
    for (uint32_t i = 0; i < k; ++i) {
      for (uint32_t sidx = 0; sidx < k; ++sidx) mt[idx * stride + sidx * k + i] = (uint8_t)row[sidx];
      // row <- X * row mod P: shift up, then X^k = -sum P_low[s] X^s
      const uint32_t top = row[k - 1];
      for (uint32_t sidx = k - 1; sidx > 0; --sidx)
        row[sidx] = (row[sidx - 1] + top * (p - f->P_low[sidx] % p)) % p;
      row[0] = (top * (p - f->P_low[0] % p)) % p;
    }
  }
  uint8_t* d = nullptr;
  FQT_HIP(hipMalloc(&d, mt.size()));
  FQT_HIP(hipMemcpy(d, mt.data(), mt.size(), hipMemcpyHostToDevice));
  f->dev_mt[dev] = d;
  *out = d;
  return ok();
}

// ---- discrete-log tables (host, then per device) ----------------------------

// Product of two elements given as k coefficients, reduced mod P.
std::vector<uint32_t> elem_mul(const fqt_field_s* f, const std::vector<uint32_t>& a,
                               const std::vector<uint32_t>& b) {
  const uint32_t k = f->k, p = f->p;
  std::vector<uint32_t> c(2 * k - 1, 0);
  for (uint32_t i = 0; i < k; ++i)
    for (uint32_t j = 0; j < k; ++j) c[i + j] = (c[i + j] + a[i] * b[j]) % p;
  return poly_mod(c, f->P_low, k, p);
}

std::vector<uint32_t> elem_pow(const fqt_field_s* f, std::vector<uint32_t> a, uint64_t e) {
  std::vector<uint32_t> r(f->k, 0);
  r[0] = 1;
  while (e) {
    if (e & 1) r = elem_mul(f, r, a);
    a = elem_mul(f, a, a);
    e >>= 1;
  }
  return r;
}

// Generator: the first element in base-p order whose order is m = p^k - 1,
// i.e. a^(m/r) != 1 for every prime r dividing m.  Then the exponent,
// binary-index and Zech tables.  Caller holds f->mu.
void log_host(fqt_field_s* f) {
  LogHost& lg = f->lg;
  if (lg.built) return;
  const uint32_t p = f->p, k = f->k, cb = f->cb;
  uint32_t pk = 1;
  for (uint32_t i = 0; i < k; ++i) pk *= p;
  const uint32_t m = pk - 1;
  std::vector<uint32_t> primes;
  for (uint32_t x = m, d = 2; x > 1; ++d) {
    if (d * d > x) d = x;
    if (x % d == 0) {
      primes.push_back(d);
      while (x % d == 0) x /= d;
    }
  }
  auto coeffs = [&](uint32_t idx) {
    std::vector<uint32_t> c(k);
    for (uint32_t i = 0; i < k; ++i, idx /= p) c[i] = idx % p;
    return c;
  };
  auto is_one = [&](const std::vector<uint32_t>& c) {
    if (c[0] != 1) return false;
    for (uint32_t i = 1; i < k; ++i)
      if (c[i]) return false;
    return true;
  };
  uint32_t gen = 0;
  for (uint32_t idx = 1; idx < pk && !gen; ++idx) {
    const auto a = coeffs(idx);
    bool full = true;
    for (uint32_t r : primes) full = full && !is_one(elem_pow(f, a, m / r));
    if (full) gen = idx;
  }
  auto word = [&](const std::vector<uint32_t>& c) {
    uint32_t w = 0;
    for (uint32_t i = 0; i < k; ++i) w |= c[i] << (8 * i);
    return w;
  };
  auto bin = [&](const std::vector<uint32_t>& c) {
    uint32_t b = 0;
    for (uint32_t i = 0; i < k; ++i) b |= c[i] << (cb * i);
    return b;
  };
  lg.gen = gen;
  lg.m = m;
  lg.expw.assign(m + 1, 0);
  lg.logt.assign((size_t)1 << (k * cb), (uint16_t)m);
  lg.zech.assign(m + 1, (uint16_t)m);
  const auto g = coeffs(gen);
  std::vector<std::vector<uint32_t>> powers(m);
  std::vector<uint32_t> x(k, 0);
  x[0] = 1;
  for (uint32_t e = 0; e < m; ++e) {
    powers[e] = x;
    lg.expw[e] = word(x);
    lg.logt[bin(x)] = (uint16_t)e;
    x = elem_mul(f, x, g);
  }
  for (uint32_t n = 0; n < m; ++n) {
    auto y = powers[n];
    y[0] = (y[0] + 1) % p;
    lg.zech[n] = lg.logt[bin(y)];
  }
  lg.built = true;
}

template <typename T>
fqt_status upload(const std::vector<T>& v, T** out) {
  FQT_HIP(hipMalloc(out, v.size() * sizeof(T)));
  FQT_HIP(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return ok();
}

fqt_status device_log_base(fqt_field_s* f, DevLogBase* out) {
  std::lock_guard<std::mutex> lk(f->mu);
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  auto it = f->dev_logb.find(dev);
  if (it != f->dev_logb.end()) {
    *out = it->second;
    return ok();
  }
  log_host(f);
  DevLogBase d;
  fqt_status st = upload(f->lg.expw, &d.expw);
  if (!st) st = upload(f->lg.logt, &d.logt);
  if (!st) st = upload(f->lg.zech, &d.zech);
  if (st) {
    hipFree(d.expw);
    hipFree(d.logt);
    hipFree(d.zech);
    return st;
  }
  f->dev_logb[dev] = d;
  *out = d;
  return ok();
}

// Packed values at q = 2^b and Thm. 3's tables mapped to codes.
fqt_status device_log_q(fqt_field_s* f, uint32_t b, DevLogQ* out) {
  std::lock_guard<std::mutex> lk(f->mu);
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  const auto key = std::make_pair(dev, b);
  auto it = f->dev_logq.find(key);
  if (it != f->dev_logq.end()) {
    *out = it->second;
    return ok();
  }
  log_host(f);
  const LogHost& lg = f->lg;
  const uint32_t k = f->k, cb = f->cb;
  const uint64_t q = 1ull << b;
  std::vector<uint32_t> pk(lg.m + 1, 0);
  for (uint32_t e = 0; e < lg.m; ++e) {
    uint64_t v = 0;
    for (int i = (int)k - 1; i >= 0; --i) v = v * q + ((lg.expw[e] >> (8 * i)) & 0xffu);
    if (v > UINT32_MAX) return fail(FQT_ERR_UNSUPPORTED, "packed value above 2^32 at q = 2^%u", b);
    pk[e] = (uint32_t)v;  // below p q^(k-1) < 2^32 for every q eq. (2) admits
  }
  const auto& ht = host_tables(f, q);
  auto to_code = [&](uint32_t w) {
    uint32_t bi = 0;
    for (uint32_t i = 0; i < k; ++i) bi |= ((w >> (8 * i)) & 0xffu) << (cb * i);
    return (uint32_t)lg.logt[bi];
  };
  std::vector<uint32_t> Lc(ht.first.size()), Hc(ht.second.size());
  for (size_t i = 0; i < Lc.size(); ++i) {
    Lc[i] = to_code(ht.first[i]);
    Hc[i] = to_code(ht.second[i]);
  }
  DevLogQ d;
  fqt_status st = upload(pk, &d.pk);
  if (!st) st = upload(Lc, &d.L);
  if (!st) st = upload(Hc, &d.H);
  if (st) {
    hipFree(d.pk);
    hipFree(d.L);
    hipFree(d.H);
    return st;
  }
  f->dev_logq[key] = d;
  *out = d;
  return ok();
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return na && nb && x < y + nb && y < x + na;
}

uint32_t max_pow2_b(uint32_t k) {  // largest b with (2k-1) b < 53, i.e. q^(2k-1) < 2^53
  return 52 / (2 * k - 1);
}

// Matrix extent in bytes for rows x cols elements with leading dimension ld.
size_t mat_bytes(int64_t rows, int64_t cols, int64_t ld, uint32_t k) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)(((rows - 1) * ld + cols) * (int64_t)k);
}

// eb = bytes per element (k coefficients, or 2 for a discrete-log code)
fqt_status check_gemm_args(const fqt_field_s* f, int64_t M, int64_t N, int64_t K,
                           const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb,
                           uint8_t* C, int64_t ldc, uint32_t eb = 0) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (!eb) eb = f->k;
  if (M < 0 || N < 0 || K < 0) return fail(FQT_ERR_INVALID_ARG, "negative dimension");
  if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
    return fail(FQT_ERR_UNSUPPORTED, "dimension above 2^31-1");
  if (lda < std::max<int64_t>(K, 1) || ldb < std::max<int64_t>(N, 1) ||
      ldc < std::max<int64_t>(N, 1))
    return fail(FQT_ERR_INVALID_ARG, "leading dimension smaller than the row length");
  if (M && N && !C) return fail(FQT_ERR_INVALID_ARG, "null C");
  if (M && K && !A) return fail(FQT_ERR_INVALID_ARG, "null A");
  if (K && N && !B) return fail(FQT_ERR_INVALID_ARG, "null B");
  const size_t nc = mat_bytes(M, N, ldc, eb);
  if (overlap(C, nc, A, mat_bytes(M, K, lda, eb)) || overlap(C, nc, B, mat_bytes(K, N, ldb, eb)))
    return fail(FQT_ERR_INVALID_ARG, "C overlaps A or B");
  return ok();
}

// Resolved parameters of the packed path.
struct PackedChoice {
  uint32_t b;
  uint32_t nq;        // MFMA slots per K-block (multiple of 4)
  uint32_t nq_real;   // products per K-block (<= nq; the rest are zero slots)
  uint32_t tile;
  bool multi;
  int mode;           // 0 single block, 1 REDQ residues, 2 digit sums
  uint32_t fold;      // boundaries between folds of the 16-bit lanes (0: never)
  bool centered;      // centred packing, digits shifted by q/2
};

// The fields of a choice as words (no padding bytes), for plan keys.
std::array<uint32_t, 8> choice_words(const PackedChoice& c) {
  return {c.b, c.nq, c.nq_real, c.tile, (uint32_t)c.multi, (uint32_t)c.mode, c.fold,
          (uint32_t)c.centered};
}

// d-split tiles: chunks of 2 coefficients packed at q = 2^17 (q^3 < 2^53).
// The largest digits are those of S_K = sum (a_lo + a_hi)(b_lo + b_hi), up
// to w (p-1)^2 per k with w = 8 for k = 4 and 4 for k = 3: one block takes
// n_q w (p-1)^2 < q.  Longer K is cut into blocks of whole 16-k steps, each
// starting from digits below p: (p-1) + n w (p-1)^2 < q.
constexpr uint32_t kSplitB = 17;

uint64_t split_unit(uint32_t p, uint32_t k) {
  return (uint64_t)(k == 4 ? 8 : 4) * (p - 1) * (p - 1);
}

fqt_status resolve_packed(const fqt_field_s* f, const fqt_gemm_opts* o, int64_t K, int64_t M,
                          int64_t N, PackedChoice* pc) {
  const uint32_t p = f->p, k = f->k;
  if (o && o->tile > (uint32_t)kPackedTiles)
    return fail(FQT_ERR_INVALID_ARG, "unknown tile id %u", o->tile);
  if (o && o->tile && is_split_tile((int)o->tile)) {
    if (o->centered)
      return fail(FQT_ERR_UNSUPPORTED, "centred packing runs on the LDS-staged tiles");
    if (k != 3 && k != 4)
      return fail(FQT_ERR_UNSUPPORTED, "d-split tiles pair coefficients of k = 3 or 4 (k = %u)", k);
    if (o->log2q && o->log2q != kSplitB)
      return fail(FQT_ERR_INVALID_ARG, "d-split tiles pack chunks at q = 2^%u", kSplitB);
    const uint64_t q = 1ull << kSplitB, unit = split_unit(p, k);
    const uint64_t nq_one = unit ? (q - 1) / unit : (uint64_t)1 << 30;
    if (o->n_q > nq_one)
      return fail(FQT_ERR_BOUNDS, "n_q = %u breaks the d-split bound %" PRIu64, o->n_q, nq_one);
    const uint64_t nq = o->n_q ? o->n_q : nq_one;
    pc->multi = (uint64_t)K > nq;
    pc->nq = 0;
    if (pc->multi) {
      const uint64_t nq_next = unit ? (q - p) / unit : nq;
      const uint64_t steps = std::min(nq, nq_next) / 16;
      if (steps == 0)
        return fail(FQT_ERR_UNSUPPORTED, "d-split blocks below 16 products (p = %u, n_q = %" PRIu64
                    ")", p, nq);
      pc->nq = (uint32_t)std::min<uint64_t>(steps * 16, 1u << 30);
    }
    pc->b = kSplitB;
    pc->nq_real = pc->nq;
    pc->tile = o->tile;
    pc->mode = 0;
    pc->fold = 0;
    pc->centered = false;
    return ok();
  }
  if (o && o->tile == (uint32_t)kWaveTile) {
    // wave-persistent tile: k = 4, q = 2^7, digit-sum block steps, blocks of
    // 4 nqg products with nqg = 1..kWaveMaxNqg fixed at compile time
    if (k != 4)
      return fail(FQT_ERR_UNSUPPORTED, "tile %d runs fields of k = 4 (k = %u)", kWaveTile, k);
    const uint32_t b = max_pow2_b(k);
    if (o->log2q && o->log2q != b)
      return fail(FQT_ERR_UNSUPPORTED, "tile %d packs at q = 2^%u", kWaveTile, b);
    const bool cenw = o->centered != 0;
    if (cenw && (p == 2 || p > 8))
      return fail(FQT_ERR_UNSUPPORTED, "tile %d centres coefficients for odd p <= 7 (p = %u)",
                  kWaveTile, p);
    const uint32_t bmode = o->boundary ? o->boundary : 2u;
    if (bmode != 2)
      return fail(FQT_ERR_UNSUPPORTED, "tile %d takes digit-sum block steps only", kWaveTile);
    const uint64_t q = 1ull << b, hc = (p - 1) / 2;
    const uint64_t unit = cenw ? (uint64_t)k * hc * hc : (uint64_t)k * (p - 1) * (p - 1);
    const uint64_t room = cenw ? q / 2 - 1 : q - 1;
    const uint64_t nq_max = room / unit;
    const uint64_t nq = o->n_q ? o->n_q : nq_max;
    if (nq > nq_max)
      return fail(FQT_ERR_BOUNDS, "n_q = %" PRIu64 " breaks the %s bound for q = 2^%u", nq,
                  cenw ? "centred" : "eq. (2)", b);
    const uint64_t nqg = std::min<uint64_t>(nq / 4, (uint64_t)kWaveMaxNqg);
    if (nqg == 0)
      return fail(FQT_ERR_UNSUPPORTED, "tile %d needs blocks of at least 4 products (n_q = %"
                  PRIu64 ")", kWaveTile, nq);
    if ((uint64_t)p * p * p * p > (uint64_t)kWaveDqtEntries)  // implied by n_q >= 4
      return fail(FQT_ERR_UNSUPPORTED, "tile %d tabulates at most %d elements (p = %u)",
                  kWaveTile, kWaveDqtEntries, p);
    // digit sums in fields of 2b bits: every absorbed block adds at most q - 1
    // to a field (its digits; centred: shifted digits), a fold leaves < p,
    // and the epilogue adds an offset below p (the centred shift's removal);
    // blocks: ceil(K / (4 nqg)) and one of the bias alone
    const uint64_t width = (1ull << (2 * b)) - 1, growth = q - 1;
    const uint64_t cap = (width - 2 * (p - 1)) / growth;
    const uint64_t nblocks = ((uint64_t)K + 4 * nqg - 1) / (4 * nqg) + 1;
    pc->b = b;
    pc->nq = pc->nq_real = (uint32_t)(4 * nqg);
    pc->tile = (uint32_t)kWaveTile;
    pc->multi = (uint64_t)K > 4 * nqg;
    pc->mode = 2;
    pc->fold = nblocks + 1 > cap ? (uint32_t)(cap - 1) : 0u;
    pc->centered = cenw;
    return ok();
  }
  const bool cen = o && o->centered;
  if (cen && p == 2) return fail(FQT_ERR_UNSUPPORTED, "centred packing needs an odd p");
  if (cen && o->tile && (int)o->tile > kStagedTiles)
    return fail(FQT_ERR_UNSUPPORTED, "centred packing runs on the LDS-staged tiles 1..%d",
                kStagedTiles);
  const uint32_t bmax = max_pow2_b(k);
  uint32_t b = (o && o->log2q) ? o->log2q : bmax;
  if (b > bmax || b < 1)
    return fail(FQT_ERR_BOUNDS, "q = 2^%u breaks (2k-1) log2 q < 53 (k = %u)", b, k);
  // residue windows [b*i, b*i+8) must stay below bit 52 of the binary64 pattern
  if (b * (2 * k - 2) + 8 > 52)
    return fail(FQT_ERR_UNSUPPORTED, "q = 2^%u leaves no room for the residue bytes (k = %u)", b,
                k);
  const uint64_t q = 1ull << b;
  // eq. (2): q > n_q k (p-1)^2; centred: n_q k ((p-1)/2)^2 <= q/2 - 1
  const uint64_t hc = (p - 1) / 2;
  const uint64_t unit = cen ? (uint64_t)k * hc * hc : (uint64_t)k * (p - 1) * (p - 1);
  if (cen && b < 2) return fail(FQT_ERR_BOUNDS, "centred packing needs q >= 4");
  const uint64_t room = cen ? q / 2 - 1 : q - 1;
  const uint64_t nq_max = unit ? room / unit : UINT32_MAX;
  uint64_t nq = (o && o->n_q) ? o->n_q : nq_max;
  if (nq > nq_max)
    return fail(FQT_ERR_BOUNDS, "n_q = %" PRIu64 " breaks the %s bound for q = 2^%u", nq,
                cen ? "centred" : "eq. (2)", b);
  nq = std::min<uint64_t>(nq, 1u << 30);
  // Blocks are whole MFMA k-groups of 4 slots.  A block of n_q % 4 != 0
  // products is padded with zero slots when the slot count divides every
  // K-tile (8 or 16); otherwise n_q is rounded down to a multiple of 4.
  // Register-direct tiles take no padded blocks.
  const bool direct = o && o->tile && is_direct_tile((int)o->tile);
  uint64_t slots = nq & ~3ull, real = slots;
  if (!direct && nq % 4 && (K > (int64_t)nq) &&
      ((nq + 3) / 4 * 4 == 8 || (nq + 3) / 4 * 4 == 16)) {
    slots = (nq + 3) / 4 * 4;
    real = nq;
  }
  if (slots < 4)
    return fail(FQT_ERR_UNSUPPORTED, "n_q below 4 (q = 2^%u, p = %u, k = %u)", b, p, k);
  const bool multi = (uint64_t)K > real;
  if (multi && b != bmax)
    return fail(FQT_ERR_UNSUPPORTED, "several K-blocks need the largest q = 2^%u", bmax);
  nq = slots;
  // default: digit sums where their fields fit (2b <= 24), else REDQ residues
  const uint32_t bmode = (o && o->boundary) ? o->boundary : (2 * b <= 24 ? 2u : 1u);
  if (bmode > 2) return fail(FQT_ERR_INVALID_ARG, "unknown boundary mode %u", bmode);
  uint32_t fold = 0;
  if (multi) {
    // lanes grow by < 2p (residues) or by at most one block's digit bound per
    // boundary; keep (p-1) + (fold+1) * growth below 2^16 (the +1 is the
    // last block, added in the epilogue)
    // REDQ residues: 16-bit lanes grow by < 2p per block.  Digit sums: fields
    // of 2b bits grow by at most the block's digit bound; they need 2b <= 24.
    if (bmode == 2 && 2 * b > 24)
      return fail(FQT_ERR_UNSUPPORTED, "digit-sum boundaries need q <= 2^12 (q = 2^%u)", b);
    const uint64_t width = bmode == 1 ? 65535 : (1ull << (2 * b)) - 1;
    // centred: every block's shifted digits are below q
    const uint64_t growth = bmode == 1 ? 2 * (uint64_t)p - 1 : cen ? q - 1 : real * unit;
    const uint64_t nblocks = ((uint64_t)K + real - 1) / real + 8;
    const uint64_t cap = (width - (p - 1)) / std::max<uint64_t>(growth, 1);
    if (cap < 2) return fail(FQT_ERR_UNSUPPORTED, "residue lanes too narrow for n_q = %" PRIu64, nq);
    if (nblocks + 1 > cap) fold = (uint32_t)(cap - 1);
  }
  uint32_t tile = (o && o->tile) ? o->tile : 0;
  if (tile > (uint32_t)kPackedTiles) return fail(FQT_ERR_INVALID_ARG, "unknown tile id %u", tile);
  if (tile && is_direct_tile((int)tile)) {
    if (multi && !direct_tile_multi_ok((int)tile))
      return fail(FQT_ERR_UNSUPPORTED, "tile %u takes single-block problems only (K <= n_q)",
                  tile);
  }
  if (!tile) {
    // default: the largest tile that still gives every CU two workgroups
    static const int pref[] = {4, 3, 2, 5, 6, 1};
    tile = 1;
    for (int id : pref) {
      if (id == 4 && k >= 3 && multi && bmode == 1) continue;  // that variant spills registers
      int bm, bn;
      packed_tile_shape(id, &bm, &bn);
      const int64_t nt = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
      if (nt >= 256) {
        tile = (uint32_t)id;
        break;
      }
    }
  }
  pc->b = b;
  pc->nq = (uint32_t)nq;
  pc->nq_real = (uint32_t)real;
  pc->tile = tile;
  pc->multi = multi;
  pc->centered = cen;
  pc->mode = multi ? (int)bmode : 0;
  pc->fold = fold;
  return ok();
}

std::string shape_key(const fqt_field_s* f, int64_t count, int64_t M, int64_t N, int64_t K) {
  auto bucket = [](int64_t x) {
    int64_t b = 1;
    while (b < x) b <<= 1;
    return b;
  };
  char buf[128];
  std::snprintf(buf, sizeof buf, "p%u_k%u_c%lld_%lld_%lld_%lld", f->p, f->k, (long long)count,
                (long long)bucket(M), (long long)bucket(N), (long long)bucket(K));
  return buf;
}

}  // namespace

// ============================================================================
extern "C" {

const char* fqt_last_error(void) { return g_last_error.c_str(); }

const char* fqt_version(void) { return "fqt-mi355x 0.1 (gfx950)"; }

uint32_t fqt_tile_count(fqt_path path) {
  return path == FQT_PATH_PACKED_F64 ? (uint32_t)kPackedTiles
         : path == FQT_PATH_INT8      ? (uint32_t)kInt8Tiles
                                      : 1u;
}

fqt_status fqt_field_create(uint32_t p, uint32_t k, const uint32_t* P_low, fqt_field* out) {
  if (!out) return fail(FQT_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!is_prime_u32(p)) return fail(FQT_ERR_NOT_PRIME, "p = %u is not prime", p);
  if (p > 127) return fail(FQT_ERR_UNSUPPORTED, "p = %u above 127", p);
  if (k < 1 || k > 4) return fail(FQT_ERR_UNSUPPORTED, "k = %u outside [1, 4]", k);
  if (k > 1 && !P_low) return fail(FQT_ERR_INVALID_ARG, "null defining polynomial");
  auto f = std::make_unique<fqt_field_s>();
  f->p = p;
  f->k = k;
  f->cb = std::max(1u, ceil_log2(p));
  for (uint32_t i = 0; i < k; ++i) {
    const uint32_t c = P_low ? P_low[i] : 0;
    if (c >= p) return fail(FQT_ERR_INVALID_ARG, "P coefficient %u not in [0, p)", c);
    f->P_low[i] = c;
  }
  if (!irreducible(f->P_low, k, p))
    return fail(FQT_ERR_REDUCIBLE, "defining polynomial is reducible over GF(%u)", p);
  f->tbl_log2 = k * f->cb;
  if (f->tbl_log2 > 12)
    return fail(FQT_ERR_UNSUPPORTED, "tables of 2^%u entries exceed 4096", f->tbl_log2);
  *out = f.release();
  return ok();
}

void fqt_field_destroy(fqt_field f) {
  if (!f) return;
  f->plans.clear();  // waits for replays in flight
  for (auto& kv : f->cap_stream) on_device(kv.first, [&] { hipStreamDestroy(kv.second); });
  for (auto& kv : f->bws) on_device(kv.first, [&] { hipFree(kv.second.ptr); });
  for (auto& kv : f->dev_tables) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      hipSetDevice(kv.first.first);
      hipFree(kv.second.L);
      hipFree(kv.second.H);
      hipSetDevice(cur);
    }
  }
  for (auto& kv : f->ws) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      hipSetDevice(kv.first);
      hipFree(kv.second.ptr);
      hipSetDevice(cur);
    }
  }
  for (auto& kv : f->wg_ws) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      hipSetDevice(kv.first);
      hipFree(kv.second.ptr);
      hipSetDevice(cur);
    }
  }
  for (auto& kv : f->dev_mt) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      hipSetDevice(kv.first);
      hipFree(kv.second);
      hipSetDevice(cur);
    }
  }
  for (auto& kv : f->dev_logb) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      hipSetDevice(kv.first);
      hipFree(kv.second.expw);
      hipFree(kv.second.logt);
      hipFree(kv.second.zech);
      hipSetDevice(cur);
    }
  }
  for (auto& kv : f->dev_logq) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      hipSetDevice(kv.first.first);
      hipFree(kv.second.pk);
      hipFree(kv.second.L);
      hipFree(kv.second.H);
      hipSetDevice(cur);
    }
  }
  delete f;
}

fqt_status fqt_field_tables(fqt_field f, uint64_t q, uint32_t* L, uint32_t* H,
                            size_t* n_entries) {
  if (!f || !n_entries) return fail(FQT_ERR_INVALID_ARG, "null argument");
  if (q < 2) return fail(FQT_ERR_INVALID_ARG, "q < 2");
  std::lock_guard<std::mutex> lk(f->mu);
  const auto& t = host_tables(f, q);
  const size_t n = t.first.size();
  if ((L || H) && *n_entries < n)
    return fail(FQT_ERR_INVALID_ARG, "table buffers hold %zu entries, need %zu", *n_entries, n);
  *n_entries = n;
  if (L) std::memcpy(L, t.first.data(), n * sizeof(uint32_t));
  if (H) std::memcpy(H, t.second.data(), n * sizeof(uint32_t));
  return ok();
}

fqt_status fqt_params(uint32_t p, uint32_t k, uint64_t n_q, int pow2_q, int carry_in,
                      uint64_t* q_out, uint64_t* nq_max_out) {
  if (!is_prime_u32(p)) return fail(FQT_ERR_NOT_PRIME, "p = %u is not prime", p);
  if (k < 1 || k > 16) return fail(FQT_ERR_UNSUPPORTED, "k = %u outside [1, 16]", k);
  if (n_q < 1) return fail(FQT_ERR_INVALID_ARG, "n_q must be at least 1");
  const uint32_t e = 2 * k - 1;
  uint64_t q;
  if (pow2_q) {
    q = 1ull << (52 / e);  // largest 2^b with b * e < 53
  } else {
    // largest integer q with q^e < 2^53
    q = (uint64_t)std::floor(std::pow(2.0, 53.0 / e));
    while (q > 1 && !pow_below(q, e, 53)) --q;
    while (pow_below(q + 1, e, 53)) ++q;
  }
  const unsigned __int128 unit = (unsigned __int128)k * (p - 1) * (p - 1);
  const unsigned __int128 extra = carry_in ? (p - 1) : 0;
  // eq. (2): q > n_q k (p-1)^2 (+ (p-1) when a reduced value re-enters)
  uint64_t nq_max = 0;
  if (unit == 0) nq_max = UINT64_MAX;
  else if ((unsigned __int128)q > extra) nq_max = (uint64_t)(((unsigned __int128)q - 1 - extra) / unit);
  if (q_out) *q_out = q;
  if (nq_max_out) *nq_max_out = nq_max;
  if (n_q > nq_max)
    return fail(FQT_ERR_BOUNDS, "no q with q^%u < 2^53 exceeds %" PRIu64 " * %u * (%u-1)^2", e,
                n_q, k, p);
  return ok();
}

fqt_status fqt_pack(fqt_field f, uint64_t q, const uint8_t* coeffs, size_t n, double* packed,
                    fqt_stream_t s) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (n && (!coeffs || !packed)) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (q < 2) return fail(FQT_ERR_INVALID_ARG, "q < 2");
  // largest packed value (p-1) * sum_{j<k} q^j must be exact in binary64
  unsigned __int128 mx = 0, qp = 1;
  for (uint32_t j = 0; j < f->k; ++j) {
    mx += (unsigned __int128)(f->p - 1) * qp;
    qp *= q;
    if (qp > ((unsigned __int128)1 << 70)) break;
  }
  if (mx > ((unsigned __int128)1 << 53) || qp > ((unsigned __int128)1 << 70))
    return fail(FQT_ERR_BOUNDS, "packed values exceed 2^53 at q = %" PRIu64, q);
  if (overlap(coeffs, n * f->k, packed, n * sizeof(double)))
    return fail(FQT_ERR_INVALID_ARG, "input and output overlap");
  const int pow2 = (q & (q - 1)) == 0;
  const uint32_t b = pow2 ? (uint32_t)__builtin_ctzll(q) : 0;
  FQT_HIP(launch_pack((int)f->k, q, pow2, b, coeffs, n, packed, (hipStream_t)s));
  return ok();
}

static fqt_status unpack_common(fqt_field f, uint64_t q, const void* packed, size_t n,
                                uint32_t ndigits, fqt_unpack_mode mode, uint8_t* out,
                                fqt_stream_t s, bool wide) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (n && (!packed || !out)) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (q < 2) return fail(FQT_ERR_INVALID_ARG, "q < 2");
  if (mode != FQT_UNPACK_POLY && mode != FQT_UNPACK_FIELD)
    return fail(FQT_ERR_INVALID_ARG, "unknown unpack mode");
  if (ndigits < 1 || ndigits > 15) return fail(FQT_ERR_UNSUPPORTED, "ndigits outside [1, 15]");
  if (mode == FQT_UNPACK_FIELD && ndigits > 2 * f->k - 1)
    return fail(FQT_ERR_INVALID_ARG, "FIELD mode takes at most 2k-1 = %u digits", 2 * f->k - 1);
  // binary64: every value is an exact integer below q^ndigits <= 2^53 (eq. (2), m = 53);
  // uint64: any value, as long as the top digit's place q^(ndigits-1) is below 2^64
  if (wide ? !pow_below(q, ndigits - 1, 64) : !pow_at_most(q, ndigits, 53))
    return fail(FQT_ERR_BOUNDS, "q^%u exceeds the %s range", ndigits, wide ? "uint64" : "binary64");
  const size_t ob = mode == FQT_UNPACK_POLY ? ndigits : f->k;
  if (overlap(packed, n * 8, out, n * ob)) return fail(FQT_ERR_INVALID_ARG, "buffers overlap");
  const int pow2 = (q & (q - 1)) == 0;
  const uint32_t b = pow2 ? (uint32_t)__builtin_ctzll(q) : 0;
  const FieldArgs fa = field_args(f, q);
  DevTables dt;
  if (mode == FQT_UNPACK_FIELD) {
    fqt_status st = device_tables(f, q, &dt);
    if (st) return st;
  }
  if (wide)
    FQT_HIP(launch_unpack_u64((int)f->k, ndigits, (int)mode, q, pow2, b, fa, dt.L, dt.H,
                              (const uint64_t*)packed, n, out, (hipStream_t)s));
  else
    FQT_HIP(launch_unpack_f64((int)f->k, ndigits, (int)mode, q, pow2, b, fa, dt.L, dt.H,
                              (const double*)packed, n, out, (hipStream_t)s));
  return ok();
}

fqt_status fqt_unpack_redq(fqt_field f, uint64_t q, const double* packed, size_t n,
                           uint32_t ndigits, fqt_unpack_mode mode, uint8_t* out, fqt_stream_t s) {
  return unpack_common(f, q, packed, n, ndigits, mode, out, s, false);
}

fqt_status fqt_unpack_redq_u64(fqt_field f, uint64_t q, const uint64_t* packed, size_t n,
                               uint32_t ndigits, fqt_unpack_mode mode, uint8_t* out,
                               fqt_stream_t s) {
  return unpack_common(f, q, packed, n, ndigits, mode, out, s, true);
}

fqt_status fqt_polymul_batch(uint32_t p, uint32_t k, uint64_t q, const uint8_t* a,
                             const uint8_t* b, size_t n, uint8_t* c, fqt_stream_t s) {
  if (!is_prime_u32(p)) return fail(FQT_ERR_NOT_PRIME, "p = %u is not prime", p);
  if (p > 127) return fail(FQT_ERR_UNSUPPORTED, "p = %u above 127", p);
  if (k < 1 || k > 8) return fail(FQT_ERR_UNSUPPORTED, "k = %u outside [1, 8]", k);
  if (n && (!a || !b || !c)) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (q < 2) return fail(FQT_ERR_INVALID_ARG, "q < 2");
  // eq. (2) with n_q = 1
  if (!((unsigned __int128)q > (unsigned __int128)k * (p - 1) * (p - 1)) ||
      !pow_below(q, 2 * k - 1, 53))
    return fail(FQT_ERR_BOUNDS, "q = %" PRIu64 " breaks eq. (2) for p = %u, k = %u", q, p, k);
  const size_t nc = n * (2 * k - 1);
  if (overlap(c, nc, a, n * k) || overlap(c, nc, b, n * k))
    return fail(FQT_ERR_INVALID_ARG, "output overlaps an input");
  fqt_field_s tmp;
  tmp.p = p;
  tmp.k = k;
  tmp.cb = std::max(1u, ceil_log2(p));
  const FieldArgs fa = field_args(&tmp, q);
  const int pow2 = (q & (q - 1)) == 0;
  const uint32_t bb = pow2 ? (uint32_t)__builtin_ctzll(q) : 0;
  FQT_HIP(launch_polymul((int)k, q, pow2, bb, fa, a, b, n, c, (hipStream_t)s));
  return ok();
}

}  // extern "C"

namespace {

// Resolved parameters of the d-FQT (Section 6) for products whose longest
// chunk-pair sum has nprod products.
struct DfqtChoice {
  uint32_t ke, bq, fold;
  uint64_t q, nq;
  int mode;
};

fqt_status resolve_dfqt(uint32_t p, uint32_t d, uint32_t log2q, uint32_t n_q, uint32_t boundary,
                        uint32_t centered, int64_t nprod, DfqtChoice* out) {
  if (!is_prime_u32(p)) return fail(FQT_ERR_NOT_PRIME, "p = %u is not prime", p);
  if (p > 127) return fail(FQT_ERR_UNSUPPORTED, "p = %u above 127", p);
  if (d > 7) return fail(FQT_ERR_UNSUPPORTED, "d = %u above 7 (chunks of at most 8 coefficients)", d);
  if (boundary > 2) return fail(FQT_ERR_INVALID_ARG, "unknown boundary mode %u", boundary);
  if (centered > 1) return fail(FQT_ERR_INVALID_ARG, "centered is 0 or 1");
  if (centered && p == 2) return fail(FQT_ERR_UNSUPPORTED, "centred chunks need an odd p");
  const uint32_t ke = d + 1;
  // eq. (2) with k = d+1 coefficients per packed number: q^(2d+1) < 2^53,
  // q > n_q (d+1)(p-1)^2; q = 2^b with (2d+1) b <= 52 so that the biased
  // accumulator holds the sum, and the residue bytes stay below bit 52
  const uint32_t bmax = 52 / (2 * ke - 1);
  const uint32_t bq = log2q ? log2q : bmax;
  if (bq < 1 || bq > bmax)
    return fail(FQT_ERR_BOUNDS, "q = 2^%u breaks q^(2d+1) < 2^53 (d = %u)", bq, d);
  if (bq * (2 * ke - 2) + 8 > 52)
    return fail(FQT_ERR_UNSUPPORTED, "q = 2^%u leaves no room for the residue bytes", bq);
  const uint64_t q = 1ull << bq;
  // centred chunks: n_q (d+1) ((p-1)/2)^2 <= q/2 - 1 instead of eq. (2)
  const uint64_t hc = (p - 1) / 2;
  const uint64_t unit = centered ? (uint64_t)ke * hc * hc : (uint64_t)ke * (p - 1) * (p - 1);
  const uint64_t room = centered ? (bq >= 2 ? q / 2 - 1 : 0) : q - 1;
  const uint64_t nq_max = unit ? room / unit : (uint64_t)1 << 30;
  if (nq_max < 1)
    return fail(FQT_ERR_BOUNDS, "q = 2^%u cannot hold one chunk product (d = %u, p = %u)", bq, d,
                p);
  const uint64_t nq = n_q ? n_q : std::min<uint64_t>(nq_max, (uint64_t)1 << 30);
  if (nq > nq_max)
    return fail(FQT_ERR_BOUNDS, "n_q = %" PRIu64 " breaks the %s bound", nq,
                centered ? "centred" : "eq. (2)");
  const bool multi = (uint64_t)nprod > nq;  // the longest S_t has nprod products
  if (multi && bq != bmax)
    return fail(FQT_ERR_UNSUPPORTED, "several blocks need the largest q = 2^%u", bmax);
  int mode = 0;
  uint32_t fold = 0;
  if (multi) {
    mode = boundary ? (int)boundary : (2 * bq <= 24 ? 2 : 1);
    if (mode == 2 && 2 * bq > 24)
      return fail(FQT_ERR_UNSUPPORTED, "digit-sum boundaries need q <= 2^12 (q = 2^%u)", bq);
    const uint64_t width = mode == 1 ? 65535 : q * q - 1;
    const uint64_t growth = mode == 1 ? 2 * (uint64_t)p - 1 : centered ? q - 1 : nq * unit;
    const uint64_t nblocks = ((uint64_t)nprod + nq - 1) / nq + 1;
    const uint64_t cap = (width - (p - 1)) / std::max<uint64_t>(growth, 1);
    if (cap < 2) return fail(FQT_ERR_UNSUPPORTED, "residue lanes too narrow for n_q = %" PRIu64, nq);
    if (nblocks + 1 > cap) fold = (uint32_t)(cap - 1);
  }
  *out = DfqtChoice{ke, bq, fold, q, nq, mode};
  return ok();
}

PackedParams dfqt_params(uint32_t p, uint32_t centered, const DfqtChoice& c) {
  fqt_field_s tmp;
  tmp.p = p;
  tmp.k = c.ke;
  tmp.cb = std::max(1u, ceil_log2(p));
  PackedParams pp{};
  pp.fa = field_args(&tmp, c.q);
  pp.qmod = (uint32_t)(c.q % p);
  pp.fold_blocks = c.fold;
  pp.b = c.bq;
  if (centered) {
    uint64_t B = 0;
    for (uint32_t j = 0; j < 2 * c.ke - 1; ++j) B = B * c.q + c.q / 2;  // below q^(2d+1) <= 2^52
    pp.centered = 1;
    pp.cbias = 4503599627370496.0 + (double)B;
    pp.c0neg = (uint32_t)((c.q / 2) % p);
  }
  return pp;
}

// Plans of uneven polynomial batches (no field handle: one process-wide
// cache, bounded like a field's, and one capture stream per device).
struct PolyPlan {
  PolyPlan() = default;
  PolyPlan(const PolyPlan&) = delete;
  PolyPlan& operator=(const PolyPlan&) = delete;
  ~PolyPlan() {
    on_device(device, [&] {
      if (exec) hipDeviceSynchronize();
      if (exec) hipGraphExecDestroy(exec);
      if (graph) hipGraphDestroy(graph);
      hipFree(d_descs);
      hipFree(d_order);
    });
  }
  PolyDesc* d_descs = nullptr;
  int32_t* d_order = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
  int32_t live = 0;  // pairs with output
};
std::mutex g_poly_mu;
fqt_detail::PlanCache<PolyPlan> g_poly_plans{kMaxPlans};
std::map<int, hipStream_t> g_poly_cap;  // per device; lives until the process ends

}  // namespace

extern "C" {

fqt_status fqt_polymul_dfqt(uint32_t p, uint32_t d, uint32_t log2q, uint32_t n_q,
                            uint32_t boundary, uint32_t centered, const uint8_t* a,
                            const uint8_t* b, int64_t count, int64_t len, uint8_t* c,
                            fqt_stream_t s) {
  if (count < 0 || len < 1) return fail(FQT_ERR_INVALID_ARG, "count < 0 or len < 1");
  if (count && (!a || !b || !c)) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (d <= 7) {
    const int64_t nch = (len + d) / (d + 1);
    if (nch > kDfqtMaxChunks)
      return fail(FQT_ERR_UNSUPPORTED, "len = %lld needs %lld chunks, above %d", (long long)len,
                  (long long)nch, kDfqtMaxChunks);
  }
  DfqtChoice ch;
  fqt_status st = resolve_dfqt(p, d, log2q, n_q, boundary, centered, (len + d) / (d + 1), &ch);
  if (st) return st;
  const int64_t nch = (len + ch.ke - 1) / ch.ke;
  const size_t nc = (size_t)count * (size_t)(2 * len - 1), ni = (size_t)count * (size_t)len;
  if (overlap(c, nc, a, ni) || overlap(c, nc, b, ni))
    return fail(FQT_ERR_INVALID_ARG, "output overlaps an input");
  DfqtArgs g{};
  g.a = a;
  g.b = b;
  g.c = c;
  g.count = count;
  g.len = (int32_t)len;
  g.nch = (int32_t)nch;
  g.cap = (int32_t)nch;
  g.nq = (uint32_t)ch.nq;
  g.lg2q = ch.bq;
  g.pp = dfqt_params(p, centered, ch);
  FQT_HIP(launch_dfqt((int)ch.ke, ch.mode, g, (hipStream_t)s));
  return ok();
}

}  // extern "C"

namespace {

// Checks of an uneven batch (every one on the host, before any device work)
// and the resolved d-FQT parameters; *live counts the pairs with output.
fqt_status poly_batch_check(uint32_t p, uint32_t d, uint32_t log2q, uint32_t n_q,
                                   uint32_t boundary, uint32_t centered, int64_t count,
                                   const fqt_poly_desc* descs, DfqtChoice* ch, int64_t* live,
                                   int32_t* cap) {
  if (count < 0 || (count && !descs)) return fail(FQT_ERR_INVALID_ARG, "bad descriptor array");
  if (count > INT32_MAX) return fail(FQT_ERR_UNSUPPORTED, "more than 2^31 - 1 pairs");
  if (d > 7) return fail(FQT_ERR_UNSUPPORTED, "d = %u above 7 (chunks of at most 8 coefficients)", d);
  const int64_t ke = d + 1;
  int64_t nprod = 1, chmax = 1;
  *live = 0;
  for (int64_t i = 0; i < count; ++i) {
    const fqt_poly_desc& e = descs[i];
    if (e.la < 0 || e.lb < 0)
      return fail(FQT_ERR_INVALID_ARG, "descriptor %lld: negative length", (long long)i);
    if (e.la == 0 || e.lb == 0) continue;
    ++*live;
    if (!e.a || !e.b || !e.c)
      return fail(FQT_ERR_INVALID_ARG, "descriptor %lld: null buffer", (long long)i);
    const int64_t nca = (e.la + ke - 1) / ke, ncb = (e.lb + ke - 1) / ke;
    if (nca > kDfqtMaxChunks || ncb > kDfqtMaxChunks)
      return fail(FQT_ERR_UNSUPPORTED, "descriptor %lld: %lld x %lld coefficients need more "
                  "than %d chunks", (long long)i, (long long)e.la, (long long)e.lb,
                  kDfqtMaxChunks);
    const size_t nc = (size_t)(e.la + e.lb - 1);
    if (overlap(e.c, nc, e.a, (size_t)e.la) || overlap(e.c, nc, e.b, (size_t)e.lb))
      return fail(FQT_ERR_INVALID_ARG, "descriptor %lld: output overlaps an input", (long long)i);
    nprod = std::max(nprod, std::min(nca, ncb));
    chmax = std::max(chmax, std::max(nca, ncb));
  }
  *cap = (int32_t)chmax;
  return resolve_dfqt(p, d, log2q, n_q, boundary, centered, nprod, ch);
}

// Pairs with output, longest first (a pair costs about nca ncb chunk products).
std::vector<int32_t> poly_order(int64_t count, const fqt_poly_desc* descs,
                                             int64_t ke) {
  std::vector<int32_t> order;
  for (int64_t i = 0; i < count; ++i)
    if (descs[i].la > 0 && descs[i].lb > 0) order.push_back((int32_t)i);
  auto cost = [&](int32_t i) {
    return ((descs[i].la + ke - 1) / ke) * ((descs[i].lb + ke - 1) / ke);
  };
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
  return order;
}

// Four waves per workgroup, each with LDS for cap chunks per operand: as
// many workgroups as fit on every CU at once, never more waves than pairs.
fqt_status poly_grid(int dev, int64_t live, const DfqtChoice& ch, uint32_t centered, int32_t cap,
                     int* grid) {
  int cus = 0;
  FQT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int per_cu = dfqt_batched_occupancy((int)ch.ke, ch.mode, centered != 0, cap);
  *grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu, (live + 3) / 4));
  return ok();
}

}  // namespace

extern "C" {

fqt_status fqt_polymul_dfqt_batched(uint32_t p, uint32_t d, uint32_t log2q, uint32_t n_q,
                                    uint32_t boundary, uint32_t centered, int64_t count,
                                    const fqt_poly_desc* descs, fqt_stream_t s) {
  if (count < 0 || (count && !descs)) return fail(FQT_ERR_INVALID_ARG, "bad descriptor array");
  // plan key: the descriptors and the call's own arguments, which decide
  // every check and every resolved parameter, and the device.  A list seen
  // before replays its plan without walking the descriptors again.
  int dev = -1;
  const bool have_dev = count > 0 && hipGetDevice(&dev) == hipSuccess;
  const uint32_t tag[8] = {p, d, log2q, n_q, boundary, centered, (uint32_t)dev, 0u};
  const fqt_detail::PlanKey key{descs, sizeof(fqt_poly_desc) * (size_t)count,
                                fqt_detail::key_tail(tag)};
  if (have_dev) {
    std::lock_guard<std::mutex> lk(g_poly_mu);
    if (PolyPlan* plan = g_poly_plans.find(key)) {
      if (plan->live > 0) FQT_HIP(hipGraphLaunch(plan->exec, (hipStream_t)s));
      return ok();
    }
  }
  DfqtChoice ch;
  int64_t live = 0;
  int32_t cap = 1;
  fqt_status st = poly_batch_check(p, d, log2q, n_q, boundary, centered, count, descs, &ch, &live,
                                   &cap);
  if (st) return st;
  if (live == 0) return ok();  // nothing to write: an empty product has no coefficient
  const int64_t ke = d + 1;
  FQT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_poly_mu);
  PolyPlan* plan = g_poly_plans.find(key);
  if (!plan) {
    const std::vector<int32_t> order = poly_order(count, descs, ke);
    auto pl = std::make_unique<PolyPlan>();
    pl->device = dev;
    pl->live = (int32_t)order.size();
    FQT_HIP(hipMalloc(&pl->d_descs, sizeof(PolyDesc) * count));
    FQT_HIP(hipMalloc(&pl->d_order, sizeof(int32_t) * std::max<size_t>(order.size(), 1)));
    static_assert(sizeof(PolyDesc) == sizeof(fqt_poly_desc), "descriptor layouts agree");
    FQT_HIP(hipMemcpy(pl->d_descs, descs, sizeof(PolyDesc) * count, hipMemcpyHostToDevice));
    if (!order.empty())
      FQT_HIP(hipMemcpy(pl->d_order, order.data(), sizeof(int32_t) * order.size(),
                        hipMemcpyHostToDevice));
    int grid = 1;
    st = poly_grid(dev, pl->live, ch, centered, cap, &grid);
    if (st) return st;
    DfqtBatchArgs g{};
    g.cap = cap;
    g.descs = pl->d_descs;
    g.order = pl->d_order;
    g.count = pl->live;
    g.nq = (uint32_t)ch.nq;
    g.lg2q = ch.bq;
    g.pp = dfqt_params(p, centered, ch);
    if (!g_poly_cap.count(dev)) {
      hipStream_t ns = nullptr;
      FQT_HIP(hipStreamCreateWithFlags(&ns, hipStreamNonBlocking));
      g_poly_cap[dev] = ns;
    }
    hipStream_t cs = g_poly_cap[dev];
    FQT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    if (pl->live > 0) le = launch_dfqt_batched((int)ch.ke, ch.mode, g, grid, cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (le != hipSuccess) return hip_fail(le, "d-FQT batched launch (capture)");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    FQT_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0));
    plan = g_poly_plans.insert(key, std::move(pl));
  }
  if (plan->live == 0) return ok();
  FQT_HIP(hipGraphLaunch(plan->exec, (hipStream_t)s));
  return ok();
}

fqt_status fqt_polymul_dfqt_batched_noalloc(uint32_t p, uint32_t d, uint32_t log2q,
                                            uint32_t n_q, uint32_t boundary, uint32_t centered,
                                            int64_t count, const fqt_poly_desc* descs,
                                            fqt_stream_t s) {
  DfqtChoice ch;
  int64_t live = 0;
  int32_t cap = 1;
  fqt_status st = poly_batch_check(p, d, log2q, n_q, boundary, centered, count, descs, &ch, &live,
                                   &cap);
  if (st) return st;
  if (live > (int64_t)kDfqtNoAllocMaxPairs)
    return fail(FQT_ERR_UNSUPPORTED, "%lld pairs with output: the allocation-free batch takes "
                "at most %zu", (long long)live, kDfqtNoAllocMaxPairs);
  if (live == 0) return ok();
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  // the descriptors in schedule order, staged in a per-thread host array that
  // keeps its capacity across calls
  thread_local std::vector<PolyDesc> ordered;
  const std::vector<int32_t> order = poly_order(count, descs, (int64_t)d + 1);
  ordered.resize(order.size());
  for (size_t i = 0; i < order.size(); ++i)
    std::memcpy(&ordered[i], &descs[order[i]], sizeof(PolyDesc));
  int grid = 1;
  st = poly_grid(dev, live, ch, centered, cap, &grid);
  if (st) return st;
  DfqtBatchArgs g{};
  g.cap = cap;
  g.count = (int32_t)live;
  g.nq = (uint32_t)ch.nq;
  g.lg2q = ch.bq;
  g.pp = dfqt_params(p, centered, ch);
  FQT_HIP(launch_dfqt_batched_noalloc((int)ch.ke, ch.mode, g, ordered.data(), grid,
                                      (hipStream_t)s));
  return ok();
}

fqt_status fqt_polymul_delayed(uint32_t p, const uint8_t* a, const uint8_t* b, int64_t count,
                               int64_t len, uint8_t* c, fqt_stream_t s) {
  if (!is_prime_u32(p)) return fail(FQT_ERR_NOT_PRIME, "p = %u is not prime", p);
  if (p > 127) return fail(FQT_ERR_UNSUPPORTED, "p = %u above 127", p);
  if (count < 0 || len < 1) return fail(FQT_ERR_INVALID_ARG, "count < 0 or len < 1");
  if (count && (!a || !b || !c)) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (len > kDelayedMaxLen)
    return fail(FQT_ERR_UNSUPPORTED, "len = %lld above %d", (long long)len, kDelayedMaxLen);
  const size_t nc = (size_t)count * (size_t)(2 * len - 1), ni = (size_t)count * (size_t)len;
  if (overlap(c, nc, a, ni) || overlap(c, nc, b, ni))
    return fail(FQT_ERR_INVALID_ARG, "output overlaps an input");
  // eq. (3), unsigned: a reduced value below p plus n_d (p-1)^2 stays below 2^32
  const uint64_t sq = (uint64_t)(p - 1) * (p - 1);
  const uint64_t lim = 0xffffffffull - p;
  DelayedArgs g{a, b, c, count, (int32_t)len, p, 0};
  if (sq && (uint64_t)len * sq > lim) g.nd = (uint32_t)(lim / sq);
  FQT_HIP(launch_polymul_delayed(g, (hipStream_t)s));
  return ok();
}

// ---- discrete-log representation (Alg. 4) -----------------------------------

fqt_status fqt_log_info(fqt_field f, uint32_t* generator_index, uint32_t* zero_code) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  std::lock_guard<std::mutex> lk(f->mu);
  log_host(f);
  if (generator_index) *generator_index = f->lg.gen;
  if (zero_code) *zero_code = f->lg.m;
  return ok();
}

fqt_status fqt_to_log(fqt_field f, const uint8_t* coeffs, int64_t n, uint16_t* codes,
                      fqt_stream_t s) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (n < 0) return fail(FQT_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return ok();
  if (!coeffs || !codes) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (overlap(coeffs, (size_t)n * f->k, codes, (size_t)n * 2))
    return fail(FQT_ERR_INVALID_ARG, "output overlaps the input");
  DevLogBase d;
  fqt_status st = device_log_base(f, &d);
  if (st) return st;
  FQT_HIP(launch_to_log((int)f->k, f->cb, coeffs, n, d.logt, codes, (hipStream_t)s));
  return ok();
}

fqt_status fqt_from_log(fqt_field f, const uint16_t* codes, int64_t n, uint8_t* coeffs,
                        fqt_stream_t s) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (n < 0) return fail(FQT_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return ok();
  if (!coeffs || !codes) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  if (overlap(coeffs, (size_t)n * f->k, codes, (size_t)n * 2))
    return fail(FQT_ERR_INVALID_ARG, "output overlaps the input");
  DevLogBase d;
  fqt_status st = device_log_base(f, &d);
  if (st) return st;
  FQT_HIP(launch_from_log((int)f->k, codes, n, f->lg.m, d.expw, coeffs, (hipStream_t)s));
  return ok();
}

fqt_status fqt_log_add(fqt_field f, const uint16_t* a, const uint16_t* b, int64_t n, uint16_t* c,
                       fqt_stream_t s) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (n < 0) return fail(FQT_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return ok();
  if (!a || !b || !c) return fail(FQT_ERR_INVALID_ARG, "null buffer");
  const size_t nb = (size_t)n * 2;
  // in place (c == a or c == b) is fine; any other overlap is not
  if ((c != a && overlap(c, nb, a, nb)) || (c != b && overlap(c, nb, b, nb)))
    return fail(FQT_ERR_INVALID_ARG, "output partly overlaps an input");
  DevLogBase d;
  fqt_status st = device_log_base(f, &d);
  if (st) return st;
  FQT_HIP(launch_log_add(a, b, n, f->lg.m, d.zech, c, (hipStream_t)s));
  return ok();
}

fqt_status fqt_gemm_log(fqt_field f, const fqt_gemm_opts* opts, int64_t M, int64_t N, int64_t K,
                        const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, uint16_t* C,
                        int64_t ldc, fqt_stream_t s) {
  const uint8_t* A8 = reinterpret_cast<const uint8_t*>(A);
  const uint8_t* B8 = reinterpret_cast<const uint8_t*>(B);
  uint8_t* C8 = reinterpret_cast<uint8_t*>(C);
  fqt_status st = check_gemm_args(f, M, N, K, A8, lda, B8, ldb, C8, ldc, 2);
  if (st) return st;
  if (M == 0 || N == 0) return ok();
  fqt_gemm_opts o = opts ? *opts : fqt_gemm_opts{0, 0, 0, 0, 0};
  if (o.tile && !is_log_tile((int)o.tile))
    return fail(FQT_ERR_UNSUPPORTED, "tile %u: the log form runs tiles 7, 9 and 11", o.tile);
  uint32_t m;
  {
    std::lock_guard<std::mutex> lk(f->mu);
    log_host(f);
    m = f->lg.m;
  }
  PackedChoice pc;
  if (!o.tile) {
    // one block: the split-K tile when its LDS fits, else tile 9; several: 11
    fqt_gemm_opts probe = o;
    probe.tile = 11;
    st = resolve_packed(f, &probe, K, M, N, &pc);
    if (st) return st;
    o.tile = pc.multi ? 11 : (log_tile_fits(7, f->tbl_log2, m) ? 7 : 9);
  }
  if (!log_tile_fits((int)o.tile, f->tbl_log2, m))
    return fail(FQT_ERR_UNSUPPORTED, "tile %u: tables of %u codes do not fit LDS", o.tile, m + 1);
  st = resolve_packed(f, &o, K, M, N, &pc);
  if (st) return st;
  DevLogBase lb;
  st = device_log_base(f, &lb);
  if (st) return st;
  DevLogQ lq;
  st = device_log_q(f, pc.b, &lq);
  if (st) return st;
  const uint64_t q = 1ull << pc.b;
  PackedParams pp{};
  pp.b = pc.b;
  pp.nq_groups = pc.nq / 4;
  pp.tbl_log2 = f->tbl_log2;
  pp.aligned = ((((uintptr_t)A) | ((uintptr_t)B)) & 3) == 0 && (lda * 2) % 4 == 0 &&
               (ldb * 2) % 4 == 0;
  pp.fold_blocks = pc.fold;
  pp.qmask = (uint32_t)(q - 1);
  pp.qmod = (uint32_t)(q % f->p);
  pp.blk_real = pc.nq_real;
  pp.fa = field_args(f, q);
  pp.L = lq.L;
  pp.H = lq.H;
  pp.pk = lq.pk;
  pp.Z = lb.zech;
  pp.zero_code = m;
  GemmArgs g{A8, B8, C8, M, N, K, lda, ldb, ldc};
  FQT_HIP(launch_gemm_log((int)f->k, (int)pc.tile, pc.mode, g, pp, (hipStream_t)s));
  return ok();
}

// Centred packing: every block starts from 2^52 + B, B = sum_{i<2k-1} (q/2) q^i,
// whose residues beta_i = floor(B / q^i) mod p shift the residues of every
// block; L + H is linear in the residues, so the result carries
// n_blocks * (L + H)(beta), taken off at the end with c0neg.
// Caller holds f->mu.
void centred_params(fqt_field_s* f, uint32_t b, PackedParams* pp) {
  const uint32_t p = f->p, k = f->k, cb = f->cb, nd = 2 * k - 1;
  const uint64_t q = 1ull << b;
  uint64_t B = 0;
  for (uint32_t i = 0; i < nd; ++i) B = B * q + q / 2;  // below q^(2k-1) <= 2^52
  std::vector<uint32_t> beta(nd);
  for (uint32_t i = 0; i < nd; ++i) beta[i] = (uint32_t)((B >> (b * i)) % p);
  const auto& ht = host_tables(f, q);
  uint32_t il = 0, ih = 0;
  for (uint32_t d = 0; d < k; ++d) {
    il |= beta[d] << (cb * d);
    ih |= beta[k - 1 + d] << (cb * d);
  }
  const uint32_t lw = ht.first[il], hw = ht.second[ih];
  uint32_t neg = 0;
  for (uint32_t i = 0; i < k; ++i) {
    const uint32_t c = (((lw >> (8 * i)) & 0xffu) + ((hw >> (8 * i)) & 0xffu)) % p;
    neg |= ((p - c) % p) << (8 * i);
  }
  pp->centered = 1;
  pp->c0neg = neg;
  pp->cbias = 4503599627370496.0 + (double)B;
}

// DQT route of the LDS-staged loaders (PackedParams::dqt_flags, fqt_packed.h
// dqt_chunk): two byte dot products per element where k = 4 and q <= 2^7;
// for centred packing with p <= 8, a byte permutation to the offset form
// (c + h) mod p = c' + h and the constant -h (1 + q + ... + q^(k-1)).
void dqt_params(const fqt_field_s* f, uint32_t b, bool centered, PackedParams* pp) {
  pp->dqt_flags = 0;
  pp->lut_lo = pp->lut_hi = 0;
  pp->dqt_off = 0;
  if (f->k == 4 && b <= 7) pp->dqt_flags |= kDqtDot4;
  if (centered && f->p <= 8) {
    const uint32_t p = f->p, h = (p - 1) / 2;
    uint32_t lut[2] = {0, 0};
    for (uint32_t c = 0; c < 8; ++c) lut[c / 4] |= ((c + h) % p) << (8 * (c % 4));
    uint64_t S = 0, qj = 1;
    for (uint32_t j = 0; j < f->k; ++j, qj <<= b) S += qj;
    pp->lut_lo = lut[0];
    pp->lut_hi = lut[1];
    pp->dqt_off = -(int32_t)(h * S);  // h S < 2^31 under eq. (2)
    pp->dqt_flags |= kDqtLut;
  }
}

// Buffered direct tiles address A and B through 32-bit offsets.
static bool extents_fit_32(const GemmArgs& g, uint32_t k) {
  const uint64_t lim = 0x7fffffffull;
  const uint64_t ea = g.M && g.K ? ((uint64_t)(g.M - 1) * g.lda + g.K) * k : 0;
  const uint64_t eb = g.K && g.N ? ((uint64_t)(g.K - 1) * g.ldb + g.N) * k : 0;
  return ea < lim && eb < lim;
}

static fqt_status batched_wave(fqt_field f, const PackedChoice& pc, int64_t count,
                               const fqt_gemm_desc* descs, hipStream_t s);

static fqt_status gemm_packed(fqt_field f, const fqt_gemm_opts* opts, const GemmArgs& g,
                              hipStream_t s) {
  PackedChoice pc;
  fqt_status st = resolve_packed(f, opts, g.K, g.M, g.N, &pc);
  if (st) return st;
  if (pc.tile == (uint32_t)kWaveTile) {  // a batch of one
    const fqt_gemm_desc d{g.M, g.N, g.K, g.lda, g.ldb, g.ldc, g.A, g.B, g.C};
    return batched_wave(f, pc, 1, &d, s);
  }
  if (direct_tile_buffered((int)pc.tile) && !extents_fit_32(g, f->k))
    return fail(FQT_ERR_UNSUPPORTED, "tile %u addresses operands below 2^31 bytes only", pc.tile);
  const uint64_t q = 1ull << pc.b;
  const bool split = is_split_tile((int)pc.tile);
  DevTables dt;
  // d-split: the tables reduce a plain coefficient vector mod P (q = p)
  st = device_tables(f, split ? f->p : q, &dt);
  if (st) return st;
  PackedParams pp{};
  pp.b = pc.b;
  pp.nq_groups = pc.nq / 4;
  pp.tbl_log2 = f->tbl_log2;
  pp.aligned = ((((uintptr_t)g.A) | ((uintptr_t)g.B)) & 3) == 0 && (g.lda * f->k) % 4 == 0 &&
               (g.ldb * f->k) % 4 == 0;
  pp.fold_blocks = pc.fold;
  pp.qmask = (uint32_t)(q - 1);
  pp.qmod = (uint32_t)(q % f->p);
  pp.blk_real = pc.nq_real;
  pp.fa = field_args(f, q);
  pp.L = dt.L;
  pp.H = dt.H;
  if (pc.centered) {
    std::lock_guard<std::mutex> lk(f->mu);
    centred_params(f, pc.b, &pp);
  }
  dqt_params(f, pc.b, pc.centered, &pp);
  if (split)
    FQT_HIP(launch_gemm_split((int)f->k, (int)pc.tile, g, pp, s));
  else if (is_direct_tile((int)pc.tile))
    FQT_HIP(launch_gemm_direct((int)f->k, (int)pc.tile, pc.mode, g, pp, s));
  else
    FQT_HIP(launch_gemm_packed((int)f->k, (int)pc.tile, pc.mode, g, pp, s));
  return ok();
}

static fqt_status workspace(fqt_field f, size_t bytes, uint8_t** out) {
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(f->mu);
  Workspace& w = f->ws[dev];
  if (w.bytes < bytes) {
    if (w.ptr) {
      // earlier launches may still read the old buffer
      FQT_HIP(hipDeviceSynchronize());
      FQT_HIP(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    if (hipMalloc(&w.ptr, bytes) != hipSuccess)
      return fail(FQT_ERR_OOM, "INT8 workspace of %zu bytes", bytes);
    w.bytes = bytes;
  }
  *out = w.ptr;
  return ok();
}

// Alignment (16, 4 or 1 bytes) shared by every row start of a matrix.
static uint32_t row_align(const void* base, int64_t row_bytes) {
  const uintptr_t b = (uintptr_t)base;
  if ((b & 15) == 0 && (row_bytes & 15) == 0) return 16;
  if ((b & 3) == 0 && (row_bytes & 3) == 0) return 4;
  return 1;
}

// K-tiles (bkk bytes of K) between reductions mod p, 0 when the whole sum
// fits: (p-1) + n (bkk (p-1)^2) < 2^31 keeps every INT32 partial sum exact.
static uint32_t i8_red_tiles(int64_t KK, int64_t p, int64_t bkk = 128) {
  const int64_t per_tile = bkk * (p - 1) * (p - 1);
  const int64_t nkt = (KK + bkk - 1) / bkk;
  if (per_tile == 0 || nkt * per_tile < (1ll << 31)) return 0;
  return (uint32_t)(((1ll << 31) - 1 - (p - 1)) / per_tile);
}

// Fused INT8 tiles hold the multiplication-matrix table in LDS beside their
// operand tiles: admissible when both fit one CU's LDS.
static bool i8f_fits(const fqt_field_s* f, uint32_t tile) {
  const size_t table = ((size_t)1 << f->tbl_log2) * mt_stride(f->k);
  const size_t st = i8f_static_lds((int)tile, (int)f->k);
  return st > 0 && st + table <= kLdsBytes;
}

static I8Args i8_args(const fqt_field_s* f, const uint8_t* A, int64_t lda, uint8_t* C,
                      int64_t ldc, int64_t M, int64_t N, int64_t K, int64_t bkk) {
  const int64_t k = f->k, p = f->p;
  I8Args a{};
  a.A = A;
  a.lda = lda * k;
  a.C = C;
  a.ldc = ldc * k;
  a.M = M;
  a.NN = N * k;
  a.KK = K * k;
  a.p = (uint32_t)p;
  a.red_tiles = i8_red_tiles(K * k, p, bkk);
  a.a_vec = row_align(A, a.lda);
  a.inv_p = 1.0 / (double)p;
  return a;
}

// Fused INT8 tiles: one kernel, B'^T built per K-tile in LDS.
static fqt_status gemm_int8_fused(fqt_field f, uint32_t tile, const GemmArgs& g, hipStream_t s) {
  const int k = (int)f->k;
  if (!i8f_fits(f, tile))
    return fail(FQT_ERR_UNSUPPORTED, "INT8 tile %u: operand tiles and the %u-bit table exceed "
                "the LDS", tile, f->tbl_log2);
  uint8_t* mt = nullptr;
  fqt_status st = device_mt(f, &mt);
  if (st) return st;
  I8Batch b{};
  b.a = i8_args(f, g.A, g.lda, g.C, g.ldc, g.M, g.N, g.K, i8f_k_bytes(k));
  b.B = g.B;
  b.ldb = g.ldb;
  b.K = g.K;
  b.N = g.N;
  FQT_HIP(launch_gemm_i8f((int)tile, k, b, mt, f->cb, f->tbl_log2, s));
  return ok();
}

// INT8 path: exact while n_d (p-1)^2 < 2^31 per accumulation run (eq. (3)).
static fqt_status batched_i8cs(fqt_field f, int64_t count, const fqt_gemm_desc* descs,
                               hipStream_t s);

static fqt_status gemm_int8(fqt_field f, const fqt_gemm_opts* opts, const GemmArgs& g,
                            hipStream_t s) {
  const int64_t k = f->k, p = f->p;
  uint32_t tile = (opts && opts->tile) ? opts->tile : 0;
  if (tile > (uint32_t)kInt8Tiles) return fail(FQT_ERR_INVALID_ARG, "unknown INT8 tile id %u", tile);
  if (tile == kInt8StripTile) {  // a batch of one
    const fqt_gemm_desc d{g.M, g.N, g.K, g.lda, g.ldb, g.ldc, g.A, g.B, g.C};
    return batched_i8cs(f, 1, &d, s);
  }
  if (i8_fused_tile(tile)) return gemm_int8_fused(f, tile, g, s);
  // B'^T rows are padded to whole 128-byte K-tiles of the INT8 GEMM
  const int64_t NN = g.N * k, KK = g.K * k, KKpad = (KK + 127) / 128 * 128;
  // untuned default, from measurements on MI355X: the 256 x 256 8-wave tile
  // for large products, 64 x 64 with 256-byte K-tiles from about 2^20
  // outputs, 64 x 64 below
  if (!tile) tile = (g.M >= 2048 && NN >= 2048) ? 7 : (g.M * NN >= (1 << 20) ? 9 : 1);
  uint8_t* ws = nullptr;
  fqt_status st = workspace(f, (size_t)std::max<int64_t>(NN * KKpad, 1), &ws);
  if (st) return st;
  uint8_t* mt = nullptr;
  st = device_mt(f, &mt);
  if (st) return st;
  FQT_HIP(launch_expand_b((int)k, g.B, g.ldb, g.K, g.N, mt, f->cb, f->tbl_log2, ws, KKpad, KKpad,
                          s));
  I8Args a{};
  a.A = g.A;
  a.lda = g.lda * k;
  a.Bt = ws;
  a.ldbt = KKpad;
  a.C = g.C;
  a.ldc = g.ldc * k;
  a.M = g.M;
  a.NN = NN;
  a.KK = KK;
  a.KKpad = KKpad;
  a.p = (uint32_t)p;
  a.red_tiles = i8_red_tiles(KK, p, i8_tile_k((int)tile));
  a.a_vec = row_align(g.A, a.lda);
  a.inv_p = 1.0 / (double)p;
  FQT_HIP(launch_gemm_i8((int)tile, a, s));
  return ok();
}

fqt_status fqt_gemm_gfpk_ex(fqt_field f, fqt_path path, const fqt_gemm_opts* opts, int64_t M,
                            int64_t N, int64_t K, const uint8_t* A, int64_t lda,
                            const uint8_t* B, int64_t ldb, uint8_t* C, int64_t ldc,
                            fqt_stream_t s) {
  fqt_status st = check_gemm_args(f, M, N, K, A, lda, B, ldb, C, ldc);
  if (st) return st;
  GemmArgs g{A, B, C, M, N, K, lda, ldb, ldc};
  if (M == 0 || N == 0) return ok();
  // Tuned options stand for a shape class (power-of-two buckets of M, N, K)
  // and were checked admissible at the K they were tuned on; a larger K of
  // the same class may need more K-blocks than they allow.  Such a refusal
  // falls back to the path's defaults.
  fqt_gemm_opts tuned{};
  bool from_tuned = false;
  if (path == FQT_PATH_AUTO) {
    std::lock_guard<std::mutex> lk(f->mu);
    auto it = f->tuned.find(shape_key(f, 1, M, N, K));
    if (it != f->tuned.end()) {
      path = it->second.path;
      if (!opts) {
        tuned = it->second.opts;
        opts = &tuned;
        from_tuned = true;
      }
    } else {
      path = FQT_PATH_PACKED_F64;
    }
  }
  if (!opts && (path == FQT_PATH_PACKED_F64 || path == FQT_PATH_INT8)) {
    std::lock_guard<std::mutex> lk(f->mu);
    auto it = f->tuned.find(shape_key(f, 1, M, N, K) +
                            (path == FQT_PATH_INT8 ? "_int8" : "_packed"));
    if (it != f->tuned.end()) {
      tuned = it->second.opts;
      opts = &tuned;
      from_tuned = true;
    }
  }
  auto run = [&](const fqt_gemm_opts* o) -> fqt_status {
    switch (path) {
      case FQT_PATH_PACKED_F64:
        return gemm_packed(f, o, g, (hipStream_t)s);
      case FQT_PATH_PLAIN: {
        const FieldArgs fa = field_args(f, 2);
        FQT_HIP(launch_gemm_plain((int)f->k, g, fa, f->P_low, (hipStream_t)s));
        return ok();
      }
      case FQT_PATH_INT8:
        return gemm_int8(f, o, g, (hipStream_t)s);
      default:
        return fail(FQT_ERR_INVALID_ARG, "unknown path %d", (int)path);
    }
  };
  st = run(opts);
  if (from_tuned && (st == FQT_ERR_UNSUPPORTED || st == FQT_ERR_BOUNDS)) st = run(nullptr);
  return st;
}

fqt_status fqt_gemm_gfpk(fqt_field f, fqt_path path, int64_t M, int64_t N, int64_t K,
                         const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb,
                         uint8_t* C, int64_t ldc, fqt_stream_t s) {
  return fqt_gemm_gfpk_ex(f, path, nullptr, M, N, K, A, lda, B, ldb, C, ldc, s);
}

// ---- Winograd's recursion over the field ---------------------------------------
// Seven block products and fifteen block additions per level (the schedule
// of the paper's Fig. 3 experiments, finite-field Winograd multiplication
// with the FQT underneath); the block products are ordinary calls of the
// chosen path, the additions coefficient-wise mod p.  Odd dimensions are
// peeled: the last row and column by plain calls, the last k as a rank-one
// product added in.

namespace {

// Temporaries of one call: S1..S4 (h x d), T1..T4 (d x w), P1..P7 (h x w),
// the rank-one term (m x n) when K is odd, then those of the next level.
size_t wg_bytes(uint32_t k, uint32_t levels, int64_t M, int64_t N, int64_t K) {
  if (!levels || M < 2 || N < 2 || K < 2) return 0;
  const int64_t m = M & ~1LL, n = N & ~1LL, kk = K & ~1LL;
  const int64_t h = m / 2, w = n / 2, d = kk / 2;
  size_t here = (size_t)(4 * h * d + 4 * d * w + 7 * h * w) * k;
  if (kk < K) here += (size_t)(m * n) * k;
  return here + wg_bytes(k, levels - 1, h, w, d);
}

struct WgRun {
  fqt_field f;
  fqt_path path;
  const fqt_gemm_opts* opts;
  hipStream_t s;
};

fqt_status wg_add(const WgRun& r, const uint8_t* X, int64_t ldx, const uint8_t* Y, int64_t ldy,
                  uint8_t* Z, int64_t ldz, int64_t rows, int64_t cols, bool sub) {
  FQT_HIP(launch_mat_addsub((int)r.f->k, r.f->p, X, ldx, Y, ldy, Z, ldz, rows, cols, sub, r.s));
  return ok();
}

fqt_status wg_rec(const WgRun& r, uint32_t levels, int64_t M, int64_t N, int64_t K,
                  const uint8_t* A, int64_t lda, const uint8_t* B, int64_t ldb, uint8_t* C,
                  int64_t ldc, uint8_t* ws) {
  if (!levels || M < 2 || N < 2 || K < 2)
    return fqt_gemm_gfpk_ex(r.f, r.path, r.opts, M, N, K, A, lda, B, ldb, C, ldc, r.s);
  const int64_t k = r.f->k;
  const int64_t m = M & ~1LL, n = N & ~1LL, kk = K & ~1LL;
  const int64_t h = m / 2, w = n / 2, d = kk / 2;
  const uint8_t *A11 = A, *A12 = A + d * k, *A21 = A + h * lda * k, *A22 = A21 + d * k;
  const uint8_t *B11 = B, *B12 = B + w * k, *B21 = B + d * ldb * k, *B22 = B21 + w * k;
  uint8_t *C11 = C, *C12 = C + w * k, *C21 = C + h * ldc * k, *C22 = C21 + w * k;
  uint8_t* cur = ws;
  auto take = [&](int64_t elems) {
    uint8_t* q = cur;
    cur += elems * k;
    return q;
  };
  uint8_t *S1 = take(h * d), *S2 = take(h * d), *S3 = take(h * d), *S4 = take(h * d);
  uint8_t *T1 = take(d * w), *T2 = take(d * w), *T3 = take(d * w), *T4 = take(d * w);
  uint8_t* P[8];
  for (int i = 1; i <= 7; ++i) P[i] = take(h * w);
  uint8_t* R = kk < K ? take(m * n) : nullptr;
  uint8_t* next = cur;
  fqt_status st;
#define FQT_WG(x)   \
  do {              \
    st = (x);       \
    if (st) return st; \
  } while (0)
  FQT_WG(wg_add(r, A21, lda, A22, lda, S1, d, h, d, false));  // S1 = A21 + A22
  FQT_WG(wg_add(r, S1, d, A11, lda, S2, d, h, d, true));      // S2 = S1 - A11
  FQT_WG(wg_add(r, A11, lda, A21, lda, S3, d, h, d, true));   // S3 = A11 - A21
  FQT_WG(wg_add(r, A12, lda, S2, d, S4, d, h, d, true));      // S4 = A12 - S2
  FQT_WG(wg_add(r, B12, ldb, B11, ldb, T1, w, d, w, true));   // T1 = B12 - B11
  FQT_WG(wg_add(r, B22, ldb, T1, w, T2, w, d, w, true));      // T2 = B22 - T1
  FQT_WG(wg_add(r, B22, ldb, B12, ldb, T3, w, d, w, true));   // T3 = B22 - B12
  FQT_WG(wg_add(r, T2, w, B21, ldb, T4, w, d, w, true));      // T4 = T2 - B21
  auto rec = [&](const uint8_t* X, int64_t ldx, const uint8_t* Y, int64_t ldy, uint8_t* Z) {
    return wg_rec(r, levels - 1, h, w, d, X, ldx, Y, ldy, Z, w, next);
  };
  FQT_WG(rec(A11, lda, B11, ldb, P[1]));
  FQT_WG(rec(A12, lda, B21, ldb, P[2]));
  FQT_WG(rec(S4, d, B22, ldb, P[3]));
  FQT_WG(rec(A22, lda, T4, w, P[4]));
  FQT_WG(rec(S1, d, T1, w, P[5]));
  FQT_WG(rec(S2, d, T2, w, P[6]));
  FQT_WG(rec(S3, d, T3, w, P[7]));
  FQT_WG(wg_add(r, P[1], w, P[2], w, C11, ldc, h, w, false));  // C11 = P1 + P2
  FQT_WG(wg_add(r, P[1], w, P[6], w, P[6], w, h, w, false));   // U2 = P1 + P6, in P6
  FQT_WG(wg_add(r, P[6], w, P[7], w, P[7], w, h, w, false));   // U3 = U2 + P7, in P7
  FQT_WG(wg_add(r, P[6], w, P[5], w, P[1], w, h, w, false));   // U4 = U2 + P5, in P1
  FQT_WG(wg_add(r, P[1], w, P[3], w, C12, ldc, h, w, false));  // C12 = U4 + P3
  FQT_WG(wg_add(r, P[7], w, P[4], w, C21, ldc, h, w, true));   // C21 = U3 - P4
  FQT_WG(wg_add(r, P[7], w, P[5], w, C22, ldc, h, w, false));  // C22 = U3 + P5
  if (R) {  // the last k: C[:m, :n] += A[:m, kk] B[kk, :n]
    FQT_WG(fqt_gemm_gfpk_ex(r.f, r.path, r.opts, m, n, K - kk, A + kk * k, lda, B + kk * ldb * k,
                            ldb, R, n, r.s));
    FQT_WG(wg_add(r, C, ldc, R, n, C, ldc, m, n, false));
  }
  if (m < M)  // the last row
    FQT_WG(fqt_gemm_gfpk_ex(r.f, r.path, r.opts, M - m, N, K, A + m * lda * k, lda, B, ldb,
                            C + m * ldc * k, ldc, r.s));
  if (n < N)  // the last column
    FQT_WG(fqt_gemm_gfpk_ex(r.f, r.path, r.opts, m, N - n, K, A, lda, B + n * k, ldb, C + n * k,
                            ldc, r.s));
#undef FQT_WG
  return ok();
}

fqt_status wg_workspace(fqt_field f, size_t bytes, uint8_t** out) {
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(f->mu);
  Workspace& w = f->wg_ws[dev];
  if (w.bytes < bytes) {
    if (w.ptr) {
      FQT_HIP(hipDeviceSynchronize());  // earlier calls may still use the old buffer
      FQT_HIP(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    if (hipMalloc(&w.ptr, bytes) != hipSuccess)
      return fail(FQT_ERR_OOM, "Winograd temporaries of %zu bytes", bytes);
    w.bytes = bytes;
  }
  *out = w.ptr;
  return ok();
}

}  // namespace

fqt_status fqt_gemm_winograd(fqt_field f, fqt_path path, const fqt_gemm_opts* opts,
                             uint32_t levels, int64_t M, int64_t N, int64_t K, const uint8_t* A,
                             int64_t lda, const uint8_t* B, int64_t ldb, uint8_t* C, int64_t ldc,
                             fqt_stream_t s) {
  fqt_status st = check_gemm_args(f, M, N, K, A, lda, B, ldb, C, ldc);
  if (st) return st;
  if (levels > 6) return fail(FQT_ERR_INVALID_ARG, "levels = %u above 6", levels);
  if (path != FQT_PATH_AUTO && path != FQT_PATH_PACKED_F64 && path != FQT_PATH_INT8 &&
      path != FQT_PATH_PLAIN)
    return fail(FQT_ERR_INVALID_ARG, "unknown path %d", (int)path);
  if (M == 0 || N == 0) return ok();
  uint8_t* ws = nullptr;
  const size_t bytes = wg_bytes(f->k, levels, M, N, K);
  if (bytes) {
    st = wg_workspace(f, bytes, &ws);
    if (st) return st;
  }
  const WgRun r{f, path, opts, (hipStream_t)s};
  return wg_rec(r, levels, M, N, K, A, lda, B, ldb, C, ldc, ws);
}

// Tile kWaveTile: wave tiles of 32 x 32 outputs, products dealt to 8 queues
// (one per XCD) longest first, the items of a queue in the order of their
// products; tables for q = 0 mod p (the epilogue reduces digit sums).
static fqt_status batched_wave(fqt_field f, const PackedChoice& pc, int64_t count,
                               const fqt_gemm_desc* descs, hipStream_t s) {
  const uint32_t k = f->k, p = f->p;
  for (int64_t d = 0; d < count; ++d) {
    const fqt_gemm_desc& e = descs[d];
    const uint64_t lim = 1ull << 30;  // buffer offsets stay below 2^31 with a far offset
    const uint64_t ea = e.M && e.K ? ((uint64_t)(e.M - 1) * e.lda + e.K) * k : 0;
    const uint64_t eb = e.K && e.N ? ((uint64_t)(e.K - 1) * e.ldb + e.N) * k : 0;
    // C: rows up to 31 past M are addressed (and their stores dropped)
    const uint64_t ec = ((uint64_t)e.M + 32) * (uint64_t)e.ldc * k;
    if (ea >= lim || eb >= lim || ec >= lim)
      return fail(FQT_ERR_UNSUPPORTED, "tile %d addresses operands below 2^30 bytes only "
                  "(descriptor %lld)", kWaveTile, (long long)d);
    if ((((uintptr_t)e.A) | ((uintptr_t)e.B) | ((uintptr_t)e.C)) & 3)
      return fail(FQT_ERR_UNSUPPORTED, "tile %d moves elements as words: A, B and C must be "
                  "4-byte aligned (descriptor %lld)", kWaveTile, (long long)d);
  }
  DevTables dt;
  fqt_status st = device_tables(f, p, &dt);  // q = 0 mod p: Q_d is the identity
  if (st) return st;
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  const fqt_detail::PlanKey key{descs, sizeof(fqt_gemm_desc) * count,
                                fqt_detail::key_tail(choice_words(pc), dev)};

  std::lock_guard<std::mutex> lk(f->mu);
  BatchPlan* plan = f->plans.find(key);
  if (!plan) {
    const int nqg = (int)(pc.nq / 4);
    const int64_t kb = 4 * nqg;
    hipDeviceProp_t prop;
    FQT_HIP(hipGetDeviceProperties(&prop, dev));
    int grid = prop.multiProcessorCount * wave_batched_occupancy(nqg, f->tbl_log2);
    grid = std::max(8, grid / 8 * 8);  // whole rounds over the 8 XCDs
    const int nwaves = grid * 4;
    // cost of a 32 x 32 tile: its K-blocks plus about one block's worth of epilogue
    auto tile_cost = [&](int64_t i) { return (descs[i].K + kb - 1) / kb + 1; };
    // products to XCDs: longest processing time first onto the lightest
    std::vector<int64_t> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = i;
    auto prod_cost = [&](int64_t i) {
      return ((descs[i].M + 31) / 32) * ((descs[i].N + 31) / 32) * tile_cost(i);
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return prod_cost(a) > prod_cost(b); });
    std::vector<std::vector<int64_t>> xcd(8);
    int64_t xload[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i : order) {
      int x = 0;
      for (int y = 1; y < 8; ++y)
        if (xload[y] < xload[x]) x = y;
      xcd[x].push_back(i);
      xload[x] += prod_cost(i);
    }
    // tiles of an XCD's products to its waves (wave w sits on XCD (w / 4) % 8),
    // longest first onto the lightest (a heap of wave loads)
    std::vector<std::vector<TileItem>> wl(nwaves);
    for (int x = 0; x < 8; ++x) {
      std::vector<int> ws;
      for (int w = 0; w < nwaves; ++w)
        if ((w / 4) % 8 == x) ws.push_back(w);
      using Slot = std::pair<int64_t, int>;  // (load, wave)
      std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
      for (int w : ws) heap.push({0, w});
      for (int64_t i : xcd[x]) {  // products already longest first
        const fqt_gemm_desc& d = descs[i];
        for (int a = 0; a < (int)((d.M + 31) / 32); ++a)
          for (int b = 0; b < (int)((d.N + 31) / 32); ++b) {
            Slot sl = heap.top();
            heap.pop();
            wl[sl.second].push_back(TileItem{(int32_t)i, a, b, 0});
            heap.push({sl.first + tile_cost(i), sl.second});
          }
      }
    }
    std::vector<GemmArgs> args(count);
    for (int64_t i = 0; i < count; ++i) {
      const fqt_gemm_desc& d = descs[i];
      args[i] = GemmArgs{d.A, d.B, d.C, d.M, d.N, d.K, d.lda, d.ldb, d.ldc};
    }
    std::vector<TileItem> items;
    std::vector<int32_t> wbeg(nwaves + 1);
    for (int w = 0; w < nwaves; ++w) {
      wbeg[w] = (int32_t)items.size();
      items.insert(items.end(), wl[w].begin(), wl[w].end());
    }
    wbeg[nwaves] = (int32_t)items.size();
    auto pl = std::make_unique<BatchPlan>();
    pl->n_items = (int32_t)items.size();
    pl->device = dev;
    pl->grid = grid;
    FQT_HIP(hipMalloc(&pl->d_descs, sizeof(GemmArgs) * std::max<int64_t>(count, 1)));
    FQT_HIP(hipMalloc(&pl->d_items, sizeof(TileItem) * std::max<size_t>(items.size(), 1)));
    FQT_HIP(hipMalloc(&pl->d_wbeg, sizeof(int32_t) * wbeg.size()));
    FQT_HIP(hipMemcpy(pl->d_descs, args.data(), sizeof(GemmArgs) * count, hipMemcpyHostToDevice));
    if (!items.empty())
      FQT_HIP(hipMemcpy(pl->d_items, items.data(), sizeof(TileItem) * items.size(),
                        hipMemcpyHostToDevice));
    FQT_HIP(hipMemcpy(pl->d_wbeg, wbeg.data(), sizeof(int32_t) * wbeg.size(),
                      hipMemcpyHostToDevice));
    const uint64_t q = 1ull << pc.b;
    PackedParams pp{};
    pp.b = pc.b;
    pp.nq_groups = (uint32_t)nqg;
    pp.tbl_log2 = f->tbl_log2;
    pp.aligned = 1;
    pp.fold_blocks = pc.fold;
    pp.qmask = (uint32_t)(q - 1);
    pp.qmod = 0;
    pp.blk_real = pc.nq_real;
    pp.fa = field_args(f, q);
    pp.L = dt.L;
    pp.H = dt.H;
    if (pc.centered) {
      centred_params(f, pc.b, &pp);  // the bias 2^52 + sum (q/2) q^i; f->mu is held
      // every digit of every block carries q/2: take off n_blocks (q/2) (L + H)(1..1)
      // with the q = 0 tables
      const auto& ht = host_tables(f, p);
      const uint32_t beta = (uint32_t)((q / 2) % p);
      uint32_t il = 0;
      for (uint32_t dd = 0; dd < k; ++dd) il |= beta << (f->cb * dd);
      const uint32_t lw = ht.first[il], hw = ht.second[il];
      uint32_t neg = 0;
      for (uint32_t i = 0; i < k; ++i) {
        const uint32_t cc = (((lw >> (8 * i)) & 0xffu) + ((hw >> (8 * i)) & 0xffu)) % p;
        neg |= ((p - cc) % p) << (8 * i);
      }
      pp.c0neg = neg;
      pp.dshift = beta;
    }
    dqt_params(f, pc.b, pc.centered, &pp);
    if (!(pp.dqt_flags & kDqtLut)) {  // the kernel always permutes: identity bytes
      pp.lut_lo = 0x03020100u;
      pp.lut_hi = 0x07060504u;
      pp.dqt_off = 0;
    }
    hipStream_t cs = nullptr;
    FQT_HIP(capture_stream(f, dev, &cs));
    FQT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    if (pl->n_items > 0)
      le = launch_gemm_wave_batched(nqg, pl->d_descs, pl->d_items, pl->d_wbeg, pl->grid, pp,
                                    cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (le != hipSuccess) return hip_fail(le, "wave batched launch (capture)");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    FQT_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0));
    plan = f->plans.insert(key, std::move(pl));
  }
  if (plan->n_items == 0) return ok();
  FQT_HIP(hipGraphLaunch(plan->exec, s));
  return ok();
}

static fqt_status batched_packed(fqt_field f, const fqt_gemm_opts* opts, int64_t count,
                                 const fqt_gemm_desc* descs, hipStream_t s) {
  int64_t Kmax = 0, Mmax = 0, Nmax = 0;
  for (int64_t i = 0; i < count; ++i) {
    Kmax = std::max(Kmax, descs[i].K);
    Mmax = std::max(Mmax, descs[i].M);
    Nmax = std::max(Nmax, descs[i].N);
  }
  PackedChoice pc;
  std::memset(&pc, 0, sizeof pc);  // the plan key copies its bytes
  fqt_gemm_opts o = opts ? *opts : fqt_gemm_opts{0, 0, 0, 0, 0};
  if (!o.tile) o.tile = 2;
  fqt_status st = resolve_packed(f, &o, Kmax, Mmax, Nmax, &pc);
  if (st) return st;
  if (pc.tile == (uint32_t)kWaveTile) return batched_wave(f, pc, count, descs, s);
  if (direct_tile_buffered((int)pc.tile))
    for (int64_t d = 0; d < count; ++d) {
      const fqt_gemm_desc& e = descs[d];
      const GemmArgs ga{e.A, e.B, e.C, e.M, e.N, e.K, e.lda, e.ldb, e.ldc};
      if (!extents_fit_32(ga, f->k))
        return fail(FQT_ERR_UNSUPPORTED, "tile %u addresses operands below 2^31 bytes only "
                    "(descriptor %lld)", pc.tile, (long long)d);
    }
  const uint64_t q = 1ull << pc.b;
  const bool split = is_split_tile((int)pc.tile);
  DevTables dt;
  st = device_tables(f, split ? f->p : q, &dt);
  if (st) return st;
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));

  // Plan key: the descriptor bytes, the resolved parameters and the device.
  const fqt_detail::PlanKey key{descs, sizeof(fqt_gemm_desc) * count,
                                fqt_detail::key_tail(choice_words(pc), dev)};

  std::lock_guard<std::mutex> lk(f->mu);
  BatchPlan* plan = f->plans.find(key);
  if (!plan) {
    int bm, bn;
    packed_tile_shape((int)pc.tile, &bm, &bn);
    std::vector<GemmArgs> args(count);
    std::vector<TileItem> items;
    bool aligned = true;
    for (int64_t i = 0; i < count; ++i) {
      const fqt_gemm_desc& d = descs[i];
      args[i] = GemmArgs{d.A, d.B, d.C, d.M, d.N, d.K, d.lda, d.ldb, d.ldc};
      aligned = aligned && ((((uintptr_t)d.A) | ((uintptr_t)d.B)) & 3) == 0 &&
                (d.lda * f->k) % 4 == 0 && (d.ldb * f->k) % 4 == 0;
      const int tm = (int)((d.M + bm - 1) / bm), tn = (int)((d.N + bn - 1) / bn);
      for (int a = 0; a < tm; ++a)
        for (int c = 0; c < tn; ++c) items.push_back(TileItem{(int32_t)i, a, c, 0});
    }
    // Longest-processing-time first: a tile costs about K (same tile area).
    std::stable_sort(items.begin(), items.end(), [&](const TileItem& x, const TileItem& y) {
      return descs[x.gemm].K > descs[y.gemm].K;
    });
    auto pl = std::make_unique<BatchPlan>();
    pl->n_items = (int32_t)items.size();
    pl->device = dev;
    FQT_HIP(hipMalloc(&pl->d_descs, sizeof(GemmArgs) * std::max<int64_t>(count, 1)));
    FQT_HIP(hipMalloc(&pl->d_items, sizeof(TileItem) * std::max<size_t>(items.size(), 1)));
    FQT_HIP(hipMalloc(&pl->d_counter, 2 * sizeof(uint32_t)));
    FQT_HIP(hipMemcpy(pl->d_descs, args.data(), sizeof(GemmArgs) * count, hipMemcpyHostToDevice));
    if (!items.empty())
      FQT_HIP(hipMemcpy(pl->d_items, items.data(), sizeof(TileItem) * items.size(),
                        hipMemcpyHostToDevice));
    FQT_HIP(hipMemset(pl->d_counter, 0, 2 * sizeof(uint32_t)));
    hipDeviceProp_t prop;
    FQT_HIP(hipGetDeviceProperties(&prop, dev));
    const bool direct = is_direct_tile((int)pc.tile);
    const int occ =
        split ? split_batched_occupancy((int)f->k, (int)pc.tile, f->tbl_log2)
        : direct ? direct_batched_occupancy((int)f->k, (int)pc.tile, pc.mode, f->tbl_log2)
                 : packed_batched_occupancy((int)f->k, (int)pc.tile, pc.mode, f->tbl_log2);
    pl->grid = std::max(1, std::min<int>(prop.multiProcessorCount * occ, pl->n_items));
    PackedParams pp{};
    pp.b = pc.b;
    pp.nq_groups = pc.nq / 4;
    pp.tbl_log2 = f->tbl_log2;
    pp.aligned = aligned;
    pp.fold_blocks = pc.fold;
    pp.qmask = (uint32_t)(q - 1);
    pp.qmod = (uint32_t)(q % f->p);
    pp.blk_real = pc.nq_real;
    pp.fa = field_args(f, q);
    pp.L = dt.L;
    pp.H = dt.H;
    if (pc.centered) centred_params(f, pc.b, &pp);  // f->mu is held
    dqt_params(f, pc.b, pc.centered, &pp);
    // Capture the persistent launch once; later calls replay the graph.
    hipStream_t cs = nullptr;
    FQT_HIP(capture_stream(f, dev, &cs));
    FQT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le =
        split    ? launch_gemm_split_batched((int)f->k, (int)pc.tile, pl->d_descs, pl->d_items,
                                             pl->n_items, pl->d_counter, pl->grid, pp,
                                             cs)
        : direct ? launch_gemm_direct_batched((int)f->k, (int)pc.tile, pc.mode, pl->d_descs,
                                              pl->d_items, pl->n_items, pl->d_counter, pl->grid,
                                              pp, cs)
                 : launch_gemm_packed_batched((int)f->k, (int)pc.tile, pc.mode, pl->d_descs,
                                              pl->d_items, pl->n_items, pl->d_counter, pl->grid,
                                              pp, cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (le != hipSuccess) return hip_fail(le, "batched launch (capture)");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    FQT_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0));
    plan = f->plans.insert(key, std::move(pl));
  }
  if (plan->n_items == 0) return ok();
  FQT_HIP(hipGraphLaunch(plan->exec, s));
  return ok();
}

// INT8 tile 11: strips of 16 output elements dealt to workgroups (products
// to XCDs longest first, then strips to the XCD's workgroups the same way).
static fqt_status batched_i8cs(fqt_field f, int64_t count, const fqt_gemm_desc* descs,
                               hipStream_t s) {
  const uint32_t k = f->k, p = f->p;
  if (k != 4)
    return fail(FQT_ERR_UNSUPPORTED, "INT8 tile %u runs fields of k = 4 (k = %u)",
                kInt8StripTile, k);
  int64_t Kmax = 0;
  for (int64_t d = 0; d < count; ++d) {
    const fqt_gemm_desc& e = descs[d];
    const uint64_t lim = 1ull << 30;
    const uint64_t ea = e.M && e.K ? ((uint64_t)(e.M - 1) * e.lda + e.K) * k : 0;
    const uint64_t eb = e.K && e.N ? ((uint64_t)(e.K - 1) * e.ldb + e.N) * k : 0;
    if (ea >= lim || eb >= lim || (uint64_t)e.lda * k * 256 >= lim ||
        (uint64_t)e.ldb * k * 256 >= lim)
      return fail(FQT_ERR_UNSUPPORTED, "INT8 tile %u addresses operands below 2^30 bytes and "
                  "rows below 2^22 bytes only (descriptor %lld)", kInt8StripTile, (long long)d);
    if ((((uintptr_t)e.A) | ((uintptr_t)e.B)) & 3)
      return fail(FQT_ERR_UNSUPPORTED, "INT8 tile %u reads operands as words: A and B must be "
                  "4-byte aligned (descriptor %lld)", kInt8StripTile, (long long)d);
    Kmax = std::max(Kmax, e.K);
  }
  uint8_t* mt = nullptr;  // before taking the field lock (device_mt takes it)
  fqt_status mst = device_mt(f, &mt);
  if (mst) return mst;
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  const int tag[2] = {-(int)kInt8StripTile, dev};
  const fqt_detail::PlanKey key{descs, sizeof(fqt_gemm_desc) * count, fqt_detail::key_tail(tag)};
  std::lock_guard<std::mutex> lk(f->mu);
  BatchPlan* plan = f->plans.find(key);
  if (!plan) {
    hipDeviceProp_t prop;
    FQT_HIP(hipGetDeviceProperties(&prop, dev));
    int grid = prop.multiProcessorCount * i8cs_occupancy(f->tbl_log2);
    grid = std::max(8, grid / 8 * 8);
    // cost of a strip: chunks of 32 rows per wave (4 waves) times K-tiles of 64
    auto strip_cost = [&](int64_t i) {
      const fqt_gemm_desc& d = descs[i];
      return ((d.M + 127) / 128) * ((d.K + 63) / 64 + 1);
    };
    auto prod_cost = [&](int64_t i) { return ((descs[i].N + 15) / 16) * strip_cost(i); };
    std::vector<int64_t> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return prod_cost(a) > prod_cost(b); });
    std::vector<std::vector<int64_t>> xcd(8);
    int64_t xload[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i : order) {
      int x = 0;
      for (int y = 1; y < 8; ++y)
        if (xload[y] < xload[x]) x = y;
      xcd[x].push_back(i);
      xload[x] += prod_cost(i);
    }
    std::vector<std::vector<int32_t>> wl(grid);  // (product, strip) pairs per workgroup
    for (int x = 0; x < 8; ++x) {
      using Slot = std::pair<int64_t, int>;
      std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
      for (int w = x; w < grid; w += 8) heap.push({0, w});
      for (int64_t i : xcd[x])
        for (int nc = 0; nc < (int)((descs[i].N + 15) / 16); ++nc) {
          Slot sl = heap.top();
          heap.pop();
          wl[sl.second].insert(wl[sl.second].end(), {(int32_t)i, nc, 0, 0});
          heap.push({sl.first + strip_cost(i), sl.second});
        }
    }
    std::vector<int32_t> items, wbeg(grid + 1);
    for (int w = 0; w < grid; ++w) {
      wbeg[w] = (int32_t)(items.size() / 4);
      items.insert(items.end(), wl[w].begin(), wl[w].end());
    }
    wbeg[grid] = (int32_t)(items.size() / 4);
    std::vector<GemmArgs> args(count);
    for (int64_t i = 0; i < count; ++i) {
      const fqt_gemm_desc& d = descs[i];
      args[i] = GemmArgs{d.A, d.B, d.C, d.M, d.N, d.K, d.lda, d.ldb, d.ldc};
    }
    auto pl = std::make_unique<BatchPlan>();
    pl->device = dev;
    pl->n_items = (int32_t)(items.size() / 4);
    pl->grid = grid;
    FQT_HIP(hipMalloc(&pl->d_descs, sizeof(GemmArgs) * std::max<int64_t>(count, 1)));
    FQT_HIP(hipMalloc(&pl->d_items, sizeof(int32_t) * std::max<size_t>(items.size(), 4)));
    FQT_HIP(hipMalloc(&pl->d_wbeg, sizeof(int32_t) * wbeg.size()));
    FQT_HIP(hipMemcpy(pl->d_descs, args.data(), sizeof(GemmArgs) * count, hipMemcpyHostToDevice));
    if (!items.empty())
      FQT_HIP(hipMemcpy(pl->d_items, items.data(), sizeof(int32_t) * items.size(),
                        hipMemcpyHostToDevice));
    FQT_HIP(hipMemcpy(pl->d_wbeg, wbeg.data(), sizeof(int32_t) * wbeg.size(),
                      hipMemcpyHostToDevice));
    // INT32 sums grow by at most 64 k (p-1)^2 per K-tile of 64 elements
    const uint64_t per_tile = 64ull * k * (p - 1) * (p - 1);
    const uint64_t cap = per_tile ? (0x7fffffffull - (p - 1)) / per_tile : 0;
    const uint64_t ktiles = ((uint64_t)Kmax + 63) / 64;
    const uint32_t red = (per_tile && ktiles > cap) ? (uint32_t)std::max<uint64_t>(cap - 1, 1) : 0;
    const uint64_t top = red ? (uint64_t)red * per_tile + p : (uint64_t)ktiles * per_tile;
    const uint32_t small = top < (1ull << 25) ? 1u : 0u;
    hipStream_t cs = nullptr;
    FQT_HIP(capture_stream(f, dev, &cs));
    FQT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    if (pl->n_items > 0)
      le = launch_gemm_i8cs_batched(pl->d_descs, reinterpret_cast<const int32_t*>(pl->d_items),
                                    pl->d_wbeg, pl->grid, mt, f->tbl_log2, p, f->cb, red, small,
                                    cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (le != hipSuccess) return hip_fail(le, "INT8 strip batched launch (capture)");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    FQT_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0));
    plan = f->plans.insert(key, std::move(pl));
  }
  if (plan->n_items == 0) return ok();
  FQT_HIP(hipGraphLaunch(plan->exec, s));
  return ok();
}

static fqt_status batched_int8(fqt_field f, const fqt_gemm_opts* opts, int64_t count,
                               const fqt_gemm_desc* descs, hipStream_t s) {
  const int64_t k = f->k, p = f->p;
  uint32_t tile = (opts && opts->tile) ? opts->tile : 8;  // measured best on uneven batches
  if (tile > (uint32_t)kInt8Tiles) return fail(FQT_ERR_INVALID_ARG, "unknown INT8 tile id %u", tile);
  if (tile == kInt8StripTile) return batched_i8cs(f, count, descs, s);
  int dev = 0;
  FQT_HIP(hipGetDevice(&dev));
  const int tag[2] = {-(int)tile, dev};  // negative: INT8 plans never match packed ones
  const fqt_detail::PlanKey key{descs, sizeof(fqt_gemm_desc) * count, fqt_detail::key_tail(tag)};

  uint8_t* mt = nullptr;  // before taking the field lock (device_mt takes it)
  fqt_status mst = device_mt(f, &mt);
  if (mst) return mst;
  const bool fused = i8_fused_tile(tile);
  if (fused && !i8f_fits(f, tile))
    return fail(FQT_ERR_UNSUPPORTED, "INT8 tile %u: operand tiles and the %u-bit table exceed "
                "the LDS", tile, f->tbl_log2);
  std::lock_guard<std::mutex> lk(f->mu);
  BatchPlan* plan = f->plans.find(key);
  if (!plan && fused) {
    // one persistent kernel over every product's tiles, no B' workspace
    const int bm = i8f_tile_m((int)tile), bne = i8f_tile_n((int)tile, (int)k);
    std::vector<I8Batch> gs(count);
    std::vector<TileItem> items;
    for (int64_t i = 0; i < count; ++i) {
      const fqt_gemm_desc& d = descs[i];
      I8Batch& b = gs[i];
      b.a = i8_args(f, d.A, d.lda, d.C, d.ldc, d.M, d.N, d.K, i8f_k_bytes((int)k));
      b.B = d.B;
      b.ldb = d.ldb;
      b.K = d.K;
      b.N = d.N;
      const int tm = (int)((d.M + bm - 1) / bm), tn = (int)((d.N + bne - 1) / bne);
      for (int a = 0; a < tm; ++a)
        for (int c = 0; c < tn; ++c) items.push_back(TileItem{(int32_t)i, a, c, 0});
    }
    std::stable_sort(items.begin(), items.end(), [&](const TileItem& x, const TileItem& y) {
      return descs[x.gemm].K > descs[y.gemm].K;
    });
    auto pl = std::make_unique<BatchPlan>();
    pl->device = dev;
    pl->n_items = (int32_t)items.size();
    FQT_HIP(hipMalloc(&pl->d_i8, sizeof(I8Batch) * count));
    FQT_HIP(hipMalloc(&pl->d_items, sizeof(TileItem) * std::max<size_t>(items.size(), 1)));
    FQT_HIP(hipMalloc(&pl->d_counter, 2 * sizeof(uint32_t)));
    FQT_HIP(hipMemcpy(pl->d_i8, gs.data(), sizeof(I8Batch) * count, hipMemcpyHostToDevice));
    if (!items.empty())
      FQT_HIP(hipMemcpy(pl->d_items, items.data(), sizeof(TileItem) * items.size(),
                        hipMemcpyHostToDevice));
    FQT_HIP(hipMemset(pl->d_counter, 0, 2 * sizeof(uint32_t)));
    hipDeviceProp_t prop;
    FQT_HIP(hipGetDeviceProperties(&prop, dev));
    pl->grid = std::max(
        1, std::min<int>(prop.multiProcessorCount *
                             i8f_batched_occupancy((int)tile, (int)k, f->tbl_log2),
                         std::max<int32_t>(pl->n_items, 1)));
    hipStream_t cs = nullptr;
    FQT_HIP(capture_stream(f, dev, &cs));
    FQT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    if (pl->n_items > 0)
      le = launch_gemm_i8f_batched((int)tile, (int)k, pl->d_i8, pl->d_items, pl->n_items,
                                   pl->d_counter, pl->grid, mt, f->cb, f->tbl_log2,
                                   cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (le != hipSuccess) return hip_fail(le, "fused INT8 batched launch (capture)");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    FQT_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0));
    plan = f->plans.insert(key, std::move(pl));
  }
  if (!plan) {
    const int bm = i8_tile_m((int)tile), bn = i8_tile_n((int)tile);
    std::vector<I8Batch> gs(count);
    std::vector<ExpandItem> exps;
    std::vector<TileItem> items;
    size_t ws_total = 0;
    std::vector<size_t> ws_off(count);
    for (int64_t i = 0; i < count; ++i) {
      const fqt_gemm_desc& d = descs[i];
      const int64_t KKpad = (d.K * k + 127) / 128 * 128;
      ws_off[i] = ws_total;
      ws_total += ((size_t)(d.N * k) * (size_t)KKpad + 255) / 256 * 256;
    }
    // B' of every product, in one buffer per device that all such plans share
    // (a plan's graph expands its own B' first); growing it destroys the
    // plans captured with the old buffer, which are rebuilt on their next call
    Workspace& bw = f->bws[dev];
    if (bw.bytes < ws_total) {
      f->plans.erase_if([&](const BatchPlan& q) { return q.shares_ws && q.device == dev; });
      if (bw.ptr) {
        FQT_HIP(hipDeviceSynchronize());
        FQT_HIP(hipFree(bw.ptr));
        bw.ptr = nullptr;
        bw.bytes = 0;
      }
      const size_t want = std::max<size_t>(ws_total, 256);
      if (hipMalloc(&bw.ptr, want) != hipSuccess)
        return fail(FQT_ERR_OOM, "INT8 batch workspace of %zu bytes", want);
      bw.bytes = want;
    }
    auto pl = std::make_unique<BatchPlan>();
    pl->device = dev;
    pl->shares_ws = true;
    for (int64_t i = 0; i < count; ++i) {
      const fqt_gemm_desc& d = descs[i];
      const int64_t KKpad = (d.K * k + 127) / 128 * 128;
      I8Batch& b = gs[i];
      b.a.A = d.A;
      b.a.lda = d.lda * k;
      b.a.Bt = bw.ptr + ws_off[i];
      b.a.ldbt = KKpad;
      b.a.C = d.C;
      b.a.ldc = d.ldc * k;
      b.a.M = d.M;
      b.a.NN = d.N * k;
      b.a.KK = d.K * k;
      b.a.KKpad = KKpad;
      b.a.p = (uint32_t)p;
      b.a.red_tiles = i8_red_tiles(d.K * k, p, i8_tile_k((int)tile));
      b.a.a_vec = row_align(d.A, d.lda * k);
      b.a.inv_p = 1.0 / (double)p;
      b.B = d.B;
      b.ldb = d.ldb;
      b.K = d.K;
      b.N = d.N;
      // kExpandL x kExpandN-element expansion blocks covering the padded row
      const int64_t lcols = (KKpad + k - 1) / k;
      if (d.K && d.N)
        for (int32_t lb = 0; lb < (int32_t)((lcols + kExpandL - 1) / kExpandL); ++lb)
          for (int32_t nb = 0; nb < (int32_t)((d.N + kExpandN - 1) / kExpandN); ++nb)
            exps.push_back(ExpandItem{(int32_t)i, lb, nb, 0});
      const int tm = (int)((d.M + bm - 1) / bm), tn = (int)((d.N * k + bn - 1) / bn);
      for (int a = 0; a < tm; ++a)
        for (int c = 0; c < tn; ++c) items.push_back(TileItem{(int32_t)i, a, c, 0});
    }
    std::stable_sort(items.begin(), items.end(), [&](const TileItem& x, const TileItem& y) {
      return descs[x.gemm].K > descs[y.gemm].K;
    });
    pl->n_items = (int32_t)items.size();
    FQT_HIP(hipMalloc(&pl->d_i8, sizeof(I8Batch) * count));
    FQT_HIP(hipMalloc(&pl->d_exp, sizeof(ExpandItem) * std::max<size_t>(exps.size(), 1)));
    FQT_HIP(hipMalloc(&pl->d_items, sizeof(TileItem) * std::max<size_t>(items.size(), 1)));
    FQT_HIP(hipMalloc(&pl->d_counter, 2 * sizeof(uint32_t)));
    FQT_HIP(hipMemcpy(pl->d_i8, gs.data(), sizeof(I8Batch) * count, hipMemcpyHostToDevice));
    if (!exps.empty())
      FQT_HIP(hipMemcpy(pl->d_exp, exps.data(), sizeof(ExpandItem) * exps.size(),
                        hipMemcpyHostToDevice));
    if (!items.empty())
      FQT_HIP(hipMemcpy(pl->d_items, items.data(), sizeof(TileItem) * items.size(),
                        hipMemcpyHostToDevice));
    FQT_HIP(hipMemset(pl->d_counter, 0, 2 * sizeof(uint32_t)));
    hipDeviceProp_t prop;
    FQT_HIP(hipGetDeviceProperties(&prop, dev));
    pl->grid = std::max(1, std::min<int>(prop.multiProcessorCount * i8_batched_occupancy((int)tile),
                                         std::max<int32_t>(pl->n_items, 1)));
    hipStream_t cs = nullptr;
    FQT_HIP(capture_stream(f, dev, &cs));
    FQT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_expand_b_batched((int)k, pl->d_i8, pl->d_exp, (int32_t)exps.size(),
                                            mt, f->cb, f->tbl_log2, cs);
    if (le == hipSuccess && pl->n_items > 0)
      le = launch_gemm_i8_batched((int)tile, pl->d_i8, pl->d_items, pl->n_items, pl->d_counter,
                                  pl->grid, cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (le != hipSuccess) return hip_fail(le, "INT8 batched launch (capture)");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    FQT_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0));
    plan = f->plans.insert(key, std::move(pl));
  }
  if (fused && plan->n_items == 0) return ok();  // nothing captured
  FQT_HIP(hipGraphLaunch(plan->exec, s));
  return ok();
}

fqt_status fqt_gemm_gfpk_batched_ex(fqt_field f, fqt_path path, const fqt_gemm_opts* opts,
                                    int64_t count, const fqt_gemm_desc* descs, fqt_stream_t s) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (count < 0 || (count && !descs)) return fail(FQT_ERR_INVALID_ARG, "bad descriptor array");
  for (int64_t i = 0; i < count; ++i) {
    const fqt_gemm_desc& d = descs[i];
    fqt_status st = check_gemm_args(f, d.M, d.N, d.K, d.A, d.lda, d.B, d.ldb, d.C, d.ldc);
    if (st) return fail(st, "descriptor %lld: %s", (long long)i, g_last_error.c_str());
  }
  if (count == 0) return ok();
  fqt_gemm_opts tuned{};
  bool from_tuned = false;
  if (path == FQT_PATH_AUTO) {
    int64_t Mmax = 0, Nmax = 0, Kmax = 0;
    for (int64_t i = 0; i < count; ++i) {
      Mmax = std::max(Mmax, descs[i].M);
      Nmax = std::max(Nmax, descs[i].N);
      Kmax = std::max(Kmax, descs[i].K);
    }
    std::lock_guard<std::mutex> lk(f->mu);
    auto it = f->tuned.find(shape_key(f, count, Mmax, Nmax, Kmax));
    path = FQT_PATH_PACKED_F64;
    if (it != f->tuned.end()) {
      path = it->second.path;
      if (!opts) {
        tuned = it->second.opts;
        opts = &tuned;
        from_tuned = true;
      }
    }
  }
  if (!opts && (path == FQT_PATH_PACKED_F64 || path == FQT_PATH_INT8)) {
    int64_t Mmax = 0, Nmax = 0, Kmax = 0;
    for (int64_t i = 0; i < count; ++i) {
      Mmax = std::max(Mmax, descs[i].M);
      Nmax = std::max(Nmax, descs[i].N);
      Kmax = std::max(Kmax, descs[i].K);
    }
    std::lock_guard<std::mutex> lk(f->mu);
    auto it = f->tuned.find(shape_key(f, count, Mmax, Nmax, Kmax) +
                            (path == FQT_PATH_INT8 ? "_int8" : "_packed"));
    if (it != f->tuned.end()) {
      tuned = it->second.opts;
      opts = &tuned;
      from_tuned = true;
    }
  }
  auto run = [&](const fqt_gemm_opts* o) -> fqt_status {
    switch (path) {
      case FQT_PATH_PACKED_F64:
        return batched_packed(f, o, count, descs, (hipStream_t)s);
      case FQT_PATH_PLAIN: {
        const FieldArgs fa = field_args(f, 2);
        for (int64_t i = 0; i < count; ++i) {
          const fqt_gemm_desc& d = descs[i];
          GemmArgs g{d.A, d.B, d.C, d.M, d.N, d.K, d.lda, d.ldb, d.ldc};
          FQT_HIP(launch_gemm_plain((int)f->k, g, fa, f->P_low, (hipStream_t)s));
        }
        return ok();
      }
      case FQT_PATH_INT8:
        return batched_int8(f, o, count, descs, (hipStream_t)s);
      default:
        return fail(FQT_ERR_INVALID_ARG, "unknown path %d", (int)path);
    }
  };
  // tuned options of the shape class may be refused at this batch's K (see
  // fqt_gemm_gfpk_ex): then the path's defaults
  fqt_status rst = run(opts);
  if (from_tuned && (rst == FQT_ERR_UNSUPPORTED || rst == FQT_ERR_BOUNDS)) rst = run(nullptr);
  return rst;
}

fqt_status fqt_gemm_gfpk_batched(fqt_field f, fqt_path path, int64_t count,
                                 const fqt_gemm_desc* descs, fqt_stream_t s) {
  return fqt_gemm_gfpk_batched_ex(f, path, nullptr, count, descs, s);
}

// ---- autotuner ---------------------------------------------------------------

namespace {

struct Candidate {
  fqt_path path;
  fqt_gemm_opts opts;
};

// Pinned host buffer (hipHostMalloc) that frees itself.
struct PinnedBuf {
  uint8_t* p = nullptr;
  size_t n = 0;
  ~PinnedBuf() {
    if (p) hipHostFree(p);
  }
  fqt_status resize(size_t bytes) {
    if (bytes <= n) return ok();
    if (p) hipHostFree(p);
    p = nullptr;
    n = 0;
    if (hipHostMalloc((void**)&p, std::max<size_t>(bytes, 1), hipHostMallocDefault) != hipSuccess)
      return fail(FQT_ERR_OOM, "pinned host buffer of %zu bytes", bytes);
    n = bytes;
    return ok();
  }
};

// Host copy of every C of the batch (rows of N*k bytes) into pinned memory.
fqt_status snapshot(const fqt_field_s* f, int64_t count, const fqt_gemm_desc* d,
                    hipStream_t s, PinnedBuf* out, size_t* total_out) {
  size_t total = 0;
  for (int64_t i = 0; i < count; ++i) total += (size_t)(d[i].M * d[i].N) * f->k;
  fqt_status st = out->resize(total);
  if (st) return st;
  *total_out = total;
  std::memset(out->p, 0, total);
  // Copies are ordered after the candidate's kernels on the same stream, then
  // the stream is drained: no reliance on null-stream ordering.
  size_t off = 0;
  for (int64_t i = 0; i < count; ++i) {
    const size_t row = (size_t)d[i].N * f->k;
    if (d[i].M && row) {
      FQT_HIP(hipMemcpy2DAsync(out->p + off, row, d[i].C, (size_t)d[i].ldc * f->k, row,
                               (size_t)d[i].M, hipMemcpyDeviceToHost, s));
    }
    off += row * (size_t)d[i].M;
  }
  FQT_HIP(hipStreamSynchronize(s));
  return ok();
}

bool read_cache(const char* path, const std::string& key, TuneEntry* e) {
  if (!path) return false;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, fp)) {
    char k[256];
    int pth = 0;
    unsigned lq = 0, nq = 0, tile = 0, bnd = 0, cen = 0;
    if (std::sscanf(line, "{\"key\": \"%255[^\"]\", \"path\": %d, \"log2q\": %u, \"n_q\": %u, \"tile\": %u, \"boundary\": %u, \"centered\": %u",
                    k, &pth, &lq, &nq, &tile, &bnd, &cen) == 7 &&
        key == k) {
      e->path = (fqt_path)pth;
      e->opts = fqt_gemm_opts{lq, nq, tile, bnd, cen};
      found = true;  // the last matching line wins
    }
  }
  std::fclose(fp);
  return found;
}

}  // namespace

fqt_status fqt_autotune(fqt_field f, fqt_path only, int64_t count, const fqt_gemm_desc* descs,
                        const char* cache_path, fqt_path* best_path, fqt_gemm_opts* best,
                        fqt_stream_t s) {
  if (!f) return fail(FQT_ERR_INVALID_ARG, "null field");
  if (only != FQT_PATH_AUTO && only != FQT_PATH_PACKED_F64 && only != FQT_PATH_INT8)
    return fail(FQT_ERR_INVALID_ARG, "autotune covers the packed and INT8 paths");
  if (count < 1 || !descs) return fail(FQT_ERR_INVALID_ARG, "empty problem");
  int64_t Mmax = 0, Nmax = 0, Kmax = 0;
  for (int64_t i = 0; i < count; ++i) {
    const fqt_gemm_desc& d = descs[i];
    fqt_status st = check_gemm_args(f, d.M, d.N, d.K, d.A, d.lda, d.B, d.ldb, d.C, d.ldc);
    if (st) return fail(st, "descriptor %lld: %s", (long long)i, g_last_error.c_str());
    Mmax = std::max(Mmax, d.M);
    Nmax = std::max(Nmax, d.N);
    Kmax = std::max(Kmax, d.K);
  }
  const std::string key = shape_key(f, count, Mmax, Nmax, Kmax) +
                          (only == FQT_PATH_AUTO ? "" : only == FQT_PATH_INT8 ? "_int8" : "_packed");
  const std::string auto_key = shape_key(f, count, Mmax, Nmax, Kmax);
  TuneEntry cached;
  if (read_cache(cache_path, key, &cached)) {
    std::lock_guard<std::mutex> lk(f->mu);
    f->tuned[key] = cached;
    if (!f->tuned.count(auto_key)) f->tuned[auto_key] = cached;
    if (best_path) *best_path = cached.path;
    if (best) *best = cached.opts;
    return ok();
  }

  // Candidates: every packed tile at the largest q and one q below (fewer
  // products per K-block), and every INT8 tile for single products.
  std::vector<Candidate> cands;
  const uint32_t bmax = max_pow2_b(f->k);
  for (uint32_t cen : {0u, 1u})
  for (uint32_t b : {bmax, bmax - 1}) {
    if (only == FQT_PATH_INT8) break;
    if (b < 1 || (cen && f->p == 2)) continue;
    const uint64_t h = (f->p - 1) / 2;
    const uint64_t unit_nq = cen ? (uint64_t)f->k * h * h : (uint64_t)f->k * (f->p - 1) * (f->p - 1);
    const uint64_t room = cen ? (1ull << (b - 1)) - 1 : (1ull << b) - 1;
    const uint32_t nq_top = unit_nq ? (uint32_t)std::min<uint64_t>(room / unit_nq, 1u << 30) : 0;
    for (uint32_t t = 1; t <= (uint32_t)kPackedTiles; ++t)
      for (uint32_t bm : {1u, 2u})
      for (uint32_t nqc : {0u, nq_top & ~3u}) {
        if (nqc && nqc == nq_top) continue;  // same as the default
        if (is_split_tile((int)t)) continue;  // below, with their own q
        if (cen && t > (uint32_t)kStagedTiles && t != (uint32_t)kWaveTile) continue;
        fqt_gemm_opts o{b, nqc, t, bm, cen};
        PackedChoice pc;
        if (resolve_packed(f, &o, Kmax, Mmax, Nmax, &pc) != FQT_OK) continue;
        if (t == 4 && f->k >= 3 && pc.mode == 1) continue;  // that variant spills registers
        if (!pc.multi && bm == 2) continue;              // one block: no boundary step
        if (cen && !pc.multi) continue;                  // one block: nothing to gain
        cands.push_back({FQT_PATH_PACKED_F64, o});
      }
  }
  // d-split tiles bring their own q (one block, no boundary step)
  if (only != FQT_PATH_INT8)
    for (uint32_t t = (uint32_t)kFirstSplitTile; t <= (uint32_t)kLastSplitTile; ++t) {
      fqt_gemm_opts o{0, 0, t, 0, 0};
      PackedChoice pc;
      if (resolve_packed(f, &o, Kmax, Mmax, Nmax, &pc) == FQT_OK)
        cands.push_back({FQT_PATH_PACKED_F64, o});
    }
  if (only != FQT_PATH_PACKED_F64)
    for (uint32_t t = 1; t <= (uint32_t)kInt8Tiles; ++t)
      if (!i8_fused_tile(t) || i8f_fits(f, t))
        cands.push_back({FQT_PATH_INT8, fqt_gemm_opts{0, 0, t, 0, 0}});
  if (cands.empty()) return fail(FQT_ERR_UNSUPPORTED, "no admissible candidate");

  hipStream_t st = (hipStream_t)s;
  auto run = [&](const Candidate& c) -> fqt_status {
    if (count == 1) {
      const fqt_gemm_desc& d = descs[0];
      return fqt_gemm_gfpk_ex(f, c.path, &c.opts, d.M, d.N, d.K, d.A, d.lda, d.B, d.ldb, d.C,
                              d.ldc, s);
    }
    return fqt_gemm_gfpk_batched_ex(f, c.path, &c.opts, count, descs, s);
  };

  hipEvent_t e0, e1;
  FQT_HIP(hipEventCreate(&e0));
  FQT_HIP(hipEventCreate(&e1));
  PinnedBuf ref, cur;
  size_t ref_n = 0, cur_n = 0;
  double best_ms = 1e30;
  size_t best_i = 0;
  std::vector<double> times(cands.size(), 0.0);
  fqt_status status = FQT_OK;
  bool have_ref = false;
  size_t ref_i = 0;
  for (size_t i = 0; i < cands.size() && status == FQT_OK; ++i) {
    status = run(cands[i]);  // warm-up: builds plans and graphs
    if (status == FQT_ERR_UNSUPPORTED) {  // refused on the host for this problem: skip it
      status = FQT_OK;
      times[i] = -1.0;
      continue;
    }
    if (status) break;
    status = !have_ref ? snapshot(f, count, descs, st, &ref, &ref_n)
                       : snapshot(f, count, descs, st, &cur, &cur_n);
    if (status) break;
    if (!have_ref) {
      have_ref = true;
      ref_i = i;
    } else if (std::memcmp(cur.p, ref.p, ref_n) != 0) {
      size_t at = 0;
      while (at < ref_n && cur.p[at] == ref.p[at]) ++at;
      size_t nbad = 0;
      for (size_t j = 0; j < ref_n; ++j) nbad += cur.p[j] != ref.p[j];
      status = fail(FQT_ERR_DEVICE, "autotune candidate %zu (path %d, q = 2^%u, tile %u, boundary "
                    "%u) is not byte-identical to candidate %zu: %zu of %zu bytes differ, first "
                    "at byte %zu (%u vs %u)", i, (int)cands[i].path, cands[i].opts.log2q,
                    cands[i].opts.tile, cands[i].opts.boundary, ref_i, nbad, ref_n, at,
                    (unsigned)cur.p[at], (unsigned)ref.p[at]);
      break;
    }
    // time enough replays to cover about 20 ms, at least three
    int reps = 3;
    if (hipEventRecord(e0, st) != hipSuccess) { status = fail(FQT_ERR_DEVICE, "event"); break; }
    for (int r = 0; r < reps && status == FQT_OK; ++r) status = run(cands[i]);
    if (status) break;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      status = fail(FQT_ERR_DEVICE, "event");
      break;
    }
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    double per = ms / reps;
    if (per * reps < 20.0) {
      reps = (int)std::min(200.0, std::ceil(20.0 / std::max(per, 1e-3)));
      hipEventRecord(e0, st);
      for (int r = 0; r < reps && status == FQT_OK; ++r) status = run(cands[i]);
      if (status) break;
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      hipEventElapsedTime(&ms, e0, e1);
      per = ms / reps;
    }
    times[i] = per;
    if (per < best_ms) {
      best_ms = per;
      best_i = i;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (status) return status;

  if (status == FQT_OK && !have_ref)
    status = fail(FQT_ERR_UNSUPPORTED, "every candidate was refused for this problem");
  if (status) return status;
  const Candidate& w = cands[best_i];
  {
    std::lock_guard<std::mutex> lk(f->mu);
    f->tuned[key] = TuneEntry{w.path, w.opts};
    if (only == FQT_PATH_AUTO || !f->tuned.count(auto_key)) f->tuned[auto_key] = TuneEntry{w.path, w.opts};
  }
  if (cache_path) {
    if (FILE* fp = std::fopen(cache_path, "a")) {
      std::fprintf(fp,
                   "{\"key\": \"%s\", \"path\": %d, \"log2q\": %u, \"n_q\": %u, \"tile\": %u, "
                   "\"boundary\": %u, \"centered\": %u, \"ms\": %.6f, \"candidates\": %zu}\n",
                   key.c_str(), (int)w.path, w.opts.log2q, w.opts.n_q, w.opts.tile, w.opts.boundary,
                   w.opts.centered, best_ms, cands.size());
      std::fclose(fp);
    }
  }
  if (best_path) *best_path = w.path;
  if (best) *best = w.opts;
  return ok();
}

// Autotuner of uneven polynomial batches: every chunk length d+1 (1..8) in
// both chunk representations (odd p), default q and n_q; a candidate counts
// only if every output byte equals the first admissible candidate's.
fqt_status fqt_autotune_polymul(uint32_t p, int64_t count, const fqt_poly_desc* descs,
                                const char* cache_path, uint32_t* best_d,
                                uint32_t* best_centered, uint32_t* best_boundary,
                                fqt_stream_t s) {
  if (count < 1 || !descs) return fail(FQT_ERR_INVALID_ARG, "empty batch");
  int64_t lmax = 0, total = 0;
  for (int64_t i = 0; i < count; ++i) {
    if (descs[i].la < 0 || descs[i].lb < 0)
      return fail(FQT_ERR_INVALID_ARG, "descriptor %lld: negative length", (long long)i);
    lmax = std::max(lmax, std::max(descs[i].la, descs[i].lb));
    if (descs[i].la && descs[i].lb) total += descs[i].la + descs[i].lb - 1;
  }
  int64_t bucket = 1;
  while (bucket < lmax) bucket <<= 1;
  char keybuf[96];
  std::snprintf(keybuf, sizeof keybuf, "poly_p%u_c%lld_L%lld", p, (long long)count,
                (long long)bucket);
  if (cache_path) {
    if (FILE* fp = std::fopen(cache_path, "r")) {
      char line[256];
      bool found = false;
      unsigned d = 0, cen = 0, bnd = 0;
      while (std::fgets(line, sizeof line, fp)) {
        char k[96];
        unsigned dd = 0, cc = 0, bb = 0;
        if (std::sscanf(line,
                        "{\"key\": \"%95[^\"]\", \"d\": %u, \"centered\": %u, \"boundary\": %u",
                        k, &dd, &cc, &bb) == 4 &&
            std::strcmp(k, keybuf) == 0) {
          d = dd;
          cen = cc;
          bnd = bb;
          found = true;  // the last matching line wins
        }
      }
      std::fclose(fp);
      if (found) {
        if (best_d) *best_d = d;
        if (best_centered) *best_centered = cen;
        if (best_boundary) *best_boundary = bnd;
        return ok();
      }
    }
  }
  hipStream_t st = (hipStream_t)s;
  PinnedBuf ref, cur;
  {
    fqt_status rs = ref.resize((size_t)total);
    if (!rs) rs = cur.resize((size_t)total);
    if (rs) return rs;
  }
  // outputs in address order, adjacent ones merged into one copy each (a
  // batch in flat buffers is one copy)
  std::vector<std::pair<uint8_t*, size_t>> runs;
  for (int64_t i = 0; i < count; ++i)
    if (descs[i].la && descs[i].lb)
      runs.push_back({descs[i].c, (size_t)(descs[i].la + descs[i].lb - 1)});
  std::sort(runs.begin(), runs.end());
  {
    size_t w = 0;
    for (size_t i = 0; i < runs.size(); ++i) {
      if (w && runs[w - 1].first + runs[w - 1].second == runs[i].first)
        runs[w - 1].second += runs[i].second;
      else
        runs[w++] = runs[i];
    }
    runs.resize(w);
  }
  auto snap = [&](PinnedBuf& b) -> fqt_status {
    size_t off = 0;
    for (const auto& r : runs) {
      FQT_HIP(hipMemcpyAsync(b.p + off, r.first, r.second, hipMemcpyDeviceToHost, st));
      off += r.second;
    }
    FQT_HIP(hipStreamSynchronize(st));
    return ok();
  };
  hipEvent_t e0, e1;
  FQT_HIP(hipEventCreate(&e0));
  FQT_HIP(hipEventCreate(&e1));
  bool have_ref = false;
  double best_ms = 1e30;
  uint32_t bd = 0, bc = 0, bb = 0;
  fqt_status status = FQT_OK;
  // chunk length d + 1, centring, and the block-boundary mode (2: digit sums,
  // for q <= 2^12; 1: REDQ residues); q and n_q are then the largest eq. (2)
  // admits, which is never slower (fewer block steps)
  for (uint32_t cen = 0; cen <= (p % 2 ? 1u : 0u) && status == FQT_OK; ++cen)
    for (uint32_t d = 0; d <= 7 && status == FQT_OK; ++d)
    for (uint32_t bnd = 2; bnd >= 1 && status == FQT_OK; --bnd) {
      auto run = [&]() {
        return fqt_polymul_dfqt_batched(p, d, 0, 0, bnd, cen, count, descs, s);
      };
      status = run();  // builds the plan and its graph
      if (status == FQT_ERR_UNSUPPORTED || status == FQT_ERR_BOUNDS) {
        status = FQT_OK;
        continue;
      }
      if (status) break;
      status = snap(have_ref ? cur : ref);
      if (status) break;
      if (have_ref && std::memcmp(cur.p, ref.p, (size_t)total) != 0) {
        status = fail(FQT_ERR_DEVICE, "polynomial autotune candidate d = %u, centered = %u, "
                      "boundary = %u is not byte-identical to the first", d, cen, bnd);
        break;
      }
      have_ref = true;
      const int reps = 5;
      hipEventRecord(e0, st);
      for (int r = 0; r < reps && status == FQT_OK; ++r) status = run();
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      if (status == FQT_OK && ms / reps < best_ms) {
        best_ms = ms / reps;
        bd = d;
        bc = cen;
        bb = bnd;
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (status) return status;
  if (!have_ref) return fail(FQT_ERR_UNSUPPORTED, "every candidate was refused for this batch");
  if (cache_path)
    if (FILE* fp = std::fopen(cache_path, "a")) {
      std::fprintf(fp,
                   "{\"key\": \"%s\", \"d\": %u, \"centered\": %u, \"boundary\": %u, "
                   "\"ms\": %.6f}\n",
                   keybuf, bd, bc, bb, best_ms);
      std::fclose(fp);
    }
  if (best_d) *best_d = bd;
  if (best_centered) *best_centered = bc;
  if (best_boundary) *best_boundary = bb;
  return ok();
}

}  // extern "C"
