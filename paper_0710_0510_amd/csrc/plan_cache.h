// Host-side cache of built launch plans (host code only, no HIP types).
//
// A plan is everything a batched call builds once for a descriptor list:
// device copies of the descriptors, the work schedule and the instantiated
// graph.  The cache key is the byte string that decides the plan (the
// descriptors, the resolved parameters, the device).  Lookup hashes the key
// where it lies (64-bit words, four multiply-rotate lanes) and compares full
// keys only among the entries of that hash, so its cost is one pass over the
// key whatever the number of plans held.
// At most `capacity` plans are kept: inserting one more destroys the least
// recently used, through the plan's own destructor, which releases what the
// plan owns.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <list>
#include <memory>
#include <unordered_map>
#include <utility>
#include <vector>

namespace fqt_detail {

inline uint64_t key_hash(const uint8_t* p, size_t n) {
  const uint64_t m = 0x9e3779b97f4a7c15ull;
  uint64_t h[4] = {0x243f6a8885a308d3ull, 0x13198a2e03707344ull, 0xa4093822299f31d0ull,
                   0x082efa98ec4e6c89ull};
  auto rotl = [](uint64_t x, int r) { return (x << r) | (x >> (64 - r)); };
  size_t i = 0;
  for (; i + 32 <= n; i += 32)
    for (int l = 0; l < 4; ++l) {
      uint64_t w;
      std::memcpy(&w, p + i + 8 * l, 8);
      h[l] = rotl(h[l] ^ w, 29) * m;
    }
  uint64_t r = (uint64_t)n * m;
  for (int l = 0; l < 4; ++l) r = rotl(r ^ h[l], 31) * m;
  for (; i < n; ++i) r = (r ^ p[i]) * 0x100000001b3ull;
  return r ^ (r >> 32);
}

// A key in two parts: the caller's descriptor array, read in place (a
// lookup copies nothing), and a short tail of resolved parameters.
struct PlanKey {
  const void* head = nullptr;
  size_t head_bytes = 0;
  std::vector<uint8_t> tail;
};

// The bytes of every argument, in order: a key tail.
template <class... T>
std::vector<uint8_t> key_tail(const T&... parts) {
  std::vector<uint8_t> v;
  (v.insert(v.end(), reinterpret_cast<const uint8_t*>(&parts),
            reinterpret_cast<const uint8_t*>(&parts) + sizeof(parts)),
   ...);
  return v;
}

inline uint64_t plan_key_hash(const PlanKey& k) {
  const uint64_t h = key_hash(static_cast<const uint8_t*>(k.head), k.head_bytes);
  const uint64_t t = key_hash(k.tail.data(), k.tail.size());
  return (h ^ (t + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2))) * 0xff51afd7ed558ccdull;
}

template <class Plan>
class PlanCache {
 public:
  explicit PlanCache(size_t capacity) : cap_(capacity ? capacity : 1) {}
  PlanCache(const PlanCache&) = delete;
  PlanCache& operator=(const PlanCache&) = delete;
  ~PlanCache() { clear(); }

  // The plan built for `key`, now the most recently used; null if none.
  Plan* find(const PlanKey& key) {
    const uint64_t h = plan_key_hash(key);
    auto range = idx_.equal_range(h);
    for (auto it = range.first; it != range.second; ++it) {
      auto e = it->second;
      if (same(e->key, key)) {
        lru_.splice(lru_.begin(), lru_, e);
        return e->plan.get();
      }
    }
    return nullptr;
  }

  // Takes ownership of `plan` under `key` (not already held) and returns it;
  // beyond the capacity, the least recently used plan is destroyed.
  Plan* insert(const PlanKey& key, std::unique_ptr<Plan> plan) {
    const uint64_t h = plan_key_hash(key);
    std::vector<uint8_t> bytes(key.head_bytes + key.tail.size());
    if (key.head_bytes) std::memcpy(bytes.data(), key.head, key.head_bytes);
    if (!key.tail.empty())
      std::memcpy(bytes.data() + key.head_bytes, key.tail.data(), key.tail.size());
    lru_.push_front(Entry{std::move(bytes), h, std::move(plan)});
    idx_.emplace(h, lru_.begin());
    while (lru_.size() > cap_) drop(std::prev(lru_.end()));
    return lru_.front().plan.get();
  }

  // Destroys every plan for which `pred(const Plan&)` holds.
  template <class Pred>
  void erase_if(Pred pred) {
    for (auto it = lru_.begin(); it != lru_.end();) {
      auto next = std::next(it);
      if (pred(*it->plan)) drop(it);
      it = next;
    }
  }

  void clear() {
    while (!lru_.empty()) drop(std::prev(lru_.end()));
  }

  size_t size() const { return lru_.size(); }
  size_t capacity() const { return cap_; }

 private:
  struct Entry {
    std::vector<uint8_t> key;  // head bytes, then tail bytes
    uint64_t hash;
    std::unique_ptr<Plan> plan;
  };
  using Iter = typename std::list<Entry>::iterator;

  static bool same(const std::vector<uint8_t>& stored, const PlanKey& k) {
    if (stored.size() != k.head_bytes + k.tail.size()) return false;
    if (k.head_bytes && std::memcmp(stored.data(), k.head, k.head_bytes) != 0) return false;
    return k.tail.empty() ||
           std::memcmp(stored.data() + k.head_bytes, k.tail.data(), k.tail.size()) == 0;
  }

  void drop(Iter e) {
    auto range = idx_.equal_range(e->hash);
    for (auto it = range.first; it != range.second; ++it)
      if (it->second == e) {
        idx_.erase(it);
        break;
      }
    lru_.erase(e);  // runs the plan's destructor
  }

  size_t cap_;
  std::list<Entry> lru_;  // most recently used first
  std::unordered_multimap<uint64_t, Iter> idx_;
};

}  // namespace fqt_detail
