"""The host-side plan cache of the batched calls (csrc/plan_cache.h), built
with the host compiler alone and run on the CPU.

Checks: lookup cost does not grow with the number of plans held (hash, then
one full-key compare); the least recently used plan is destroyed beyond the
capacity, through its destructor; erase_if destroys exactly the plans it
names; a plan whose construction stops half way releases what it holds.
"""
import shutil
import subprocess
from pathlib import Path

import pytest

HERE = Path(__file__).resolve().parent
CSRC = HERE.parent / "paper_0710_0510_amd" / "csrc"

DRIVER = r"""
#include "plan_cache.h"

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

static int g_live = 0;  // plans constructed and not yet destroyed
struct Plan {
  int id;
  std::vector<char> owned;  // stands for device buffers
  explicit Plan(int i) : id(i), owned(64) { ++g_live; }
  ~Plan() { --g_live; }
};

using fqt_detail::PlanCache;
using fqt_detail::PlanKey;

// keys of `bytes` bytes, equal except in the last 8 (a worst case for a
// cache that compares keys one after another)
// (the head lives in the caller's memory: kept alive in a pool)
static std::vector<std::vector<uint8_t>> g_heads;
static PlanKey make_key(size_t bytes, uint64_t tag) {
  g_heads.emplace_back(bytes, 0x5a);
  std::vector<uint8_t>& k = g_heads.back();
  for (int i = 0; i < 8; ++i) k[bytes - 8 + i] = (uint8_t)(tag >> (8 * i));
  return PlanKey{k.data(), k.size(), fqt_detail::key_tail(int(7))};
}

static double lookup_ns(size_t nplans, size_t bytes) {
  PlanCache<Plan> c(100000);
  for (size_t i = 0; i < nplans; ++i) c.insert(make_key(bytes, i), std::make_unique<Plan>((int)i));
  const auto probe = make_key(bytes, 0);  // the oldest plan
  volatile int sink = 0;
  double best = 1e30;
  for (int rep = 0; rep < 7; ++rep) {
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < 50; ++r) {
      Plan* p = c.find(probe);
      if (!p || p->id != 0) std::abort();
      sink = sink + p->id;
    }
    const auto t1 = std::chrono::steady_clock::now();
    best = std::min(best, std::chrono::duration<double, std::nano>(t1 - t0).count() / 50);
  }
  return best;
}

int main() {
  // LRU: capacity 4
  {
    PlanCache<Plan> c(4);
    for (int i = 0; i < 4; ++i) c.insert(make_key(16, i), std::make_unique<Plan>(i));
    if (g_live != 4 || c.size() != 4) return 10;
    if (!c.find(make_key(16, 0))) return 11;         // 0 is now the most recent
    c.insert(make_key(16, 4), std::make_unique<Plan>(4));  // drops 1
    if (g_live != 4 || c.find(make_key(16, 1))) return 12;
    if (!c.find(make_key(16, 0)) || !c.find(make_key(16, 2))) return 13;
    c.insert(make_key(16, 5), std::make_unique<Plan>(5));  // drops 3
    if (c.find(make_key(16, 3)) || !c.find(make_key(16, 4))) return 14;
    // different sizes, and different tails, never match
    if (c.find(make_key(24, 0))) return 15;
    PlanKey other = make_key(16, 0);
    other.tail = fqt_detail::key_tail(int(8));
    if (c.find(other)) return 18;
    c.erase_if([](const Plan& p) { return p.id % 2 == 0; });  // 0, 2, 4
    if (c.size() != 1 || g_live != 1 || !c.find(make_key(16, 5))) return 16;
    c.clear();
    if (c.size() != 0 || g_live != 0) return 17;
  }
  // a plan whose building stops half way is destroyed with what it holds
  {
    auto build = [](bool fail_midway, PlanCache<Plan>& c) -> Plan* {
      auto pl = std::make_unique<Plan>(99);
      pl->owned.resize(1 << 20);
      if (fail_midway) return nullptr;  // an error return inside plan creation
      return c.insert(make_key(16, 99), std::move(pl));
    };
    PlanCache<Plan> c(2);
    if (build(true, c) || g_live != 0 || c.size() != 0) return 20;
    if (!build(false, c) || g_live != 1) return 21;
  }
  if (g_live != 0) return 22;  // the cache's destructor released its plans
  // lookup cost: one pass over a 300 KB key, whatever the number of plans
  const size_t bytes = 300000;
  const double t1 = lookup_ns(1, bytes), t256 = lookup_ns(256, bytes);
  std::printf("%.0f %.0f\n", t1, t256);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("plan_cache")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([cxx, "-std=c++17", "-O2", "-Wall", "-Werror", "-I", str(CSRC), str(src),
                    "-o", str(exe)], check=True)
    return exe


def test_plan_cache_lru_erase_and_failure(driver):
    out = subprocess.run([str(driver)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)


def test_plan_cache_lookup_independent_of_plan_count(driver):
    out = subprocess.run([str(driver)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0
    t1, t256 = (float(x) for x in out.stdout.split())
    # a linear scan would compare 256 keys of 300 KB: ~256x the cost of one
    assert t256 < 3.0 * t1 + 20000, (t1, t256)
