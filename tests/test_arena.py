"""Host test of the server's device-memory arena (slim_serve.hip): the class
is compiled on its own with a malloc-backed stand-in for the HIP allocator
and driven through random allocations and frees.  Checked: every block is at
least the requested size, live blocks never overlap, freed ranges coalesce
(after everything is freed a whole chunk is allocatable again without new
runtime allocations), and entirely free chunks go back under the cap."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1912_08950_amd", "csrc", "slim_serve.hip")

HARNESS = r'''
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <vector>
typedef int hipError_t;
const int hipSuccess = 0;
static uint64_t g_mallocs = 0, g_frees = 0, g_live_bytes = 0, g_peak_bytes = 0;
static std::map<void*, uint64_t> g_sizes;
hipError_t hipMalloc(void** p, uint64_t n) {
  *p = malloc(n);
  if (!*p) return 1;
  ++g_mallocs;
  g_sizes[*p] = n;
  g_live_bytes += n;
  g_peak_bytes = std::max(g_peak_bytes, g_live_bytes);
  return 0;
}
hipError_t hipFree(void* p) {
  ++g_frees;
  g_live_bytes -= g_sizes[p];
  g_sizes.erase(p);
  free(p);
  return 0;
}
hipError_t hipGetLastError() { return 0; }
@ARENA@
int main() {
  Arena A;
  const uint64_t cap = uint64_t(12) << 30;
  A.set_cap(cap);
  std::mt19937_64 rng(7);
  struct Blk { char* p; uint64_t n; };
  std::vector<Blk> live;
  for (int it = 0; it < 100000; ++it) {
    if (live.empty() || rng() % 2) {
      const uint64_t n = (rng() % 8 == 0) ? (rng() % (uint64_t(3) << 30)) + 1 : (rng() % (1 << 22)) + 1;
      uint64_t got = 0;
      char* p = (char*)A.alloc(n, &got);
      if (!p) { printf("FAIL alloc %llu\n", (unsigned long long)n); return 1; }
      if (got < n) { printf("FAIL short block\n"); return 1; }
      live.push_back({p, got});
      if (live.size() > 24) {
        const size_t i = rng() % live.size();
        A.free(live[i].p, live[i].n);
        live.erase(live.begin() + i);
      }
    } else {
      const size_t i = rng() % live.size();
      A.free(live[i].p, live[i].n);
      live.erase(live.begin() + i);
    }
    if (it % 997 == 0) {
      auto v = live;
      std::sort(v.begin(), v.end(), [](const Blk& x, const Blk& y) { return x.p < y.p; });
      for (size_t k = 1; k < v.size(); ++k)
        if (v[k - 1].p + v[k - 1].n > v[k].p) { printf("FAIL overlap\n"); return 1; }
    }
  }
  for (auto& b : live) A.free(b.p, b.n);
  const uint64_t before = g_mallocs;
  uint64_t got = 0;
  if (!A.alloc(uint64_t(2) << 30, &got) || g_mallocs != before) { printf("FAIL no coalescing\n"); return 1; }
  A.release_all();
  if (g_live_bytes != 0) { printf("FAIL leak\n"); return 1; }
  printf("OK mallocs=%llu frees=%llu peak=%llu\n", (unsigned long long)g_mallocs,
         (unsigned long long)g_frees, (unsigned long long)g_peak_bytes);
  return 0;
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_random_alloc_free(tmp_path):
    src = open(SRC).read()
    start = src.index("class Arena {")
    end = src.index("enum State {", start)
    prog = HARNESS.replace("@ARENA@", src[start:end])
    cpp = tmp_path / "arena.cpp"
    exe = tmp_path / "arena"
    cpp.write_text(prog)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    str(cpp), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("OK"), out.stdout + out.stderr
