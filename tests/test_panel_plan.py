"""Host planning of the row-panel jobs (paper_2510_23446_amd/csrc/
tcf_panel_plan.h), built with g++ (with AddressSanitizer and UBSan where
the host has them) and checked on seeded job lists:
split_jobs covers every tile once, in order, at the offsets the stored
tiles take, in parts of nearly equal length that add atomically when a
panel is split; xcd_order is a permutation that keeps each run of
kXcdRun consecutive jobs on one XCD (block b runs on XCD b % 8)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r'''
#include <cstdio>
#include <random>
#include "tcf_panel_plan.h"
using namespace tcf;
static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { std::printf("FAIL " __VA_ARGS__); std::printf("\n"); ++fails; } } while (0)
int main() {
  std::mt19937 rng(7);
  for (int trial = 0; trial < 200; ++trial) {
    // whole panels: random tile counts and tile widths, back to back
    std::vector<PanelTile> tl;
    std::vector<PanelJob> whole;
    const int eb = trial % 2 ? 8 : 4;
    int64_t off = 0;
    const int nj = 1 + rng() % 40;
    for (int j = 0; j < nj; ++j) {
      PanelJob p{off, (int)tl.size(), 1 + (int)(rng() % 70), (int)(rng() % 1000), 1 + (int)(rng() % 64),
                 (int)(rng() % 1000), (int)(rng() % 16) & ~1};
      for (int k = 0; k < p.nt; ++k) {
        tl.push_back(PanelTile{(int)(rng() % 5000), 1 + (int)(rng() % 64)});
        off += panel_tile_elems(tl.back().nc, eb);
      }
      whole.push_back(p);
    }
    const int chunks[] = {1, 3, 4, 16, 32, 1 << 20};
    for (int chunk : chunks) {
      const std::vector<PanelJob> v = split_jobs(whole, chunk, tl, eb);
      size_t i = 0;
      for (const PanelJob& w : whole) {
        const int parts = (w.nt + chunk - 1) / chunk;
        int t = w.t0, nmin = 1 << 30, nmax = 0;
        int64_t o = w.m_off;
        for (int q = 0; q < parts; ++q, ++i) {
          CHECK(i < v.size(), "too few parts");
          if (i >= v.size()) return 1;
          const PanelJob& c = v[i];
          CHECK(c.t0 == t && c.m_off == o, "part %d of a panel starts at tile %d offset %lld", q, c.t0, (long long)c.m_off);
          CHECK(c.nt >= 1 && c.nt <= chunk, "part length %d at split %d", c.nt, chunk);
          CHECK(c.yr_off == w.yr_off && c.nr == w.nr && c.xr_off == w.xr_off, "rows changed");
          CHECK(c.flags == (parts > 1 ? (w.flags | 1) : w.flags), "flags %d", c.flags);
          for (int k = 0; k < c.nt; ++k) o += panel_tile_elems(tl[c.t0 + k].nc, eb);
          t += c.nt;
          nmin = std::min(nmin, c.nt);
          nmax = std::max(nmax, c.nt);
        }
        CHECK(t == w.t0 + w.nt, "tiles not covered");
        CHECK(nmax - nmin <= 1, "parts of uneven length %d..%d", nmin, nmax);
      }
      CHECK(i == v.size(), "extra parts");
    }
    // dispatch order
    std::vector<PanelJob> jobs(rng() % 700);
    for (size_t k = 0; k < jobs.size(); ++k) jobs[k].t0 = (int)k;  // identity tag
    const std::vector<PanelJob> o = xcd_order(jobs);
    CHECK(o.size() == jobs.size(), "size");
    std::vector<int> seen(jobs.size(), 0), xcd_of_run((jobs.size() + kXcdRun - 1) / kXcdRun, -1);
    const int n = (int)jobs.size();
    // every XCD's queue is full for this many positions
    const int full = (n / (8 * kXcdRun)) * 8 * kXcdRun;
    for (int b = 0; b < (int)o.size(); ++b) {
      const int k = o[b].t0;
      CHECK(k >= 0 && k < n && !seen[k], "not a permutation at %d", b);
      if (k < 0 || k >= n) return 1;
      seen[k] = 1;
      if (b < full) {
        const int r = k / kXcdRun;
        CHECK(r % 8 == b % 8, "run %d at position %d", r, b);
        if (xcd_of_run[r] < 0) xcd_of_run[r] = b % 8;
        CHECK(xcd_of_run[r] == b % 8, "run %d split over XCDs", r);
      }
    }
    // within one XCD, jobs come in their original order
    for (int x = 0; x < 8; ++x) {
      int last = -1;
      for (int b = x; b < full; b += 8) {
        CHECK(o[b].t0 > last, "order inside XCD %d", x);
        last = o[b].t0;
      }
    }
  }
  std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
'''


def test_split_and_dispatch_order(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    src = tmp_path / "plan_test.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "plan_test"
    csrc = os.path.join(ROOT, "paper_2510_23446_amd", "csrc")
    # host code only: AddressSanitizer and UBSan catch an out-of-range tile
    # or job index in the planning
    flags = ["-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    b = subprocess.run([gxx, *flags, "-I", csrc, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if b.returncode != 0:  # no sanitizer runtime here: plain build
        subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", csrc, str(src), "-o", str(exe)],
                       check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:]


def test_committed_tune_table_matches_the_key_format():
    """Every entry of the committed tune table carries the key the library
    builds (same version tag and fields), so the bench finds it instead of
    re-timing at setup."""
    import re
    src = open(os.path.join(ROOT, "paper_2510_23446_amd", "csrc", "tcf_api.hip")).read()
    fmt = re.search(r'snprintf\(buf, sizeof buf, "(panels-v\d+[^"]*)"', src).group(1)
    pat = "^" + re.escape(fmt).replace("%d", r"-?\d+") + r" chunks( \d+){4}$"
    table = os.path.join(ROOT, "paper_2510_23446_amd", "tune", "panels_mi355x.txt")
    lines = [l.rstrip("\n") for l in open(table) if l.strip()]
    assert lines
    for l in lines:
        assert re.match(pat, l), l
