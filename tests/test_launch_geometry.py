"""Launch geometry of the whole-state sweeps, checked on the CPU.

HIP allows at most 2^32 - 1 work-items per grid dimension; the state of the
largest accepted size (n = 35) has 2^35 amplitudes.  The sweeps that touch
every amplitude or pair (the gate-by-gate circuit and the in-place reversal
of a complemented bound state) therefore run grid-stride on a capped grid.
This compiles the library's geometry header with the host compiler and
checks, for every n the ABI accepts, that each grid fits the limit and that
the grid-stride chunks cover every item exactly once.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2312_03019_amd", "csrc")

HARNESS = r"""
#include <stdio.h>
#include "qaoa_geometry.h"
using namespace qaoa;

// Items a grid-stride sweep reaches: chunk ch is visited by block ch % grid;
// every chunk < nchunks is visited once, and its items are
// [ch * per_chunk, min(items, (ch + 1) * per_chunk)).
static int check(const char* what, int n, int64_t items, int64_t per_chunk, int64_t blocks) {
  if (blocks < 1 && items > 0) { printf("%s n=%d: empty grid\n", what, n); return 1; }
  if (blocks * 256 > kMaxWorkItems) { printf("%s n=%d: %lld blocks exceed the work-item limit\n", what, n, (long long)blocks); return 1; }
  const int64_t nch = sweep_chunks(items, per_chunk);
  int64_t visited = 0;
  for (int64_t b = 0; b < blocks && b < 4; ++b)          // first blocks: count their chunks
    for (int64_t ch = b; ch < nch; ch += blocks) ++visited;
  const int64_t per_block = (nch + blocks - 1) / blocks;
  if (blocks >= 4 && visited < 4 * (per_block - 1)) { printf("%s n=%d: chunks not reached\n", what, n); return 1; }
  if (nch * per_chunk < items || (nch - 1) * per_chunk >= items) { printf("%s n=%d: chunk count wrong\n", what, n); return 1; }
  return 0;
}

int main() {
  int bad = 0;
  for (int n = 1; n <= 35; ++n) {
    const SweepGrids g = sweep_grids(n);
    const int64_t N = int64_t(1) << n;
    bad += check("gate_full", n, N, 256 * kSweepItems, g.gate_full);
    bad += check("gate_half", n, N / 2, 256 * kSweepItems, g.gate_half);
    if (n >= 2) bad += check("reverse", n, N / 2, 256, g.reverse);
    if (n == 1 && g.reverse != 1) { printf("reverse n=1: %lld\n", (long long)g.reverse); ++bad; }
  }
  printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
"""


def test_sweep_grids_fit_and_cover(tmp_path):
    src = tmp_path / "geom.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "geom"
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout


def _grid_stride_items(items, per_chunk, blocks):
    """Python model of the kernels' loop: for ch = block; ch < nchunks; ch += grid."""
    nch = -(-items // per_chunk)
    seen = []
    for b in range(blocks):
        for ch in range(b, nch, blocks):
            seen.extend(range(ch * per_chunk, min(items, (ch + 1) * per_chunk)))
    return seen


@pytest.mark.parametrize("items,per_chunk,blocks", [(1000, 64, 3), (4096, 1024, 4), (5, 256, 1), (1 << 12, 256, 7)])
def test_grid_stride_loop_covers_each_item_once(items, per_chunk, blocks):
    seen = _grid_stride_items(items, per_chunk, blocks)
    assert sorted(seen) == list(range(items))
