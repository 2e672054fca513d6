// Launch geometry of the whole-state sweeps (plain C++, no HIP: the CPU
// tests compile it on its own).
//
// A HIP launch may hold at most 2^32 - 1 work-items per grid dimension, and a
// state of 2^33 or more amplitudes has more items than that.  Such sweeps therefore
// run grid-stride: the grid is capped at kMaxSweepBlocks workgroups, and each
// workgroup walks chunks blockIdx.x, blockIdx.x + gridDim.x, ... until the
// chunk count is reached.
#pragma once
#include <stdint.h>

namespace qaoa {

constexpr int64_t kMaxSweepBlocks = int64_t(1) << 20;   // x 256 threads = 2^28 work-items
constexpr int64_t kMaxWorkItems = (int64_t(1) << 32) - 1;

// Chunks of `per_chunk` items covering `items`.
constexpr int64_t sweep_chunks(int64_t items, int64_t per_chunk) { return (items + per_chunk - 1) / per_chunk; }

// Workgroups launched for a grid-stride sweep over `items` in chunks of `per_chunk`.
constexpr int64_t sweep_blocks(int64_t items, int64_t per_chunk) {
  const int64_t c = sweep_chunks(items, per_chunk);
  return c < kMaxSweepBlocks ? c : kMaxSweepBlocks;
}

// Workgroups (of 256 threads) of the sweeps over an n-qubit state: the
// gate-by-gate circuit's per-amplitude sweeps (init, edge phases) and
// per-pair sweeps (H, RX), 4 items per thread, and the in-place reversal
// (one pair per item).
struct SweepGrids {
  int64_t gate_full, gate_half, reverse;
};
constexpr int kSweepItems = 4;
constexpr SweepGrids sweep_grids(int n) {
  const int64_t N = int64_t(1) << n;
  return SweepGrids{sweep_blocks(N, 256 * kSweepItems), sweep_blocks(N / 2, 256 * kSweepItems),
                    sweep_blocks(N / 2, 256)};
}

}  // namespace qaoa
