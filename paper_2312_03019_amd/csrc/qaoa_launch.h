// Host-side launchers of the gfx950 kernels (defined in qaoa_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qaoa_plan.h"

namespace qaoa {

// Tile bits per precision: 2^13 complex64 = 2^12 complex128 = 64 KiB of LDS.
constexpr int kTileBitsC64 = 13;
constexpr int kTileBitsC128 = 12;
constexpr int kLogRC64 = 5;     // 32 amplitudes per thread
constexpr int kLogRC128 = 4;    // 16 amplitudes per thread
constexpr int kPassengerC64 = 4;   // high passes keep >= 16 contiguous complex64 (128 B)
constexpr int kPassengerC128 = 3;  // ... >= 8 contiguous complex128 (128 B)

// Forward pass shapes with a specialised kernel (at full register width):
// shape = rounds * 8 + code; 0 selects the generic kernel.
enum : int {
  kShapeFirst = 1,     // |+>^n synthesised, cost phase, one mixer segment
  kShapeSingle = 2,    // one mixer segment
  kShapeMerged = 3,    // mixer segment, cost phase, mixer segment
  kShapeLast = 4,      // one mixer segment, then <C> and norm
  kShapeLastLam = 5,   // ... and lam = C psi
};

// prec: 1 = complex64, 0 = complex128.  One workgroup per tile; descriptors
// are found by tile_begin when ndesc > 1.  All descriptors of one launch
// share logr and (forward) shape.
hipError_t launch_pass(int prec, bool backward, int logr, int shape, const PassDesc* d, int ndesc, int64_t nblocks,
                       int nthreads, hipStream_t st);
hipError_t launch_reduce(const ReduceJob* jobs, const Span* spans, int njobs, hipStream_t st);
hipError_t launch_cut_table(const GraphDev* g, bool weighted, void* out, int64_t N, hipStream_t st);
hipError_t launch_overlap(int prec_a, const void* a, int prec_b, const void* b, int64_t N, double* part,
                          int nblocks, int rev_b, hipStream_t st);
// x[z] <-> x[N-1-z] in place (complements every index bit).
hipError_t launch_reverse(int prec, void* x, int64_t N, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, int64_t n16, hipStream_t st);
// Per-tile cut table (kTileCutStride doubles per tile) of one qubit set.
hipError_t launch_tile_cut(const GraphDev* g, int K, int L, int h, int64_t ntiles, double* out, hipStream_t st);

}  // namespace qaoa
