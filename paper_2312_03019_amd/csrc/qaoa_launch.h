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
  kShapeMergedChunk = 6,   // merged, launched per chunk as a pass pair's second pass
};

// prec: 1 = complex64, 0 = complex128.  One workgroup per tile; descriptors
// are found by tile_begin when ndesc > 1.  All descriptors of one launch
// share logr and (forward) shape.
// lm: the launch's tile map (identity_launch() for every tile of the pass;
// must be the identity when ndesc > 1).
// done: if not null, the launch marks this event when its kernel completes (a
// forward pass; no separate marker enters the queue).
hipError_t launch_pass(int prec, bool backward, int logr, int shape, const PassDesc* d, int ndesc, int64_t nblocks,
                       int nthreads, hipStream_t st, const LaunchMap& lm = identity_launch(),
                       hipEvent_t done = nullptr);
// Name of the kernel launch_pass runs for these arguments, as the profiler
// reports it without the parameter list (e.g. "k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>").
void pass_kernel_name(int prec, bool backward, int logr, int shape, char* buf, size_t len);
hipError_t launch_reduce(const ReduceJob* jobs, const Span* spans, int njobs, hipStream_t st);
hipError_t launch_cut_table(const GraphDev* g, bool weighted, void* out, int64_t N, hipStream_t st);
hipError_t launch_overlap(int prec_a, const void* a, int prec_b, const void* b, int64_t N, double* part,
                          int nblocks, int rev_b, hipStream_t st);
// Workspace of the fidelity sums, one device buffer: per-block partials
// (4 rows of nblocks doubles), the reduce jobs and spans, and the four sums
// Re<a|b>, Im<a|b>, <a|a>, <b|b> at off_out.  Sub-buffers are 256-byte aligned.
struct FidelityWork {
  size_t off_part, off_jobs, off_spans, off_out, bytes;
};
constexpr int kFidelityMaxBlocks = 2048;
inline size_t round_up_256(size_t x) { return (x + 255) & ~(size_t)255; }
inline FidelityWork fidelity_work(int nblocks) {
  FidelityWork w;
  w.off_part = 0;
  w.off_jobs = round_up_256(4 * (size_t)nblocks * sizeof(double));
  w.off_spans = round_up_256(w.off_jobs + 4 * sizeof(ReduceJob));
  w.off_out = round_up_256(w.off_spans + 4 * sizeof(Span));
  w.bytes = round_up_256(w.off_out + 4 * sizeof(double));
  return w;
}
inline int fidelity_blocks(int64_t N) {
  const int64_t b = (N + 255) / 256;
  return (int)(b < kFidelityMaxBlocks ? b : kFidelityMaxBlocks);
}
// Overlap partials, then the fixed-order reduction of each row, all in `work`
// (fidelity_work(nblocks).bytes of device memory).
hipError_t launch_fidelity_sums(int prec_a, const void* a, int prec_b, const void* b, int64_t N, int rev_b, char* work,
                                int nblocks, hipStream_t st);
// Whole small requests, one workgroup each (SmallDesc array in device memory).
hipError_t launch_small(int prec, const SmallDesc* d, int count, hipStream_t st);
// x[z] <-> x[N-1-z] in place (complements every index bit).
hipError_t launch_reverse(int prec, void* x, int64_t N, hipStream_t st);
// block_bytes: bytes per workgroup, 4096 or 16384.
hipError_t launch_copy(const void* src, void* dst, int64_t n16, int block_bytes, hipStream_t st);
// Per-tile cut table (kTileCutStride doubles per tile) of one qubit set.
hipError_t launch_tile_cut(const GraphDev* g, int K, int nfree, const TileMap& map, int64_t ntiles, double* out,
                           hipStream_t st);

// Gate-by-gate circuit (Algorithm 1): |0> -> H on every qubit -> per level one
// diagonal sweep per edge and one RX sweep per qubit.  Host arrays, canonical
// edge order; weights may be NULL (all 1).
struct GateRun {
  int n, m, p;
  const int32_t *eu, *ev;
  const double *weights, *gamma, *beta;
  void* psi;
};
hipError_t launch_gate_run(int prec, const GateRun& r, hipStream_t st);
// Blocks of the full-state reductions below (part needs 2 doubles per block).
int gate_reduce_blocks(int n);
// out[0] = sum |psi|^2 C(z), out[1] = sum |psi|^2, FP64, fixed order.
hipError_t launch_expect_state(int prec, const GraphDev* g, const void* psi, int n, double* part, double* out,
                               hipStream_t st);
// Inverse-CDF samples of |psi|^2 in natural index order (rev: the state is
// stored complemented).  sums: sample_chunks(n) doubles; prefix: one more;
// bsums: 64 per chunk; u and out: count entries, device memory.
int64_t sample_chunks(int n);
hipError_t launch_sample(int prec, const void* psi, int n, int rev, double* sums, double* prefix, double* bsums,
                         const double* u, int64_t count, uint64_t* out, hipStream_t st);
// Maximum cut value and its lowest index (pv / pz: one entry per block).
hipError_t launch_max_cut(const GraphDev* g, int n, double* pv, uint64_t* pz, double* ov, uint64_t* oz,
                          hipStream_t st);

}  // namespace qaoa
