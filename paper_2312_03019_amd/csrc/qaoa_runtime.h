// Host runtime internals shared by the single-run API and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "qaoa_launch.h"
#include "qaoa_plan.h"

namespace qaoa {

void set_error(const char* fmt, ...);

// Canonical graph on the host.
struct HostGraph {
  int n = 0;
  std::vector<int32_t> eu, ev;   // u < v, lexicographic
  std::vector<double> w;         // empty = unweighted
  bool weighted() const { return !w.empty(); }
  int m() const { return (int)eu.size(); }
  double weight(int e) const { return w.empty() ? 1.0 : w[e]; }
};

// Validates and canonicalises; returns QAOA_OK or QAOA_EINVAL (message set).
int make_graph(int n, int num_edges, const int32_t* edges, const double* weights, HostGraph* out);

// Device copy of a graph: one allocation holding GraphDev and its arrays.
struct DevGraph {
  void* mem = nullptr;
  size_t bytes = 0;
  GraphDev* g = nullptr;
};
size_t dev_graph_bytes(const HostGraph& hg);
// Fill `host_buf` (dev_graph_bytes long) with the image of the graph as it
// will sit at device address `dev_base`.
void build_dev_graph_image(const HostGraph& hg, void* host_buf, void* dev_base);

// The qubit sets the mixer is split into and their tile geometry.
struct SetGeom {
  int K, L, k;                  // tile bits, passenger tile bits, qubits in set
  TileMap map;                  // where tile bits and tile-index bits sit in memory
  int nr;                       // rounds
  int rb[kMaxRounds];
  int rxmask[kMaxRounds];
};

struct PrecCfg {
  int prec;       // 1 = c64, 0 = c128
  int kmax;       // tile bits
  int logr_max;
  int passenger;
  size_t elem;    // bytes per amplitude
};
PrecCfg prec_cfg(int prec);

// Whether a plan's rounds overlap by one tile bit (complex64 2^13 tiles,
// moved through half the LDS by the specialised forward kernels).
bool half_tile_rounds(int K, int logr, const PrecCfg& pc);

// Tile bits and register bits used for an n-qubit state.
void tile_shape(int n, const PrecCfg& pc, int* K, int* logr);
std::vector<SetGeom> make_sets(int n, const PrecCfg& pc);

// One pass of the forward schedule.
struct PassSpec {
  int set;
  std::vector<int> seg_layer;   // layer index of each segment
  std::vector<int> seg_phase;   // 1 if the segment starts with the cost phase of its layer
  bool gen = false, expect = false;
};
std::vector<PassSpec> make_schedule(int nsets, int p);

// Everything uploaded for one run (descriptors and tables), built on the host.
struct RunImage {
  std::vector<PassDesc> fwd, bwd;   // device pointers filled in
  std::vector<SegDesc> segs;
  std::vector<double> dtab;
  std::vector<double> ctab;          // complex values, interleaved, as doubles (converted on pack)
  std::vector<ReduceJob> jobs;
  std::vector<Span> spans;
  int64_t part_doubles = 0;
  int nout = 0;
  std::vector<double> pass_bytes;    // algorithmic HBM bytes per forward pass
  std::vector<double> bwd_bytes;     // ... and per backward pass
  std::vector<int> fwd_set, bwd_set; // qubit set (0 = low set) of each forward / backward pass
  bool complemented = false;         // final state stored at z ^ (2^n - 1)
  // Chunked pass pairs (three-set plans): forward passes 2i-1 (low set) and
  // 2i (a high set X) run chunk by chunk, 2^chunk_bits chunks each, a chunk
  // fixing pair_fixed[i-1] (memory bits of the third set Y) to its index.
  int chunk_bits = 0;
  std::vector<uint64_t> pair_fixed;
};

struct RunRequest {
  const HostGraph* hg;
  int prec;
  int p;
  const double* gamma;
  const double* beta;
  bool grad;
  void* psi;                // device
  void* lam;                // device (grad)
  const GraphDev* g;        // device
  size_t chunk_bytes = 0;   // forward pass pairs in chunks of about this many state bytes (0 = off)
};

// Layout of the device region holding one run image.
struct ImageLayout {
  size_t off_segs, off_dtab, off_ctab, off_jobs, off_spans, off_fwd, off_bwd, total;
};

// Build the run image.  Device pointers inside descriptors are computed from
// `dev_region` (the device address the packed image will occupy), `part`
// (device partial buffer) and `out_index0` (first output slot).
void build_run(const RunRequest& rq, RunImage* img);
ImageLayout image_layout(const RunImage& img, int prec);
// Pack the image for upload: writes `lay.total` bytes into host_buf and
// patches device pointers to point into dev_region, the partial buffer
// `part` and the output array `out` (nout doubles, device).
void pack_run(RunImage& img, const ImageLayout& lay, int prec, void* host_buf, char* dev_region,
              double* part, double* out, const double* tcut);
// Chunk bits F of the pass pairs of a plan (0 = no chunking) and, per pair,
// the memory bits the chunks fix (see build_run).
int chunk_plan(const std::vector<SetGeom>& sets, const std::vector<PassSpec>& sched, int p, double state_bytes,
               size_t chunk_bytes, std::vector<uint64_t>* fixed_out);
// Launch map of chunk k of a pass whose tile index g spans nfree bits with
// g bit i at memory bit map.gpos[i]: the chunk fixes the memory bits in
// fixed_mem to the bits of k (in ascending order of the memory bits) and
// enumerates the remaining index bits in ascending order.
LaunchMap chunk_launch_map(const TileMap& map, int nfree, uint64_t fixed_mem, int64_t k);
// Doubles of the per-tile cut tables of all qubit sets of an n-qubit plan.
size_t tile_cut_doubles(int n, int prec);
// Fill them (device memory `tcut`) for the graph at device address g.
hipError_t launch_tile_cuts(int n, int prec, const GraphDev* g, double* tcut, hipStream_t st);

}  // namespace qaoa
