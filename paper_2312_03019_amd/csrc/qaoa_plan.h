// Work descriptors shared by the host runtime and the gfx950 pass kernels.
//
// A run is a list of HBM passes.  Each pass streams the whole state through
// on-chip memory one tile at a time: a tile is 2^K amplitudes whose indices
// differ in a fixed set of K bits (the "tile bits"), the rest of the index
// (the tile id) being fixed.  Tile bits [0, L) are memory bits [0, L)
// (contiguous, so loads coalesce); where the others go is the set's TileMap.
// Inside the tile, each thread holds 2^LOGR amplitudes in
// registers whose indices differ in LOGR consecutive tile bits [b, b + LOGR)
// (a "round"); LDS transposes move from one round's register bits to the
// next.  The mixer qubits of a pass are applied round by round.
#pragma once
#include <stdint.h>

namespace qaoa {

enum : int32_t {
  PF_GEN = 1,         // generate |+>^n in registers instead of loading
  PF_EXPECT = 2,      // accumulate <C> and norm partials after the last segment
  PF_WRITE_LAM = 4,   // forward: also store lam = C psi (start of the adjoint sweep)
  PF_NO_STORE = 8,    // backward: state is not written back (undoing the first pass)
  PF_SITE0 = 16,      // per-thread cut values needed at the round-0 mapping
  PF_SITE1 = 32,      // ... and at the last round's mapping
  PF_SCALE = 64,      // multiply by fscale after the last segment
};

constexpr int kMaxLogR = 5;
constexpr int kMaxRounds = 4;
constexpr int kMaxN = 35;   // a complex64 state of 2^35 amplitudes is 256 GiB
constexpr int kMaxThreads = 256;
constexpr int kMaxTileBits = 16;

// Where a tile sits in the state: tile bit i is memory (qubit) bit tpos[i],
// bit i of the tile index g is memory bit gpos[i], and the two lists
// together cover every memory bit once.  A tile's passengers (low memory
// bits carried along for coalescing) are its lowest tile bits.  The index
// map is also kept as runs of consecutive bits, so a tile's base offset is
// OR over r of (g & gmask[r]) << gshift[r] (unused runs have gmask 0).
constexpr int kMaxRuns = 12;
struct alignas(8) TileMap {
  uint64_t gmask[kMaxRuns];
  int8_t gshift[kMaxRuns];
  int8_t tpos[kMaxTileBits];
  int8_t gpos[kMaxN];
  int8_t pad[2];
};

// Graph in device memory.  Masks hold one bit per vertex.
struct GraphDev {
  int32_t n, m, weighted, pad;
  uint64_t adj[kMaxN];      // all neighbours of v
  uint64_t upper[kMaxN];    // neighbours j > v (graph_I of Algorithm 3)
  int32_t off[kMaxN + 2];   // CSR row offsets into nbr/nw
  const int32_t *eu;        // edge endpoints (canonical order), weighted cut sum
  const int32_t *ev;
  const double *ew;
  const int32_t *nbr;       // CSR neighbour lists
  const double *nw;
};

// Where the cost phase / cut value is evaluated: the register mapping of one
// round.  A thread's amplitudes there have indices z0 ^ J, with z0 the
// thread's index with its register bits clear and J over the register bits;
// C(z0 ^ J) = C(z0) + sum_{k in J} d_k + RT[J].  Per thread, with S the tile
// vertices set in the thread's part of the tile index, P all tile vertices
// that are not register vertices, and dout_u the cut change of flipping tile
// vertex u alone against the out-of-tile vertices (from the tile's base):
//   C(z0) = C(zbase) + sum_{u in S} dout_u + F[tid],  F = w(S, tile \ S)
//   d_k   = dout_{q_k} + G[k][tid],  G = sum_{v in P} w_{q_k v} (1 - 2 [v in S])
// C(zbase) and dout are computed once per tile; F, G, RT are host tables.
struct SiteDesc {
  int32_t q[kMaxLogR];      // memory bit (vertex) of register bit k
  int32_t rt_off;           // offsets (doubles) into dtab: RT[2^LOGR],
  int32_t f_off;            //   F[nthreads],
  int32_t g_off;            //   G[LOGR][nthreads]
};

// One segment = optional cost phase exp(-i gamma C) then the mixer on the
// pass's qubit set.  Segments alternate their round order.
// The forward sweep applies exp(-i beta X) = cos(beta) (I - i tan(beta) X)
// (mode 0, |cos| >= |sin|) or, with b' = beta - pi/2,
// (-i sin(beta)) X (I - i tan(b') X) (mode 1): always 4 FMAs per amplitude
// pair with |t| <= 1.  All qubits of a layer share beta, so a mode-1 layer
// leaves the state complemented on every qubit once it is complete; since
// C(z) = C(~z) that commutes with every cost phase and leaves <C> unchanged,
// and the run just records it (RunImage::complemented) when the count of
// mode-1 layers is odd: the stored state is then psi(~z), i.e. reversed.
// The product sigma of the factored scalars is carried on the host and
// folded into the next cost phase (pre) or applied after the last pass
// (PassDesc::fscale).  The adjoint sweep uses the unitary form.
struct SegDesc {
  double gamma, beta;
  double cb, sb;            // cos(beta), sin(beta) in FP64
  double coef;              // tan(beta) (mode 0) or tan(beta - pi/2) = -cot(beta) (mode 1)
  double pre_re, pre_im;    // sigma of the previous segment of this pass (forward only)
  int32_t mode;
  int32_t has_phase;
  int32_t ph_off;           // offset (complex elements) into ctab of exp(-i gamma RT[J])
  int32_t pad;
  // Adjoint sweep.  Undoing the mixer is factored the same way:
  // exp(+i beta X) = cos(beta) (I + i tan(beta) X), or (i sin(beta)) X (I - i cot(beta) X),
  // so the kernel applies (I - i bcoef X) and drops the scalar q per qubit
  // (and the X, a frame flip under which every gradient term is invariant).
  // With P the product of the scalars dropped so far, the vectors held are
  // the true ones divided by P: each round's dbeta sum is weighted by |P|^2
  // at that round (bw, by round index), the dgamma sum by bwg, and P is
  // folded into the next undone cost phase (bpre) and then reset.
  double bcoef;
  double bpre_re, bpre_im;
  double bw[kMaxRounds];
  double bwg;
};

struct PassDesc {
  void *psi;                // state (complex, working precision)
  void *lam;                // adjoint vector (gradient only)
  const GraphDev *g;
  const double *dtab;       // FP64 tables of this descriptor's run
  const void *ctab;         // complex tables (working precision)
  const SegDesc *segs;      // this pass's segments
  double *part;             // partial-sum slots: part[slot * ntiles + tile]
  int64_t tile_begin;       // first workgroup of this descriptor within the launch
  int64_t ntiles;
  int32_t n, K;
  int32_t nfree;            // tile-index bits: n - K
  int32_t pad0_;
  int32_t nrounds;
  int32_t rb[kMaxRounds];   // register-bit base of each round
  int32_t rxmask[kMaxRounds];  // which register bits get the mixer in that round
  int32_t flags;
  int32_t nseg;
  int32_t shape;            // forward kernel specialisation (see launch_pass)
  int32_t pad_;
  SiteDesc site[2];         // site 0: mapping of round 0; site 1: of the last round
  double amp0;              // 2^(-n/2)
  double fscale_re, fscale_im;  // pending mixer scalars, applied at the end when PF_SCALE
  const double *tcut;       // per tile: C(zbase), dout[0..K) (kTileCutStride doubles each)
  TileMap map;
  uint64_t rbit0[kMaxLogR];  // memory bit (as a mask) of each register bit of round 0
};

// Which tiles one launch covers: workgroup-local tile index t -> the pass's
// tile index g = gfix | OR over r of (t & mask[r]) << shift[r].  The identity
// (one run, gfix 0) covers every tile; a chunked launch deposits t into the
// index bits left free by the chunk and ORs the chunk's fixed bits in.
constexpr int kLaunchRuns = 10;
struct LaunchMap {
  uint64_t gfix;
  uint64_t mask[kLaunchRuns];
  int8_t shift[kLaunchRuns];
  int32_t nruns;
};
// The pass tile index of launch-local tile t (used by the pass kernels and
// by the host-side inspection of chunk plans).
__host__ __device__ inline uint64_t launch_tile(const LaunchMap& m, uint64_t t) {
  uint64_t g = m.gfix;
#pragma unroll
  for (int r = 0; r < kLaunchRuns; ++r)
    if (r < m.nruns) g |= (t & m.mask[r]) << m.shift[r];
  return g;
}
inline LaunchMap identity_launch() {
  LaunchMap m{};
  m.mask[0] = ~0ull;
  m.nruns = 1;
  return m;
}

// Per-tile cut table row: [C(zbase), dout_0 .. dout_{K-1}, 0...].
constexpr int kTileCutStride = 16;

// A whole small request evaluated by one workgroup (serving): the state
// (2^n amplitudes, n <= kSmallMaxN for the precision) lives in LDS for all p
// layers, so the request needs no HBM passes and completes within one launch.
constexpr int kSmallMaxNC64 = 14;    // 2^14 complex64 = 128 KiB of LDS
constexpr int kSmallMaxNC128 = 13;   // 2^13 complex128 = 128 KiB
constexpr int kSmallThreads = 1024;
struct SmallDesc {
  const GraphDev *g;
  const double *gamma, *beta;   // p values each
  double *out;                  // <C>, norm
  int32_t n, p;
};

// One output value: *out = scale * (sum of the listed spans, in order).
struct ReduceJob {
  int32_t span_begin, span_end;  // into the span array
  double scale;
  double *out;
};

struct Span {
  const double *ptr;   // partial sums (device)
  int64_t count;
};

}  // namespace qaoa
