// gfx950 kernels of the QAOA max-cut state-vector simulator.
//
// Hot path (one launch per HBM pass, see qaoa_plan.h for the tile layout):
//   k_fwd      : load a tile (or synthesise |+>^n, launch control), run the
//                pass's segments -- each an optional diagonal cost phase
//                exp(-i gamma C(z)) (rotation compression, Eq. UC_opt /
//                Algorithm 2, cut counted with Algorithm 3's popcount form
//                for unweighted graphs) followed by exp(-i beta X_q) on the
//                pass's qubits -- then optionally accumulate <C> and the norm
//                in FP64, and store.
//   k_bwd      : the adjoint sweep: undo a forward pass on (phi, lam) while
//                accumulating Im<lam|X_q|phi> and Im<lam|C|phi> in FP64.
// Support: k_tile_cut (per-tile cut values), k_reduce (deterministic
// second-stage sums), k_cut_table_*, k_overlap (fidelity), k_reverse
// (complemented state back to natural order), k_copy (bandwidth reference).
//
// Design notes.  The state streams through each CU once per pass: every
// amplitude is read and written exactly once, and all butterflies of the
// pass happen in registers, with LDS used only to transpose which tile bits
// are register bits.  The cost phase of a tile is never evaluated per
// amplitude from scratch: each thread evaluates C at one index z0 (its
// register bits zero) and, for each register bit k, the change d_k of the
// cut when that bit flips alone; C(z0 ^ J) = C(z0) + sum_{k in J} d_k + RT[J]
// with RT the cut among the register vertices (a per-pass table).  The
// phase is then a product tree of 1 + LOGR complex exponentials.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "qaoa_geometry.h"
#include "qaoa_plan.h"
#include "qaoa_launch.h"

namespace qaoa {

// Device memory reached through descriptors arrives as generic pointers;
// state goes through the global address space (global_load/store), tables
// and graph data through the constant space (scalar loads when uniform).
// (The host pass only sees these bodies for the kernel stubs; it gets no
// address spaces.)
#if defined(__HIP_DEVICE_COMPILE__)
#define QGLOBAL __attribute__((address_space(1)))
#define QCONST __attribute__((address_space(4)))
#else
#define QGLOBAL
#define QCONST
#endif

template <typename T>
__device__ __forceinline__ QGLOBAL T* gmem(void* p) {
  return (QGLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const QCONST T* cmem(const void* p) {
  return (const QCONST T*)p;
}

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
struct Prec;
template <>
struct Prec<float> {
  static constexpr int kSwz = 5;   // 32 complex64 = 256 B per swizzle group
  typedef float V __attribute__((ext_vector_type(2)));
};
template <>
struct Prec<double> {
  static constexpr int kSwz = 4;   // 16 complex128 = 256 B per swizzle group
  typedef double V __attribute__((ext_vector_type(2)));
};

template <typename R>
__device__ __forceinline__ cx<R> ldg(const QGLOBAL cx<R>* p) {
  const typename Prec<R>::V v = *reinterpret_cast<const QGLOBAL typename Prec<R>::V*>(p);
  return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void stg(QGLOBAL cx<R>* p, cx<R> a) {
  typename Prec<R>::V v;
  v.x = a.re;
  v.y = a.im;
  *reinterpret_cast<QGLOBAL typename Prec<R>::V*>(p) = v;
}

// The pass kernels stream the state: every amplitude is read once and written
// once per pass, with no reuse through the caches.  Non-temporal loads and
// stores (streaming cache policy) together measured about 9% faster than the
// default policy for a contiguous in-place sweep of 8 GiB, and a few percent
// for the strided high-set tiles; either one alone gained nothing.
template <typename R>
__device__ __forceinline__ cx<R> ldg_nt(const QGLOBAL cx<R>* p) {
  const typename Prec<R>::V v = __builtin_nontemporal_load(reinterpret_cast<const QGLOBAL typename Prec<R>::V*>(p));
  return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void stg_nt(QGLOBAL cx<R>* p, cx<R> a) {
  typename Prec<R>::V v;
  v.x = a.re;
  v.y = a.im;
  __builtin_nontemporal_store(v, reinterpret_cast<QGLOBAL typename Prec<R>::V*>(p));
}

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// LDS index swizzle: XOR-fold the higher groups of the tile index into the
// lowest group.  GF(2)-linear and a bijection on the tile.
template <typename R>
__device__ __forceinline__ uint32_t swz(uint32_t t) {
  constexpr int G = Prec<R>::kSwz;
  constexpr uint32_t M = (1u << G) - 1u;
  return t ^ (((t >> G) ^ (t >> (2 * G)) ^ (t >> (3 * G))) & M);
}

// Tile index of (thread tid, register 0) in a round whose register bits are [b, b+LOGR).
template <int LOGR>
__device__ __forceinline__ uint32_t tbase(uint32_t tid, int b) {
  return (tid & ((1u << b) - 1u)) | ((tid >> b) << (b + LOGR));
}

// Memory offset of tile index t: tile bit i -> memory bit tpos[i] (bits of t
// at KB and above are zero).  The positions are read as whole words.
template <int KB>
__device__ __forceinline__ uint64_t tmem(uint32_t t, const QCONST int8_t* tpos) {
  const QCONST uint32_t* w = reinterpret_cast<const QCONST uint32_t*>(tpos);
  uint32_t pw[(KB + 3) / 4];
#pragma unroll
  for (int i = 0; i < (KB + 3) / 4; ++i) pw[i] = w[i];
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < KB; ++i) r |= (uint64_t)((t >> i) & 1u) << ((pw[i >> 2] >> (8 * (i & 3))) & 63u);
  return r;
}

// Memory offset of register index j: the OR of the memory bits (given as
// masks) of the register bits set in j.
template <int LOGR>
struct RegOffsets {
  uint64_t bit[LOGR];
  __device__ __forceinline__ explicit RegOffsets(const QCONST uint64_t* bits) {
#pragma unroll
    for (int k = 0; k < LOGR; ++k) bit[k] = bits[k];
  }
  __device__ __forceinline__ uint64_t operator()(int j) const {
    uint64_t o = 0;
#pragma unroll
    for (int k = 0; k < LOGR; ++k)
      if ((j >> k) & 1) o |= bit[k];
    return o;
  }
};

template <typename R, int LOGR, bool NT>
__device__ __forceinline__ void load_tile(cx<R> (&v)[1 << LOGR], const QGLOBAL cx<R>* __restrict__ src,
                                          uint64_t zt, const RegOffsets<LOGR>& ro) {
  const QGLOBAL cx<R>* base = src + zt;
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) v[j] = NT ? ldg_nt(base + ro(j)) : ldg(base + ro(j));
}

template <typename R, int LOGR, bool NT>
__device__ __forceinline__ void store_tile(const cx<R> (&v)[1 << LOGR], QGLOBAL cx<R>* __restrict__ dst,
                                           uint64_t zt, const RegOffsets<LOGR>& ro) {
  QGLOBAL cx<R>* base = dst + zt;
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) {
    if (NT) stg_nt(base + ro(j), v[j]);
    else stg(base + ro(j), v[j]);
  }
}

// Cache policy and occupancy per pass shape, as measured on the n = 30 plans
// (complex64 and complex128, 8 / 16 GiB): the streaming (non-temporal)
// policy pays for the passes over high-set tiles and for the complex128
// passes launched whole.  The plain low-set pass (complex64: three rounds;
// complex128: four, a shape only chunked pass pairs use) takes the default
// policy, so the chunk it writes is still cached when the high-set pass
// reads it (complex64 contiguous tiles also stream better that way whole),
// and runs four workgroups per CU.  The two-round merged complex64 pass runs
// four workgroups per CU as well (127 VGPRs) when launched whole; its chunk
// launches in a pass pair (HALF = 2) run three, which leaves the low-set chunk
// beside it more of each CU (n = 30, three runs each: 59.06 / 59.43 / 59.45 ->
// 58.70 / 59.14 / 59.22 ms per run; whole passes are faster at four).
template <typename R, int NRC, int NSC, int GEN, int EXP>
constexpr bool low_single() {
  return NSC == 1 && GEN == 0 && EXP == 0 && NRC == (sizeof(R) == 4 ? 3 : 4);
}
template <typename R, int NRC, int NSC, int GEN, int EXP>
__device__ constexpr bool fwd_streaming() {
  return !low_single<R, NRC, NSC, GEN, EXP>() && (sizeof(R) == 8 || GEN == 1 || EXP > 0 || NSC == 2);
}
template <typename R, int NRC, int NSC, int GEN, int EXP, int HALF>
constexpr int fwd_waves() {
  return !HALF ? 2 : HALF == 2 ? 3 : (low_single<R, NRC, NSC, GEN, EXP>() || (sizeof(R) == 4 && NSC == 2 && NRC == 2)) ? 4 : 3;
}
template <typename R, int NRC, int NSC, int NOSTORE>
__device__ constexpr bool bwd_streaming() {
  // not for the low-set passes (three rounds complex64, four complex128) nor the complex64 merged pass
  return NRC > 0 && !(sizeof(R) == 4 && NRC == 3 && NSC == 1) && !(sizeof(R) == 8 && NRC == 4) &&
         !(sizeof(R) == 4 && NSC == 2);
}

// Move the register contents from round mapping `from` to round mapping `to` through LDS.
template <typename R, int LOGR>
__device__ __forceinline__ void transpose(cx<R>* lds, cx<R> (&v)[1 << LOGR], uint32_t tid, int from, int to) {
  const uint32_t s0 = swz<R>(tbase<LOGR>(tid, from));
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) lds[s0 ^ swz<R>((uint32_t)j << from)] = v[j];
  __syncthreads();
  const uint32_t s1 = swz<R>(tbase<LOGR>(tid, to));
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) v[j] = lds[s1 ^ swz<R>((uint32_t)j << to)];
  __syncthreads();
}

// Half-tile transposes: consecutive rounds' register windows overlap in at
// least one tile bit s (the highest shared one is used), so the tile splits
// into the two halves s = 0 / s = 1 that move one after the other through
// half the LDS (index with bit s removed).  Three workgroups then share a CU
// (the register budget of three waves per SIMD) instead of two.
//
// Bank model (gfx950, 64 banks of 4 bytes): an LDS access of 8 or 16 bytes
// per lane is served in groups of lanes, and the lanes of a group conflict
// when their byte ranges share a bank.  The counters show the groups are
// 128 bytes wide for some accesses (16 lanes x 8 B, 8 lanes x 16 B) and the
// swizzles are built to be conflict-free for 256-byte groups (32 x 8 B,
// 16 x 16 B) as well.  The swizzle XORs into the bank bits of the LDS index
// a GF(2)-linear function of its higher bits, each bit flipping only bits
// below itself (triangular, hence a bijection).  The patterns were found by
// a search over such functions and checked for every access of every round
// transition of the tile shape (tests/test_lds_swizzle.py repeats the check).
template <typename R>
__device__ __forceinline__ uint32_t swz_half(uint32_t c);
template <>
__device__ __forceinline__ uint32_t swz_half<float>(uint32_t c) {
  constexpr uint32_t P[8] = {1u, 2u, 6u, 11u, 16u, 0u, 16u, 0u};   // for index bits 4..11
  uint32_t f = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) f ^= ((c >> (4 + i)) & 1u) * P[i];
  return c ^ f;
}
template <>
__device__ __forceinline__ uint32_t swz_half<double>(uint32_t c) {
  constexpr uint32_t P[8] = {1u, 3u, 6u, 8u, 1u, 0u, 0u, 0u};      // for index bits 3..10
  uint32_t f = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) f ^= ((c >> (3 + i)) & 1u) * P[i];
  return c ^ f;
}
__device__ __forceinline__ uint32_t drop_bit(uint32_t x, int s) {
  return (x & ((1u << s) - 1u)) | ((x >> (s + 1)) << s);
}
template <typename R, int LOGR>
__device__ __forceinline__ void transpose_half(cx<R>* lds, cx<R> (&v)[1 << LOGR], uint32_t tid, int from, int to) {
  const int s = from > to ? from : to;   // the shared tile bit
  const int kf = s - from, kt = s - to;  // its register bit in each round
  const uint32_t cf = swz_half<R>(drop_bit(tbase<LOGR>(tid, from), s));
  const uint32_t ct = swz_half<R>(drop_bit(tbase<LOGR>(tid, to), s));
  // The first half's reads must not land on registers the second half still
  // has to write out, so they go to a second array (register renaming in the
  // unrolled code: no extra live registers).
  cx<R> w[1 << LOGR];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
    for (int j = 0; j < (1 << LOGR); ++j)
      if (((j >> kf) & 1) == hh) lds[cf ^ swz_half<R>(drop_bit((uint32_t)j << from, s))] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (1 << LOGR); ++j)
      if (((j >> kt) & 1) == hh) w[j] = lds[ct ^ swz_half<R>(drop_bit((uint32_t)j << to, s))];
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) v[j] = w[j];
}

// Factored mixer on the register bits of one round: for every bit in mask,
// (a, b) -> (a - i t b, b - i t a).  The dropped scalar per qubit (cos beta,
// or -i sin beta when the segment uses the shifted angle; for the adjoint
// sweep the corresponding undo scalars) is applied elsewhere.  `cand` (a
// compile-time constant in the shaped kernels) lists the bits that can be in
// the mask at all; the others generate no code.  Bits outside the (runtime)
// mask are skipped by a uniform branch: rounds often hold only a few mask
// bits, and a branch-free form (t = 0) lets the scheduler overlap every bit's
// work and run out of registers.
template <typename R, int LOGR>
__device__ __forceinline__ void rx_round_br(cx<R> (&v)[1 << LOGR], int mask, R t, int cand) {
#pragma unroll
  for (int k = 0; k < LOGR; ++k) {
    if (!(((cand & mask) >> k) & 1)) continue;
#pragma unroll
    for (int j = 0; j < (1 << LOGR); ++j) {
      if (!(j & (1 << k))) {
        cx<R>& a = v[j];
        cx<R>& b = v[j | (1 << k)];
        const cx<R> A = a, B = b;
        a.re = fma(t, B.im, A.re);
        a.im = fma(-t, B.re, A.im);
        b.re = fma(t, A.im, B.re);
        b.im = fma(-t, A.re, B.im);
      }
    }
  }
}


// exp(-i th) = cos th - i sin th in the working precision, for the moderate
// angles the cost phase produces.  Reduction (Cody-Waite): k = rint(th * 2/pi),
// r = th - k * pi/2 in double with pi/2 split into two doubles, each product
// taken exactly inside an FMA, so r in [-pi/4, pi/4] carries only rounding of
// the last step.  sin r and cos r are their Taylor series, truncated where the
// next term is below half an ulp of the working precision on [-pi/4, pi/4]
// (float: through r^9 and r^10; double: through r^17 and r^16).  The quadrant
// k mod 4 then swaps and negates the pair.  No large-argument path is needed
// (or generated), unlike a general sincos.
template <typename R>
__device__ __forceinline__ void sincos_poly(R r, R& s, R& c);
template <>
__device__ __forceinline__ void sincos_poly<float>(float r, float& s, float& c) {
  const float r2 = r * r;
  float ps = 1.0f / 362880.0f;                   // 1/9!
  ps = fmaf(ps, r2, -1.0f / 5040.0f);
  ps = fmaf(ps, r2, 1.0f / 120.0f);
  ps = fmaf(ps, r2, -1.0f / 6.0f);
  s = fmaf(ps * r2, r, r);
  float pc = -1.0f / 3628800.0f;                 // -1/10!
  pc = fmaf(pc, r2, 1.0f / 40320.0f);
  pc = fmaf(pc, r2, -1.0f / 720.0f);
  pc = fmaf(pc, r2, 1.0f / 24.0f);
  pc = fmaf(pc, r2, -0.5f);
  c = fmaf(pc, r2, 1.0f);
}
template <>
__device__ __forceinline__ void sincos_poly<double>(double r, double& s, double& c) {
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0;           // 1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0);      // -1/15!
  ps = fma(ps, r2, 1.0 / 6227020800.0);          // 1/13!
  ps = fma(ps, r2, -1.0 / 39916800.0);           // -1/11!
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  s = fma(ps * r2, r, r);
  double pc = 1.0 / 20922789888000.0;            // 1/16!
  pc = fma(pc, r2, -1.0 / 87178291200.0);        // -1/14!
  pc = fma(pc, r2, 1.0 / 479001600.0);           // 1/12!
  pc = fma(pc, r2, -1.0 / 3628800.0);
  pc = fma(pc, r2, 1.0 / 40320.0);
  pc = fma(pc, r2, -1.0 / 720.0);
  pc = fma(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  c = fma(pc, r2, 1.0);
}

template <typename R>
__device__ __forceinline__ cx<R> expmi(double th) {
  const double k = rint(th * 0.63661977236758134);       // 2/pi
  double r = fma(-k, 1.5707963267948966, th);            // pi/2, high part
  r = fma(-k, 6.123233995736766e-17, r);                 // pi/2, low part
  R sr, cr;
  sincos_poly<R>((R)r, sr, cr);
  const int q = (int)k & 3;
  const R c0 = (q & 1) ? sr : cr, s0 = (q & 1) ? cr : sr;
  const R cs = ((q + 1) & 2) ? -c0 : c0;                  // cos(r + q pi/2)
  const R sn = (q & 2) ? -s0 : s0;                        // sin(r + q pi/2)
  return {cs, -sn};
}

// Sum over the 64-lane wave, then across waves; result valid on thread 0.
__device__ __forceinline__ void block_reduce2(double& a, double& b, double* red, int nthreads) {
  const int wsz = nthreads < 64 ? nthreads : 64;
  for (int off = wsz >> 1; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, wsz);
    b += __shfl_xor(b, off, wsz);
  }
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6)] = a;
    red[2 * (tid >> 6) + 1] = b;
  }
  __syncthreads();
  if (tid == 0) {
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < (nthreads + 63) / 64; ++w) {
      a += red[2 * w];
      b += red[2 * w + 1];
    }
  }
  __syncthreads();
}

struct SiteVals {
  double cz0;
  double d[kMaxLogR];
};

// Per-tile part of the cut decomposition: C(zbase) and, for each tile bit i,
// dout_i = sum over out-of-tile neighbours v of the tile vertex u_i of
// w_uv (1 - 2 zbase_v).  It depends only on the graph and the tile
// geometry, so it is tabulated once per qubit set (k_tile_cut) and read by
// the pass kernels with uniform loads.
__global__ void __launch_bounds__(256) k_tile_cut(const GraphDev* __restrict__ gp, int K, int nfree, TileMap map,
                                                  int64_t ntiles, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= ntiles) return;
  const QCONST GraphDev* g_ = cmem<GraphDev>(gp);
  const QCONST int32_t* eu = cmem<int32_t>(g_->eu);
  const QCONST int32_t* ev = cmem<int32_t>(g_->ev);
  const QCONST double* ew = cmem<double>(g_->ew);
  const QCONST int32_t* nbr = cmem<int32_t>(g_->nbr);
  const QCONST double* nw = cmem<double>(g_->nw);
  uint64_t zb = 0, tmask = 0;
  for (int i = 0; i < nfree; ++i) zb |= (((uint64_t)g >> i) & 1ull) << map.gpos[i];
  for (int i = 0; i < K; ++i) tmask |= 1ull << map.tpos[i];
  double cb = 0.0;
  for (int e = 0; e < g_->m; ++e)
    if (((zb >> eu[e]) ^ (zb >> ev[e])) & 1ull) cb += ew[e];
  double* row = out + g * kTileCutStride;
  row[0] = cb;
  for (int i = 0; i < kTileCutStride - 1; ++i) {
    double d = 0.0;
    if (i < K) {
      const int u = map.tpos[i];
      for (int k = g_->off[u]; k < g_->off[u + 1]; ++k) {
        const int v = nbr[k];
        if (!((tmask >> v) & 1ull)) d += ((zb >> v) & 1ull) ? -nw[k] : nw[k];
      }
    }
    row[1 + i] = d;
  }
}

template <int LOGR>
__device__ __forceinline__ SiteVals site_values(const QCONST double* __restrict__ dtab, const SiteDesc& S,
                                                const QCONST double* __restrict__ tcrow, uint32_t tb, int b, int K,
                                                uint32_t tid, int nthreads) {
  SiteVals r;
  double c = tcrow[0];
#pragma unroll
  for (int i = 0; i < kTileCutStride - 1; ++i)
    if (i < K && ((tb >> i) & 1u)) c += tcrow[1 + i];
  r.cz0 = c + dtab[S.f_off + tid];
#pragma unroll
  for (int k = 0; k < LOGR; ++k) r.d[k] = tcrow[1 + b + k] + dtab[S.g_off + k * nthreads + tid];
#pragma unroll
  for (int k = LOGR; k < kMaxLogR; ++k) r.d[k] = 0.0;
  return r;
}

// v[J] *= exp(-i gamma C(z0 ^ J)), or its conjugate when `undo`.  The
// per-amplitude phase is exp(-i gamma C(z0)) * prod_{k in J} exp(-i gamma d_k)
// * exp(-i gamma RT[J]); the product over J is split into a low and a high
// half-tree so only 2^3 + 2^(LOGR-3) partial products stay in registers.
// `pre` multiplies every factor (a carried scalar).
template <typename R, int LOGR>
struct PhaseTrees {
  static constexpr int LO = LOGR < 3 ? LOGR : 3;
  static constexpr int HI = LOGR - LO;
  cx<R> lo[1 << LO], hi[1 << HI];
  __device__ __forceinline__ PhaseTrees(const SiteVals& sv, double gamma, bool undo, cx<R> pre) {
    const double gs = undo ? -gamma : gamma;
    lo[0] = cmul(expmi<R>(gs * sv.cz0), pre);
#pragma unroll
    for (int k = 0; k < LO; ++k) {
      const cx<R> e = expmi<R>(gs * sv.d[k]);
#pragma unroll
      for (int j = 0; j < (1 << k); ++j) lo[j | (1 << k)] = cmul(lo[j], e);
    }
    hi[0] = {(R)1, (R)0};
#pragma unroll
    for (int k = 0; k < HI; ++k) {
      const cx<R> e = expmi<R>(gs * sv.d[LO + k]);
#pragma unroll
      for (int j = 0; j < (1 << k); ++j) hi[j | (1 << k)] = cmul(hi[j], e);
    }
  }
  // the factor of register index j
  __device__ __forceinline__ cx<R> at(int j, cx<R> rt, bool undo) const {
    const cx<R> t = cmul(lo[j & ((1 << LO) - 1)], hi[j >> LO]);
    return undo ? cmulc(t, rt) : cmul(t, rt);
  }
};

template <typename R, int LOGR>
__device__ __forceinline__ void apply_phase(cx<R> (&v)[1 << LOGR], const SiteVals& sv, double gamma,
                                            const QCONST cx<R>* __restrict__ rtph, bool undo,
                                            cx<R> pre = {(R)1, (R)0}) {
  const PhaseTrees<R, LOGR> T(sv, gamma, undo, pre);
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) v[j] = cmul(v[j], T.at(j, rtph[j], undo));
}

// The same phase on two vectors (the adjoint sweep's phi and lam), factors computed once.
template <typename R, int LOGR>
__device__ __forceinline__ void apply_phase2(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR], const SiteVals& sv,
                                             double gamma, const QCONST cx<R>* __restrict__ rtph, bool undo,
                                             cx<R> pre) {
  const PhaseTrees<R, LOGR> T(sv, gamma, undo, pre);
#pragma unroll
  for (int j = 0; j < (1 << LOGR); ++j) {
    const cx<R> t = T.at(j, rtph[j], undo);
    f[j] = cmul(f[j], t);
    l[j] = cmul(l[j], t);
  }
}

__device__ __forceinline__ int find_desc(const PassDesc* __restrict__ descs, int ndesc, int64_t wg) {
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= wg) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Tile handled by this workgroup.  Workgroups are dealt round-robin to the
// eight XCDs; for a single-descriptor launch, give each XCD a contiguous run
// of the launch's tiles so its L2 and the HBM pages it opens see neighbouring
// addresses, then map the launch-local index to the pass's tile index (the
// identity unless the launch covers one chunk of the state).  The map is a
// kernel argument, so this is scalar arithmetic on registers.
__device__ __forceinline__ int64_t tile_of_block(const PassDesc& D, int ndesc, const LaunchMap& lm) {
  const int64_t wg = blockIdx.x;
  if (ndesc > 1) return wg - D.tile_begin;
  const uint64_t t = (gridDim.x & 7u) == 0 ? (wg & 7) * (int64_t)(gridDim.x >> 3) + (wg >> 3) : wg;
  return (int64_t)launch_tile(lm, t);
}

// Memory offset of tile g's index-0 amplitude (scalar arithmetic on the
// descriptor's runs, so the tile's loads can issue at once).
__device__ __forceinline__ uint64_t tile_zbase(const PassDesc& D, int64_t g) {
  uint64_t z = 0;
#pragma unroll
  for (int r = 0; r < kMaxRuns; ++r) z |= ((uint64_t)g & D.map.gmask[r]) << D.map.gshift[r];
  return z;
}

// One forward pass over one tile.  Template knobs, each either fixed at
// compile time or -1 / 0 = read from the descriptor (the generic kernel):
//   NRC rounds per mixer segment, NSC segments, PHM bit s = segment s starts
//   with the cost phase, GEN synthesise |+>^n instead of loading, EXP 1 =
//   accumulate <C> and the norm, 2 = also store lam = C psi; HALF 0 = the
//   tile moves through the full LDS, 1 = through half of it, 2 = as 1, at
//   three waves per SIMD (the chunk launches of a complex64 merged pass).
// With everything fixed the pass is straight-line code (no register merges).
template <typename R, int LOGR, int KB, int NRC, int NSC, int PHM, int GEN, int EXP, int HALF>
__global__ void __launch_bounds__(kMaxThreads)
    __attribute__((amdgpu_waves_per_eu(fwd_waves<R, NRC, NSC, GEN, EXP, HALF>(),
                                       fwd_waves<R, NRC, NSC, GEN, EXP, HALF>())))
k_fwd(const PassDesc* __restrict__ descs, int ndesc, LaunchMap lm) {
  constexpr int NR = 1 << LOGR;
  constexpr bool NT = NRC > 0 ? fwd_streaming<R, NRC, NSC, GEN, EXP>() : sizeof(R) == 8;
  __shared__ cx<R> lds[1 << (KB - (HALF ? 1 : 0))];
  __shared__ double red[2 * (kMaxThreads / 64)];
  const uint32_t tid = threadIdx.x;
  const PassDesc& D = descs[ndesc > 1 ? find_desc(descs, ndesc, blockIdx.x) : 0];
  const int64_t g = tile_of_block(D, ndesc, lm);
  const int nth = blockDim.x;
  const int nr = NRC > 0 ? NRC : D.nrounds;
  const int nseg = NSC > 0 ? NSC : D.nseg;
  const int flags = D.flags;
  const bool gen = GEN >= 0 ? GEN != 0 : (flags & PF_GEN) != 0;
  const int exp = EXP >= 0 ? EXP : ((flags & PF_EXPECT) ? ((flags & PF_WRITE_LAM) ? 2 : 1) : 0);
  const QCONST cx<R>* __restrict__ ctab = cmem<cx<R>>(D.ctab);
  const QCONST SegDesc* __restrict__ segs = cmem<SegDesc>(D.segs);
  const QCONST double* __restrict__ dtab = cmem<double>(D.dtab);
  const QCONST double* __restrict__ tcrow = cmem<double>(D.tcut) + g * kTileCutStride;

  const RegOffsets<LOGR> ro0(cmem<uint64_t>(D.rbit0));
  const uint64_t zt0 = tile_zbase(D, g) | tmem<KB>(tbase<LOGR>(tid, D.rb[0]), cmem<int8_t>(D.map.tpos));
  cx<R> v[NR];
  if (gen) {
    const R a = (R)D.amp0;
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = {a, (R)0};
  } else {
    load_tile<R, LOGR, NT>(v, gmem<cx<R>>(D.psi), zt0, ro0);
  }
  // Site values: the per-thread cut decomposition; segment s uses site s & 1,
  // at the round it starts in, and <C> uses site 0.  Full-LDS kernels run two
  // workgroups per CU whatever their register count, so they read every site
  // they need with the tile load (latency hidden, registers free).  Half-LDS
  // kernels are register-limited: only the first phase's site is read up
  // front, a later phase's where it is used, and <C>'s just before the last
  // mixer round when that round is round 0, else after the way back to it.
  constexpr bool kEarly = HALF == 0;
  auto site = [&](int which) __attribute__((always_inline)) {
    const int b = which ? D.rb[nr - 1] : D.rb[0];
    return site_values<LOGR>(dtab, D.site[which], tcrow, tbase<LOGR>(tid, b), b, D.K, tid, nth);
  };
  auto has_phase = [&](int s) __attribute__((always_inline)) {
    return PHM >= 0 ? ((PHM >> s) & 1) != 0 : segs[s].has_phase != 0;
  };
  const bool need0 = PHM >= 0 ? ((PHM & 1) || EXP > 0) : (flags & PF_SITE0) != 0;
  const bool need1 = PHM >= 0 ? ((PHM & 2) != 0) : (flags & PF_SITE1) != 0;
  SiteVals s0{}, s1{}, sve{};
  if (kEarly ? need0 : has_phase(0)) s0 = site(0);
  if (kEarly && need1) s1 = site(1);

  // HALF: rounds are [K-LOGR, K), then each LOGR-1 lower, the last clamped at
  // 0 (compile-time bases).
  // (lambdas forced inline: an outlined call would move v[] to scratch memory)
  auto rbase = [&](int i) __attribute__((always_inline)) {
    return HALF ? (KB - LOGR - i * (LOGR - 1) > 0 ? KB - LOGR - i * (LOGR - 1) : 0) : D.rb[i];
  };
  auto step = [&](int from, int to) __attribute__((always_inline)) {
    if (HALF) transpose_half<R, LOGR>(lds, v, tid, rbase(from), rbase(to));
    else transpose<R, LOGR>(lds, v, tid, rbase(from), rbase(to));
  };
  int cur = 0;
#pragma unroll
  for (int s = 0; s < (NSC > 0 ? NSC : 64); ++s) {
    if (NSC <= 0 && s >= nseg) break;
    const SegDesc sg = segs[s];
    if (has_phase(s)) {
      __builtin_amdgcn_sched_barrier(0);
      apply_phase<R, LOGR>(v, s == 0 ? s0 : kEarly ? ((s & 1) ? s1 : s0) : site(s & 1), sg.gamma,
                           ctab + sg.ph_off, false, cx<R>{(R)sg.pre_re, (R)sg.pre_im});
      __builtin_amdgcn_sched_barrier(0);
    }
    const R t = (R)sg.coef;
#pragma unroll
    for (int u = 0; u < (NRC > 0 ? NRC : kMaxRounds); ++u) {
      if (NRC <= 0 && u >= nr) break;
      const int i = (s & 1) ? nr - 1 - u : u;
      if (i != cur) {
        step(cur, i);
        cur = i;
      }
      if (!kEarly && exp > 0 && s == nseg - 1 && u == nr - 1 && i == 0) sve = site(0);
      // Half tiles: round i > 0 shares its top bits with round i-1, which
      // mixed them (the masks give each qubit to the first round holding it).
      const int cand = (HALF && i > 0) ? ((1 << LOGR) - 1) >> (rbase(i) + LOGR - rbase(i - 1)) : (1 << LOGR) - 1;
      rx_round_br<R, LOGR>(v, D.rxmask[i], t, cand);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // back to round 0 for the coalesced store (adjacent steps for half tiles)
  if (HALF) {
#pragma unroll
    for (int i = (NRC > 0 ? NRC : kMaxRounds) - 1; i > 0; --i)
      if (i <= cur) step(i, i - 1);
  } else if (cur != 0) {
    step(cur, 0);
  }
  if (kEarly) sve = s0;
  else if (exp > 0 && (nseg == 0 || cur != 0)) sve = site(0);

  if (flags & PF_SCALE) {
    const cx<R> fs = {(R)D.fscale_re, (R)D.fscale_im};
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = cmul(v[j], fs);
  }

  if (exp > 0) {
    // Gray-code walk over the register index: one FP64 add per amplitude.
    const QCONST double* __restrict__ rt = dtab + D.site[0].rt_off;
    QGLOBAL cx<R>* __restrict__ lam = gmem<cx<R>>(D.lam);
    double aE = 0.0, aN = 0.0, c = sve.cz0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      if (i % 8 == 0) __builtin_amdgcn_sched_barrier(0);   // RT eight entries at a time
      const int J = i ^ (i >> 1);
      if (i > 0) {
        const int k = __builtin_ctz(i);
        c += ((J >> k) & 1) ? sve.d[k] : -sve.d[k];
      }
      const double cj = c + rt[J];
      const double pr = (double)v[J].re * v[J].re + (double)v[J].im * v[J].im;
      aE = fma(pr, cj, aE);
      aN += pr;
      if (exp == 2) {
        const cx<R> lv = {(R)(cj * v[J].re), (R)(cj * v[J].im)};
        if (NT) stg_nt(lam + (zt0 | ro0(J)), lv);
        else stg(lam + (zt0 | ro0(J)), lv);
      }
    }
    block_reduce2(aE, aN, red, blockDim.x);
    if (tid == 0) {
      QGLOBAL double* part = gmem<double>(D.part);
      part[g] = aE;
      part[D.ntiles + g] = aN;
    }
  }
  if (!(flags & PF_NO_STORE)) store_tile<R, LOGR, NT>(v, gmem<cx<R>>(D.psi), zt0, ro0);
}

// Im sum over register pairs of conj(l_a) f_b + conj(l_b) f_a, for the qubits
// in mask.  Each pair's four-product term is formed in the working precision
// (like every other product of two amplitudes) and the sum over pairs and
// qubits runs in FP64.
template <typename R, int LOGR>
__device__ __forceinline__ double dbeta_round(const cx<R> (&f)[1 << LOGR], const cx<R> (&l)[1 << LOGR],
                                              int mask, int cand = (1 << LOGR) - 1) {
  // Bits outside the mask are skipped by a uniform branch.
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < LOGR; ++k) {
    if (!(((cand & mask) >> k) & 1)) continue;
#pragma unroll
    for (int j = 0; j < (1 << LOGR); ++j) {
      if (!(j & (1 << k))) {
        const int b = j | (1 << k);
        R a = l[j].re * f[b].im;
        a = fma(-l[j].im, f[b].re, a);
        a = fma(l[b].re, f[j].im, a);
        a = fma(-l[b].im, f[j].re, a);
        acc += (double)a;
      }
    }
  }
  return acc;
}

// One pass of the adjoint sweep: undo a forward pass on (phi, lam) while
// accumulating the dbeta terms Im <lam| X_q |phi> of every mixer qubit (at any
// point of its layer's undo, since X_q commutes with the layer's other RX) and
// the dgamma term Im <lam| C |phi> at each cost phase, before undoing it.
// Template knobs as for k_fwd (0 / -1 = from the descriptor); NOSTORE: the
// pass that undoes the first forward pass stores nothing.  Rounds of shaped
// kernels follow the full-width pattern; both vectors move through the full
// LDS (two workgroups per CU either way, with 2 x 2^LOGR amplitudes per thread).
template <typename R, int LOGR, int KB, int NRC, int NSC, int PHM, int NOSTORE>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_bwd(const PassDesc* __restrict__ descs, int ndesc, LaunchMap lm) {
  constexpr int NR = 1 << LOGR;
  constexpr bool NT = bwd_streaming<R, NRC, NSC, NOSTORE>();
  constexpr bool SHAPED = NRC > 0;
  __shared__ cx<R> lds[1 << KB];
  __shared__ double red[2 * (kMaxThreads / 64)];
  const uint32_t tid = threadIdx.x;
  const PassDesc& D = descs[ndesc > 1 ? find_desc(descs, ndesc, blockIdx.x) : 0];
  const int64_t g = tile_of_block(D, ndesc, lm);
  const int nth = blockDim.x;
  const int nr = NRC > 0 ? NRC : D.nrounds;
  const int nseg = NSC > 0 ? NSC : D.nseg;
  const bool nostore = NOSTORE >= 0 ? NOSTORE != 0 : (D.flags & PF_NO_STORE) != 0;
  const int64_t nt = D.ntiles;
  QGLOBAL cx<R>* __restrict__ phi = gmem<cx<R>>(D.psi);
  QGLOBAL cx<R>* __restrict__ lamp = gmem<cx<R>>(D.lam);
  QGLOBAL double* __restrict__ part = gmem<double>(D.part);
  const QCONST cx<R>* __restrict__ ctab = cmem<cx<R>>(D.ctab);
  const QCONST SegDesc* __restrict__ segs = cmem<SegDesc>(D.segs);
  const QCONST double* __restrict__ dtab = cmem<double>(D.dtab);
  const QCONST double* __restrict__ tcrow = cmem<double>(D.tcut) + g * kTileCutStride;

  const RegOffsets<LOGR> ro0(cmem<uint64_t>(D.rbit0));
  const uint64_t zt0 = tile_zbase(D, g) | tmem<KB>(tbase<LOGR>(tid, D.rb[0]), cmem<int8_t>(D.map.tpos));
  cx<R> f[NR], l[NR];
  load_tile<R, LOGR, NT>(f, phi, zt0, ro0);
  load_tile<R, LOGR, NT>(l, lamp, zt0, ro0);

  auto has_phase = [&](int s) __attribute__((always_inline)) {
    return PHM >= 0 ? ((PHM >> s) & 1) != 0 : segs[s].has_phase != 0;
  };
  // Site 0 is read with the tile; site 1 (the second segment's phase) where
  // it is used, which keeps it out of the registers of the rounds before.
  const bool need0 = PHM >= 0 ? (PHM & 1) != 0 : (D.flags & PF_SITE0) != 0;
  SiteVals s0{};
  if (need0) s0 = site_values<LOGR>(dtab, D.site[0], tcrow, tbase<LOGR>(tid, D.rb[0]), D.rb[0], D.K, tid, nth);

  // (lambdas forced inline: an outlined call would move f[], l[] to scratch memory)
  auto rbase = [&](int i) __attribute__((always_inline)) {
    return SHAPED ? (KB - LOGR - i * (LOGR - 1) > 0 ? KB - LOGR - i * (LOGR - 1) : 0) : D.rb[i];
  };
  auto step = [&](int from, int to) __attribute__((always_inline)) {
    transpose<R, LOGR>(lds, f, tid, rbase(from), rbase(to));
    transpose<R, LOGR>(lds, l, tid, rbase(from), rbase(to));
  };
  int cur = 0;
  if ((nseg & 1) && nr > 1) {   // the last forward segment ended in the last round
    step(0, nr - 1);
    cur = nr - 1;
  }
#pragma unroll
  for (int s = (NSC > 0 ? NSC : 64) - 1; s >= 0; --s) {
    if (NSC <= 0 && s >= nseg) continue;
    const SegDesc sg = segs[s];
    const R t = (R)sg.bcoef;
    double dB = 0.0;
#pragma unroll
    for (int u = 0; u < (NRC > 0 ? NRC : kMaxRounds); ++u) {
      if (NRC <= 0 && u >= nr) break;
      const int i = (s & 1) ? u : nr - 1 - u;   // forward order reversed
      if (i != cur) {
        step(cur, i);
        cur = i;
      }
      const int cand = (SHAPED && i > 0) ? ((1 << LOGR) - 1) >> (rbase(i) + LOGR - rbase(i - 1)) : (1 << LOGR) - 1;
      dB = fma(sg.bw[i], dbeta_round<R, LOGR>(f, l, D.rxmask[i], cand), dB);
      __builtin_amdgcn_sched_barrier(0);
      rx_round_br<R, LOGR>(f, D.rxmask[i], t, cand);
      __builtin_amdgcn_sched_barrier(0);
      rx_round_br<R, LOGR>(l, D.rxmask[i], t, cand);
      __builtin_amdgcn_sched_barrier(0);
    }
    double dG = 0.0;
    if (has_phase(s)) {
      const SiteVals sv =
          (s & 1) ? site_values<LOGR>(dtab, D.site[1], tcrow, tbase<LOGR>(tid, D.rb[nr - 1]), D.rb[nr - 1], D.K, tid, nth)
                  : s0;
      const QCONST double* __restrict__ rt = dtab + D.site[s & 1].rt_off;
      double c0 = sv.cz0;
#pragma unroll
      for (int ii = 0; ii < NR; ++ii) {
        // (RT read eight entries at a time: hoisting all of them would push
        // the uniform values out of scalar registers into vector ones)
        if (ii % 8 == 0) __builtin_amdgcn_sched_barrier(0);
        const int J = ii ^ (ii >> 1);
        if (ii > 0) {
          const int k = __builtin_ctz(ii);
          c0 += ((J >> k) & 1) ? sv.d[k] : -sv.d[k];
        }
        // Im(conj(l) f): products of two working-precision values are exact in FP64
        const double im = fma((double)l[J].re, (double)f[J].im, -((double)l[J].im * (double)f[J].re));
        dG = fma(c0 + rt[J], im, dG);
      }
      dG *= sg.bwg;
      if (!(nostore && s == 0)) {
        __builtin_amdgcn_sched_barrier(0);
        apply_phase2<R, LOGR>(f, l, sv, sg.gamma, ctab + sg.ph_off, true, cx<R>{(R)sg.bpre_re, (R)sg.bpre_im});
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    block_reduce2(dB, dG, red, nth);
    if (tid == 0) {
      part[(int64_t)(2 * s) * nt + g] = dB;
      part[(int64_t)(2 * s + 1) * nt + g] = dG;
    }
  }
  if (!nostore) {
    if (cur != 0) step(cur, 0);
    // An opaque copy of the tile base: the store addresses are recomputed
    // instead of keeping all load addresses of both vectors live meanwhile.
    uint64_t zs = zt0;
    asm volatile("" : "+v"(zs));
    store_tile<R, LOGR, NT>(f, phi, zs, ro0);
    store_tile<R, LOGR, NT>(l, lamp, zs, ro0);
  }
}

// ---------------------------------------------------------------------------
// A whole small request in one workgroup (serving).  The state stays in LDS
// for every layer: |+>^n, then per layer the cost phase exp(-i gamma C(z))
// (C from Algorithm 3's popcounts when unweighted, else the FP64 sum over the
// cut edges in canonical order; computed once per amplitude and kept in
// registers as FP64) and exp(-i beta X) on every qubit, four (complex128:
// three) qubits at a time in registers (the unitary 2x2 form), then <C> and the norm in FP64 with
// a fixed reduction order.  Thread t owns amplitudes z = t + 1024 k for the
// phase and the sums; for the mixer window [b, b + W) it holds the 2^W
// amplitudes whose other bits are t's.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kSmallThreads) k_small(const SmallDesc* __restrict__ descs) {
  constexpr int MAXN = sizeof(R) == 4 ? kSmallMaxNC64 : kSmallMaxNC128;
  constexpr int KPT = (1 << MAXN) / kSmallThreads;   // amplitudes per thread at the largest n
  __shared__ cx<R> st[1 << MAXN];
  __shared__ double red[2 * (kSmallThreads / 64)];
  const SmallDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (n < 1 || n > MAXN) return;   // the host routes only sizes that fit (uniform: the whole workgroup)
  const int N = 1 << n;
  const uint32_t tid = threadIdx.x;
  const QCONST GraphDev* g = cmem<GraphDev>(D.g);
  const QCONST double* gam = cmem<double>(D.gamma);
  const QCONST double* bet = cmem<double>(D.beta);
  double cz[KPT];
  const R amp0 = (R)exp2(-0.5 * n);
#pragma unroll
  for (int k = 0; k < KPT; ++k) {
    const int z = (int)tid + k * kSmallThreads;
    cz[k] = 0.0;
    if (z < N) {
      const uint64_t b = (uint64_t)z;
      if (!g->weighted) {
        int c = 0;
        for (int v = 0; v < n; ++v) c += (int)__popcll(g->upper[v] & ((0ull - ((b >> v) & 1ull)) ^ b));
        cz[k] = (double)c;
      } else {
        const QCONST int32_t* eu = cmem<int32_t>(g->eu);
        const QCONST int32_t* ev = cmem<int32_t>(g->ev);
        const QCONST double* ew = cmem<double>(g->ew);
        double c = 0.0;
        for (int e = 0; e < g->m; ++e)
          if (((b >> eu[e]) ^ (b >> ev[e])) & 1ull) c += ew[e];
        cz[k] = c;
      }
      st[z] = {amp0, (R)0};
    }
  }
  __syncthreads();
  constexpr int WMAX = sizeof(R) == 4 ? 4 : 3;   // register window (complex128: fewer registers)
  const int W = n < WMAX ? n : WMAX;
  const uint32_t active = 1u << (n - W);
  for (int l = 0; l < D.p; ++l) {
    const double gl = gam[l];
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const int z = (int)tid + k * kSmallThreads;
      if (z < N) st[z] = cmul(st[z], expmi<R>(gl * cz[k]));
    }
    __syncthreads();
    const R c = (R)cos(bet[l]), s = (R)sin(bet[l]);
    for (int b0 = 0; b0 < n; b0 += WMAX) {
      const int b = b0 + W <= n ? b0 : n - W;    // window [b, b + W); bits below b0 are done
      if (tid < active) {
        const uint32_t base = ((tid >> b) << (b + W)) | (tid & ((1u << b) - 1u));
        cx<R> v[1 << WMAX];
#pragma unroll
        for (int j = 0; j < (1 << WMAX); ++j)
          if (j < (1 << W)) v[j] = st[base | ((uint32_t)j << b)];
#pragma unroll
        for (int k = 0; k < WMAX; ++k) {
          if (k >= W || b + k < b0) continue;
#pragma unroll
          for (int j = 0; j < (1 << WMAX); ++j) {
            if (j >= (1 << W) || (j & (1 << k))) continue;
            const cx<R> a = v[j], e = v[j | (1 << k)];
            v[j] = {c * a.re + s * e.im, c * a.im - s * e.re};             // c a - i s e
            v[j | (1 << k)] = {c * e.re + s * a.im, c * e.im - s * a.re};  // -i s a + c e
          }
        }
#pragma unroll
        for (int j = 0; j < (1 << WMAX); ++j)
          if (j < (1 << W)) st[base | ((uint32_t)j << b)] = v[j];
      }
      __syncthreads();
    }
  }
  double aE = 0.0, aN = 0.0;
#pragma unroll
  for (int k = 0; k < KPT; ++k) {
    const int z = (int)tid + k * kSmallThreads;
    if (z < N) {
      const double pr = (double)st[z].re * st[z].re + (double)st[z].im * st[z].im;
      aE = fma(pr, cz[k], aE);
      aN += pr;
    }
  }
  block_reduce2(aE, aN, red, kSmallThreads);
  if (tid == 0) {
    QGLOBAL double* o = gmem<double>(D.out);
    o[0] = aE;
    o[1] = aN;
  }
}

hipError_t launch_small(int prec, const SmallDesc* d, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (prec == 1) hipLaunchKernelGGL(k_small<float>, dim3(count), dim3(kSmallThreads), 0, st, d);
  else hipLaunchKernelGGL(k_small<double>, dim3(count), dim3(kSmallThreads), 0, st, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic second-stage sums: one workgroup per output, Neumaier
// compensation per thread over a fixed stride, then a fixed-order combine.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void nadd(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

__global__ void __launch_bounds__(256) k_reduce(const ReduceJob* __restrict__ jobs, const Span* __restrict__ spans) {
  __shared__ double ss[256], cc[256];
  const ReduceJob J = jobs[blockIdx.x];
  double s = 0.0, c = 0.0;
  for (int k = J.span_begin; k < J.span_end; ++k) {
    const Span sp = spans[k];
    const QGLOBAL double* p = (const QGLOBAL double*)sp.ptr;
    int64_t i = threadIdx.x;
    // eight independent loads in flight, then added in index order
    for (; i + 7 * 256 < sp.count; i += 8 * 256) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = p[i + u * 256];
#pragma unroll
      for (int u = 0; u < 8; ++u) nadd(s, c, x[u]);
    }
    for (; i < sp.count; i += 256) nadd(s, c, p[i]);
  }
  ss[threadIdx.x] = s;
  cc[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ts = 0.0, tc = 0.0;
    for (int i = 0; i < 256; ++i) {
      nadd(ts, tc, ss[i]);
      nadd(ts, tc, cc[i]);
    }
    *(QGLOBAL double*)J.out = J.scale * (ts + tc);
  }
}

// Cut values, unweighted: Algorithm 3's popcount count of cut edges.
__global__ void k_cut_table_i32(const GraphDev* __restrict__ gp, int32_t* __restrict__ out, int64_t N) {
  const QCONST GraphDev* g = cmem<GraphDev>(gp);
  const int n = g->n;
  for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < N; z += (int64_t)gridDim.x * blockDim.x) {
    int c = 0;
    const uint64_t b = (uint64_t)z;
    for (int v = 0; v < n; ++v) c += (int)__popcll(g->upper[v] & ((0ull - ((b >> v) & 1ull)) ^ b));
    out[z] = c;
  }
}

// Cut values, weighted: FP64 sum over cut edges in canonical edge order.
__global__ void k_cut_table_f64(const GraphDev* __restrict__ gp, double* __restrict__ out, int64_t N) {
  const QCONST GraphDev* g = cmem<GraphDev>(gp);
  const int m = g->m;
  const QCONST int32_t* eu = cmem<int32_t>(g->eu);
  const QCONST int32_t* ev = cmem<int32_t>(g->ev);
  const QCONST double* ew = cmem<double>(g->ew);
  for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < N; z += (int64_t)gridDim.x * blockDim.x) {
    double c = 0.0;
    const uint64_t b = (uint64_t)z;
    for (int e = 0; e < m; ++e)
      if (((b >> eu[e]) ^ (b >> ev[e])) & 1ull) c += ew[e];
    out[z] = c;
  }
}

// Per-block partials of Re<a|b>, Im<a|b>, <a|a>, <b|b> in FP64 (fixed grid).
// rev_b: read b at the complemented index N-1-z.
template <typename Ra, typename Rb>
__global__ void __launch_bounds__(256) k_overlap(const cx<Ra>* __restrict__ a, const cx<Rb>* __restrict__ b,
                                                 int64_t N, double* __restrict__ part, int rev_b) {
  __shared__ double red[2 * 4];
  double sr = 0.0, si = 0.0, sa = 0.0, sb = 0.0;
  for (int64_t z = (int64_t)blockIdx.x * 256 + threadIdx.x; z < N; z += (int64_t)gridDim.x * 256) {
    const cx<Ra> x = ldg((const QGLOBAL cx<Ra>*)(a + z));
    const cx<Rb> y = ldg((const QGLOBAL cx<Rb>*)(b + (rev_b ? N - 1 - z : z)));
    const double ar = x.re, ai = x.im, br = y.re, bi = y.im;
    sr += ar * br + ai * bi;
    si += ar * bi - ai * br;
    sa += ar * ar + ai * ai;
    sb += br * br + bi * bi;
  }
  block_reduce2(sr, si, red, 256);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sr;
    part[gridDim.x + blockIdx.x] = si;
  }
  block_reduce2(sa, sb, red, 256);
  if (threadIdx.x == 0) {
    part[2 * gridDim.x + blockIdx.x] = sa;
    part[3 * gridDim.x + blockIdx.x] = sb;
  }
}

// Reduce jobs for `njobs` equal rows of partials: job k sums part[k * count ..
// (k + 1) * count) into out[k].  Filled on the device, so a caller needs no
// host-to-device copy (and no host staging) before k_reduce.
__global__ void k_row_jobs(ReduceJob* __restrict__ jobs, Span* __restrict__ spans, const double* part, int64_t count,
                           int njobs, double* out) {
  const int k = threadIdx.x;
  if (k >= njobs) return;
  ReduceJob j;
  j.span_begin = k;
  j.span_end = k + 1;
  j.scale = 1.0;
  j.out = out + k;
  jobs[k] = j;
  spans[k] = Span{part + (int64_t)k * count, count};
}

// Streaming copy through the global address space: each thread moves ITEMS
// 16-byte vectors (all loads issued before the stores), one workgroup per
// 256 * ITEMS * 16 bytes (4 KiB for ITEMS = 1, 16 KiB for ITEMS = 4).
template <int ITEMS>
__global__ void __launch_bounds__(256) k_copy(const float4* __restrict__ s_, float4* __restrict__ d_, int64_t n) {
  const QGLOBAL float4* s = (const QGLOBAL float4*)s_;
  QGLOBAL float4* d = (QGLOBAL float4*)d_;
  const int64_t base = (int64_t)blockIdx.x * (256 * ITEMS) + threadIdx.x;
  float4 x[ITEMS];
#pragma unroll
  for (int u = 0; u < ITEMS; ++u)
    if (base + u * 256 < n) x[u] = s[base + u * 256];
#pragma unroll
  for (int u = 0; u < ITEMS; ++u)
    if (base + u * 256 < n) d[base + u * 256] = x[u];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// A pass launch; with `done` the launch itself marks that event when the kernel
// completes (no separate marker on the queue), for a wait on another stream.
template <typename K>
static void launch_fwd_kernel(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t done, const PassDesc* d,
                              int ndesc, const LaunchMap& lm) {
  if (done) hipExtLaunchKernelGGL(kernel, grid, block, 0, st, nullptr, done, 0, d, ndesc, lm);
  else hipLaunchKernelGGL(kernel, grid, block, 0, st, d, ndesc, lm);
}

template <typename R, int KB, int LOGR>
static void launch_fwd_shaped(int shape, const PassDesc* d, int ndesc, const LaunchMap& lm, dim3 grid, dim3 block,
                              hipStream_t st, hipEvent_t done) {
  constexpr int HALF = 1;   // full-width tiles move through half the LDS
  switch (shape) {
#define QAOA_FWD(NRC, CODE, NSC, PHM, GEN, EXP)                                                              \
  case NRC * 8 + CODE:                                                                                      \
    launch_fwd_kernel(k_fwd<R, LOGR, KB, NRC, NSC, PHM, GEN, EXP, HALF>, grid, block, st, done, d, ndesc, lm);  \
    return;
#define QAOA_FWD_NR(NRC)                                      \
  QAOA_FWD(NRC, kShapeFirst, 1, 1, 1, 0)                      \
  QAOA_FWD(NRC, kShapeSingle, 1, 0, 0, 0)                     \
  QAOA_FWD(NRC, kShapeMerged, 2, 2, 0, 0)                     \
  QAOA_FWD(NRC, kShapeLast, 1, 0, 0, 1)                       \
  QAOA_FWD(NRC, kShapeLastLam, 1, 0, 0, 2)
    QAOA_FWD_NR(1)
    QAOA_FWD_NR(2)
    QAOA_FWD_NR(3)
    case 2 * 8 + kShapeMergedChunk:   // the planner gives it to complex64 passes only
      if constexpr (sizeof(R) == 4)
        launch_fwd_kernel(k_fwd<R, LOGR, KB, 2, 2, 2, 0, 0, 2>, grid, block, st, done, d, ndesc, lm);
      else
        launch_fwd_kernel(k_fwd<R, LOGR, KB, 2, 2, 2, 0, 0, HALF>, grid, block, st, done, d, ndesc, lm);
      return;
    // Four rounds (the complex128 low set): a merged pass would spill.  A
    // plain single pass launched whole takes the generic full-LDS kernel (it
    // streams at copy speed there); chunked beside a high-set pass it takes
    // this half-LDS kernel, since two full-LDS workgroups per CU leave too
    // little LDS for the high-set chunk's workgroups.  The planner gives the
    // shape only to chunked passes.
    QAOA_FWD(4, kShapeFirst, 1, 1, 1, 0)
    QAOA_FWD(4, kShapeSingle, 1, 0, 0, 0)
    QAOA_FWD(4, kShapeLast, 1, 0, 0, 1)
    QAOA_FWD(4, kShapeLastLam, 1, 0, 0, 2)
#undef QAOA_FWD_NR
#undef QAOA_FWD
    default:
      launch_fwd_kernel(k_fwd<R, LOGR, KB, 0, 0, -1, -1, -1, 0>, grid, block, st, done, d, ndesc, lm);
  }
}

template <typename R, int KB>
static hipError_t launch_pass_t(bool backward, int logr, int shape, const PassDesc* d, int ndesc, const LaunchMap& lm,
                                int64_t nblocks, int nthreads, hipStream_t st, hipEvent_t done) {
  if (backward && done) return hipErrorInvalidValue;   // completion events: forward passes only
  const dim3 grid((unsigned)nblocks), block((unsigned)nthreads);
  constexpr int LMAX = sizeof(R) == 4 ? kLogRC64 : kLogRC128;
  if (logr < 1 || logr > LMAX) return hipErrorInvalidValue;
  if (backward) {
    if (logr == LMAX) {
      switch (shape) {
#define QAOA_BWD(NRC, CODE, NSC, PHM, NOSTORE)                                                            \
  case NRC * 8 + CODE:                                                                                    \
    hipLaunchKernelGGL((k_bwd<R, LMAX, KB, NRC, NSC, PHM, NOSTORE>), grid, block, 0, st, d, ndesc, lm);   \
    return hipGetLastError();
#define QAOA_BWD_NR(NRC)                              \
  QAOA_BWD(NRC, kShapeFirst, 1, 1, 1)                 \
  QAOA_BWD(NRC, kShapeSingle, 1, 0, 0)                \
  QAOA_BWD(NRC, kShapeMerged, 2, 2, 0)
        QAOA_BWD_NR(1)
        QAOA_BWD_NR(2)
        QAOA_BWD_NR(3)
        QAOA_BWD(4, kShapeSingle, 1, 0, 0)   // the complex128 low set
#undef QAOA_BWD_NR
#undef QAOA_BWD
        default:
          break;
      }
    }
#define QAOA_BWD(LR) \
  if (logr == LR) hipLaunchKernelGGL((k_bwd<R, LR, KB, 0, 0, -1, -1>), grid, block, 0, st, d, ndesc, lm);
    QAOA_BWD(1)
    QAOA_BWD(2)
    QAOA_BWD(3)
    QAOA_BWD(4)
    if constexpr (LMAX >= 5) QAOA_BWD(5)
#undef QAOA_BWD
    return hipGetLastError();
  }
  if (logr == LMAX) {
    launch_fwd_shaped<R, KB, LMAX>(shape, d, ndesc, lm, grid, block, st, done);
    return hipGetLastError();
  }
#define QAOA_GEN(LR) \
  if (logr == LR) launch_fwd_kernel(k_fwd<R, LR, KB, 0, 0, -1, -1, -1, 0>, grid, block, st, done, d, ndesc, lm);
  QAOA_GEN(1)
  QAOA_GEN(2)
  QAOA_GEN(3)
  if constexpr (LMAX >= 5) QAOA_GEN(4)
#undef QAOA_GEN
  return hipGetLastError();
}

hipError_t launch_pass(int prec, bool backward, int logr, int shape, const PassDesc* d, int ndesc, int64_t nblocks,
                       int nthreads, hipStream_t st, const LaunchMap& lm, hipEvent_t done) {
  if (prec == 1)
    return launch_pass_t<float, kTileBitsC64>(backward, logr, shape, d, ndesc, lm, nblocks, nthreads, st, done);
  return launch_pass_t<double, kTileBitsC128>(backward, logr, shape, d, ndesc, lm, nblocks, nthreads, st, done);
}

// Mirrors the specialisations launch_pass_t selects (same cases, same
// template arguments); anything else is the generic kernel.
void pass_kernel_name(int prec, bool backward, int logr, int shape, char* buf, size_t len) {
  const char* R = prec == 1 ? "float" : "double";
  const int KB = prec == 1 ? kTileBitsC64 : kTileBitsC128;
  const int LMAX = prec == 1 ? kLogRC64 : kLogRC128;
  const int nrc = shape >> 3, code = shape & 7;
  if (backward) {
    bool shaped = logr == LMAX && ((code == kShapeFirst && nrc >= 1 && nrc <= 3) ||
                                   (code == kShapeSingle && nrc >= 1 && nrc <= 4) ||
                                   (code == kShapeMerged && nrc >= 1 && nrc <= 3));
    if (shaped) {
      const int nsc = code == kShapeMerged ? 2 : 1, phm = code == kShapeFirst ? 1 : code == kShapeMerged ? 2 : 0;
      snprintf(buf, len, "k_bwd<%s, %d, %d, %d, %d, %d, %d>", R, LMAX, KB, nrc, nsc, phm, code == kShapeFirst ? 1 : 0);
    } else {
      snprintf(buf, len, "k_bwd<%s, %d, %d, 0, 0, -1, -1>", R, logr, KB);
    }
    return;
  }
  bool shaped = logr == LMAX && (((code == kShapeFirst || code == kShapeSingle || code == kShapeLast ||
                                   code == kShapeLastLam) && nrc >= 1 && nrc <= 4) ||
                                 (code == kShapeMerged && nrc >= 1 && nrc <= 3) ||
                                 (code == kShapeMergedChunk && nrc == 2));
  if (!shaped) {
    snprintf(buf, len, "k_fwd<%s, %d, %d, 0, 0, -1, -1, -1, 0>", R, logr, KB);
    return;
  }
  const bool merged = code == kShapeMerged || code == kShapeMergedChunk;
  const int nsc = merged ? 2 : 1;
  const int phm = code == kShapeFirst ? 1 : merged ? 2 : 0;
  const int gen = code == kShapeFirst ? 1 : 0;
  const int exp = code == kShapeLast ? 1 : code == kShapeLastLam ? 2 : 0;
  const int half = code == kShapeMergedChunk && prec == 1 ? 2 : 1;
  snprintf(buf, len, "k_fwd<%s, %d, %d, %d, %d, %d, %d, %d, %d>", R, LMAX, KB, nrc, nsc, phm, gen, exp, half);
}

hipError_t launch_reduce(const ReduceJob* jobs, const Span* spans, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(njobs), dim3(256), 0, st, jobs, spans);
  return hipGetLastError();
}

hipError_t launch_cut_table(const GraphDev* g, bool weighted, void* out, int64_t N, hipStream_t st) {
  const int64_t blocks64 = (N + 255) / 256;
  const unsigned blocks = (unsigned)(blocks64 < 65536 ? blocks64 : 65536);
  if (weighted) hipLaunchKernelGGL(k_cut_table_f64, dim3(blocks), dim3(256), 0, st, g, (double*)out, N);
  else hipLaunchKernelGGL(k_cut_table_i32, dim3(blocks), dim3(256), 0, st, g, (int32_t*)out, N);
  return hipGetLastError();
}

hipError_t launch_fidelity_sums(int prec_a, const void* a, int prec_b, const void* b, int64_t N, int rev_b, char* work,
                                int nblocks, hipStream_t st) {
  const FidelityWork w = fidelity_work(nblocks);
  double* part = (double*)(work + w.off_part);
  ReduceJob* jobs = (ReduceJob*)(work + w.off_jobs);
  Span* spans = (Span*)(work + w.off_spans);
  double* out = (double*)(work + w.off_out);
  hipError_t e = launch_overlap(prec_a, a, prec_b, b, N, part, nblocks, rev_b, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_jobs, dim3(1), dim3(64), 0, st, jobs, spans, (const double*)part, (int64_t)nblocks, 4, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_reduce(jobs, spans, 4, st);
}

hipError_t launch_overlap(int prec_a, const void* a, int prec_b, const void* b, int64_t N, double* part,
                          int nblocks, int rev_b, hipStream_t st) {
  const dim3 grid(nblocks), block(256);
  if (prec_a == 1 && prec_b == 1)
    hipLaunchKernelGGL((k_overlap<float, float>), grid, block, 0, st, (const cx<float>*)a, (const cx<float>*)b, N, part,
                       rev_b);
  else if (prec_a == 1)
    hipLaunchKernelGGL((k_overlap<float, double>), grid, block, 0, st, (const cx<float>*)a, (const cx<double>*)b, N,
                       part, rev_b);
  else if (prec_b == 1)
    hipLaunchKernelGGL((k_overlap<double, float>), grid, block, 0, st, (const cx<double>*)a, (const cx<float>*)b, N,
                       part, rev_b);
  else
    hipLaunchKernelGGL((k_overlap<double, double>), grid, block, 0, st, (const cx<double>*)a, (const cx<double>*)b, N,
                       part, rev_b);
  return hipGetLastError();
}

// In-place reversal z <-> N-1-z (the complement of every index bit): item
// i < N/2 swaps one pair, so no element is read after another thread wrote
// it.  Grid-stride over items (the grid is capped, see qaoa_geometry.h).
template <typename T>
__global__ void __launch_bounds__(256) k_reverse(T* __restrict__ x, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N / 2; i += (int64_t)gridDim.x * 256) {
    const T a = x[i], b = x[N - 1 - i];
    x[i] = b;
    x[N - 1 - i] = a;
  }
}

hipError_t launch_reverse(int prec, void* x, int64_t N, hipStream_t st) {
  const int64_t blocks = N < 2 ? 0 : sweep_grids(63 - __builtin_clzll((unsigned long long)N)).reverse;
  if (blocks < 1) return hipSuccess;
  if (prec == 1) hipLaunchKernelGGL((k_reverse<float2>), dim3((unsigned)blocks), dim3(256), 0, st, (float2*)x, N);
  else hipLaunchKernelGGL((k_reverse<double2>), dim3((unsigned)blocks), dim3(256), 0, st, (double2*)x, N);
  return hipGetLastError();
}

hipError_t launch_tile_cut(const GraphDev* g, int K, int nfree, const TileMap& map, int64_t ntiles, double* out,
                           hipStream_t st) {
  const int64_t blocks = (ntiles + 255) / 256;
  hipLaunchKernelGGL(k_tile_cut, dim3((unsigned)blocks), dim3(256), 0, st, g, K, nfree, map, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t n16, int block_bytes, hipStream_t st) {
  const int items = block_bytes / (256 * 16);
  if (items != 1 && items != 4) return hipErrorInvalidValue;
  const int64_t blocks = (n16 + 256 * items - 1) / (256 * items);
  if (blocks < 1 || blocks * 256 > kMaxWorkItems) return hipErrorInvalidValue;
  if (items == 1)
    hipLaunchKernelGGL(k_copy<1>, dim3((unsigned)blocks), dim3(256), 0, st, (const float4*)src, (float4*)dst, n16);
  else
    hipLaunchKernelGGL(k_copy<4>, dim3((unsigned)blocks), dim3(256), 0, st, (const float4*)src, (float4*)dst, n16);
  return hipGetLastError();
}

}  // namespace qaoa
