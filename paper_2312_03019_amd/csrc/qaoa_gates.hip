// The uncompressed gate-by-gate circuit (Algorithm 1) on the same state
// layout, as the reference the fused passes are measured against, plus the
// full-state sweeps that go with the QAOA loop: <C> of a given state, the
// maximum cut max_z C(z) (the denominator of the approximation ratio), and
// sampling bitstrings from |psi|^2 (the solutions a QAOA run hands back).
//
// Every gate is one sweep over the state (read + write of 2^n amplitudes):
// n Hadamards, then per level one diagonal sweep per edge (the RZZ gate of
// Algorithm 1, as exp(-i gamma w) on the basis states that cut the edge,
// which is exp(-i gamma w_uv [z_u != z_v]) -- the same unitary as the fused
// cost phase, with no global phase left over) and one RX sweep per qubit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qaoa_geometry.h"
#include "qaoa_launch.h"
#include "qaoa_plan.h"

namespace qaoa {
namespace {

template <typename R>
struct V2;
template <>
struct V2<float> {
  typedef float T __attribute__((ext_vector_type(2)));
};
template <>
struct V2<double> {
  typedef double T __attribute__((ext_vector_type(2)));
};

constexpr int kItems = kSweepItems;   // pairs (or amplitudes) per thread

__device__ __forceinline__ int64_t insert_zero(int64_t i, int q) {
  return ((i >> q) << (q + 1)) | (i & ((int64_t(1) << q) - 1));
}

// The sweeps below run grid-stride over chunks of 256 * kItems items (the
// grid is capped, see qaoa_geometry.h).
template <typename R>
__global__ void __launch_bounds__(256) k_gate_init(typename V2<R>::T* __restrict__ psi, int64_t N) {
  const int64_t nchunks = sweep_chunks(N, 256 * kItems);
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t base = ch * 256 * kItems + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      const int64_t z = base + u * 256;
      if (z < N) {
        typename V2<R>::T v;
        v.x = z == 0 ? (R)1 : (R)0;
        v.y = (R)0;
        psi[z] = v;
      }
    }
  }
}

// kind 0: Hadamard (a, b) -> ((a + b) c, (a - b) c) with c = 1/sqrt(2)
// kind 1: exp(-i beta X): (a, b) -> (c a - i s b, -i s a + c b)
template <typename R, int KIND>
__global__ void __launch_bounds__(256) k_gate_pair(typename V2<R>::T* __restrict__ psi, int64_t half, int q, R c,
                                                   R s) {
  const int64_t bit = int64_t(1) << q;
  const int64_t nchunks = sweep_chunks(half, 256 * kItems);
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t base = ch * 256 * kItems + threadIdx.x;
    typename V2<R>::T a[kItems], b[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      const int64_t i = base + u * 256;
      if (i < half) {
        const int64_t z = insert_zero(i, q);
        a[u] = psi[z];
        b[u] = psi[z | bit];
      }
    }
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      const int64_t i = base + u * 256;
      if (i < half) {
        const int64_t z = insert_zero(i, q);
        typename V2<R>::T x, y;
        if (KIND == 0) {
          x.x = (a[u].x + b[u].x) * c;
          x.y = (a[u].y + b[u].y) * c;
          y.x = (a[u].x - b[u].x) * c;
          y.y = (a[u].y - b[u].y) * c;
        } else {
          x.x = c * a[u].x + s * b[u].y;
          x.y = c * a[u].y - s * b[u].x;
          y.x = c * b[u].x + s * a[u].y;
          y.y = c * b[u].y - s * a[u].x;
        }
        psi[z] = x;
        psi[z | bit] = y;
      }
    }
  }
}

// One edge (u, v): psi_z *= (pr + i pi) where z_u != z_v.
template <typename R>
__global__ void __launch_bounds__(256) k_gate_zz(typename V2<R>::T* __restrict__ psi, int64_t N, int u, int v, R pr,
                                                 R pi) {
  const int64_t nchunks = sweep_chunks(N, 256 * kItems);
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t base = ch * 256 * kItems + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t z = base + k * 256;
      if (z < N && (((z >> u) ^ (z >> v)) & 1)) {
        const typename V2<R>::T a = psi[z];
        typename V2<R>::T r;
        r.x = a.x * pr - a.y * pi;
        r.y = a.x * pi + a.y * pr;
        psi[z] = r;
      }
    }
  }
}

// C(z): Algorithm 3's popcount form (unweighted, exact integer) or the FP64
// sum over cut edges in canonical edge order (weighted).
__device__ __forceinline__ double cut_value(const GraphDev* g, uint64_t b) {
  if (!g->weighted) {
    int c = 0;
    for (int v = 0; v < g->n; ++v) c += (int)__popcll(g->upper[v] & ((0ull - ((b >> v) & 1ull)) ^ b));
    return (double)c;
  }
  double c = 0.0;
  for (int e = 0; e < g->m; ++e)
    if (((b >> g->eu[e]) ^ (b >> g->ev[e])) & 1ull) c += g->ew[e];
  return c;
}

// Per-block partials of sum |psi|^2 C(z) and sum |psi|^2 (fixed grid, fixed order).
template <typename R>
__global__ void __launch_bounds__(256) k_expect_state(const GraphDev* __restrict__ g,
                                                      const typename V2<R>::T* __restrict__ psi, int64_t N,
                                                      double* __restrict__ part) {
  __shared__ double red[2][256];
  double e = 0.0, nn = 0.0;
  for (int64_t z = (int64_t)blockIdx.x * 256 + threadIdx.x; z < N; z += (int64_t)gridDim.x * 256) {
    const typename V2<R>::T a = psi[z];
    const double pr = (double)a.x * a.x + (double)a.y * a.y;
    e = fma(pr, cut_value(g, (uint64_t)z), e);
    nn += pr;
  }
  red[0][threadIdx.x] = e;
  red[1][threadIdx.x] = nn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = red[0][0];
    part[gridDim.x + blockIdx.x] = red[1][0];
  }
}

// out[k] = sum over blocks of part[k * nb + i], k < nsum, in block order.
__global__ void __launch_bounds__(64) k_sum_parts(const double* __restrict__ part, int nb, int nsum,
                                                  double* __restrict__ out) {
  if (threadIdx.x < nsum) {
    double s = 0.0, c = 0.0;   // Neumaier
    for (int i = 0; i < nb; ++i) {
      const double x = part[(int64_t)threadIdx.x * nb + i];
      const double t = s + x;
      c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    out[threadIdx.x] = s + c;
  }
}

// (value, index) order for the maximum cut: larger value first, then lower index.
__device__ __forceinline__ bool better(double v, uint64_t z, double bv, uint64_t bz) {
  return v > bv || (v == bv && z < bz);
}

__global__ void __launch_bounds__(256) k_max_cut(const GraphDev* __restrict__ g, int64_t N, double* __restrict__ pv,
                                                 uint64_t* __restrict__ pz) {
  __shared__ double sv[256];
  __shared__ uint64_t sz[256];
  double bv = -INFINITY;
  uint64_t bz = ~0ull;
  for (int64_t z = (int64_t)blockIdx.x * 256 + threadIdx.x; z < N; z += (int64_t)gridDim.x * 256) {
    const double c = cut_value(g, (uint64_t)z);
    if (better(c, (uint64_t)z, bv, bz)) {
      bv = c;
      bz = (uint64_t)z;
    }
  }
  sv[threadIdx.x] = bv;
  sz[threadIdx.x] = bz;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && better(sv[threadIdx.x + s], sz[threadIdx.x + s], sv[threadIdx.x], sz[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + s];
      sz[threadIdx.x] = sz[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pz[blockIdx.x] = sz[0];
  }
}

__global__ void __launch_bounds__(64) k_max_final(const double* __restrict__ pv, const uint64_t* __restrict__ pz,
                                                  int nb, double* __restrict__ ov, uint64_t* __restrict__ oz) {
  if (threadIdx.x == 0) {
    double bv = -INFINITY;
    uint64_t bz = ~0ull;
    for (int i = 0; i < nb; ++i)
      if (better(pv[i], pz[i], bv, bz)) {
        bv = pv[i];
        bz = pz[i];
      }
    *ov = bv;
    *oz = bz;
  }
}

// ---------------------------------------------------------------------------
// Sampling z with probability |psi_z|^2 / sum |psi|^2 by inverse CDF over the
// natural index order: sample = min{z : CDF(z) > u * total}, for uniforms u in
// [0, 1) supplied by the caller.  `rev` reads a complemented state (stored at
// N-1-z).  Chunks of kChunk amplitudes: one pass over the state gives the
// per-chunk sums and, inside each chunk, the sums of its 64 blocks of 64
// amplitudes (fixed order); one workgroup turns the chunk sums into their
// exclusive prefix.  Then each wave serves 64 samples: every lane binary-
// searches the chunk prefix for its own sample, and per sample the wave reads
// that chunk's 64 block sums, takes their prefix, and scans the one block
// that holds the target, 64 amplitudes across the lanes.
// ---------------------------------------------------------------------------
constexpr int kChunk = 4096;

template <typename R>
__device__ __forceinline__ double prob_at(const typename V2<R>::T* psi, int64_t N, int rev, int64_t z) {
  const typename V2<R>::T a = psi[rev ? N - 1 - z : z];
  return (double)a.x * a.x + (double)a.y * a.y;
}

template <typename R>
__global__ void __launch_bounds__(256) k_chunk_sums(const typename V2<R>::T* __restrict__ psi, int64_t N, int rev,
                                                    double* __restrict__ sums, double* __restrict__ bsums) {
  __shared__ double pv[kChunk + kChunk / 64];   // one pad slot per 64 keeps the block walks conflict-free
  __shared__ double red[256];
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  const int len = N - c0 < kChunk ? (int)(N - c0) : kChunk;
  for (int i = threadIdx.x; i < len; i += 256) pv[i + (i >> 6)] = prob_at<R>(psi, N, rev, c0 + i);
  __syncthreads();
  if (threadIdx.x < 64) {   // block sums, each in index order
    double a = 0.0;
    for (int i = 0; i < 64; ++i) {
      const int j = (int)threadIdx.x * 64 + i;
      if (j < len) a += pv[j + (j >> 6)];
    }
    bsums[blockIdx.x * 64 + threadIdx.x] = a;
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < len; i += 256) s += pv[i + (i >> 6)];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Exclusive prefix of sums[0..nc) into prefix[0..nc], prefix[nc] = total.
// One workgroup of 1024: each thread scans a contiguous segment in order.
__global__ void __launch_bounds__(1024) k_scan_chunks(const double* __restrict__ sums, int64_t nc,
                                                      double* __restrict__ prefix) {
  __shared__ double seg[1024];
  const int64_t per = (nc + 1023) / 1024;
  const int64_t b = (int64_t)threadIdx.x * per;
  const int64_t e = b + per < nc ? b + per : nc;
  double s = 0.0;
  for (int64_t i = b; i < e; ++i) s += sums[i];
  seg[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int i = 0; i < 1024; ++i) {
      const double x = seg[i];
      seg[i] = run;
      run += x;
    }
    prefix[nc] = run;
  }
  __syncthreads();
  double run = seg[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    prefix[i] = run;
    run += sums[i];
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_sample(const typename V2<R>::T* __restrict__ psi, int64_t N, int rev,
                                                const double* __restrict__ prefix, const double* __restrict__ bsums,
                                                int64_t nc, const double* __restrict__ u, int64_t count,
                                                uint64_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t k0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;   // this wave's 64 samples
  // (kept below the total, so trailing chunks without mass are never chosen)
  const double total = prefix[nc];
  const int64_t kl = k0 + lane;
  double t = kl < count ? u[kl] * total : 0.0;
  if (t >= total) t = nextafter(total, 0.0);
  // last chunk c with prefix[c] <= t (prefix is non-decreasing, prefix[0] = 0), one search per lane
  int64_t lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const int64_t my_c = lo;
  const double my_tl = t - prefix[lo];
  for (int smp = 0; smp < 64; ++smp) {   // uniform trip count: every lane takes part in every shuffle
    const int64_t c = __shfl(my_c, smp, 64);
    const double tl = __shfl(my_tl, smp, 64);
    const int64_t c0 = c * kChunk;
    const int64_t len = N - c0 < kChunk ? N - c0 : kChunk;
    const double bs = bsums[c * 64 + lane];
    double incl = bs;   // inclusive wave prefix of the block sums
    for (int off = 1; off < 64; off <<= 1) {
      const double y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    // The first block with mass whose inclusive sum exceeds the target holds
    // the sample (the CDF only steps up at elements of nonzero probability;
    // the lanes' sums associate differently, so an empty block can round one
    // ulp above its predecessor).  If rounding (block sums re-added in another
    // order than the chunk sums) leaves no such block, the sample is the
    // chunk's last element with nonzero probability, found in the highest
    // block with mass.
    const unsigned long long ball = __ballot(bs > 0.0 && incl > tl);
    const bool found = ball != 0ull;
    const unsigned long long mass = __ballot(bs > 0.0);
    const int L = found ? __ffsll(ball) - 1 : (mass ? 63 - __clzll(mass) : 0);
    const double base = __shfl(incl - bs, L, 64);   // sum of the blocks before L
    const int64_t j = (int64_t)L * 64 + lane;
    const double pz = j < len ? prob_at<R>(psi, N, rev, c0 + j) : 0.0;
    double run = pz;
    for (int off = 1; off < 64; off <<= 1) {
      const double y = __shfl_up(run, off, 64);
      if (lane >= off) run += y;
    }
    run += base;
    const unsigned long long hit = __ballot(found && pz > 0.0 && run > tl);
    const unsigned long long nz = __ballot(pz > 0.0);
    const int64_t z = hit ? c0 + (int64_t)L * 64 + (__ffsll(hit) - 1)
                          : (nz ? c0 + (int64_t)L * 64 + (63 - __clzll(nz)) : c0);
    if (lane == 0 && k0 + smp < count) out[k0 + smp] = (uint64_t)z;
  }
}

template <typename R>
hipError_t gate_run_t(const GateRun& r, hipStream_t st) {
  typedef typename V2<R>::T T;
  T* psi = (T*)r.psi;
  const int64_t N = int64_t(1) << r.n, half = N >> 1;
  const dim3 blk(256);
  const SweepGrids sg = sweep_grids(r.n);
  const dim3 gfull((unsigned)sg.gate_full);
  const dim3 ghalf((unsigned)sg.gate_half);
  hipLaunchKernelGGL(k_gate_init<R>, gfull, blk, 0, st, psi, N);
  const R h = (R)0.70710678118654752440;
  for (int q = 0; q < r.n; ++q) hipLaunchKernelGGL((k_gate_pair<R, 0>), ghalf, blk, 0, st, psi, half, q, h, (R)0);
  for (int l = 0; l < r.p; ++l) {
    for (int e = 0; e < r.m; ++e) {
      const double th = r.gamma[l] * (r.weights ? r.weights[e] : 1.0);
      hipLaunchKernelGGL(k_gate_zz<R>, gfull, blk, 0, st, psi, N, r.eu[e], r.ev[e], (R)cos(th), (R)(-sin(th)));
    }
    const R c = (R)cos(r.beta[l]), s = (R)sin(r.beta[l]);
    for (int q = 0; q < r.n; ++q) hipLaunchKernelGGL((k_gate_pair<R, 1>), ghalf, blk, 0, st, psi, half, q, c, s);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gate_run(int prec, const GateRun& r, hipStream_t st) {
  if (r.n < 1 || r.n > kMaxN) return hipErrorInvalidValue;
  return prec == 1 ? gate_run_t<float>(r, st) : gate_run_t<double>(r, st);
}

int gate_reduce_blocks(int n) {
  const int64_t b = ((int64_t(1) << n) + 255) / 256;
  return (int)(b < 4096 ? b : 4096);
}

hipError_t launch_expect_state(int prec, const GraphDev* g, const void* psi, int n, double* part, double* out,
                               hipStream_t st) {
  const int nb = gate_reduce_blocks(n);
  const int64_t N = int64_t(1) << n;
  if (prec == 1)
    hipLaunchKernelGGL(k_expect_state<float>, dim3(nb), dim3(256), 0, st, g, (const V2<float>::T*)psi, N, part);
  else
    hipLaunchKernelGGL(k_expect_state<double>, dim3(nb), dim3(256), 0, st, g, (const V2<double>::T*)psi, N, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, part, nb, 2, out);
  return hipGetLastError();
}

int64_t sample_chunks(int n) { return ((int64_t(1) << n) + kChunk - 1) / kChunk; }

hipError_t launch_sample(int prec, const void* psi, int n, int rev, double* sums, double* prefix, double* bsums,
                         const double* u, int64_t count, uint64_t* out, hipStream_t st) {
  const int64_t N = int64_t(1) << n, nc = sample_chunks(n);
  if (prec == 1)
    hipLaunchKernelGGL(k_chunk_sums<float>, dim3((unsigned)nc), dim3(256), 0, st, (const V2<float>::T*)psi, N, rev,
                       sums, bsums);
  else
    hipLaunchKernelGGL(k_chunk_sums<double>, dim3((unsigned)nc), dim3(256), 0, st, (const V2<double>::T*)psi, N,
                       rev, sums, bsums);
  hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, st, sums, nc, prefix);
  if (count > 0) {
    const int64_t waves = (count + 63) / 64;
    const dim3 grid((unsigned)((waves + 3) / 4));
    if (prec == 1)
      hipLaunchKernelGGL(k_sample<float>, grid, dim3(256), 0, st, (const V2<float>::T*)psi, N, rev, prefix, bsums, nc,
                         u, count, out);
    else
      hipLaunchKernelGGL(k_sample<double>, grid, dim3(256), 0, st, (const V2<double>::T*)psi, N, rev, prefix, bsums,
                         nc, u, count, out);
  }
  return hipGetLastError();
}

hipError_t launch_max_cut(const GraphDev* g, int n, double* pv, uint64_t* pz, double* ov, uint64_t* oz,
                          hipStream_t st) {
  const int nb = gate_reduce_blocks(n);
  hipLaunchKernelGGL(k_max_cut, dim3(nb), dim3(256), 0, st, g, int64_t(1) << n, pv, pz);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, st, pv, pz, nb, ov, oz);
  return hipGetLastError();
}

}  // namespace qaoa
