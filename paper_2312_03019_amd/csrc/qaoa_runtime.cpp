// Host-side planning: graph encoding, qubit sets, pass schedule and the
// descriptor/table image uploaded for every run.
#include "qaoa_runtime.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <complex>
#include <numeric>

#include "../../include/qaoa.h"

namespace qaoa {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char* last_error() { return g_err.c_str(); }

// Table 1 encoding: one weight per unordered pair, stored with u < v.
int make_graph(int n, int num_edges, const int32_t* edges, const double* weights, HostGraph* out) {
  if (n < 1 || n > kMaxN) {
    set_error("n=%d out of range [1, %d]", n, kMaxN);
    return QAOA_EINVAL;
  }
  if (num_edges < 0 || (num_edges > 0 && !edges)) {
    set_error("invalid edge list");
    return QAOA_EINVAL;
  }
  std::vector<int> idx(num_edges);
  std::vector<std::pair<int, int>> e(num_edges);
  for (int k = 0; k < num_edges; ++k) {
    const int u = edges[2 * k], v = edges[2 * k + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) {
      set_error("edge %d = (%d, %d) invalid for n=%d", k, u, v, n);
      return QAOA_EINVAL;
    }
    if (weights && !std::isfinite(weights[k])) {
      set_error("weight %d is not finite", k);
      return QAOA_EINVAL;
    }
    e[k] = {std::min(u, v), std::max(u, v)};
    idx[k] = k;
  }
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return e[a] < e[b]; });
  HostGraph g;
  g.n = n;
  for (int k = 0; k < num_edges; ++k) {
    if (k > 0 && e[idx[k]] == e[idx[k - 1]]) {
      set_error("duplicate edge (%d, %d)", e[idx[k]].first, e[idx[k]].second);
      return QAOA_EINVAL;
    }
    g.eu.push_back(e[idx[k]].first);
    g.ev.push_back(e[idx[k]].second);
    if (weights) g.w.push_back(weights[idx[k]]);
  }
  *out = std::move(g);
  return QAOA_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t dev_graph_bytes(const HostGraph& hg) {
  const size_t m = hg.m();
  size_t b = align_up(sizeof(GraphDev), 256);
  b += align_up(4 * m, 256) * 2 + align_up(8 * m, 256);          // eu, ev, ew
  b += align_up(4 * 2 * m, 256) + align_up(8 * 2 * m, 256);      // nbr, nw
  return b;
}

void build_dev_graph_image(const HostGraph& hg, void* host_buf, void* dev_base) {
  const size_t m = hg.m();
  char* h = (char*)host_buf;
  char* d = (char*)dev_base;
  memset(h, 0, dev_graph_bytes(hg));
  size_t off = align_up(sizeof(GraphDev), 256);
  const size_t o_eu = off; off += align_up(4 * m, 256);
  const size_t o_ev = off; off += align_up(4 * m, 256);
  const size_t o_ew = off; off += align_up(8 * m, 256);
  const size_t o_nb = off; off += align_up(8 * m, 256);
  const size_t o_nw = off;
  GraphDev G;
  memset(&G, 0, sizeof G);
  G.n = hg.n;
  G.m = (int)m;
  G.weighted = hg.weighted() ? 1 : 0;
  std::vector<std::vector<std::pair<int, double>>> nb(hg.n);
  for (size_t e = 0; e < m; ++e) {
    const int u = hg.eu[e], v = hg.ev[e];
    G.adj[u] |= 1ull << v;
    G.adj[v] |= 1ull << u;
    G.upper[u] |= 1ull << v;
    nb[u].push_back({v, hg.weight((int)e)});
    nb[v].push_back({u, hg.weight((int)e)});
    ((int32_t*)(h + o_eu))[e] = u;
    ((int32_t*)(h + o_ev))[e] = v;
    ((double*)(h + o_ew))[e] = hg.weight((int)e);
  }
  int pos = 0;
  for (int v = 0; v < hg.n; ++v) {
    std::sort(nb[v].begin(), nb[v].end());
    G.off[v] = pos;
    for (auto& x : nb[v]) {
      ((int32_t*)(h + o_nb))[pos] = x.first;
      ((double*)(h + o_nw))[pos] = x.second;
      ++pos;
    }
  }
  for (int v = hg.n; v <= kMaxN + 1; ++v) G.off[v] = pos;
  G.eu = (const int32_t*)(d + o_eu);
  G.ev = (const int32_t*)(d + o_ev);
  G.ew = (const double*)(d + o_ew);
  G.nbr = (const int32_t*)(d + o_nb);
  G.nw = (const double*)(d + o_nw);
  memcpy(h, &G, sizeof G);
}

bool half_tile_rounds(int K, int logr, const PrecCfg& pc) {
  return K == pc.kmax && logr == pc.logr_max;
}

PrecCfg prec_cfg(int prec) {
  if (prec == QAOA_C64) return {1, kTileBitsC64, kLogRC64, kPassengerC64, 8};
  return {0, kTileBitsC128, kLogRC128, kPassengerC128, 16};
}

void tile_shape(int n, const PrecCfg& pc, int* K, int* logr) {
  *K = std::min(n, pc.kmax);
  *logr = std::min(pc.logr_max, *K);
}

// Rounds that put every tile bit of [sL, K) into registers once, starting
// from the top tile bits (so round 0 leaves the low tile bits on lanes and
// loads/stores coalesce).
// overlap: register windows of consecutive rounds share that many tile bits
// (one for full-width tiles, which transpose through half the LDS).
static void make_rounds(SetGeom& s, int sL, int logr, int overlap) {
  uint32_t want = 0, covered = 0;
  for (int t = sL; t < s.K; ++t) want |= 1u << t;
  int b = s.K - logr;
  s.nr = 0;
  for (;;) {
    if (b < 0) b = 0;
    int mask = 0;
    for (int k = 0; k < logr; ++k) {
      const int t = b + k;
      if (t >= sL && t < s.K && !((covered >> t) & 1u)) mask |= 1 << k;
    }
    s.rb[s.nr] = b;
    s.rxmask[s.nr] = mask;
    ++s.nr;
    covered |= (uint32_t)mask << b;
    if ((covered & want) == want) break;
    b -= logr - overlap;
  }
}

// Tile map of a set whose tile bit i is memory bit mem[i]; the tile index
// takes the remaining memory bits in ascending order.  False if the index
// map needs more than kMaxRuns runs.
static bool tile_map(int n, const std::vector<int>& mem, TileMap* m) {
  memset(m, 0, sizeof *m);
  uint64_t used = 0;
  for (size_t i = 0; i < mem.size(); ++i) {
    m->tpos[i] = (int8_t)mem[i];
    used |= 1ull << mem[i];
  }
  int k = 0, r = -1;
  for (int b = 0; b < n; ++b) {
    if ((used >> b) & 1ull) continue;
    m->gpos[k] = (int8_t)b;
    if (k == 0 || m->gpos[k - 1] != b - 1) {   // a new run starts at index bit k
      if (++r == kMaxRuns) return false;
      m->gshift[r] = (int8_t)(b - k);
    }
    m->gmask[r] |= 1ull << k;
    ++k;
  }
  return true;
}

// Memory layout of the low set (all tile bits are qubits [0, K)).  In round 0
// a thread's tile bits are [0, K - logr): lanes [0, 6), the wave index above
// them, the registers on top.  Placing the register bits right above the lane
// bits and the wave bits at the top makes each wave's loads cover one
// contiguous block of 64 * 2^logr amplitudes.
static std::vector<int> low_set_bits(int K, int logr) {
  const int t0 = K - logr, lanes = t0 < 6 ? t0 : 6, w = t0 - lanes;
  std::vector<int> mem(K);
  for (int i = 0; i < K; ++i) mem[i] = i < lanes ? i : (i < t0 ? i + logr : i - w);
  return mem;
}

// The qubits above the low set are dealt to the high sets in turn (set j
// takes K + j, K + j + mh, ...).  Each high tile then spreads over every
// part of the address range in similar measure; a set made of the top
// qubits alone sends a tile's 2^(K-L) runs to addresses 2^(n-k) apart
// across the whole state, which HBM serves markedly slower.
std::vector<SetGeom> make_sets(int n, const PrecCfg& pc) {
  int K, logr;
  tile_shape(n, pc, &K, &logr);
  const int ov = half_tile_rounds(K, logr, pc) ? 1 : 0;
  std::vector<SetGeom> sets;
  SetGeom a{};
  a.K = K; a.L = K; a.k = K;
  tile_map(n, low_set_bits(K, logr), &a.map);   // one run
  make_rounds(a, 0, logr, ov);
  sets.push_back(a);
  if (n <= pc.kmax) return sets;
  const int rem = n - K, cap = K - pc.passenger;
  const int mh = (rem + cap - 1) / cap;
  int start = K;
  for (int i = 0; i < mh; ++i) {
    const int k = (n - K) / mh + (i < (n - K) % mh ? 1 : 0);
    SetGeom s{};
    s.K = K; s.k = k; s.L = K - k;
    std::vector<int> mem;
    for (int t = 0; t < s.L; ++t) mem.push_back(t);
    for (int t = K + i; t < n; t += mh) mem.push_back(t);
    if (!tile_map(n, mem, &s.map)) {          // too many index runs: a contiguous block
      mem.resize(s.L);
      for (int t = start; t < start + k; ++t) mem.push_back(t);
      tile_map(n, mem, &s.map);
    }
    start += k;
    make_rounds(s, s.L, logr, ov);
    sets.push_back(s);
  }
  return sets;
}

// Layer l applies its qubit sets in forward order when l is even and in
// reverse order when l is odd, so the last set of one layer is the first of
// the next and both land in one pass (the cost phase of the next layer,
// diagonal, sits between the two mixer segments inside the tile).
//
// The first and last sets of the order carry two mixer segments and a cost
// phase in their (merged) passes, the others one segment.  With three or
// more sets the low set -- the largest -- goes second, so it is never a
// merged pass.
std::vector<PassSpec> make_schedule(int nsets, int p) {
  std::vector<int> order(nsets);
  for (int j = 0; j < nsets; ++j) order[j] = j;
  if (nsets >= 3) std::swap(order[0], order[1]);
  std::vector<PassSpec> passes;
  for (int l = 0; l < p; ++l) {
    for (int j = 0; j < nsets; ++j) {
      const int s = (l % 2 == 0) ? order[j] : order[nsets - 1 - j];
      if (!passes.empty() && passes.back().set == s) {
        passes.back().seg_layer.push_back(l);
        passes.back().seg_phase.push_back(j == 0);
      } else {
        PassSpec ps;
        ps.set = s;
        ps.seg_layer.push_back(l);
        ps.seg_phase.push_back(j == 0);
        passes.push_back(ps);
      }
    }
  }
  if (passes.empty()) {
    PassSpec ps;
    ps.set = order[0];
    passes.push_back(ps);
  }
  passes.front().gen = true;
  passes.back().expect = true;
  return passes;
}

// Memory bit carried by tile bit t.
static int tile_to_mem(const SetGeom& s, int t) { return s.map.tpos[t]; }

// Host tables of one round mapping (see SiteDesc): RT over the register
// vertices, and per thread F and G over the thread's set tile vertices.
static SiteDesc make_site(const SetGeom& s, int round, int logr, const HostGraph& hg, std::vector<double>& dtab) {
  SiteDesc sd;
  memset(&sd, 0, sizeof sd);
  const int b = s.rb[round];
  const int K = s.K;
  const int nth = 1 << (K - logr);
  int vtile[64];                // tile bit of each vertex, -1 outside the tile
  for (int v = 0; v < 64; ++v) vtile[v] = -1;
  for (int i = 0; i < K; ++i) vtile[tile_to_mem(s, i)] = i;
  for (int k = 0; k < logr; ++k) sd.q[k] = tile_to_mem(s, b + k);
  const int NR = 1 << logr;
  sd.rt_off = (int32_t)dtab.size();
  std::vector<double> rt(NR, 0.0);
  for (int e = 0; e < hg.m(); ++e) {
    const int iu = vtile[hg.eu[e]], iv = vtile[hg.ev[e]];
    if (iu < b || iu >= b + logr || iv < b || iv >= b + logr) continue;
    const int ku = iu - b, kv = iv - b;
    for (int J = 0; J < NR; ++J)
      if (((J >> ku) ^ (J >> kv)) & 1) rt[J] += hg.weight(e);
  }
  dtab.insert(dtab.end(), rt.begin(), rt.end());
  // in-tile edges only
  std::vector<int> ti, tj;
  std::vector<double> tw;
  for (int e = 0; e < hg.m(); ++e) {
    const int iu = vtile[hg.eu[e]], iv = vtile[hg.ev[e]];
    if (iu < 0 || iv < 0) continue;
    ti.push_back(iu);
    tj.push_back(iv);
    tw.push_back(hg.weight(e));
  }
  const uint32_t regmask = ((1u << logr) - 1u) << b;
  std::vector<double> F(nth, 0.0), G((size_t)logr * nth, 0.0);
  for (int tid = 0; tid < nth; ++tid) {
    const uint32_t tb = (tid & ((1u << b) - 1u)) | ((uint32_t)(tid >> b) << (b + logr));
    for (size_t e = 0; e < ti.size(); ++e) {
      const int su = (tb >> ti[e]) & 1, sv = (tb >> tj[e]) & 1;
      if (su != sv) F[tid] += tw[e];
      const bool ru = (regmask >> ti[e]) & 1u, rv = (regmask >> tj[e]) & 1u;
      if (ru && !rv) G[(size_t)(ti[e] - b) * nth + tid] += sv ? -tw[e] : tw[e];
      if (rv && !ru) G[(size_t)(tj[e] - b) * nth + tid] += su ? -tw[e] : tw[e];
    }
  }
  sd.f_off = (int32_t)dtab.size();
  dtab.insert(dtab.end(), F.begin(), F.end());
  sd.g_off = (int32_t)dtab.size();
  dtab.insert(dtab.end(), G.begin(), G.end());
  return sd;
}

// Which specialised forward kernel runs a pass (0 = the generic one).
// Compiled pass shapes exist for full-width tiles (K and LOGR at their
// maxima), whose rounds follow the half-tile pattern: [K-LOGR, K), then each
// LOGR-1 lower, the last clamped at 0.  Anything else takes the generic kernel.
// A four-round plain pass (the complex128 low set) is shaped only when it runs
// chunked (`chunked`, the first pass of a pair): whole, the generic full-LDS
// kernel is faster.  A complex64 two-round merged pass that runs chunked (the
// second pass of a pair, `chunked2`) gets its own occupancy.
static int forward_shape(const PassDesc& d, const PrecCfg& pc, int logr, const SegDesc* segs, bool chunked,
                         bool chunked2) {
  if (d.K != pc.kmax || logr != pc.logr_max || d.nrounds < 1 || d.nrounds > 4) return 0;
  for (int i = 0; i < d.nrounds; ++i)
    if (d.rb[i] != std::max(0, d.K - logr - i * (logr - 1))) return 0;
  const bool gen = d.flags & PF_GEN, ex = d.flags & PF_EXPECT, lam = d.flags & PF_WRITE_LAM;
  const bool ph0 = d.nseg >= 1 && segs[0].has_phase, ph1 = d.nseg >= 2 && segs[1].has_phase;
  int code = 0;
  if (d.nseg == 1 && gen && ph0 && !ex) code = kShapeFirst;
  else if (d.nseg == 1 && !gen && !ph0 && !ex && (d.nrounds <= 3 || chunked)) code = kShapeSingle;
  else if (d.nseg == 2 && !gen && !ph0 && ph1 && !ex && d.nrounds <= 3)
    code = chunked2 && pc.prec == 1 && d.nrounds == 2 ? kShapeMergedChunk : kShapeMerged;
  else if (d.nseg == 1 && !gen && !ph0 && ex) code = lam ? kShapeLastLam : kShapeLast;
  return code ? d.nrounds * 8 + code : 0;
}

// Backward shapes: the pass undoing the first forward pass (one segment with
// its phase, nothing stored), a single segment without phase, and a merged
// pass (phase in the second segment).  Same round condition as forward_shape.
static int backward_shape(const PassDesc& d, const PrecCfg& pc, int logr, const SegDesc* segs) {
  if (d.K != pc.kmax || logr != pc.logr_max || d.nrounds < 1 || d.nrounds > 4) return 0;
  for (int i = 0; i < d.nrounds; ++i)
    if (d.rb[i] != std::max(0, d.K - logr - i * (logr - 1))) return 0;
  const bool nost = d.flags & PF_NO_STORE;
  const bool ph0 = d.nseg >= 1 && segs[0].has_phase, ph1 = d.nseg >= 2 && segs[1].has_phase;
  int code = 0;
  if (d.nseg == 1 && ph0 && nost && d.nrounds <= 3) code = kShapeFirst;
  else if (d.nseg == 1 && !ph0 && !nost) code = kShapeSingle;
  else if (d.nseg == 2 && !ph0 && ph1 && !nost && d.nrounds <= 3) code = kShapeMerged;
  return code ? d.nrounds * 8 + code : 0;
}

// Chunked pass pairs: with three sets the schedule is a high set (the first
// pass), then per layer the low set and a high set X (sets 1 and 2 alternate).
// Each pair (low, X) is closed under chunks that fix qubits of the third set
// Y, so the pair can run chunk by chunk, the second pass finding its chunk in
// cache.  The top F qubits of Y are fixed, F from the chunk size (a launch map
// holds F + 1 runs).  Returns F (0 = no chunking) and the fixed memory bits of
// every pair.
int chunk_plan(const std::vector<SetGeom>& sets, const std::vector<PassSpec>& sched, int p, double state_bytes,
               size_t chunk_bytes, std::vector<uint64_t>* fixed_out) {
  fixed_out->clear();
  if (chunk_bytes == 0 || sets.size() != 3 || p < 1 || sched.size() != (size_t)(2 * p + 1)) return 0;
  int F = 0;
  while (F < kLaunchRuns - 1 && state_bytes / (double)((int64_t)1 << (F + 1)) >= (double)chunk_bytes) ++F;
  for (int i = 1; i <= p && F > 0; ++i) {
    const int x = sched[2 * i].set, y = 3 - x;
    if (sched[2 * i - 1].set != 0 || x < 1 || x > 2) return fixed_out->clear(), 0;
    F = std::min(F, sets[y].k);
  }
  if (F == 0) return 0;
  for (int i = 1; i <= p; ++i) {
    const SetGeom& Y = sets[3 - sched[2 * i].set];
    uint64_t fixed = 0;
    for (int t = Y.K - 1, c = 0; c < F; --t, ++c) fixed |= 1ull << Y.map.tpos[t];   // Y's top qubits
    fixed_out->push_back(fixed);
  }
  return F;
}

void build_run(const RunRequest& rq, RunImage* img) {
  const HostGraph& hg = *rq.hg;
  const int n = hg.n;
  const PrecCfg pc = prec_cfg(rq.prec);
  int K, logr;
  tile_shape(n, pc, &K, &logr);
  const std::vector<SetGeom> sets = make_sets(n, pc);
  const std::vector<PassSpec> sched = make_schedule((int)sets.size(), rq.p);
  const int64_t ntiles = (int64_t)1 << (n - K);
  const double state_bytes = (double)((int64_t)1 << n) * (double)pc.elem;
  const int NR = 1 << logr;

  *img = RunImage();
  img->chunk_bits = chunk_plan(sets, sched, rq.p, state_bytes, rq.chunk_bytes, &img->pair_fixed);
  // site tables depend only on (set, round): build each once
  std::vector<std::array<SiteDesc, 2>> sites(sets.size());
  for (size_t k = 0; k < sets.size(); ++k) {
    sites[k][0] = make_site(sets[k], 0, logr, hg, img->dtab);
    sites[k][1] = sets[k].nr > 1 ? make_site(sets[k], sets[k].nr - 1, logr, hg, img->dtab) : sites[k][0];
  }
  // Mixer scalars still to be applied; folded into the next cost phase, or
  // applied at the end of the last pass.
  std::complex<double> pending(1.0, 0.0);
  // parity of shifted-angle (mode 1) layers: the final state is complemented when odd
  int mode1_layers = 0;
  for (int l = 0; l < rq.p; ++l) mode1_layers += fabs(cos(rq.beta[l])) >= fabs(sin(rq.beta[l])) ? 0 : 1;
  int64_t part = 0;
  std::vector<int64_t> bwd_part(sched.size(), 0);
  std::vector<int> seg_begin(sched.size(), 0);
  int64_t fwd_part = 0;

  for (size_t i = 0; i < sched.size(); ++i) {
    const PassSpec& ps = sched[i];
    const SetGeom& s = sets[ps.set];
    PassDesc d;
    memset(&d, 0, sizeof d);
    d.n = n;
    d.K = s.K;
    d.nfree = n - s.K;
    d.map = s.map;
    for (int k = 0; k < logr; ++k) d.rbit0[k] = 1ull << s.map.tpos[s.rb[0] + k];
    d.nrounds = s.nr;
    for (int r = 0; r < s.nr; ++r) {
      d.rb[r] = s.rb[r];
      d.rxmask[r] = s.rxmask[r];
    }
    d.ntiles = ntiles;
    d.nseg = (int)ps.seg_layer.size();
    d.amp0 = pow(2.0, -0.5 * n);
    d.site[0] = sites[ps.set][0];
    d.site[1] = sites[ps.set][1];
    // segments; seg pointer patched at pack time (stored as index in `segs`)
    const int seg0 = (int)img->segs.size();
    seg_begin[i] = seg0;
    bool ph_even = false, ph_odd = false;
    int kq = 0;   // mixer qubits of this pass
    for (int r = 0; r < s.nr; ++r) kq += __builtin_popcount(s.rxmask[r]);
    for (int k = 0; k < d.nseg; ++k) {
      const int l = ps.seg_layer[k];
      SegDesc sg;
      memset(&sg, 0, sizeof sg);
      sg.gamma = rq.gamma[l];
      sg.beta = rq.beta[l];
      sg.cb = cos(rq.beta[l]);
      sg.sb = sin(rq.beta[l]);
      std::complex<double> sigma;
      if (fabs(sg.cb) >= fabs(sg.sb)) {
        sg.mode = 0;
        sg.coef = sg.sb / sg.cb;
        sigma = std::pow(std::complex<double>(sg.cb, 0.0), kq);
      } else {
        // exp(-i b X) = (-i X) exp(-i (b - pi/2) X): factored with t = tan(b - pi/2)
        // = -cot(b); the X on every mixer qubit is tracked as an index flip.
        sg.mode = 1;
        sg.coef = -sg.cb / sg.sb;
        sigma = std::pow(std::complex<double>(0.0, -sg.sb), kq);
      }
      sg.has_phase = ps.seg_phase[k];
      if (sg.has_phase) {
        sg.pre_re = pending.real();
        sg.pre_im = pending.imag();
        pending = 1.0;
      }
      pending *= sigma;
      if (sg.has_phase) {
        (k & 1 ? ph_odd : ph_even) = true;
        const SiteDesc& site = d.site[k & 1];
        sg.ph_off = (int32_t)(img->ctab.size() / 2);
        for (int J = 0; J < NR; ++J) {
          const double th = rq.gamma[l] * img->dtab[site.rt_off + J];
          img->ctab.push_back(cos(th));
          img->ctab.push_back(-sin(th));
        }
      }
      img->segs.push_back(sg);
    }
    d.segs = (const SegDesc*)(intptr_t)seg0;   // index until packed
    if (ps.expect && pending != std::complex<double>(1.0, 0.0)) {
      d.fscale_re = pending.real();
      d.fscale_im = pending.imag();
      pending = 1.0;
      d.flags |= PF_SCALE;
    }
    int flags = 0;
    if (ps.gen) flags |= PF_GEN;
    if (ps.expect) {
      flags |= PF_EXPECT;
      if (rq.grad) flags |= PF_WRITE_LAM;
    }
    int fflags = flags;
    if (ph_even || ps.expect) fflags |= PF_SITE0;
    if (ph_odd) fflags |= PF_SITE1;
    d.flags |= fflags;
    const bool chunked = img->chunk_bits > 0 && (i & 1) && i + 1 < sched.size();   // first pass of a pair
    const bool chunked2 = img->chunk_bits > 0 && i >= 2 && !(i & 1);               // second pass of a pair
    d.shape = forward_shape(d, pc, logr, img->segs.data() + seg0, chunked, chunked2);
    d.psi = rq.psi;
    d.lam = rq.lam;
    d.g = rq.g;
    d.tcut = (const double*)(intptr_t)((int64_t)ps.set * ntiles * kTileCutStride);   // offset until packed
    if (ps.expect) {
      fwd_part = part;
      d.part = (double*)(intptr_t)part;   // offset until packed
      part += 2 * ntiles;
    }
    d.tile_begin = 0;
    img->fwd.push_back(d);
    img->fwd_set.push_back(ps.set);
    double by = ps.gen ? state_bytes : 2.0 * state_bytes;
    if (ps.expect && rq.grad) by += state_bytes;
    img->pass_bytes.push_back(by);
    if (rq.grad && d.nseg > 0) {
      PassDesc b = d;
      int bf = 0;
      if (ph_even) bf |= PF_SITE0;
      if (ph_odd) bf |= PF_SITE1;
      if (ps.gen) bf |= PF_NO_STORE;
      b.flags = bf;
      bwd_part[i] = part;
      b.part = (double*)(intptr_t)part;
      part += 2 * (int64_t)d.nseg * ntiles;
      img->bwd.push_back(b);
      img->bwd_set.push_back(ps.set);
      img->bwd_bytes.push_back(ps.gen ? 2.0 * state_bytes : 4.0 * state_bytes);   // phi and lam
    }
  }
  img->complemented = (mode1_layers & 1) != 0;
  if (rq.grad) {
    // Scalars of the factored adjoint sweep (SegDesc): walk the passes and
    // segments in the order the sweep undoes them, with the rounds of each
    // segment in reverse forward order.
    std::complex<double> P(1.0, 0.0);
    for (int i = (int)sched.size() - 1; i >= 0; --i) {
      const PassSpec& ps = sched[i];
      const SetGeom& st = sets[ps.set];
      for (int k = (int)ps.seg_layer.size() - 1; k >= 0; --k) {
        SegDesc& sg = img->segs[seg_begin[i] + k];
        const double cb = sg.cb, sb = sg.sb;
        std::complex<double> q;
        if (fabs(cb) >= fabs(sb)) {
          sg.bcoef = -sb / cb;                          // (I + i tan(beta) X)
          q = std::complex<double>(cb, 0.0);
        } else {
          sg.bcoef = cb / sb;                           // (I - i cot(beta) X), then X
          q = std::complex<double>(0.0, sb);
        }
        for (int u = 0; u < st.nr; ++u) {
          const int r = (k & 1) ? u : st.nr - 1 - u;
          sg.bw[r] = std::norm(P);
          P *= std::pow(q, __builtin_popcount(st.rxmask[r]));
        }
        if (ps.seg_phase[k]) {
          sg.bwg = std::norm(P);
          sg.bpre_re = P.real();
          sg.bpre_im = P.imag();
          P = 1.0;
        }
      }
    }
    for (PassDesc& b : img->bwd) b.shape = backward_shape(b, pc, logr, img->segs.data() + (intptr_t)b.segs);
  }
  // backward launches run from the last forward pass to the first
  std::reverse(img->bwd.begin(), img->bwd.end());
  std::reverse(img->bwd_bytes.begin(), img->bwd_bytes.end());
  std::reverse(img->bwd_set.begin(), img->bwd_set.end());
  img->part_doubles = part;

  // outputs: [E, N, dgamma[p], dbeta[p]]
  // spans and outputs hold offsets (into part / out) until packed
  auto add_job = [&](int dst, double scale, const std::vector<Span>& sp) {
    ReduceJob j;
    memset(&j, 0, sizeof j);
    j.span_begin = (int32_t)img->spans.size();
    img->spans.insert(img->spans.end(), sp.begin(), sp.end());
    j.span_end = (int32_t)img->spans.size();
    j.out = (double*)(intptr_t)dst;
    j.scale = scale;
    img->jobs.push_back(j);
  };
  auto span = [&](int64_t off) { return Span{(const double*)(intptr_t)off, ntiles}; };
  add_job(0, 1.0, {span(fwd_part)});
  add_job(1, 1.0, {span(fwd_part + ntiles)});
  img->nout = 2;
  if (rq.grad) {
    for (int l = 0; l < rq.p; ++l) {
      std::vector<Span> sg, sb;
      for (size_t i = 0; i < sched.size(); ++i) {
        const PassSpec& ps = sched[i];
        for (size_t k = 0; k < ps.seg_layer.size(); ++k) {
          if (ps.seg_layer[k] != l) continue;
          sb.push_back(span(bwd_part[i] + (int64_t)(2 * k) * ntiles));
          if (ps.seg_phase[k]) sg.push_back(span(bwd_part[i] + (int64_t)(2 * k + 1) * ntiles));
        }
      }
      add_job(2 + l, 2.0, sg);
      add_job(2 + rq.p + l, 2.0, sb);
    }
    img->nout = 2 + 2 * rq.p;
  }
}

ImageLayout image_layout(const RunImage& img, int prec) {
  const PrecCfg pc = prec_cfg(prec);
  ImageLayout L;
  size_t off = 0;
  L.off_segs = off; off = align_up(off + img.segs.size() * sizeof(SegDesc), 256);
  L.off_dtab = off; off = align_up(off + img.dtab.size() * sizeof(double), 256);
  L.off_ctab = off; off = align_up(off + (img.ctab.size() / 2) * pc.elem, 256);
  L.off_jobs = off; off = align_up(off + img.jobs.size() * sizeof(ReduceJob), 256);
  L.off_spans = off; off = align_up(off + img.spans.size() * sizeof(Span), 256);
  L.off_fwd = off; off = align_up(off + img.fwd.size() * sizeof(PassDesc), 256);
  L.off_bwd = off; off = align_up(off + img.bwd.size() * sizeof(PassDesc), 256);
  L.total = off;
  return L;
}

LaunchMap chunk_launch_map(const TileMap& map, int nfree, uint64_t fixed_mem, int64_t k) {
  LaunchMap m{};
  int j = 0, t = 0, r = -1;
  for (int b = 0; b < 64 && j < 64; ++b) {   // fixed memory bits in ascending order -> bits of k
    if (!((fixed_mem >> b) & 1ull)) continue;
    for (int i = 0; i < nfree; ++i)
      if (map.gpos[i] == b) m.gfix |= (uint64_t)((k >> j) & 1) << i;
    ++j;
  }
  for (int i = 0; i < nfree; ++i) {           // free index bits: local bit t -> index bit i
    if ((fixed_mem >> map.gpos[i]) & 1ull) continue;
    if (r < 0 || (i - t) != m.shift[r]) {      // a skipped (fixed) bit starts a new run
      ++r;
      m.shift[r] = (int8_t)(i - t);
    }
    m.mask[r] |= 1ull << t;
    ++t;
  }
  m.nruns = r + 1;
  return m;
}

size_t tile_cut_doubles(int n, int prec) {
  const PrecCfg pc = prec_cfg(prec);
  int K, logr;
  tile_shape(n, pc, &K, &logr);
  return make_sets(n, pc).size() * ((size_t)1 << (n - K)) * kTileCutStride;
}

hipError_t launch_tile_cuts(int n, int prec, const GraphDev* g, double* tcut, hipStream_t st) {
  const PrecCfg pc = prec_cfg(prec);
  int K, logr;
  tile_shape(n, pc, &K, &logr);
  const int64_t ntiles = (int64_t)1 << (n - K);
  const std::vector<SetGeom> sets = make_sets(n, pc);
  for (size_t k = 0; k < sets.size(); ++k) {
    hipError_t e = launch_tile_cut(g, sets[k].K, n - sets[k].K, sets[k].map, ntiles,
                                   tcut + (int64_t)k * ntiles * kTileCutStride, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void pack_run(RunImage& img, const ImageLayout& lay, int prec, void* host_buf, char* dev_region, double* part,
              double* out, const double* tcut) {
  char* h = (char*)host_buf;
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) memcpy(h + off, src, bytes);
  };
  put(lay.off_segs, img.segs.data(), img.segs.size() * sizeof(SegDesc));
  put(lay.off_dtab, img.dtab.data(), img.dtab.size() * sizeof(double));
  const size_t nc = img.ctab.size() / 2;
  if (prec == QAOA_C64) {
    float* c = (float*)(h + lay.off_ctab);
    for (size_t i = 0; i < 2 * nc; ++i) c[i] = (float)img.ctab[i];
  } else {
    put(lay.off_ctab, img.ctab.data(), 2 * nc * sizeof(double));
  }
  for (auto& j : img.jobs) j.out = out + (intptr_t)j.out;
  for (auto& sp : img.spans) sp.ptr = part + (intptr_t)sp.ptr;
  put(lay.off_jobs, img.jobs.data(), img.jobs.size() * sizeof(ReduceJob));
  put(lay.off_spans, img.spans.data(), img.spans.size() * sizeof(Span));
  auto patch = [&](PassDesc& d) {
    const intptr_t seg0 = (intptr_t)d.segs;
    d.segs = (const SegDesc*)(dev_region + lay.off_segs) + seg0;
    d.dtab = (const double*)(dev_region + lay.off_dtab);
    d.ctab = (const void*)(dev_region + lay.off_ctab);
    d.part = part + (intptr_t)d.part;
    d.tcut = tcut + (intptr_t)d.tcut;
  };
  for (auto& d : img.fwd) patch(d);
  for (auto& d : img.bwd) patch(d);
  put(lay.off_fwd, img.fwd.data(), img.fwd.size() * sizeof(PassDesc));
  put(lay.off_bwd, img.bwd.data(), img.bwd.size() * sizeof(PassDesc));
}

}  // namespace qaoa
