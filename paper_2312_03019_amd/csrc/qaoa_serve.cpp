// Serving: continuous batching of <C> and gradient requests on one GPU.
//
// One scheduler thread owns the device side.  Requests queue in FIFO order
// and are admitted while a slot is free and their device footprint (state,
// adjoint vector, graph, descriptors, partial sums) fits in a sub-allocated
// arena of the HBM budget.  Every step advances each active request by one
// HBM pass; all of a step's forward passes go out in one launch (and all
// backward passes in a second), each workgroup finding its request's
// descriptor by its tile range.  A request whose last pass is in the step
// also gets its deterministic reduction and the copy of its results.  Two
// steps may be in flight; admission, retirement and the host bookkeeping
// of one step overlap the kernels of the previous one.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/qaoa.h"
#include "qaoa_runtime.h"

using namespace qaoa;

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// First-fit sub-allocator over one device allocation, coalescing on release.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  void init(char* b, size_t s) {
    base = b;
    size = s;
    free_.clear();
    free_[0] = s;
    used = 0;
  }
  bool alloc(size_t sz, size_t* off) {
    sz = align256(sz);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= sz) {
        *off = it->first;
        const size_t rest = it->second - sz;
        const size_t roff = it->first + sz;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used += sz;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t sz) {
    sz = align256(sz);
    used -= sz;
    auto it = free_.emplace(off, sz).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct SReq {
  uint64_t ticket = 0;
  HostGraph hg;
  int p = 0;
  std::vector<double> gamma, beta;
  bool grad = false;
  bool small = false;   // whole request in one workgroup (state in LDS), no HBM passes
  double t_arrival = 0, t_admit = -1, t_done = -1;
  int status = QAOA_EPENDING;
  double expect = 0, norm = 0;
  std::vector<double> dg, db;
  bool canceled = false;
  bool finished = false;
  // device side (scheduler thread)
  RunImage img;
  ImageLayout lay{};
  size_t graph_bytes = 0, sz_psi = 0, sz_lam = 0, sz_aux = 0, tcut_doubles = 0;
  size_t off_psi = 0, off_lam = 0, off_aux = 0;
  bool has_mem = false;
  int slot = -1;
  int next = 0, nlaunch = 0, nf = 0;
  int64_t ntiles = 0;
  int nthreads = 0, logr = 0;
  bool uploaded = false;
  bool reduce_issued = false;
  char* dev_aux = nullptr;
  size_t footprint() const { return align256(sz_psi) + align256(sz_lam) + align256(sz_aux); }
};

constexpr int kServeMaxP = 1024;

}  // namespace

struct qaoa_server {
  int prec = QAOA_C64;
  int max_slots = 1;
  size_t budget = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  char* arena_mem = nullptr;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<SReq*> queue;
  std::vector<SReq*> active;
  std::unordered_map<uint64_t, SReq*> all;
  uint64_t next_ticket = 1;
  std::vector<int> free_slots;
  bool stop = false;
  std::thread th;
  std::chrono::steady_clock::time_point t0;
  // statistics over completed requests
  std::vector<double> lat;
  double t_first = -1, t_last = -1;
  // per-parity staging
  char* hstage[2] = {nullptr, nullptr};
  size_t hstage_cap[2] = {0, 0};
  char* dstage[2] = {nullptr, nullptr};
  size_t dstage_cap[2] = {0, 0};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool inflight[2] = {false, false};
  std::vector<SReq*> finishers[2];
  double* host_out = nullptr;   // pinned, max_slots * out_stride
  int out_stride = 0;
  int dev_error = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void run();
  int step_once(uint64_t step);
  void complete(int par);
  void release_mem(SReq* r);
  void finish_locked(SReq* r, int status);
};

void qaoa_server::release_mem(SReq* r) {
  if (!r->has_mem) return;
  if (r->sz_psi) arena.release(r->off_psi, r->sz_psi);
  if (r->sz_lam) arena.release(r->off_lam, r->sz_lam);
  arena.release(r->off_aux, r->sz_aux);
  r->has_mem = false;
}

void qaoa_server::finish_locked(SReq* r, int status) {
  r->status = status;
  r->finished = true;
  r->t_done = now();
  if (status == QAOA_OK) {
    lat.push_back(r->t_done - r->t_arrival);
    if (t_first < 0 || r->t_arrival < t_first) t_first = r->t_arrival;
    t_last = std::max(t_last, r->t_done);
  }
  if (r->slot >= 0) {
    free_slots.push_back(r->slot);
    r->slot = -1;
  }
  cv_done.notify_all();
}

// Results of the requests whose final work was in step parity `par`.
void qaoa_server::complete(int par) {
  (void)hipEventSynchronize(ev[par]);
  inflight[par] = false;
  std::lock_guard<std::mutex> lk(mu);
  for (SReq* r : finishers[par]) {
    const double* o = host_out + (size_t)r->slot * out_stride;
    r->expect = o[0];
    r->norm = o[1];
    if (r->grad) {
      r->dg.assign(o + 2, o + 2 + r->p);
      r->db.assign(o + 2 + r->p, o + 2 + 2 * r->p);
    }
    finish_locked(r, r->canceled ? QAOA_ECANCELED : (dev_error ? QAOA_EDEVICE : QAOA_OK));
  }
  finishers[par].clear();
}

static int grow_pinned(char** p, size_t* cap, size_t need) {
  if (*cap >= need) return 0;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  const size_t sz = std::max<size_t>(need + need / 2, 1 << 16);
  if (hipHostMalloc((void**)p, sz, hipHostMallocDefault) != hipSuccess) {
    *cap = 0;
    return -1;
  }
  *cap = sz;
  return 0;
}

static int grow_dev(char** p, size_t* cap, size_t need) {
  if (*cap >= need) return 0;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  const size_t sz = std::max<size_t>(need + need / 2, 1 << 16);
  if (hipMalloc((void**)p, sz) != hipSuccess) {
    *cap = 0;
    return -1;
  }
  *cap = sz;
  return 0;
}

// Admit, launch one step, retire.  Returns 1 if work was launched, 0 if
// there was nothing to launch, <0 on a device error.
int qaoa_server::step_once(uint64_t step) {
  const int par = (int)(step & 1);
  if (inflight[par]) complete(par);

  std::vector<SReq*> fresh, act;
  {
    std::lock_guard<std::mutex> lk(mu);
    // retire cancelled requests that have no reduction in flight
    for (size_t i = 0; i < active.size();) {
      SReq* r = active[i];
      if (r->canceled && !r->reduce_issued) {
        release_mem(r);
        finish_locked(r, QAOA_ECANCELED);
        active.erase(active.begin() + i);
      } else {
        ++i;
      }
    }
    while (!queue.empty() && (int)active.size() < max_slots && !free_slots.empty()) {
      SReq* r = queue.front();
      size_t a = 0, b = 0, c = 0;
      if (r->sz_psi && !arena.alloc(r->sz_psi, &a)) break;
      if (r->sz_lam && !arena.alloc(r->sz_lam, &b)) {
        if (r->sz_psi) arena.release(a, r->sz_psi);
        break;
      }
      if (!arena.alloc(r->sz_aux, &c)) {
        if (r->sz_psi) arena.release(a, r->sz_psi);
        if (r->sz_lam) arena.release(b, r->sz_lam);
        break;
      }
      r->off_psi = a;
      r->off_lam = b;
      r->off_aux = c;
      r->has_mem = true;
      r->slot = free_slots.back();
      free_slots.pop_back();
      r->t_admit = now();
      queue.pop_front();
      active.push_back(r);
      fresh.push_back(r);
    }
    for (SReq* r : active)
      if (!r->canceled && !r->reduce_issued) act.push_back(r);
  }
  if (act.empty()) return 0;

  // ---- host staging: new requests' graph + run images, then step descriptors
  size_t hneed = 0;
  for (SReq* r : fresh)
    hneed += align256(r->graph_bytes) + (r->small ? align256((2 * (size_t)r->p + 2) * sizeof(double))
                                                    : align256(r->lay.total));
  struct Group {
    bool bwd;
    int logr, nthreads, shape;
    std::vector<PassDesc> d;
    int64_t tiles;
  };
  std::vector<Group> groups;
  std::vector<SReq*> fin;
  for (SReq* r : act) {
    if (r->next >= r->nlaunch) continue;
    const bool bwd = r->next >= r->nf;
    PassDesc d = bwd ? r->img.bwd[r->next - r->nf] : r->img.fwd[r->next];
    const int shape = d.shape;
    Group* g = nullptr;
    for (auto& x : groups)
      if (x.bwd == bwd && x.logr == r->logr && x.nthreads == r->nthreads && x.shape == shape) g = &x;
    if (!g) {
      groups.push_back(Group{bwd, r->logr, r->nthreads, shape, {}, 0});
      g = &groups.back();
    }
    d.tile_begin = g->tiles;
    g->tiles += d.ntiles;
    g->d.push_back(d);
  }
  size_t nsmall = 0;
  for (SReq* r : fresh) nsmall += r->small ? 1 : 0;
  size_t dneed = align256(nsmall * sizeof(SmallDesc));
  for (auto& g : groups) dneed += align256(g.d.size() * sizeof(PassDesc));
  if (grow_pinned(&hstage[par], &hstage_cap[par], hneed + dneed + 256) ||
      grow_dev(&dstage[par], &dstage_cap[par], dneed + 256))
    return QAOA_ENOMEM;

  size_t hoff = 0;
  std::vector<SmallDesc> smalls;
  std::vector<SReq*> small_reqs;
  for (SReq* r : fresh) {
    if (r->small) {
      // graph image, then gamma, beta and the two outputs
      char* aux = arena.base + r->off_aux;
      r->dev_aux = aux;
      build_dev_graph_image(r->hg, hstage[par] + hoff, aux);
      double* hg = (double*)(hstage[par] + hoff + align256(r->graph_bytes));
      std::copy(r->gamma.begin(), r->gamma.end(), hg);
      std::copy(r->beta.begin(), r->beta.end(), hg + r->p);
      hg[2 * r->p] = hg[2 * r->p + 1] = 0.0;
      double* dg = (double*)(aux + align256(r->graph_bytes));
      const size_t bytes = align256(r->graph_bytes) + (2 * (size_t)r->p + 2) * sizeof(double);
      if (hipMemcpyAsync(aux, hstage[par] + hoff, bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
        return QAOA_EDEVICE;
      SmallDesc sd;
      sd.g = (const GraphDev*)aux;
      sd.gamma = dg;
      sd.beta = dg + r->p;
      sd.out = dg + 2 * r->p;
      sd.n = r->hg.n;
      sd.p = r->p;
      smalls.push_back(sd);
      small_reqs.push_back(r);
      hoff += align256(r->graph_bytes) + align256((2 * (size_t)r->p + 2) * sizeof(double));
      r->uploaded = true;
      continue;
    }
    char* psi = arena.base + r->off_psi;
    char* lam = r->sz_lam ? arena.base + r->off_lam : nullptr;
    char* aux = arena.base + r->off_aux;
    r->dev_aux = aux;
    char* dgraph = aux;
    char* dimg = aux + align256(r->graph_bytes);
    double* dpart = (double*)(dimg + align256(r->lay.total));
    double* dout = dpart + r->img.part_doubles;
    double* dtcut = (double*)((char*)dpart + align256((r->img.part_doubles + r->img.nout) * sizeof(double)));
    build_dev_graph_image(r->hg, hstage[par] + hoff, dgraph);
    for (auto& d : r->img.fwd) {
      d.psi = psi;
      d.lam = lam;
      d.g = (const GraphDev*)dgraph;
    }
    for (auto& d : r->img.bwd) {
      d.psi = psi;
      d.lam = lam;
      d.g = (const GraphDev*)dgraph;
    }
    pack_run(r->img, r->lay, prec, hstage[par] + hoff + align256(r->graph_bytes), dimg, dpart, dout, dtcut);
    if (hipMemcpyAsync(dgraph, hstage[par] + hoff, align256(r->graph_bytes) + r->lay.total, hipMemcpyHostToDevice,
                       stream) != hipSuccess)
      return QAOA_EDEVICE;
    if (launch_tile_cuts(r->hg.n, prec, (const GraphDev*)dgraph, dtcut, stream) != hipSuccess) return QAOA_EDEVICE;
    hoff += align256(r->graph_bytes) + align256(r->lay.total);
    r->uploaded = true;
  }
  // descriptors reference the packed (device-pointer) versions: rebuild groups now that
  // fresh requests are packed
  groups.clear();
  for (SReq* r : act) {
    if (r->next >= r->nlaunch) continue;
    const bool bwd = r->next >= r->nf;
    PassDesc d = bwd ? r->img.bwd[r->next - r->nf] : r->img.fwd[r->next];
    const int shape = d.shape;
    Group* g = nullptr;
    for (auto& x : groups)
      if (x.bwd == bwd && x.logr == r->logr && x.nthreads == r->nthreads && x.shape == shape) g = &x;
    if (!g) {
      groups.push_back(Group{bwd, r->logr, r->nthreads, shape, {}, 0});
      g = &groups.back();
    }
    d.tile_begin = g->tiles;
    g->tiles += d.ntiles;
    g->d.push_back(d);
    ++r->next;
    if (r->next == r->nlaunch) fin.push_back(r);
  }
  size_t doff = 0;
  const size_t small_off = doff;
  if (!smalls.empty()) {
    memcpy(hstage[par] + hoff + doff, smalls.data(), smalls.size() * sizeof(SmallDesc));
    doff += align256(smalls.size() * sizeof(SmallDesc));
  }
  std::vector<size_t> goff;
  for (auto& g : groups) {
    memcpy(hstage[par] + hoff + doff, g.d.data(), g.d.size() * sizeof(PassDesc));
    goff.push_back(doff);
    doff += align256(g.d.size() * sizeof(PassDesc));
  }
  if (doff && hipMemcpyAsync(dstage[par], hstage[par] + hoff, doff, hipMemcpyHostToDevice, stream) != hipSuccess)
    return QAOA_EDEVICE;
  for (size_t i = 0; i < groups.size(); ++i) {
    const Group& g = groups[i];
    if (launch_pass(prec == QAOA_C64 ? 1 : 0, g.bwd, g.logr, g.shape, (const PassDesc*)(dstage[par] + goff[i]),
                    (int)g.d.size(), g.tiles, g.nthreads, stream) != hipSuccess)
      return QAOA_EDEVICE;
  }
  if (!smalls.empty()) {
    if (launch_small(prec == QAOA_C64 ? 1 : 0, (const SmallDesc*)(dstage[par] + small_off), (int)smalls.size(),
                     stream) != hipSuccess)
      return QAOA_EDEVICE;
    for (size_t i = 0; i < small_reqs.size(); ++i) {
      SReq* r = small_reqs[i];
      if (hipMemcpyAsync(host_out + (size_t)r->slot * out_stride, smalls[i].out, 2 * sizeof(double),
                         hipMemcpyDeviceToHost, stream) != hipSuccess)
        return QAOA_EDEVICE;
      r->reduce_issued = true;
    }
  }
  for (SReq* r : fin) {
    char* dimg = r->dev_aux + align256(r->graph_bytes);
    double* dout = (double*)(dimg + align256(r->lay.total)) + r->img.part_doubles;
    if (launch_reduce((const ReduceJob*)(dimg + r->lay.off_jobs), (const Span*)(dimg + r->lay.off_spans),
                      (int)r->img.jobs.size(), stream) != hipSuccess)
      return QAOA_EDEVICE;
    if (hipMemcpyAsync(host_out + (size_t)r->slot * out_stride, dout, r->img.nout * sizeof(double),
                       hipMemcpyDeviceToHost, stream) != hipSuccess)
      return QAOA_EDEVICE;
    r->reduce_issued = true;
  }
  if (hipEventRecord(ev[par], stream) != hipSuccess) return QAOA_EDEVICE;
  inflight[par] = true;
  {
    // Later users of this memory are ordered after these kernels on the one
    // stream, so finished requests give their memory back immediately.
    std::lock_guard<std::mutex> lk(mu);
    fin.insert(fin.end(), small_reqs.begin(), small_reqs.end());
    for (SReq* r : fin) {
      release_mem(r);
      active.erase(std::find(active.begin(), active.end(), r));
    }
    finishers[par] = fin;
  }
  return 1;
}

void qaoa_server::run() {
  (void)hipSetDevice(device);
  uint64_t step = 0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_sched.wait(lk, [&] { return stop || !queue.empty() || !active.empty() || inflight[0] || inflight[1]; });
      if (stop) break;
    }
    int rc = dev_error ? 0 : step_once(step);
    if (rc < 0) {
      std::lock_guard<std::mutex> lk(mu);
      dev_error = rc;
      for (SReq* r : active) {
        release_mem(r);
        finish_locked(r, rc);
      }
      active.clear();
      for (SReq* r : queue) finish_locked(r, rc);
      queue.clear();
    }
    if (rc == 1) {
      ++step;
      continue;
    }
    // nothing launched: drain the older in-flight step, else wait for work
    const int a = (int)(step & 1), b = a ^ 1;
    if (inflight[b]) complete(b);
    else if (inflight[a]) complete(a);
    else {
      std::unique_lock<std::mutex> lk(mu);
      bool launchable = false;
      for (SReq* r : active)
        if (!r->canceled && r->next < r->nlaunch) launchable = true;
      if (!launchable && queue.empty())
        cv_sched.wait_for(lk, std::chrono::milliseconds(50));
      else if (!launchable && !queue.empty())
        cv_sched.wait_for(lk, std::chrono::milliseconds(1));
    }
  }
  for (int k = 0; k < 2; ++k)
    if (inflight[k]) complete(k);
}

extern "C" {

int qaoa_serve_create(size_t hbm_budget_bytes, int max_slots, int prec, qaoa_server** out) {
  if (!out || max_slots < 1 || max_slots > 4096 || hbm_budget_bytes < (1u << 20) ||
      (prec != QAOA_C64 && prec != QAOA_C128)) {
    set_error("invalid server arguments");
    return QAOA_EINVAL;
  }
  *out = nullptr;
  qaoa_server* s = new qaoa_server();
  s->prec = prec;
  s->max_slots = max_slots;
  s->budget = hbm_budget_bytes & ~(size_t)255;
  s->t0 = std::chrono::steady_clock::now();
  s->out_stride = 2 + 2 * kServeMaxP;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void**)&s->arena_mem, s->budget);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&s->host_out, (size_t)max_slots * s->out_stride * sizeof(double), hipHostMallocDefault);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    set_error("server setup: %s", hipGetErrorString(e));
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->host_out) (void)hipHostFree(s->host_out);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return e == hipErrorOutOfMemory ? QAOA_ENOMEM : QAOA_EDEVICE;
  }
  s->arena.init(s->arena_mem, s->budget);
  for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->th = std::thread([s] { s->run(); });
  *out = s;
  return QAOA_OK;
}

int qaoa_serve_submit(qaoa_server* s, const qaoa_request* q, double arrival_time, uint64_t* ticket) {
  if (!s || !q || !ticket) {
    set_error("invalid arguments");
    return QAOA_EINVAL;
  }
  if (q->p < 0 || q->p > kServeMaxP || (q->p > 0 && (!q->gamma || !q->beta))) {
    set_error("p must be in [0, %d] with gamma/beta arrays", kServeMaxP);
    return QAOA_EINVAL;
  }
  for (int l = 0; l < q->p; ++l)
    if (!std::isfinite(q->gamma[l]) || !std::isfinite(q->beta[l])) {
      set_error("angle %d is not finite", l);
      return QAOA_EINVAL;
    }
  SReq* r = new SReq();
  int rc = make_graph(q->n, q->num_edges, q->edges, q->weights, &r->hg);
  if (rc) {
    delete r;
    return rc;
  }
  r->p = q->p;
  r->gamma.assign(q->gamma, q->gamma + q->p);
  r->beta.assign(q->beta, q->beta + q->p);
  r->grad = q->want_grad != 0;
  const PrecCfg pc = prec_cfg(s->prec);
  r->small = !r->grad && r->hg.n <= (s->prec == QAOA_C64 ? kSmallMaxNC64 : kSmallMaxNC128);
  if (r->small) {
    r->graph_bytes = dev_graph_bytes(r->hg);
    r->sz_aux = align256(r->graph_bytes) + align256((2 * (size_t)r->p + 2) * sizeof(double));
    r->nf = r->nlaunch = 0;
  }
  RunRequest rq{&r->hg, s->prec, r->p, r->gamma.data(), r->beta.data(), r->grad, nullptr, nullptr, nullptr};
  if (!r->small) {
    build_run(rq, &r->img);
    r->lay = image_layout(r->img, s->prec);
    r->graph_bytes = dev_graph_bytes(r->hg);
    r->sz_psi = ((size_t)1 << r->hg.n) * pc.elem;
    r->sz_lam = r->grad ? r->sz_psi : 0;
    r->tcut_doubles = tile_cut_doubles(r->hg.n, s->prec);
    r->sz_aux = align256(r->graph_bytes) + align256(r->lay.total) +
                align256((r->img.part_doubles + r->img.nout) * sizeof(double)) +
                align256(r->tcut_doubles * sizeof(double));
    r->nf = (int)r->img.fwd.size();
    r->nlaunch = r->nf + (int)r->img.bwd.size();
    int K;
    tile_shape(r->hg.n, pc, &K, &r->logr);
    r->nthreads = 1 << (K - r->logr);
    r->ntiles = (int64_t)1 << (r->hg.n - K);
  }
  if (r->footprint() > s->budget) {
    set_error("request needs %zu bytes, budget is %zu", r->footprint(), s->budget);
    delete r;
    return QAOA_ENOMEM;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->dev_error) {
    delete r;
    set_error("server stopped after a device error");
    return QAOA_EDEVICE;
  }
  r->ticket = s->next_ticket++;
  r->t_arrival = arrival_time >= 0 ? arrival_time : s->now();
  s->all[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_sched.notify_one();
  return QAOA_OK;
}

static int collect_locked(qaoa_server* s, SReq* r, qaoa_result* out) {
  const int st = r->status;
  if (out) {
    out->status = st;
    out->expect = r->expect;
    out->norm = r->norm;
    out->t_arrival = r->t_arrival;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    if (st == QAOA_OK && r->grad) {
      if (out->dgamma) std::copy(r->dg.begin(), r->dg.end(), out->dgamma);
      if (out->dbeta) std::copy(r->db.begin(), r->db.end(), out->dbeta);
    }
  }
  s->all.erase(r->ticket);
  delete r;
  return st;
}

int qaoa_serve_poll(qaoa_server* s, uint64_t ticket, qaoa_result* out) {
  if (!s) return QAOA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    set_error("unknown ticket");
    return QAOA_EINVAL;
  }
  if (!it->second->finished) return QAOA_EPENDING;
  return collect_locked(s, it->second, out);
}

int qaoa_serve_wait(qaoa_server* s, uint64_t ticket, qaoa_result* out, double timeout_s) {
  if (!s) return QAOA_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto pred = [&] {
    auto it = s->all.find(ticket);
    return it == s->all.end() || it->second->finished;
  };
  if (timeout_s < 0) s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return QAOA_EPENDING;
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    set_error("unknown ticket");
    return QAOA_EINVAL;
  }
  return collect_locked(s, it->second, out);
}

int qaoa_serve_cancel(qaoa_server* s, uint64_t ticket) {
  if (!s) return QAOA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    set_error("unknown ticket");
    return QAOA_EINVAL;
  }
  SReq* r = it->second;
  if (r->finished) return QAOA_OK;
  r->canceled = true;
  auto q = std::find(s->queue.begin(), s->queue.end(), r);
  if (q != s->queue.end()) {
    s->queue.erase(q);
    s->finish_locked(r, QAOA_ECANCELED);
  }
  s->cv_sched.notify_one();
  return QAOA_OK;
}

int qaoa_serve_stats(qaoa_server* s, double* rps, double* p50, double* p99) {
  if (!s) return QAOA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->lat;
  const size_t n = v.size();
  if (rps) *rps = (n && s->t_last > s->t_first) ? n / (s->t_last - s->t_first) : 0.0;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) {
    if (!n) return 0.0;
    const size_t k = (size_t)std::min<double>(n - 1, std::ceil(q * n) - 1);
    return v[k];
  };
  if (p50) *p50 = pct(0.50);
  if (p99) *p99 = pct(0.99);
  return QAOA_OK;
}

double qaoa_serve_clock(qaoa_server* s) { return s ? s->now() : 0.0; }

int qaoa_serve_destroy(qaoa_server* s) {
  if (!s) return QAOA_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
  }
  s->th.join();
  (void)hipStreamSynchronize(s->stream);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (SReq* r : s->active) {
      s->release_mem(r);
      if (!r->finished) s->finish_locked(r, QAOA_ECANCELED);
    }
    for (SReq* r : s->queue)
      if (!r->finished) s->finish_locked(r, QAOA_ECANCELED);
    for (auto& kv : s->all) delete kv.second;
    s->all.clear();
  }
  for (int k = 0; k < 2; ++k) {
    if (s->hstage[k]) (void)hipHostFree(s->hstage[k]);
    if (s->dstage[k]) (void)hipFree(s->dstage[k]);
    if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
  }
  if (s->host_out) (void)hipHostFree(s->host_out);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return QAOA_OK;
}

}  // extern "C"
