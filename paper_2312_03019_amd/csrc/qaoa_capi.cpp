// C ABI: simulator contexts (qaoa_create ... qaoa_destroy).
#include <math.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/qaoa.h"
#include "qaoa_runtime.h"

namespace qaoa {
const char* last_error();
}

using namespace qaoa;

#define HIPCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));               \
      return e_ == hipErrorOutOfMemory ? QAOA_ENOMEM : QAOA_EDEVICE;          \
    }                                                                         \
  } while (0)

struct qaoa_ctx {
  HostGraph hg;
  int prec = QAOA_C128;
  int device = 0;
  bool dev_ready = false;
  hipStream_t stream = nullptr;
  bool stream_bound = false;
  void* psi = nullptr;
  bool own_psi = false;
  size_t state_bytes = 0;
  void* lam = nullptr;
  void* dgraph = nullptr;
  double* dtcut = nullptr;   // per-tile cut tables of the plan's qubit sets
  char* dev_img = nullptr;
  size_t dev_img_cap = 0;
  double* dev_part = nullptr;
  size_t dev_part_cap = 0;
  double* dev_out = nullptr;
  size_t dev_out_cap = 0;
  char* host_img = nullptr;
  size_t host_img_cap = 0;
  double* host_out = nullptr;
  size_t host_out_cap = 0;
  hipEvent_t upload_done = nullptr;
  // chunked pass pairs: the second pass of each chunk runs on stream2
  // (defaults set by precision in qaoa_create)
  size_t chunk_bytes = 0;
  size_t chunk_min_state = 0;   // chunking only for states at least this large
  int chunk_streams = 2;               // 2: P2 chunks on one extra stream; 3: on two; 4: P1 on two as well
  hipStream_t xs[3] = {nullptr, nullptr, nullptr};   // the device's library streams 1..3
  std::vector<hipEvent_t> chunk_ev;
  hipEvent_t join_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool upload_pending = false;
  bool have_state = false;
  bool have_expect = false;
  bool complemented = false;   // the state buffer holds psi(~z) (reversed order)
  bool profiling = false;
  std::vector<hipEvent_t> ev;
  int ntimed = 0;
  std::vector<double> pass_bytes;
  std::vector<int> pass_set, pass_shape;   // per pass of the last run (forward, then backward)
  int pass_logr = 0, pass_nfwd = 0;
  std::atomic<int> busy{0};
};

namespace {

struct Busy {
  qaoa_ctx* c;
  bool ok;
  explicit Busy(qaoa_ctx* ctx) : c(ctx), ok(ctx && ctx->busy.exchange(1) == 0) {}
  ~Busy() {
    if (ok) c->busy.store(0);
  }
};

int grow_device(void** p, size_t* cap, size_t need, hipStream_t st) {
  if (*cap >= need && *p) return QAOA_OK;
  if (*p) {
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(*p));
    *p = nullptr;
    *cap = 0;
  }
  size_t sz = need < 4096 ? 4096 : need + need / 2;
  HIPCHK(hipMalloc(p, sz));
  *cap = sz;
  return QAOA_OK;
}

int grow_host(void** p, size_t* cap, size_t need, qaoa_ctx* c) {
  if (*cap >= need && *p) return QAOA_OK;
  if (*p) {
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipHostFree(*p));
    *p = nullptr;
    *cap = 0;
  }
  size_t sz = need < 4096 ? 4096 : need + need / 2;
  HIPCHK(hipHostMalloc(p, sz, hipHostMallocDefault));
  *cap = sz;
  return QAOA_OK;
}

// Library streams, shared by every context on a device and kept until the
// process ends: stream 0 is the stream of contexts not bound to a caller's
// stream, 1..3 are the extra streams of chunked pass pairs.  A device has a
// few hardware queues, which its streams share in turn; with streams of their
// own per context, a context's second-pass stream can land on the queue of its
// own first-pass chain, which serialises the pair (complex128 n = 30 with a
// complex64 context alive: 144 ms per run with private extra streams, 115 ms
// with shared ones, as alone).  Contexts that run at once on different threads
// then queue their launches behind each other on these streams: still correct
// (every wait is on the context's own events), not concurrent.
static hipError_t device_streams(int device, int count, hipStream_t* out) {
  static std::mutex mu;
  static std::map<int, std::vector<hipStream_t>> pool;
  std::lock_guard<std::mutex> lock(mu);
  std::vector<hipStream_t>& v = pool[device];
  while ((int)v.size() < count) {
    hipStream_t st = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);   // default priority
    if (e != hipSuccess) return e;
    v.push_back(st);
  }
  for (int i = 0; i < count; ++i) out[i] = v[i];
  return hipSuccess;
}

int ensure_device(qaoa_ctx* c) {
  if (c->dev_ready) return QAOA_OK;
  HIPCHK(hipGetDevice(&c->device));
  if (!c->stream && !c->stream_bound) HIPCHK(device_streams(c->device, 1, &c->stream));   // the library stream
  const size_t gb = dev_graph_bytes(c->hg);
  HIPCHK(hipMalloc(&c->dgraph, gb));
  std::vector<char> img(gb);
  build_dev_graph_image(c->hg, img.data(), c->dgraph);
  HIPCHK(hipMemcpy(c->dgraph, img.data(), gb, hipMemcpyHostToDevice));
  HIPCHK(hipMalloc((void**)&c->dtcut, tile_cut_doubles(c->hg.n, c->prec) * sizeof(double)));
  HIPCHK(launch_tile_cuts(c->hg.n, c->prec, (const GraphDev*)c->dgraph, c->dtcut, c->stream));
  if (!c->psi) {
    HIPCHK(hipMalloc(&c->psi, c->state_bytes));
    c->own_psi = true;
  }
  HIPCHK(hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming));
  c->dev_ready = true;
  return QAOA_OK;
}

int check_angles(int p, const double* g, const double* b) {
  if (p < 0 || p > 100000 || (p > 0 && (!g || !b))) {
    set_error("invalid p or angle arrays");
    return QAOA_EINVAL;
  }
  for (int l = 0; l < p; ++l)
    if (!std::isfinite(g[l]) || !std::isfinite(b[l])) {
      set_error("angle %d is not finite", l);
      return QAOA_EINVAL;
    }
  return QAOA_OK;
}

// One forward pass pair (passes a and a + 1) chunk by chunk: chunk k's first
// pass on a first-pass stream, its second pass on a second-pass stream once the
// first pass's launch has marked chunk k written (the launch's own completion
// event: no marker packet between consecutive first-pass chunks), while the
// first-pass streams go on with the next chunks.  First-pass streams: the
// context stream (and xs[2] with four streams, alternating); second-pass
// streams: xs[0] (and xs[1] with three or four, alternating).  The pair starts
// after the context stream's earlier work and ends with all streams joined back
// into it.  With profiling, the first pass's time spans its chunk launches on
// the context stream and the second's runs from its first chunk launch to the
// join, so the pair's span is qaoa_pass_span(a, a+1).
static int launch_pair_chunks(qaoa_ctx* c, const RunImage& img, const PassDesc* dlist, size_t a, uint64_t fixed,
                              int logr, int64_t ntiles, int nthreads) {
  const std::vector<PassDesc>& list = img.fwd;
  const size_t b = a + 1;
  const int prec = prec_cfg(c->prec).prec;
  const int64_t nch = (int64_t)1 << img.chunk_bits, per = ntiles >> img.chunk_bits;
  const int S = c->chunk_streams;
  const int nx = S - 1;
  if (!c->xs[nx - 1]) {
    hipStream_t all[4];
    HIPCHK(device_streams(c->device, nx + 1, all));
    for (int x = 0; x < nx; ++x) c->xs[x] = all[x + 1];
  }
  while ((int64_t)c->chunk_ev.size() < nch) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->chunk_ev.push_back(e);
  }
  for (int x = 0; x < 4; ++x)
    if (!c->join_ev[x]) HIPCHK(hipEventCreateWithFlags(&c->join_ev[x], hipEventDisableTiming));
  hipStream_t p1s[2] = {c->stream, S >= 4 ? c->xs[2] : c->stream};
  hipStream_t p2s[2] = {c->xs[0], S >= 3 ? c->xs[1] : c->xs[0]};
  const int nfree = c->hg.n - list[a].K;
  if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * a], c->stream));
  HIPCHK(hipEventRecord(c->join_ev[3], c->stream));
  for (int x = 0; x < nx; ++x) HIPCHK(hipStreamWaitEvent(c->xs[x], c->join_ev[3], 0));
  for (int64_t k = 0; k < nch; ++k) {
    hipStream_t s1 = p1s[k & 1], s2 = p2s[k & 1];
    const LaunchMap la = chunk_launch_map(list[a].map, nfree, fixed, k);
    HIPCHK(launch_pass(prec, false, logr, list[a].shape, dlist + a, 1, per, nthreads, s1, la, c->chunk_ev[k]));
    HIPCHK(hipStreamWaitEvent(s2, c->chunk_ev[k], 0));
    if (c->profiling && k == 0) HIPCHK(hipEventRecord(c->ev[2 * b], s2));
    const LaunchMap lb = chunk_launch_map(list[b].map, nfree, fixed, k);
    HIPCHK(launch_pass(prec, false, logr, list[b].shape, dlist + b, 1, per, nthreads, s2, lb));
  }
  if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * a + 1], c->stream));
  for (int x = 0; x < nx; ++x) {
    HIPCHK(hipEventRecord(c->join_ev[x], c->xs[x]));
    HIPCHK(hipStreamWaitEvent(c->stream, c->join_ev[x], 0));
  }
  if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * b + 1], c->stream));
  return QAOA_OK;
}

// Build, upload and launch one run (forward, and the adjoint sweep if grad).
int launch_run(qaoa_ctx* c, int p, const double* gamma, const double* beta, bool grad) {
  int rc = ensure_device(c);
  if (rc) return rc;
  if (grad && !c->lam) HIPCHK(hipMalloc(&c->lam, c->state_bytes));
  RunRequest rq{&c->hg, c->prec, p, gamma, beta, grad, c->psi, c->lam, (const GraphDev*)c->dgraph};
  rq.chunk_bytes = c->state_bytes >= c->chunk_min_state ? c->chunk_bytes : 0;
  RunImage img;
  build_run(rq, &img);
  const ImageLayout lay = image_layout(img, c->prec);
  if (c->upload_pending) {
    HIPCHK(hipEventSynchronize(c->upload_done));
    c->upload_pending = false;
  }
  if ((rc = grow_device((void**)&c->dev_img, &c->dev_img_cap, lay.total, c->stream))) return rc;
  if ((rc = grow_device((void**)&c->dev_part, &c->dev_part_cap, img.part_doubles * sizeof(double), c->stream)))
    return rc;
  if ((rc = grow_device((void**)&c->dev_out, &c->dev_out_cap, img.nout * sizeof(double), c->stream))) return rc;
  if ((rc = grow_host((void**)&c->host_img, &c->host_img_cap, lay.total, c))) return rc;
  if ((rc = grow_host((void**)&c->host_out, &c->host_out_cap, img.nout * sizeof(double), c))) return rc;
  pack_run(img, lay, c->prec, c->host_img, c->dev_img, c->dev_part, c->dev_out, c->dtcut);
  HIPCHK(hipMemcpyAsync(c->dev_img, c->host_img, lay.total, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipEventRecord(c->upload_done, c->stream));
  c->upload_pending = true;

  const PrecCfg pc = prec_cfg(c->prec);
  int K, logr;
  tile_shape(c->hg.n, pc, &K, &logr);
  const int nthreads = 1 << (K - logr);
  const int64_t ntiles = (int64_t)1 << (c->hg.n - K);
  const size_t nf = img.fwd.size(), nb = img.bwd.size();
  if (c->profiling) {
    while (c->ev.size() < 2 * (nf + nb)) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      c->ev.push_back(e);
    }
  }
  const PassDesc* dfwd = (const PassDesc*)(c->dev_img + lay.off_fwd);
  if (img.chunk_bits == 0) {
    for (size_t i = 0; i < nf; ++i) {
      if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * i], c->stream));
      HIPCHK(launch_pass(pc.prec, false, logr, img.fwd[i].shape, dfwd + i, 1, ntiles, nthreads, c->stream));
      if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * i + 1], c->stream));
    }
  } else {
    if (c->profiling) HIPCHK(hipEventRecord(c->ev[0], c->stream));
    HIPCHK(launch_pass(pc.prec, false, logr, img.fwd[0].shape, dfwd, 1, ntiles, nthreads, c->stream));
    if (c->profiling) HIPCHK(hipEventRecord(c->ev[1], c->stream));
    for (size_t pr = 0; pr < img.pair_fixed.size(); ++pr)
      if ((rc = launch_pair_chunks(c, img, dfwd, 2 * pr + 1, img.pair_fixed[pr], logr, ntiles, nthreads)))
        return rc;
  }
  c->ntimed = c->profiling ? (int)(nf + nb) : 0;
  c->pass_bytes = img.pass_bytes;
  c->pass_bytes.insert(c->pass_bytes.end(), img.bwd_bytes.begin(), img.bwd_bytes.end());
  c->pass_set = img.fwd_set;
  c->pass_set.insert(c->pass_set.end(), img.bwd_set.begin(), img.bwd_set.end());
  c->pass_shape.clear();
  for (const PassDesc& d : img.fwd) c->pass_shape.push_back(d.shape);
  for (const PassDesc& d : img.bwd) c->pass_shape.push_back(d.shape);
  c->pass_logr = logr;
  c->pass_nfwd = (int)nf;
  const PassDesc* dbwd = (const PassDesc*)(c->dev_img + lay.off_bwd);
  // The adjoint sweep runs whole passes: paired and chunked like the forward
  // passes (both vectors of a chunk per launch) it measured slower.
  for (size_t i = 0; i < nb; ++i) {
    if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * (nf + i)], c->stream));
    HIPCHK(launch_pass(pc.prec, true, logr, img.bwd[i].shape, dbwd + i, 1, ntiles, nthreads, c->stream));
    if (c->profiling) HIPCHK(hipEventRecord(c->ev[2 * (nf + i) + 1], c->stream));
  }
  HIPCHK(launch_reduce((const ReduceJob*)(c->dev_img + lay.off_jobs), (const Span*)(c->dev_img + lay.off_spans),
                       (int)img.jobs.size(), c->stream));
  HIPCHK(hipMemcpyAsync(c->host_out, c->dev_out, img.nout * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  c->complemented = img.complemented;
  // A caller-owned state buffer is left in natural order.
  if (c->complemented && !c->own_psi && !grad) {
    HIPCHK(launch_reverse(c->prec == QAOA_C64 ? 1 : 0, c->psi, (int64_t)1 << c->hg.n, c->stream));
    c->complemented = false;
  }
  return QAOA_OK;
}

// Shared by qaoa_fidelity and qaoa_fidelity_noalloc: argument and state checks.
int fidelity_check(qaoa_ctx* a, qaoa_ctx* b, double* f_out, const Busy& ba, const Busy& bb) {
  if (!a || !b || !f_out || a == b) {
    set_error("invalid arguments");
    return QAOA_EINVAL;
  }
  if (!ba.ok || !bb.ok) {
    set_error("context busy");
    return QAOA_ESTATE;
  }
  if (a->hg.n != b->hg.n) {
    set_error("qubit counts differ");
    return QAOA_EINVAL;
  }
  if (!a->have_state || !b->have_state) {
    set_error("both contexts need a state");
    return QAOA_ESTATE;
  }
  if (a->device != b->device) {
    set_error("the two contexts live on different devices");
    return QAOA_EINVAL;
  }
  return QAOA_OK;
}

// The overlap sums of a and b in the device workspace d (fidelity_work(nb)
// bytes), on a's stream after b's work; F = |<a|b>|^2 / (<a|a><b|b>).
int fidelity_core(qaoa_ctx* a, qaoa_ctx* b, char* d, int nb, double* f_out) {
  HIPCHK(hipStreamSynchronize(b->stream));
  const int64_t N = (int64_t)1 << a->hg.n;
  const int rev = a->complemented != b->complemented ? 1 : 0;
  double h[4] = {0, 0, 0, 0};
  hipError_t e = launch_fidelity_sums(a->prec, a->psi, b->prec, b->psi, N, rev, d, nb, a->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h, d + fidelity_work(nb).off_out, sizeof h, hipMemcpyDeviceToHost, a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  if (e != hipSuccess) {
    set_error("fidelity: %s", hipGetErrorString(e));
    return QAOA_EDEVICE;
  }
  *f_out = (h[0] * h[0] + h[1] * h[1]) / (h[2] * h[3]);
  return QAOA_OK;
}

// Static device workspace of qaoa_fidelity_noalloc: one copy per GPU, held
// until the process ends; every call on a GPU reuses it.  In host code the
// array's name is only a stand-in for the symbol, so the device address is
// looked up once per device (with that device current) and kept.
constexpr size_t kScratchBytes = 66 * 1024;
static __device__ __align__(256) char scratch[kScratchBytes];
static_assert(sizeof(scratch) >= 4 * kFidelityMaxBlocks * sizeof(double) + 1024, "fidelity workspace must fit");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d out of range", device);
    return QAOA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIPCHK(hipSetDevice(cur));
    HIPCHK(e);
    if (!p) {
      set_error("hipGetSymbolAddress returned NULL for the static workspace");
      return QAOA_EDEVICE;
    }
    g_scratch_ptr[device] = (char*)p;
  }
  *out = g_scratch_ptr[device];
  return QAOA_OK;
}

}  // namespace

extern "C" {

const char* qaoa_last_error(void) { return qaoa::last_error(); }

int qaoa_create(int n, int num_edges, const int32_t* edges, const double* weights, int prec, qaoa_ctx** out) {
  if (!out) {
    set_error("out is NULL");
    return QAOA_EINVAL;
  }
  *out = nullptr;
  if (prec != QAOA_C128 && prec != QAOA_C64) {
    set_error("prec must be QAOA_C128 or QAOA_C64");
    return QAOA_EINVAL;
  }
  HostGraph hg;
  int rc = make_graph(n, num_edges, edges, weights, &hg);
  if (rc) return rc;
  qaoa_ctx* c = new qaoa_ctx();
  c->hg = std::move(hg);
  c->prec = prec;
  c->state_bytes = ((size_t)1 << n) * prec_cfg(prec).elem;
  // measured on three-set plans with 128 MiB chunks and the high-set chunks
  // alternating over two streams: complex64 n = 30 runs 10% faster chunked
  // (3% at n = 26, 28), complex128 n = 30 10% (8% at n = 26, 28); from 512
  // MiB states on, smaller ones run faster whole
  c->chunk_bytes = (size_t)128 << 20;
  c->chunk_min_state = (size_t)512 << 20;
  c->chunk_streams = 3;
  *out = c;
  return QAOA_OK;
}

void qaoa_destroy(qaoa_ctx* c) {
  if (!c) return;
  if (c->dev_ready && c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->own_psi && c->psi) (void)hipFree(c->psi);
  if (c->lam) (void)hipFree(c->lam);
  if (c->dgraph) (void)hipFree(c->dgraph);
  if (c->dtcut) (void)hipFree(c->dtcut);
  if (c->dev_img) (void)hipFree(c->dev_img);
  if (c->dev_part) (void)hipFree(c->dev_part);
  if (c->dev_out) (void)hipFree(c->dev_out);
  for (hipEvent_t e : c->chunk_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->join_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->host_img) (void)hipHostFree(c->host_img);
  if (c->host_out) (void)hipHostFree(c->host_out);
  if (c->upload_done) (void)hipEventDestroy(c->upload_done);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

int qaoa_max_qubits(int prec, int with_grad) {
  if (prec != QAOA_C128 && prec != QAOA_C64) return 0;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 0;
  const size_t elem = prec_cfg(prec).elem;
  const size_t margin = (size_t)256 << 20;
  int best = 0;
  for (int n = 1; n <= kMaxN; ++n) {
    const size_t need = ((size_t)1 << n) * elem * (with_grad ? 2 : 1) + tile_cut_doubles(n, prec) * sizeof(double) +
                        margin;
    if (need <= fr) best = n;
  }
  return best;
}

int qaoa_run(qaoa_ctx* c, int p, const double* gamma, const double* beta) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  int rc = check_angles(p, gamma, beta);
  if (rc) return rc;
  c->have_state = c->have_expect = false;
  rc = launch_run(c, p, gamma, beta, false);
  if (rc) return rc;
  c->have_state = c->have_expect = true;
  return QAOA_OK;
}

int qaoa_expect(qaoa_ctx* c, double* expect_out, double* norm_out) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (!c->have_expect) {
    set_error("no run to take the expectation of");
    return QAOA_ESTATE;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  if (expect_out) *expect_out = c->host_out[0];
  if (norm_out) *norm_out = c->host_out[1];
  return QAOA_OK;
}

int qaoa_run_gates(qaoa_ctx* c, int p, const double* gamma, const double* beta) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  int rc = check_angles(p, gamma, beta);
  if (rc) return rc;
  if ((rc = ensure_device(c))) return rc;
  c->have_state = c->have_expect = false;
  if (c->upload_pending) {   // the host image buffers are reused below
    HIPCHK(hipEventSynchronize(c->upload_done));
    c->upload_pending = false;
  }
  const int nb = gate_reduce_blocks(c->hg.n);
  if ((rc = grow_device((void**)&c->dev_part, &c->dev_part_cap, 2 * nb * sizeof(double), c->stream))) return rc;
  if ((rc = grow_device((void**)&c->dev_out, &c->dev_out_cap, 2 * sizeof(double), c->stream))) return rc;
  if ((rc = grow_host((void**)&c->host_out, &c->host_out_cap, 2 * sizeof(double), c))) return rc;
  GateRun r{c->hg.n, c->hg.m(), p, c->hg.eu.data(), c->hg.ev.data(), c->hg.weighted() ? c->hg.w.data() : nullptr,
            gamma, beta, c->psi};
  HIPCHK(launch_gate_run(c->prec == QAOA_C64 ? 1 : 0, r, c->stream));
  HIPCHK(launch_expect_state(c->prec == QAOA_C64 ? 1 : 0, (const GraphDev*)c->dgraph, c->psi, c->hg.n, c->dev_part,
                             c->dev_out, c->stream));
  HIPCHK(hipMemcpyAsync(c->host_out, c->dev_out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  c->complemented = false;
  c->ntimed = 0;
  c->pass_shape.clear();
  c->pass_set.clear();
  c->have_state = c->have_expect = true;
  return QAOA_OK;
}

int qaoa_sample(qaoa_ctx* c, int64_t count, const double* uniforms, uint64_t* out) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (count < 0 || count > (int64_t(1) << 31) || (count > 0 && (!uniforms || !out))) {
    set_error("invalid sample count or NULL arrays");
    return QAOA_EINVAL;
  }
  for (int64_t k = 0; k < count; ++k)
    if (!(uniforms[k] >= 0.0 && uniforms[k] < 1.0)) {
      set_error("uniform %lld is not in [0, 1)", (long long)k);
      return QAOA_EINVAL;
    }
  if (!c->have_state) {
    set_error("no state to sample");
    return QAOA_ESTATE;
  }
  const int n = c->hg.n;
  const int64_t nc = sample_chunks(n);
  const size_t bytes = (size_t)(66 * nc + 1) * 8 + (size_t)count * 16;
  char* tmp = nullptr;
  HIPCHK(hipMalloc((void**)&tmp, bytes));
  double* sums = (double*)tmp;
  double* prefix = sums + nc;
  double* bsums = prefix + nc + 1;
  double* du = bsums + 64 * nc;
  uint64_t* dout = (uint64_t*)(du + count);
  hipError_t e = hipSuccess;
  if (count > 0) e = hipMemcpyAsync(du, uniforms, (size_t)count * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_sample(c->prec == QAOA_C64 ? 1 : 0, c->psi, n, c->complemented ? 1 : 0, sums, prefix, bsums, du, count,
                      dout, c->stream);
  if (e == hipSuccess && count > 0) e = hipMemcpyAsync(out, dout, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(tmp);
  HIPCHK(e);
  return QAOA_OK;
}

int qaoa_max_cut(qaoa_ctx* c, double* value_out, uint64_t* argmax_out) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (!value_out && !argmax_out) {
    set_error("value_out and argmax_out are NULL");
    return QAOA_EINVAL;
  }
  int rc = ensure_device(c);
  if (rc) return rc;
  const int nb = gate_reduce_blocks(c->hg.n);
  char* tmp = nullptr;
  const size_t bytes = (size_t)nb * 16 + 16;
  HIPCHK(hipMalloc((void**)&tmp, bytes));
  double* pv = (double*)tmp;
  uint64_t* pz = (uint64_t*)(tmp + (size_t)nb * 8);
  double* ov = (double*)(tmp + (size_t)nb * 16);
  uint64_t* oz = (uint64_t*)(tmp + (size_t)nb * 16 + 8);
  hipError_t e = launch_max_cut((const GraphDev*)c->dgraph, c->hg.n, pv, pz, ov, oz, c->stream);
  double v = 0.0;
  uint64_t z = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&v, ov, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&z, oz, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(tmp);
  HIPCHK(e);
  if (value_out) *value_out = v;
  if (argmax_out) *argmax_out = z;
  return QAOA_OK;
}

int qaoa_grad(qaoa_ctx* c, int p, const double* gamma, const double* beta, double* expect_out, double* dgamma,
              double* dbeta) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  int rc = check_angles(p, gamma, beta);
  if (rc) return rc;
  if (p > 0 && (!dgamma || !dbeta)) {
    set_error("dgamma/dbeta are NULL");
    return QAOA_EINVAL;
  }
  c->have_state = c->have_expect = false;
  rc = launch_run(c, p, gamma, beta, true);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (expect_out) *expect_out = c->host_out[0];
  for (int l = 0; l < p; ++l) {
    dgamma[l] = c->host_out[2 + l];
    dbeta[l] = c->host_out[2 + p + l];
  }
  c->have_expect = true;     // the state buffer now holds an intermediate of the adjoint sweep
  return QAOA_OK;
}

int qaoa_cut_table(qaoa_ctx* c, void* host_out, size_t bytes) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  const size_t N = (size_t)1 << c->hg.n;
  const size_t need = N * (c->hg.weighted() ? 8 : 4);
  if (!host_out || bytes != need) {
    set_error("cut table needs %zu bytes", need);
    return QAOA_EINVAL;
  }
  int rc = ensure_device(c);
  if (rc) return rc;
  void* d = nullptr;
  HIPCHK(hipMalloc(&d, need));
  hipError_t e = launch_cut_table((const GraphDev*)c->dgraph, c->hg.weighted(), d, (int64_t)N, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(host_out, d, need, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e != hipSuccess) {
    set_error("cut table: %s", hipGetErrorString(e));
    return QAOA_EDEVICE;
  }
  return QAOA_OK;
}

int qaoa_get_state(qaoa_ctx* c, void* host_out, size_t bytes) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (!c->have_state) {
    set_error("no state: run first (a gradient run leaves no final state)");
    return QAOA_ESTATE;
  }
  if (!host_out || bytes != c->state_bytes) {
    set_error("state needs %zu bytes", c->state_bytes);
    return QAOA_EINVAL;
  }
  HIPCHK(hipMemcpyAsync(host_out, c->psi, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->complemented) {   // stored as psi(~z): reverse into natural order
    const size_t N = (size_t)1 << c->hg.n, el = prec_cfg(c->prec).elem;
    char* h = (char*)host_out;
    char tmp[16];
    for (size_t i = 0; i < N / 2; ++i) {
      memcpy(tmp, h + i * el, el);
      memcpy(h + i * el, h + (N - 1 - i) * el, el);
      memcpy(h + (N - 1 - i) * el, tmp, el);
    }
  }
  return QAOA_OK;
}

int qaoa_fidelity(qaoa_ctx* a, qaoa_ctx* b, double* f_out) {
  Busy ba(a), bb(b);
  int rc = fidelity_check(a, b, f_out, ba, bb);
  if (rc) return rc;
  const int nb = fidelity_blocks((int64_t)1 << a->hg.n);
  char* d = nullptr;
  HIPCHK(hipMalloc((void**)&d, fidelity_work(nb).bytes));
  rc = fidelity_core(a, b, d, nb, f_out);
  (void)hipFree(d);
  return rc;
}

int qaoa_fidelity_noalloc(qaoa_ctx* a, qaoa_ctx* b, double* f_out) {
  Busy ba(a), bb(b);
  int rc = fidelity_check(a, b, f_out, ba, bb);
  if (rc) return rc;
  const int nb = fidelity_blocks((int64_t)1 << a->hg.n);
  if (fidelity_work(nb).bytes > sizeof(scratch)) {
    set_error("fidelity workspace of %zu bytes exceeds the %zu-byte static buffer", fidelity_work(nb).bytes,
              sizeof(scratch));
    return QAOA_EINVAL;
  }
  char* d = nullptr;
  if ((rc = scratch_address(a->device, &d))) return rc;
  return fidelity_core(a, b, d, nb, f_out);
}

int qaoa_bind_stream(qaoa_ctx* c, void* hip_stream) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (c->dev_ready) HIPCHK(hipStreamSynchronize(c->stream));
  c->stream = (hipStream_t)hip_stream;
  c->stream_bound = true;
  return QAOA_OK;
}

int qaoa_bind_state(qaoa_ctx* c, void* dev_ptr, size_t bytes) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (!dev_ptr || bytes != c->state_bytes || ((uintptr_t)dev_ptr & 255u)) {
    set_error("state buffer must be %zu bytes, 256-byte aligned", c->state_bytes);
    return QAOA_EINVAL;
  }
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  if (c->own_psi && c->psi) HIPCHK(hipFree(c->psi));
  c->psi = dev_ptr;
  c->own_psi = false;
  c->have_state = c->have_expect = false;
  return QAOA_OK;
}

int qaoa_set_profiling(qaoa_ctx* c, int enable) {
  if (!c) {
    set_error("context is NULL");
    return QAOA_EINVAL;
  }
  c->profiling = enable != 0;
  return QAOA_OK;
}

int qaoa_pass_times(qaoa_ctx* c, float* ms, double* bytes, int max, int* count) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (!count || max < 0) {
    set_error("count is NULL");
    return QAOA_EINVAL;
  }
  *count = c->ntimed;
  if (c->ntimed == 0) return QAOA_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < c->ntimed && i < max; ++i) {
    if (ms) HIPCHK(hipEventElapsedTime(&ms[i], c->ev[2 * i], c->ev[2 * i + 1]));
    if (bytes) bytes[i] = c->pass_bytes[i];
  }
  return QAOA_OK;
}

int qaoa_chunk_plan(int n, int prec, int p, size_t chunk_bytes, int* chunk_bits, uint64_t* pair_fixed,
                    int max_pairs, int* npairs) {
  if (n < 1 || n > kMaxN || (prec != QAOA_C64 && prec != QAOA_C128) || p < 0 || !chunk_bits || !npairs) {
    set_error("invalid arguments");
    return QAOA_EINVAL;
  }
  const PrecCfg pc = prec_cfg(prec);
  const std::vector<SetGeom> sets = make_sets(n, pc);
  const std::vector<PassSpec> sch = make_schedule((int)sets.size(), p);
  std::vector<uint64_t> fixed;
  *chunk_bits = chunk_plan(sets, sch, p, (double)((int64_t)1 << n) * (double)pc.elem, chunk_bytes, &fixed);
  *npairs = (int)fixed.size();
  for (int i = 0; pair_fixed && i < (int)fixed.size() && i < max_pairs; ++i) pair_fixed[i] = fixed[i];
  return QAOA_OK;
}

int qaoa_chunk_tiles(int n, int prec, int set, uint64_t fixed_mem, int chunk_bits, int64_t k, int64_t* g_out) {
  if (n < 1 || n > kMaxN || (prec != QAOA_C64 && prec != QAOA_C128) || !g_out || chunk_bits < 0 ||
      chunk_bits >= kLaunchRuns || __builtin_popcountll(fixed_mem) != chunk_bits || k < 0 ||
      k >= ((int64_t)1 << chunk_bits)) {
    set_error("invalid arguments");
    return QAOA_EINVAL;
  }
  const PrecCfg pc = prec_cfg(prec);
  const std::vector<SetGeom> s = make_sets(n, pc);
  if (set < 0 || set >= (int)s.size()) {
    set_error("the plan has %d qubit sets", (int)s.size());
    return QAOA_EINVAL;
  }
  const int nfree = n - s[set].K;
  if (nfree < chunk_bits) {
    set_error("too few tile-index bits");
    return QAOA_EINVAL;
  }
  uint64_t index_bits = 0;
  for (int i = 0; i < nfree; ++i) index_bits |= 1ull << s[set].map.gpos[i];
  if (fixed_mem & ~index_bits) {
    set_error("fixed bits must be tile-index bits of the set");
    return QAOA_EINVAL;
  }
  const LaunchMap m = chunk_launch_map(s[set].map, nfree, fixed_mem, k);
  const int64_t per = ((int64_t)1 << nfree) >> chunk_bits;
  for (int64_t t = 0; t < per; ++t) g_out[t] = (int64_t)launch_tile(m, (uint64_t)t);
  return QAOA_OK;
}

int qaoa_set_chunking(qaoa_ctx* c, size_t chunk_bytes, size_t min_state_bytes, int streams) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (streams < 2 || streams > 4) {
    set_error("streams must be 2, 3 or 4");
    return QAOA_EINVAL;
  }
  c->chunk_bytes = chunk_bytes;
  c->chunk_min_state = min_state_bytes;
  c->chunk_streams = streams;
  return QAOA_OK;
}

int qaoa_pass_kernel(qaoa_ctx* c, int index, int* set_out, char* name, size_t len) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (index < 0 || index >= (int)c->pass_shape.size()) {
    set_error("the last run has %d passes", (int)c->pass_shape.size());
    return QAOA_EINVAL;
  }
  if (set_out) *set_out = c->pass_set[index];
  if (name && len > 0)
    pass_kernel_name(c->prec == QAOA_C64 ? 1 : 0, index >= c->pass_nfwd, c->pass_logr, c->pass_shape[index], name,
                     len);
  return QAOA_OK;
}

int qaoa_pass_span(qaoa_ctx* c, int first, int last, float* ms) {
  Busy b(c);
  if (!b.ok) {
    set_error(c ? "context busy" : "context is NULL");
    return c ? QAOA_ESTATE : QAOA_EINVAL;
  }
  if (!ms || first < 0 || last < first || last >= c->ntimed) {
    set_error("the last timed run has %d passes", c->ntimed);
    return QAOA_EINVAL;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipEventElapsedTime(ms, c->ev[2 * first], c->ev[2 * last + 1]));
  return QAOA_OK;
}

int qaoa_plan_info(qaoa_ctx* c, int p, int* passes, int* sets, int* sizes, int max_sets) {
  if (!c || p < 0) {
    set_error("invalid arguments");
    return QAOA_EINVAL;
  }
  const std::vector<SetGeom> s = make_sets(c->hg.n, prec_cfg(c->prec));
  const std::vector<PassSpec> sch = make_schedule((int)s.size(), p);
  if (passes) *passes = (int)sch.size();
  if (sets) *sets = (int)s.size();
  for (int i = 0; sizes && i < (int)s.size() && i < max_sets; ++i) sizes[i] = s[i].k;
  return QAOA_OK;
}

int qaoa_tile_map(int n, int prec, int set, int* k_out, int8_t* tpos, int8_t* gpos, uint64_t* gmask,
                  int8_t* gshift) {
  if (n < 1 || n > kMaxN || (prec != QAOA_C64 && prec != QAOA_C128) || !k_out || !tpos || !gpos) {
    set_error("invalid arguments");
    return QAOA_EINVAL;
  }
  const std::vector<SetGeom> s = make_sets(n, prec_cfg(prec));
  if (set < 0 || set >= (int)s.size()) {
    set_error("the plan has %d qubit sets", (int)s.size());
    return QAOA_EINVAL;
  }
  const SetGeom& g = s[set];
  *k_out = g.K;
  for (int i = 0; i < g.K; ++i) tpos[i] = g.map.tpos[i];
  for (int i = 0; i < n - g.K; ++i) gpos[i] = g.map.gpos[i];
  for (int r = 0; gmask && gshift && r < kMaxRuns; ++r) {
    gmask[r] = g.map.gmask[r];
    gshift[r] = g.map.gshift[r];
  }
  return QAOA_OK;
}

int qaoa_copy_probe(const void* src, void* dst, size_t bytes, int block_bytes, void* hip_stream) {
  if (!src || !dst || bytes == 0 || bytes % 16 || (block_bytes != 4096 && block_bytes != 16384)) {
    set_error("copy probe needs non-NULL pointers, a multiple of 16 bytes and 4096 or 16384 bytes per workgroup");
    return QAOA_EINVAL;
  }
  HIPCHK(launch_copy(src, dst, (int64_t)(bytes / 16), block_bytes, (hipStream_t)hip_stream));
  return QAOA_OK;
}

}  // extern "C"
