/*
 * qaoa.h -- C ABI of the MI355X (gfx950) QAOA max-cut state-vector simulator.
 *
 * The simulated circuit is the max-cut QAOA of Lin, Wang, Tu and Hung,
 * "Towards Optimizations of Quantum Circuit Simulation for Solving Max-Cut
 * Problems with QAOA" (arXiv:2312.03019):
 *   - n qubits, a dense state vector of 2^n complex amplitudes indexed by z,
 *     qubit q <-> bit q of z (the bit extraction (b >> i) & 1 of Algorithm 3);
 *   - start |+>^n: every amplitude 2^(-n/2) ("launch control", Section
 *     Mathematical Optimizations);
 *   - p layers; layer l applies the diagonal cost unitary exp(-i gamma_l C(z))
 *     (rotation compression, Eq. UC_opt / Algorithm 2), with the cut value
 *     C(z) = sum over edges of w_uv [z_u != z_v] (bitwise popcount form of
 *     Algorithm 3 for unweighted graphs), then the mixer exp(-i beta_l X_q) =
 *     RX(2 beta_l) on every qubit (mixer layer of Algorithm 1);
 *   - the objective <C> = sum_z |psi_z|^2 C(z).
 * The paper prints its cost layer as exp(-i gamma/2 sum w Z_i Z_j) and its
 * mixer as RX(beta); those equal this ABI's gamma -> -gamma, beta -> beta/2 up
 * to a global phase.  The ABI fixes the convention above and takes no flag.
 *
 * Conventions for every call:
 *   - Return value: QAOA_OK (0) or a negative QAOA_E* code; nothing throws or
 *     aborts.  qaoa_last_error() gives a thread-local message for the last
 *     failure on the calling thread.
 *   - Ownership: the caller owns every input array; the library copies what
 *     it keeps before returning.  Output arrays are caller-provided host
 *     memory unless stated.  Device state is owned by the library unless the
 *     caller lends a buffer with qaoa_bind_state.
 *   - Threads: one context must not be used from two threads at once (the
 *     second caller gets QAOA_ESTATE).  A server handle is thread-safe.
 *   - Streams: a context runs on the stream given to qaoa_bind_stream, else
 *     on a library stream that all unbound contexts on the device share;
 *     chunked pass pairs add up to three more library streams per device,
 *     shared the same way.  Library streams live until the process ends.
 *   - Device errors (HIP) are reported as QAOA_EDEVICE with the HIP message.
 */
#ifndef QAOA_H
#define QAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QAOA_OK = 0,
  QAOA_EINVAL = -1,    /* invalid argument */
  QAOA_ENOMEM = -2,    /* device or host memory, or serving budget, exhausted */
  QAOA_EDEVICE = -3,   /* HIP runtime error */
  QAOA_EPENDING = -4,  /* serving: result not ready yet */
  QAOA_ECANCELED = -5, /* serving: request was cancelled */
  QAOA_ESTATE = -6     /* call out of order, or context busy on another thread */
};

enum { QAOA_C128 = 0, QAOA_C64 = 1 }; /* state precision: complex double / complex float */

typedef struct qaoa_ctx qaoa_ctx;
typedef struct qaoa_server qaoa_server;

/* Create a simulator for one max-cut instance (Table 1's N, graph and w).
 * n: qubits = vertices, 1 <= n <= qaoa_max_qubits(prec, 0).
 * edges: 2*num_edges int32 vertex ids u0,v0,u1,v1,... with 0 <= u,v < n,
 *   u != v, each unordered pair at most once (the paper's upper-triangular
 *   graph holds one weight per pair).  num_edges = 0 is valid (C = 0).
 * weights: num_edges finite doubles, or NULL for the unweighted graph (all
 *   weights 1; cut values are then exact integers).
 * prec: QAOA_C128 or QAOA_C64.  With QAOA_C64 the state is complex float;
 *   phase angles gamma*C(z) are formed and reduced in double before the
 *   single-precision sine/cosine, and all reductions run in double.
 * The context binds to the current HIP device and allocates no state until
 * the first run.  Validation happens before any device call. */
int qaoa_create(int n, int num_edges, const int32_t *edges, const double *weights,
                int prec, qaoa_ctx **out);

/* Release everything the context owns (a bound state buffer is not freed). */
void qaoa_destroy(qaoa_ctx *ctx);

/* Largest n whose state (times two vectors when with_grad) fits the current
 * device's free memory for the given precision; 0 when no device. */
int qaoa_max_qubits(int prec, int with_grad);

/* Evolve |+>^n through p layers (p >= 0) with angles gamma[p], beta[p]
 * (finite doubles): the circuit of Algorithm 1 (Section 2.1) with each
 * level's RZZ gates compressed into one diagonal phase exp(-i gamma_l C(z))
 * per basis state (Eq. UC_opt, Algorithm 2; launch control of Section 2.2
 * for the start state), followed by exp(-i beta_l X) on every qubit.
 * Enqueues work on the bound stream and returns; the state stays on the
 * device.  p = 0 leaves |+>^n.  QAOA_EINVAL for p < 0, NULL angle arrays
 * with p > 0 or a non-finite angle; QAOA_ENOMEM / QAOA_EDEVICE when the
 * state cannot be allocated or a launch fails. */
int qaoa_run(qaoa_ctx *ctx, int p, const double *gamma, const double *beta);

/* <C> = sum_z |psi_z|^2 C(z), the expected cut the classical optimiser of
 * the QAOA workflow (Section 1) consumes, and the norm sum |psi|^2, of the
 * last qaoa_run or qaoa_run_gates (both double, accumulated in FP64 in a
 * fixed order; the norm pointer may be NULL).  Synchronises the stream.
 * QAOA_ESTATE before any run. */
int qaoa_expect(qaoa_ctx *ctx, double *expect_out, double *norm_out);

/* <C> and its gradient d<C>/dgamma_l, d<C>/dbeta_l for l < p, by one forward
 * sweep and one adjoint backward sweep on the device (two state vectors).
 * dgamma and dbeta are caller arrays of p doubles.  Synchronises the stream.
 * The backward sweep overwrites the state buffer, so afterwards there is no
 * state to read: qaoa_get_state / qaoa_fidelity return QAOA_ESTATE until the
 * next qaoa_run. */
int qaoa_grad(qaoa_ctx *ctx, int p, const double *gamma, const double *beta,
              double *expect_out, double *dgamma, double *dbeta);

/* The same evolution as qaoa_run, computed gate by gate as Algorithm 1
 * (Section 2.1) lays the circuit out: |0>, a Hadamard on every qubit, then
 * per level one diagonal two-qubit sweep per edge (exp(-i gamma_l w_uv) on the
 * basis states that cut edge (u, v), i.e. the RZZ gate up to the global phase
 * the ABI convention drops) and one RX sweep per qubit; every gate is one pass
 * over the state.  It is the uncompressed reference for the fused passes'
 * speedup (Tables "cpu"/"gpu" and the p-scan of Section 3.4 compare the
 * paper's optimisations with such a gate-level simulation).  <C> and the norm
 * are then computed by a separate sweep, so qaoa_expect, qaoa_get_state and
 * qaoa_fidelity work as after qaoa_run.  Asynchronous like qaoa_run. */
int qaoa_run_gates(qaoa_ctx *ctx, int p, const double *gamma, const double *beta);

/* The maximum cut max_z C(z) and the lowest z attaining it (the denominator of
 * the approximation ratio <C> / max C of Section 3.4), by one device sweep
 * evaluating C(z) as qaoa_cut_table does (so bit-exact in both cases).
 * Either output pointer may be NULL, not both.  Synchronises the stream. */
int qaoa_max_cut(qaoa_ctx *ctx, double *value_out, uint64_t *argmax_out);

/* Draw count bitstrings z from |psi_z|^2 of the last run's state (the
 * solutions a QAOA run hands to the classical side, Section 1's workflow):
 * sample k is the smallest z with CDF(z) > uniforms[k] * sum|psi|^2, the CDF
 * taken over z in natural order in FP64 (so the result is a deterministic
 * function of the caller's uniforms, each in [0, 1), else QAOA_EINVAL).
 * uniforms and out are host arrays of count entries.  QAOA_ESTATE without a
 * state (no run yet, or after qaoa_grad).  Allocates a device workspace of
 * about 2^n / 8 + 16 * count bytes for the call (QAOA_EDEVICE if that
 * fails).  Synchronises the stream. */
int qaoa_sample(qaoa_ctx *ctx, int64_t count, const double *uniforms, uint64_t *out);

/* Cut value C(z) for all 2^n z (the per-state totals of Algorithms 2/3, in the
 * max-cut form).  Unweighted: int32 values (bytes = 4*2^n), exact.
 * Weighted: double values (bytes = 8*2^n).  host_out is host memory. */
int qaoa_cut_table(qaoa_ctx *ctx, void *host_out, size_t bytes);

/* Copy the state of the last run (the 2^n amplitudes the paper's simulator
 * evolves, Section 2.1; amplitude z at index z, qubit q = bit q of z) to
 * host memory: 2^n interleaved (re, im) pairs of double (C128) or float
 * (C64).  bytes must equal 2^n * 16 (C128) or 2^n * 8 (C64), else
 * QAOA_EINVAL; QAOA_ESTATE without a state (no run, or after qaoa_grad).
 * Synchronises the stream. */
int qaoa_get_state(qaoa_ctx *ctx, void *host_out, size_t bytes);

/* F = |<a|b>|^2 / (<a|a><b|b>) between the states of two contexts with the
 * same n (precisions may differ), accumulated in double on the device: the
 * agreement measure for the complex64 state against the complex128 one (the
 * paper leaves its precision unstated, so both are offered).  QAOA_EINVAL
 * for a == b, NULL pointers or different n; QAOA_ESTATE when a context has
 * no state.  Allocates a device workspace of about 65 KiB for the call
 * (qaoa_fidelity_noalloc does not).  Synchronises both streams. */
int qaoa_fidelity(qaoa_ctx *a, qaoa_ctx *b, double *f_out);

/* qaoa_fidelity for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, computed by the same kernels in the same order (so equal
 * bit for bit), but the per-block partial sums and reduction bookkeeping live
 * in a static device buffer of 66 KiB that the library holds on each GPU it
 * runs on until the process ends, instead of a per-call allocation.  The
 * workspace needed is 32 bytes per block of 256 amplitudes, capped at 2048
 * blocks (about 65 KiB) at every n; a size beyond the static buffer returns
 * QAOA_EINVAL.  The first call on a device looks the buffer up (no
 * allocation).  Both contexts must be on the same device.  Calls that
 * overlap on one GPU (from several threads) share the buffer and race: the
 * caller serialises them.  Synchronises a's stream. */
int qaoa_fidelity_noalloc(qaoa_ctx *a, qaoa_ctx *b, double *f_out);

/* Launch all further work of this context on an existing HIP stream
 * (hipStream_t passed as void*; NULL = the null stream).  The caller keeps
 * the stream alive while the context uses it.  Not a step of the paper's
 * method: it lets the simulator share a caller's (e.g. torch's) stream.
 * Synchronises the previous stream first. */
int qaoa_bind_stream(qaoa_ctx *ctx, void *hip_stream);

/* Use caller-owned device memory (e.g. a torch tensor) as the state vector
 * (the 2^n-amplitude array of Section 2.1, in the layout of qaoa_get_state).
 * bytes must be exactly 2^n * (16 for C128, 8 for C64); dev_ptr must be
 * 256-byte aligned device memory that outlives the context's use of it
 * (borrowed, never freed), else QAOA_EINVAL.  After a run the buffer holds
 * the final state in natural index order. */
int qaoa_bind_state(qaoa_ctx *ctx, void *dev_ptr, size_t bytes);

/* Per-pass kernel timing of later runs: when enabled, every pass launch is
 * bracketed by HIP events on the bound stream. */
int qaoa_set_profiling(qaoa_ctx *ctx, int enable);

/* Kernel times (ms) of the passes of the last run, in launch order (the
 * forward passes, then after qaoa_grad the backward passes; a chunked pass's
 * time spans its chunk launches on its stream), plus each pass's
 * algorithmic HBM bytes (state bytes read + written, both vectors for a
 * backward pass).  Fills at most max entries of ms[] and bytes[] (either may
 * be NULL) and returns the pass count through *count.  Synchronises the
 * stream.  Only runs made while profiling is enabled are timed. */
int qaoa_pass_times(qaoa_ctx *ctx, float *ms, double *bytes, int max, int *count);

/* Chunked pass pairs (tuning).  With three qubit sets, every layer is one
 * pass over the low set followed by one over a high set X; the pair is closed
 * under chunks that fix the top qubits of the third set.  Runs whose state
 * has at least min_state_bytes then execute each pair chunk by chunk (chunks
 * of at least chunk_bytes), the high-set pass of chunk k on a second stream
 * beside the low-set pass of chunk k + 1, so it reads its chunk while it is
 * still cached.  The result is bitwise the same as unchunked.  chunk_bytes =
 * 0 turns chunking off.  streams (2, 3 or 4, else QAOA_EINVAL): 2 runs the
 * high-set chunks on one extra stream, 3 alternates them over two, 4 also
 * alternates the low-set chunks over two streams.  Defaults: 128 MiB chunks
 * for states from 512 MiB (complex64 n >= 26, complex128 n >= 25) on three
 * streams. */
int qaoa_set_chunking(qaoa_ctx *ctx, size_t chunk_bytes, size_t min_state_bytes, int streams);

/* Inspection of the chunked pass pairs, no GPU needed (tests).  Chunk bits
 * F of an n-qubit depth-p plan for the given chunk size (0 = not chunked)
 * and, per pair, the memory bits its chunks fix (pair_fixed: up to max_pairs
 * entries; the pair count through *npairs). */
int qaoa_chunk_plan(int n, int prec, int p, size_t chunk_bytes, int *chunk_bits, uint64_t *pair_fixed,
                    int max_pairs, int *npairs);
/* The tile indices g of qubit set `set` that chunk k's launch covers, in
 * launch order: 2^(n - K - chunk_bits) entries into g_out (K = tile bits).
 * fixed_mem holds chunk_bits memory bits, all tile-index bits of the set, and
 * 0 <= k < 2^chunk_bits; QAOA_EINVAL otherwise. */
int qaoa_chunk_tiles(int n, int prec, int set, uint64_t fixed_mem, int chunk_bits, int64_t k, int64_t *g_out);

/* Measurement hook: pass `index` of the last run (forward passes in launch
 * order, then after qaoa_grad the backward passes), the qubit set it mixes
 * (0 = the low set) and the name of the kernel it ran, as the profiler
 * reports it without the parameter list (NUL-terminated, truncated to len).
 * QAOA_EINVAL for an index outside the last run. */
int qaoa_pass_kernel(qaoa_ctx *ctx, int index, int *set_out, char *name, size_t len);

/* Measurement hook: ms from the start of pass `first` to the end of pass
 * `last` of the last timed run (for chunked pass pairs, whose two passes
 * overlap on two streams, the pair's span is first = its low-set pass, last =
 * its high-set pass).  Synchronises the stream. */
int qaoa_pass_span(qaoa_ctx *ctx, int first, int last, float *ms);

/* Plan of a run of depth p: number of HBM passes, number of qubit sets the
 * mixer is split into, and the qubits per set (sizes[] up to max_sets). */
int qaoa_plan_info(qaoa_ctx *ctx, int p, int *passes, int *sets, int *sizes, int max_sets);

/* Memory layout of qubit set `set` (0 = the low set) of an n-qubit plan in
 * precision prec, for inspection and tests; needs no GPU and no context.
 * Writes the tile-bit count K to *k_out, then tpos[0..K): the memory bit of
 * each tile bit, gpos[0..n-K): the memory bit of each tile-index bit, and
 * (if not NULL) the same index map as runs, gmask[0..12) / gshift[0..12):
 * base offset of tile g = OR over r of (g & gmask[r]) << gshift[r].  tpos
 * needs 16 entries, gpos 64.  QAOA_EINVAL for n outside [1, 35] or a set
 * the plan does not have. */
int qaoa_tile_map(int n, int prec, int set, int *k_out, int8_t *tpos, int8_t *gpos, uint64_t *gmask,
                  int8_t *gshift);

/* Bandwidth reference (not a step of the method): copy bytes (a multiple of
 * 16) from src to dst, both device pointers, with a plain streaming kernel
 * on the given stream; block_bytes = 4096 or 16384 bytes per workgroup
 * (one or four 16-byte vectors per thread), else QAOA_EINVAL. */
int qaoa_copy_probe(const void *src, void *dst, size_t bytes, int block_bytes, void *hip_stream);

/* Thread-local message describing the last failure on this thread. */
const char *qaoa_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of <C> and gradient requests.
 * A scheduler thread admits queued requests while the sum of their device
 * footprints stays within hbm_budget_bytes and fewer than max_slots are
 * active, then advances every active request by one HBM pass per step, all
 * of a step's passes in one batched kernel launch.  Requests that arrive
 * while others run join at the next step; finished ones retire and free
 * their memory at once.  Each request's arithmetic (tiles, per-tile partial
 * slots, reduction order) is independent of what it shares a step with, so
 * its result is bitwise the same alone or in a mix.
 * ------------------------------------------------------------------------- */
typedef struct {
  int n;                  /* 1 <= n <= 35 */
  int num_edges;
  const int32_t *edges;   /* as in qaoa_create */
  const double *weights;  /* NULL = unweighted */
  int p;                  /* >= 0 */
  const double *gamma;    /* p values */
  const double *beta;     /* p values */
  int want_grad;          /* also return d<C>/dgamma, d<C>/dbeta */
} qaoa_request;

typedef struct {
  int status;             /* QAOA_OK or an error code */
  double expect, norm;
  double *dgamma, *dbeta; /* caller arrays of p doubles, filled when want_grad */
  double t_arrival, t_admit, t_done;  /* seconds on the server's clock */
} qaoa_result;

/* Start a server on the current device.  prec: QAOA_C64 or QAOA_C128. */
int qaoa_serve_create(size_t hbm_budget_bytes, int max_slots, int prec, qaoa_server **out);

/* Queue a request (inputs are copied).  A request whose footprint exceeds the
 * whole budget is refused with QAOA_ENOMEM.  *ticket identifies it.
 * arrival_time < 0 stamps the submit time; otherwise it is taken as the
 * arrival instant (server clock) for latency accounting. */
int qaoa_serve_submit(qaoa_server *srv, const qaoa_request *req, double arrival_time,
                      uint64_t *ticket);

/* Non-blocking: QAOA_OK with *out filled, QAOA_EPENDING, or the request's
 * error.  A collected result is forgotten by the server. */
int qaoa_serve_poll(qaoa_server *srv, uint64_t ticket, qaoa_result *out);

/* Blocking form of poll with a timeout in seconds (< 0 waits forever). */
int qaoa_serve_wait(qaoa_server *srv, uint64_t ticket, qaoa_result *out, double timeout_s);

/* Cancel a queued or running request; its result becomes QAOA_ECANCELED. */
int qaoa_serve_cancel(qaoa_server *srv, uint64_t ticket);

/* Throughput and latency (arrival -> done) over completed requests. */
int qaoa_serve_stats(qaoa_server *srv, double *req_per_s, double *p50_s, double *p99_s);

/* Seconds on the server's clock (the time base of t_arrival and friends). */
double qaoa_serve_clock(qaoa_server *srv);

/* Stop the scheduler; queued and running requests are cancelled. */
int qaoa_serve_destroy(qaoa_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* QAOA_H */
