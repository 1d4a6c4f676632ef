// C ABI of the vertex-tensor library: argument checks, workspace management and launch
// sequencing.  All device work is enqueued on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <sstream>

#include "eprl_internal.hpp"

using namespace eprl;

// One configuration of a batch: its plan, where its data sits in the batch workspace, and how
// its shell sum is split.
struct BatchEntry {
  Plan plan;
  bool ring = false;
  size_t tables = 0, boff = 0, kr = 0, sched = 0, partial = 0;  // byte offsets in the workspace
  int nchunk = 0;
  int64_t chunk = 0;
  std::vector<int> bounds;      // chunk bounds of the factorised path
  std::vector<double> ccost;    // estimated cost of each (i1, chunk), in x iterations
};

// The launch sequence of a laid-out batch (host data): replayed from a captured graph, or
// enqueued directly when per-kernel timing is on.
struct BatchSeq {
  std::vector<BatchEntry> ent;
  std::vector<const double *> B;
  std::vector<double *> A;
  int nring = 0, max_nd = 1, ncu = 256;
  int cls_begin[kRingClasses + 1] = {0};
  size_t params_off = 0, items_off = 0, counters_off = 0;
};

struct eprl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // grow-only device workspace
  char *ws = nullptr;
  size_t ws_size = 0;
  // Pinned staging for small host->device uploads: a ring of buffers, each reused once its
  // last copy has finished, so that the host waits for the device only when it runs
  // kStages calls ahead (never in steady state), not once per call.
  static constexpr int kStages = 8;
  char *stage[kStages] = {};
  size_t stage_size[kStages] = {};
  hipEvent_t stage_done[kStages] = {};
  bool stage_pending[kStages] = {};
  int stage_cur = 0;
  // Device address of the contraction's fixed scratch array on this context's device (looked
  // up once at creation, with the device current).
  double *scratch = nullptr;
  // Recorded on the old stream when the context moves to another one, which then waits for it:
  // work enqueued earlier still uses the workspace that later calls reuse.
  hipEvent_t handoff = nullptr;
  // factorial prime-exponent table (device), valid for arguments <= fact_max
  uint16_t *fexp = nullptr;
  int *primes = nullptr;
  int fact_max = -1;
  int nprime = 0;
  // algorithm: EPRL_ALGO_AUTO, EPRL_ALGO_SHELL or EPRL_ALGO_RING
  int algo = 0;
  // optional per-kernel timing
  bool timing = false;
  struct Rec {
    int kernel;
    hipEvent_t start, stop;
  };
  std::vector<Rec> recs;
  bool capturing = false;
  // Schedule per tile class of the factorised path (set by eprl_autotune or eprl_set_tuning):
  // workgroup target of the cost schedule (0: default) and booster staging level (-1: the
  // most that fits).
  int tune_wg[kRingClasses] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int tune_stg[kRingClasses] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
  // Cost schedule of the last configuration run in the factorised order (host data only; it
  // depends on the spins, dl and the workgroup target, and is recomputed when they change).
  std::vector<int> sched_key, sched_bounds;
  int sched_nchunk = 0;
  // Plan of the last configuration asked for (host data only, keyed by spins and dl).
  std::vector<int> plan_key;
  Plan plan_last;
  // Batched path: a dedicated workspace and the instantiated graph of the last batch.
  struct Batch {
    std::vector<int64_t> key;
    char *ws = nullptr;
    size_t ws_size = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;  // private stream the graph is captured on (default priority)
    BatchSeq seq;
  } batch;
};

namespace {

int fail(eprl_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(eprl_ctx *c, hipError_t e, const char *what) {
  std::ostringstream os;
  os << what << ": " << hipGetErrorString(e);
  return fail(c, EPRL_EHIP, os.str());
}

#define HIP_TRY(ctx, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// Brackets a launch with timing events when timing is enabled.
struct TimedLaunch {
  eprl_ctx *c;
  int kernel;
  hipEvent_t start = nullptr, stop = nullptr;
  TimedLaunch(eprl_ctx *c_, int k) : c(c_), kernel(k) {
    if (!c->timing || c->capturing) return;
    if (hipEventCreate(&start) != hipSuccess || hipEventCreate(&stop) != hipSuccess) {
      (void)hipGetLastError();
      start = stop = nullptr;
      return;
    }
    (void)hipEventRecord(start, c->stream);
  }
  ~TimedLaunch() {
    if (!start) return;
    (void)hipEventRecord(stop, c->stream);
    c->recs.push_back({kernel, start, stop});
  }
};

void clear_timing(eprl_ctx *c) {
  for (auto &r : c->recs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  c->recs.clear();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int ensure_workspace(eprl_ctx *c, size_t bytes) {
  if (bytes <= c->ws_size) return EPRL_OK;
  if (c->ws) {
    // Earlier work on the stream may still read the old workspace.
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_size = 0;
  }
  size_t want = std::max(bytes, c->ws_size * 3 / 2);
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    c->ws = nullptr;
    if (hipMalloc(&c->ws, bytes) != hipSuccess) {
      c->ws = nullptr;
      (void)hipGetLastError();
      return fail(c, EPRL_ENOMEM, "device workspace allocation failed");
    }
    want = bytes;
  }
  c->ws_size = want;
  return EPRL_OK;
}

// The next pinned staging buffer of the ring, at least `bytes` long; waits only for the last
// upload from that buffer (kStages uploads ago).
int staging(eprl_ctx *c, size_t bytes, char **out) {
  const int k = c->stage_cur = (c->stage_cur + 1) % eprl_ctx::kStages;
  if (c->stage_pending[k]) {
    HIP_TRY(c, hipEventSynchronize(c->stage_done[k]));
    c->stage_pending[k] = false;
  }
  if (bytes > c->stage_size[k]) {
    if (c->stage[k]) HIP_TRY(c, hipHostFree(c->stage[k]));
    c->stage[k] = nullptr;
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipHostMalloc((void **)&c->stage[k], want, hipHostMallocDefault) != hipSuccess) {
      c->stage[k] = nullptr;
      c->stage_size[k] = 0;
      (void)hipGetLastError();
      return fail(c, EPRL_ENOMEM, "pinned staging allocation failed");
    }
    c->stage_size[k] = want;
  }
  *out = c->stage[k];
  return EPRL_OK;
}

// Copies the first `bytes` of the current staging buffer to dst and marks it in flight.
int upload(eprl_ctx *c, void *dst, size_t bytes) {
  const int k = c->stage_cur;
  HIP_TRY(c, hipMemcpyAsync(dst, c->stage[k], bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipEventRecord(c->stage_done[k], c->stream));
  c->stage_pending[k] = true;
  return EPRL_OK;
}

// Forgets the instantiated graph of the last batch (it holds device pointers of the context,
// such as the factorial table, that are about to change).
void drop_batch_graph(eprl_ctx *c) {
  if (c->batch.exec) (void)hipGraphExecDestroy(c->batch.exec);
  if (c->batch.graph) (void)hipGraphDestroy(c->batch.graph);
  c->batch.exec = nullptr;
  c->batch.graph = nullptr;
  c->batch.key.clear();
}

int ensure_fexp(eprl_ctx *c, int fact_max) {
  if (fact_max <= c->fact_max) return EPRL_OK;
  fact_max = std::max(fact_max, 256);
  std::vector<int> pr = primes_upto(fact_max);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // A captured batch reads the table through its old address: it must be captured again.
  drop_batch_graph(c);
  if (c->fexp) HIP_TRY(c, hipFree(c->fexp));
  if (c->primes) HIP_TRY(c, hipFree(c->primes));
  c->fexp = nullptr;
  c->primes = nullptr;
  c->fact_max = -1;
  if (hipMalloc(&c->primes, pr.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&c->fexp, (size_t)(fact_max + 1) * pr.size() * sizeof(uint16_t)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, EPRL_ENOMEM, "factorial table allocation failed");
  }
  char *st;
  int rc = staging(c, pr.size() * sizeof(int), &st);
  if (rc) return rc;
  std::memcpy(st, pr.data(), pr.size() * sizeof(int));
  rc = upload(c, c->primes, pr.size() * sizeof(int));
  if (rc) return rc;
  HIP_TRY(c, launch_fexp_table(c->fexp, fact_max, c->primes, (int)pr.size(), c->stream));
  c->fact_max = fact_max;
  c->nprime = (int)pr.size();
  return EPRL_OK;
}

// The plan of (two_j, dl), made once and kept on the context until another configuration is
// asked for.  *out stays valid until the next call of plan_for on c.
int plan_for(eprl_ctx *c, const int two_j[10], int dl, const Plan **out) {
  std::vector<int> key(two_j, two_j + 10);
  key.push_back(dl);
  if (key != c->plan_key) {
    c->plan_key.clear();
    int rc = make_plan(two_j, dl, c->plan_last, c->err);
    if (rc) return rc;
    c->plan_key = key;
  }
  *out = &c->plan_last;
  return EPRL_OK;
}

// Device-side state of one configuration: tables built, metadata uploaded.
// Workgroups per launch of the factorised path: enough for several rounds of resident
// workgroups on 256 CUs, so that cost-balanced chunks finish together.  A batch uses the same
// schedule per configuration, which keeps its tensors bitwise equal to those of plain calls.
constexpr int kRingTargetWG = 8192;

struct Prepared {
  Plan plan;
  double *tables = nullptr;
  int64_t *boff = nullptr;
  int *kr = nullptr;
  int *sched = nullptr;  // chunk bounds of the factorised path, when asked for
  char *tail = nullptr;  // first free byte of the workspace after the above
};

// Plan, size the workspace (tables + metadata + `extra` bytes), upload metadata (and `sched`,
// if given) and build the 6j tables.  `extra` is placed at `prep.tail`.
int prepare(eprl_ctx *c, const int two_j[10], int dl, size_t extra, Prepared &prep,
            bool ring_tables = false, const std::vector<int> *sched = nullptr,
            const Plan *known = nullptr, bool any_dims = false) {
  int rc = EPRL_OK;
  if (known)
    prep.plan = *known;
  else
    rc = make_plan(two_j, dl, prep.plan, c->err);
  if (rc) return rc;
  Plan &p = prep.plan;
  if (!any_dims && (p.D == 0 || p.kmax > 16))
    return fail(c, EPRL_ERANGE, "intertwiner dimensions above 16 are not supported");
  rc = ensure_fexp(c, p.fact_max);
  if (rc) return rc;
  const size_t tbytes = align_up((size_t)p.toff[5] * sizeof(double), 256);
  const size_t bbytes = align_up(p.boff.size() * sizeof(int64_t), 256);
  const size_t kbytes = align_up(p.kr.size() * sizeof(int), 256);
  const size_t sbytes = sched ? align_up(sched->size() * sizeof(int), 256) : 0;
  rc = ensure_workspace(c, tbytes + bbytes + kbytes + sbytes + extra);
  if (rc) return rc;
  prep.tables = reinterpret_cast<double *>(c->ws);
  prep.boff = reinterpret_cast<int64_t *>(c->ws + tbytes);
  prep.kr = reinterpret_cast<int *>(c->ws + tbytes + bbytes);
  prep.sched = sched ? reinterpret_cast<int *>(c->ws + tbytes + bbytes + kbytes) : nullptr;
  prep.tail = c->ws + tbytes + bbytes + kbytes + sbytes;
  char *st;
  rc = staging(c, bbytes + kbytes + sbytes, &st);
  if (rc) return rc;
  std::memcpy(st, p.boff.data(), p.boff.size() * sizeof(int64_t));
  std::memcpy(st + bbytes, p.kr.data(), p.kr.size() * sizeof(int));
  if (sched) std::memcpy(st + bbytes + kbytes, sched->data(), sched->size() * sizeof(int));
  rc = upload(c, prep.boff, bbytes + kbytes + sbytes);
  if (rc) return rc;
  TableParams tp;
  std::memcpy(tp.two_j, p.two_j, sizeof(tp.two_j));
  tp.nd = p.nd;
  tp.i1_lo2 = p.i[0].lo2;
  tp.i1_n = p.i[0].n;
  for (int e = 0; e < 4; ++e) {
    tp.K_lo2[e] = p.K[e].lo2;
    tp.K_n[e] = p.K[e].n;
  }
  tp.X_lo2 = p.X.lo2;
  tp.NX = p.X.n;
  for (int t = 0; t < 6; ++t) tp.toff[t] = p.toff[t];
  tp.tables = prep.tables;
  tp.fexp = c->fexp;
  tp.primes = c->primes;
  tp.nprime = c->nprime;
  {
    TimedLaunch tl(c, 0);
    if (ring_tables)
      HIP_TRY(c, launch_ring_tables(tp, p.toff[5], c->stream));
    else
      HIP_TRY(c, launch_sixj_tables(tp, p.toff[5], c->stream));
  }
  return EPRL_OK;
}

VertexParams vertex_params(const Prepared &prep, const double *B) {
  const Plan &p = prep.plan;
  VertexParams vp;
  std::memset(&vp, 0, sizeof(vp));
  std::memcpy(vp.two_j, p.two_j, sizeof(vp.two_j));
  vp.nd = p.nd;
  for (int e = 0; e < 5; ++e) {
    vp.i_lo2[e] = p.i[e].lo2;
    vp.i_n[e] = p.i[e].n;
  }
  for (int e = 0; e < 4; ++e) {
    vp.K_lo2[e] = p.K[e].lo2;
    vp.K_n[e] = p.K[e].n;
  }
  vp.X_lo2 = p.X.lo2;
  vp.NX = p.X.n;
  for (int t = 0; t < 5; ++t) {
    const double *tab = prep.tables + p.toff[t];
    if (t == 0) vp.T1 = tab;
    if (t == 1) vp.T2 = tab;
    if (t == 2) vp.T3 = tab;
    if (t == 3) vp.T4 = tab;
    if (t == 4) vp.T5 = tab;
  }
  vp.B = B;
  vp.boff = prep.boff;
  vp.kr = prep.kr;
  return vp;
}

int check_ctx(eprl_ctx *c) { return c ? EPRL_OK : EPRL_EINVAL; }

ReduceParams reduce_params(const Plan &p, const double *partial, int nchunk, double *A,
                           int accumulate) {
  ReduceParams rp;
  rp.partial = partial;
  rp.nchunk = nchunk;
  rp.a_size = p.a_size;
  for (int e = 0; e < 5; ++e) {
    rp.i_lo2[e] = p.i[e].lo2;
    rp.i_n[e] = p.i[e].n;
  }
  rp.A = A;
  rp.accumulate = accumulate;
  return rp;
}

// Kernel parameters of the factorised order for a prepared configuration (ring tables).
RingParams ring_params(const Prepared &prep, const double *B) {
  const Plan &p = prep.plan;
  RingParams rp;
  std::memset(&rp, 0, sizeof(rp));
  std::memcpy(rp.two_j, p.two_j, sizeof(rp.two_j));
  rp.nd = p.nd;
  for (int e = 0; e < 5; ++e) {
    rp.i_lo2[e] = p.i[e].lo2;
    rp.i_n[e] = p.i[e].n;
  }
  for (int e = 0; e < 4; ++e) {
    rp.K_lo2[e] = p.K[e].lo2;
    rp.K_n[e] = p.K[e].n;
  }
  rp.X_lo2 = p.X.lo2;
  rp.NX = p.X.n;
  rp.U1 = prep.tables + p.toff[0];
  rp.U2 = prep.tables + p.toff[1];
  rp.U3 = prep.tables + p.toff[2];
  rp.U4 = prep.tables + p.toff[3];
  rp.U5 = prep.tables + p.toff[4];
  rp.B = B;
  rp.boff = prep.boff;
  rp.kr = prep.kr;
  rp.kw = p.ring_kw;
  rp.nrb = ring_row_blocks(p);
  return rp;
}

// Factorised evaluation over the cores [core_lo, core_hi) (core_hi < 0: all cores), every
// l23 and l45 inside: one launch of the ring kernel, then the reduction.
int ring_impl(eprl_ctx *c, const int two_j[10], int dl, const double *B, int accumulate,
              double *A, const Plan &probe, int core_lo = 0, int core_hi = -1) {
  const int cls = probe.ring_cls;
  const int target = c->tune_wg[cls] > 0 ? c->tune_wg[cls] : kRingTargetWG;
  std::vector<int> key(two_j, two_j + 10);
  key.push_back(dl);
  key.push_back(target);
  key.push_back(cls);
  key.push_back(core_lo);
  key.push_back(core_hi);
  if (key != c->sched_key) {
    c->sched_nchunk = ring_schedule(probe, target, c->sched_bounds, nullptr, core_lo, core_hi);
    c->sched_key = key;
  }
  const std::vector<int> &bounds = c->sched_bounds;
  const int nchunk = c->sched_nchunk;
  const size_t pbytes = align_up((size_t)nchunk * probe.a_size * sizeof(double), 256);
  Prepared prep;
  int rc = prepare(c, two_j, dl, pbytes, prep, true, &bounds, &probe);
  if (rc) return rc;
  const Plan &p = prep.plan;
  RingParams rp = ring_params(prep, B);
  rp.partial = reinterpret_cast<double *>(prep.tail);
  rp.bounds = prep.sched;
  rp.nchunk = nchunk;
  rp.kw = p.ring_kw;
  rp.nrb = ring_row_blocks(p);
  {
    TimedLaunch tl(c, 4);
    if (p.ring_cls == kWideClass)
      HIP_TRY(c, launch_wide(rp, c->stream));
    else
      HIP_TRY(c, launch_ring(rp, p.ring_cls, c->tune_stg[p.ring_cls], c->stream));
  }
  ReduceParams red = reduce_params(p, rp.partial, nchunk, A, accumulate);
  {
    TimedLaunch tl(c, 2);
    HIP_TRY(c, launch_reduce(red, c->stream));
  }
  return EPRL_OK;
}

int vertex_range_impl(eprl_ctx *c, const int two_j[10], int dl, double gamma, const double *B,
                      int64_t sb, int64_t se, int accumulate, double *A) {
  if (!(gamma > 0.0) || !std::isfinite(gamma))
    return fail(c, EPRL_EINVAL, "gamma must be finite and positive");
  if (!B || !A) return fail(c, EPRL_EINVAL, "null booster or output pointer");
  const Plan *pp = nullptr;
  int rc = plan_for(c, two_j, dl, &pp);
  if (rc) return rc;
  const Plan &probe = *pp;
  if (sb < 0 || se > probe.nshell || sb > se)
    return fail(c, EPRL_EINVAL, "shell range outside [0, (dl+1)^6]");
  const int D = probe.D;
  if (D == 0) return fail(c, EPRL_ERANGE, "intertwiner dimensions above 16 are not supported");
  const bool full = sb == 0 && se == probe.nshell;
  const bool ring_forced = c->algo == EPRL_ALGO_RING || c->algo == EPRL_ALGO_RING_VALU;
  if (ring_forced && (!full || probe.ring_KW == 0))
    return fail(c, EPRL_ERANGE,
                "the factorised path needs the full shell range, i and k ranges <= 16 and core "
                "windows <= 32");
  if (full && c->algo != EPRL_ALGO_SHELL && probe.ring_KW != 0) {
    if (c->algo == EPRL_ALGO_RING_VALU && probe.ring_cls != probe.ring_cls8) {
      Plan q = probe;
      q.ring_cls = q.ring_cls8;
      return ring_impl(c, two_j, dl, B, accumulate, A, q);
    }
    return ring_impl(c, two_j, dl, B, accumulate, A, probe);
  }
  const int64_t nrange = std::max<int64_t>(se - sb, 1);
  const int target_wg = D == 8 ? 4096 : 1024;
  int nchunk = std::max(1, target_wg / probe.i[0].n);
  int64_t chunk = (nrange + nchunk - 1) / nchunk;
  nchunk = (int)((nrange + chunk - 1) / chunk);
  const size_t pbytes = align_up((size_t)nchunk * probe.a_size * sizeof(double), 256);
  Prepared prep;
  rc = prepare(c, two_j, dl, pbytes, prep, false, nullptr, &probe);
  if (rc) return rc;
  VertexParams vp = vertex_params(prep, B);
  vp.partial = reinterpret_cast<double *>(prep.tail);
  vp.shell_begin = sb;
  vp.shell_end = se;
  vp.chunk = chunk;
  vp.nchunk = nchunk;
  {
    TimedLaunch tl(c, 1);
    HIP_TRY(c, launch_assemble(vp, D, c->stream));
  }
  ReduceParams rp;
  rp.partial = vp.partial;
  rp.nchunk = nchunk;
  rp.a_size = prep.plan.a_size;
  for (int e = 0; e < 5; ++e) {
    rp.i_lo2[e] = prep.plan.i[e].lo2;
    rp.i_n[e] = prep.plan.i[e].n;
  }
  rp.A = A;
  rp.accumulate = accumulate;
  {
    TimedLaunch tl(c, 2);
    HIP_TRY(c, launch_reduce(rp, c->stream));
  }
  return EPRL_OK;
}

int vertex_cores_impl(eprl_ctx *c, const int two_j[10], int dl, double gamma, const double *B,
                      int64_t cb, int64_t ce, int accumulate, double *A) {
  if (!(gamma > 0.0) || !std::isfinite(gamma))
    return fail(c, EPRL_EINVAL, "gamma must be finite and positive");
  if (!B || !A) return fail(c, EPRL_EINVAL, "null booster or output pointer");
  if (c->algo == EPRL_ALGO_SHELL)
    return fail(c, EPRL_EINVAL, "core ranges are units of the factorised order, not of the per-shell order");
  const Plan *pp = nullptr;
  int rc = plan_for(c, two_j, dl, &pp);
  if (rc) return rc;
  const Plan &probe = *pp;
  const int64_t ncore = (int64_t)probe.nd * probe.nd * probe.nd * probe.nd;
  if (cb < 0 || ce > ncore || cb > ce)
    return fail(c, EPRL_EINVAL, "core range outside [0, (dl+1)^4]");
  if (probe.D == 0) return fail(c, EPRL_ERANGE, "intertwiner dimensions above 16 are not supported");
  if (probe.ring_KW == 0)
    return fail(c, EPRL_ERANGE,
                "the factorised path needs i and k ranges <= 16 and core windows <= 32");
  if (c->algo == EPRL_ALGO_RING_VALU && probe.ring_cls != probe.ring_cls8) {
    Plan q = probe;
    q.ring_cls = q.ring_cls8;
    return ring_impl(c, two_j, dl, B, accumulate, A, q, (int)cb, (int)ce);
  }
  return ring_impl(c, two_j, dl, B, accumulate, A, probe, (int)cb, (int)ce);
}

// ---- batched path ------------------------------------------------------------------------
//
// All configurations of a batch share one dedicated workspace laid out once per batch shape:
// for each configuration its 6j tables, booster offsets and k ranges, and its per-chunk partial
// sums; then the RingParams array and the work list of the persistent ring kernel.  The
// device work (table builds, one persistent ring launch for every configuration the
// factorised path handles, per-shell launches for the others, reductions) is captured once
// into a hipGraph and replayed while the batch (spins, shell counts, pointers, algorithm)
// stays the same.  Chunking per configuration equals the single-configuration path, so every
// tensor is bitwise identical to a separate eprl_vertex_tensor call.


int batch_chunks(const Plan &p, bool ring, int target_wg, int &nchunk, int64_t &chunk,
                 std::vector<int> &bounds, std::vector<double> &ccost) {
  if (ring) {
    nchunk = ring_schedule(p, target_wg > 0 ? target_wg : kRingTargetWG, bounds, &ccost);
    chunk = 0;
  } else {
    const int target_wg = p.D == 8 ? 4096 : 1024;
    nchunk = std::max(1, target_wg / p.i[0].n);
    chunk = (p.nshell + nchunk - 1) / nchunk;
    nchunk = (int)((p.nshell + chunk - 1) / chunk);
  }
  return EPRL_OK;
}

TableParams table_params(const Plan &p, double *tables, const eprl_ctx *c) {
  TableParams tp;
  std::memcpy(tp.two_j, p.two_j, sizeof(tp.two_j));
  tp.nd = p.nd;
  tp.i1_lo2 = p.i[0].lo2;
  tp.i1_n = p.i[0].n;
  for (int e = 0; e < 4; ++e) {
    tp.K_lo2[e] = p.K[e].lo2;
    tp.K_n[e] = p.K[e].n;
  }
  tp.X_lo2 = p.X.lo2;
  tp.NX = p.X.n;
  for (int t = 0; t < 6; ++t) tp.toff[t] = p.toff[t];
  tp.tables = tables;
  tp.fexp = c->fexp;
  tp.primes = c->primes;
  tp.nprime = c->nprime;
  return tp;
}

// Enqueues the device work of the laid-out batch on c->stream: the 6j tables of every
// configuration, the work-queue counters (reset by a kernel, so that graph replays start from
// 0), one persistent ring launch per tile class, per-shell launches for configurations the
// factorised order does not handle, and the reductions.  Outside a capture each launch is
// bracketed by the timing events when timing is on.
hipError_t enqueue_batch(eprl_ctx *c) {
  const BatchSeq &seq = c->batch.seq;
  char *ws = c->batch.ws;
  const int n = (int)seq.ent.size();
  hipError_t e = hipSuccess;
  for (int q = 0; q < n && e == hipSuccess; ++q) {
    const BatchEntry &b = seq.ent[q];
    TableParams tp = table_params(b.plan, reinterpret_cast<double *>(ws + b.tables), c);
    TimedLaunch tl(c, 0);
    e = b.ring ? launch_ring_tables(tp, b.plan.toff[5], c->stream)
               : launch_sixj_tables(tp, b.plan.toff[5], c->stream);
  }
  int *counters = reinterpret_cast<int *>(ws + seq.counters_off);
  if (e == hipSuccess && seq.nring > 0) e = launch_reset_counters(counters, kRingClasses, c->stream);
  for (int cls = 0; cls < kRingClasses && e == hipSuccess; ++cls) {
    const int nit = seq.cls_begin[cls + 1] - seq.cls_begin[cls];
    if (nit == 0) continue;
    if (cls == kWideClass) {
      // One 8-wavefront workgroup per CU, LDS sized for the largest configuration of the class;
      // booster blocks staged when every configuration's fit.
      size_t shm = 0, shm_stg = 0;
      bool stg = true;
      for (const BatchEntry &b : seq.ent)
        if (b.ring && b.plan.ring_cls == kWideClass) {
          int dims[5];
          for (int q = 0; q < 5; ++q) dims[q] = b.plan.i[q].n;
          shm = std::max(shm, wide_smem_bytes(b.plan.nd, dims, b.plan.ring_kw, b.plan.ring_nrb, false));
          shm_stg = std::max(shm_stg, wide_smem_bytes(b.plan.nd, dims, b.plan.ring_kw, b.plan.ring_nrb, true));
          stg = stg && wide_fits(b.plan.nd, dims, b.plan.ring_kw, b.plan.ring_nrb, true);
        }
      TimedLaunch tl(c, 6);
      e = launch_wide_batch(reinterpret_cast<const RingParams *>(ws + seq.params_off),
                            reinterpret_cast<const int *>(ws + seq.items_off) + 4 * seq.cls_begin[cls],
                            nit, stg ? shm_stg : shm, stg, std::min(nit, seq.ncu), counters + cls, c->stream);
      continue;
    }
    // Enough workgroups to fill the chip at the occupancy the tile class allows.
    const size_t shm = ring_smem_bytes(cls, seq.max_nd, c->tune_stg[cls]);
    const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / std::max<size_t>(shm, 1))));
    const int grid = (int)std::min<int>(nit, seq.ncu * per_cu);
    TimedLaunch tl(c, 6);
    e = launch_ring_batch(reinterpret_cast<const RingParams *>(ws + seq.params_off),
                          reinterpret_cast<const int *>(ws + seq.items_off) + 4 * seq.cls_begin[cls],
                          nit, cls, seq.max_nd, c->tune_stg[cls], grid, counters + cls, c->stream);
  }
  for (int q = 0; q < n && e == hipSuccess; ++q) {
    const BatchEntry &b = seq.ent[q];
    if (b.ring) continue;
    Prepared prep;
    prep.plan = b.plan;
    prep.tables = reinterpret_cast<double *>(ws + b.tables);
    prep.boff = reinterpret_cast<int64_t *>(ws + b.boff);
    prep.kr = reinterpret_cast<int *>(ws + b.kr);
    VertexParams vp = vertex_params(prep, seq.B[q]);
    vp.partial = reinterpret_cast<double *>(ws + b.partial);
    vp.shell_begin = 0;
    vp.shell_end = b.plan.nshell;
    vp.chunk = b.chunk;
    vp.nchunk = b.nchunk;
    TimedLaunch tl(c, 1);
    e = launch_assemble(vp, b.plan.D, c->stream);
  }
  for (int q = 0; q < n && e == hipSuccess; ++q) {
    const BatchEntry &b = seq.ent[q];
    ReduceParams red = reduce_params(b.plan, reinterpret_cast<double *>(ws + b.partial), b.nchunk,
                                     seq.A[q], 0);
    TimedLaunch tl(c, 2);
    e = launch_reduce(red, c->stream);
  }
  return e;
}

// Runs the current batch: a replay of its graph, or, with per-kernel timing on, the same
// launch sequence enqueued directly so that every launch can be timed.
int run_batch(eprl_ctx *c) {
  if (c->timing) {
    hipError_t e = enqueue_batch(c);
    if (e != hipSuccess) return hip_fail(c, e, "batched launch sequence");
    return EPRL_OK;
  }
  HIP_TRY(c, hipGraphLaunch(c->batch.exec, c->stream));
  return EPRL_OK;
}

// layout_dl (may be null): configuration q reads its boosters from a buffer packed for
// layout_dl[q] >= dl[q] shells per link (the blocks of its own spins found by their offsets in
// that larger layout).
int batched_impl(eprl_ctx *c, int n, const int *two_j, const int *dl,
                 const double *const *boosters, double *const *A, const int *layout_dl = nullptr) {
  std::vector<int64_t> key;
  key.push_back(n);
  key.push_back(c->algo);
  key.push_back(layout_dl != nullptr);
  if (layout_dl)
    for (int q = 0; q < n; ++q) key.push_back(layout_dl[q]);
  for (int q = 0; q < kRingClasses; ++q) {
    key.push_back(c->tune_wg[q]);
    key.push_back(c->tune_stg[q]);
  }
  for (int q = 0; q < n; ++q) {
    for (int t = 0; t < 10; ++t) key.push_back(two_j[10 * q + t]);
    key.push_back(dl[q]);
    key.push_back((int64_t)(uintptr_t)boosters[q]);
    key.push_back((int64_t)(uintptr_t)A[q]);
    if (!boosters[q] || !A[q]) return fail(c, EPRL_EINVAL, "null booster or output pointer");
  }
  if (c->batch.exec && key == c->batch.key) return run_batch(c);
  // New batch shape: plan every configuration and lay out the workspace.
  std::vector<BatchEntry> ent(n);
  size_t off = 0;
  int fact_max = 0, max_nd = 1;
  for (int q = 0; q < n; ++q) {
    BatchEntry &b = ent[q];
    std::string err;
    int rc = make_plan(two_j + 10 * q, dl[q], b.plan, err);
    if (rc) {
      std::ostringstream os;
      os << "configuration " << q << ": " << err;
      return fail(c, rc, os.str());
    }
    if (layout_dl && layout_dl[q] != dl[q]) {
      Plan pl;
      if (layout_dl[q] < dl[q]) return fail(c, EPRL_EINVAL, "booster layout smaller than the shells");
      rc = make_plan(two_j + 10 * q, layout_dl[q], pl, err);
      if (rc) return fail(c, rc, err);
      const int nd = b.plan.nd, nd3 = nd * nd * nd, ndl = pl.nd, ndl3 = ndl * ndl * ndl;
      for (int e = 0; e < 4; ++e)
        for (int t = 0; t < nd3; ++t) {
          const int tl = ((t / (nd * nd)) * ndl + (t / nd) % nd) * ndl + t % nd;
          b.plan.boff[(size_t)e * nd3 + t] = pl.boff[(size_t)e * ndl3 + tl];
        }
      b.plan.boff[4 * (size_t)nd3] = pl.boff[4 * (size_t)ndl3];
    }
    const Plan &p = b.plan;
    if (p.D == 0) return fail(c, EPRL_ERANGE, "intertwiner dimensions above 16 are not supported");
    b.ring = c->algo != EPRL_ALGO_SHELL && p.ring_KW != 0;
    if ((c->algo == EPRL_ALGO_RING || c->algo == EPRL_ALGO_RING_VALU) && !b.ring)
      return fail(c, EPRL_ERANGE, "the factorised path does not apply to every configuration");
    if (c->algo == EPRL_ALGO_RING_VALU) b.plan.ring_cls = b.plan.ring_cls8;
    batch_chunks(p, b.ring, p.ring_cls >= 0 ? c->tune_wg[p.ring_cls] : 0, b.nchunk, b.chunk,
                 b.bounds, b.ccost);
    fact_max = std::max(fact_max, p.fact_max);
    if (b.ring) max_nd = std::max(max_nd, p.nd);
    b.tables = off;
    off += align_up((size_t)p.toff[5] * sizeof(double), 256);
    b.boff = off;
    off += align_up(p.boff.size() * sizeof(int64_t), 256);
    b.kr = off;
    off += align_up(p.kr.size() * sizeof(int), 256);
    b.sched = off;
    off += align_up(b.bounds.size() * sizeof(int), 256);
    b.partial = off;
    off += align_up((size_t)b.nchunk * p.a_size * sizeof(double), 256);
  }
  // Work lists of the persistent kernels, one per tile class: (configuration, chunk, i1, row
  // block), longest first.
  struct Item {
    double cost;
    int cfg, chunk, n1, rb;
  };
  std::vector<Item> cls_items[kRingClasses];
  std::vector<int> ring_index(n, -1);
  int nring = 0;
  for (int q = 0; q < n; ++q) {
    if (!ent[q].ring) continue;
    ring_index[q] = nring++;
    // Cost of an item: the chunk's x iterations (from the schedule) times the size of the
    // A(i1) slice, which sets the work of the final contraction of each iteration.
    const Plan &p = ent[q].plan;
    const double slice = (double)p.i[1].n * p.i[2].n * p.i[3].n * p.i[4].n;
    const int cls = p.ring_cls, nrb = ring_row_blocks(p), nch = ent[q].nchunk;
    for (int ch = 0; ch < nch; ++ch)
      for (int n1 = 0; n1 < p.i[0].n; ++n1) {
        const double cost = ent[q].ccost[(size_t)n1 * nch + ch] * slice;
        for (int rb = 0; rb < nrb; ++rb) cls_items[cls].push_back({cost, ring_index[q], ch, n1, rb});
      }
  }
  std::vector<Item> items;
  int cls_begin[kRingClasses + 1] = {0};
  for (int cls = 0; cls < kRingClasses; ++cls) {
    std::stable_sort(cls_items[cls].begin(), cls_items[cls].end(),
                     [](const Item &a, const Item &b) { return a.cost > b.cost; });
    items.insert(items.end(), cls_items[cls].begin(), cls_items[cls].end());
    cls_begin[cls + 1] = (int)items.size();
  }
  const size_t params_off = off;
  off += align_up((size_t)std::max(nring, 1) * sizeof(RingParams), 256);
  const size_t items_off = off;
  off += align_up(std::max<size_t>(items.size(), 1) * 4 * sizeof(int), 256);
  const size_t counters_off = off;  // one work-queue counter per tile class
  off += 256;
  int rc = ensure_fexp(c, fact_max);
  if (rc) return rc;
  // Drop the previous graph and workspace.
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  drop_batch_graph(c);
  if (off > c->batch.ws_size) {
    if (c->batch.ws) (void)hipFree(c->batch.ws);
    c->batch.ws = nullptr;
    c->batch.ws_size = 0;
    if (hipMalloc(&c->batch.ws, off) != hipSuccess) {
      (void)hipGetLastError();
      c->batch.ws = nullptr;
      return fail(c, EPRL_ENOMEM, "batch workspace allocation failed");
    }
    c->batch.ws_size = off;
  }
  char *ws = c->batch.ws;
  // Metadata upload (outside the graph; the workspace belongs to this batch only).
  std::vector<RingParams> params(std::max(nring, 1));
  for (int q = 0; q < n; ++q) {
    if (!ent[q].ring) continue;
    const Plan &p = ent[q].plan;
    RingParams &rp = params[ring_index[q]];
    std::memset(&rp, 0, sizeof(rp));
    std::memcpy(rp.two_j, p.two_j, sizeof(rp.two_j));
    rp.nd = p.nd;
    for (int e = 0; e < 5; ++e) {
      rp.i_lo2[e] = p.i[e].lo2;
      rp.i_n[e] = p.i[e].n;
    }
    for (int e = 0; e < 4; ++e) {
      rp.K_lo2[e] = p.K[e].lo2;
      rp.K_n[e] = p.K[e].n;
    }
    rp.X_lo2 = p.X.lo2;
    rp.NX = p.X.n;
    const double *tab = reinterpret_cast<const double *>(ws + ent[q].tables);
    rp.U1 = tab + p.toff[0];
    rp.U2 = tab + p.toff[1];
    rp.U3 = tab + p.toff[2];
    rp.U4 = tab + p.toff[3];
    rp.U5 = tab + p.toff[4];
    rp.B = boosters[q];
    rp.boff = reinterpret_cast<const int64_t *>(ws + ent[q].boff);
    rp.kr = reinterpret_cast<const int *>(ws + ent[q].kr);
    rp.partial = reinterpret_cast<double *>(ws + ent[q].partial);
    rp.bounds = reinterpret_cast<const int *>(ws + ent[q].sched);
    rp.nchunk = ent[q].nchunk;
    rp.kw = p.ring_kw;
    rp.nrb = ring_row_blocks(p);
  }
  // Compact staging of the metadata blocks: (workspace offset, bytes) in staging order.
  std::vector<std::pair<size_t, size_t>> blocks;
  size_t sbytes = 0;
  for (int q = 0; q < n; ++q) {
    blocks.push_back({ent[q].boff, ent[q].partial - ent[q].boff});  // boff and kr
    sbytes += ent[q].partial - ent[q].boff;
  }
  blocks.push_back({params_off, off - params_off});                  // params and items
  sbytes += off - params_off;
  char *st;
  rc = staging(c, sbytes, &st);
  if (rc) return rc;
  {
    size_t so = 0;
    for (int q = 0; q < n; ++q) {
      const Plan &p = ent[q].plan;
      std::memcpy(st + so, p.boff.data(), p.boff.size() * sizeof(int64_t));
      std::memcpy(st + so + (ent[q].kr - ent[q].boff), p.kr.data(), p.kr.size() * sizeof(int));
      if (!ent[q].bounds.empty())
        std::memcpy(st + so + (ent[q].sched - ent[q].boff), ent[q].bounds.data(),
                    ent[q].bounds.size() * sizeof(int));
      so += ent[q].partial - ent[q].boff;
    }
    std::memcpy(st + so, params.data(), params.size() * sizeof(RingParams));
    std::vector<int> flat(std::max<size_t>(items.size(), 1) * 4, 0);
    for (size_t k = 0; k < items.size(); ++k) {
      flat[4 * k] = items[k].cfg;
      flat[4 * k + 1] = items[k].chunk;
      flat[4 * k + 2] = items[k].n1;
      flat[4 * k + 3] = items[k].rb;
    }
    std::memcpy(st + so + (items_off - params_off), flat.data(), flat.size() * sizeof(int));
    so = 0;
    for (auto &b : blocks) {
      HIP_TRY(c, hipMemcpyAsync(ws + b.first, st + so, b.second, hipMemcpyHostToDevice, c->stream));
      so += b.second;
    }
  }
  HIP_TRY(c, hipEventRecord(c->stage_done[c->stage_cur], c->stream));
  c->stage_pending[c->stage_cur] = true;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  BatchSeq &seq = c->batch.seq;
  seq.ent = std::move(ent);
  seq.B.assign(boosters, boosters + n);
  seq.A.assign(A, A + n);
  seq.nring = nring;
  seq.max_nd = max_nd;
  std::copy(cls_begin, cls_begin + kRingClasses + 1, seq.cls_begin);
  seq.params_off = params_off;
  seq.items_off = items_off;
  seq.counters_off = counters_off;
  seq.ncu = 256;
  (void)hipDeviceGetAttribute(&seq.ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  // Capture the device work on a private stream (the caller's stream may be the null stream,
  // which cannot be captured); the graph is then launched on the caller's stream.
  if (!c->batch.cap) HIP_TRY(c, hipStreamCreateWithFlags(&c->batch.cap, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  c->stream = c->batch.cap;
  hipError_t eb = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) {
    c->stream = user;
    return hip_fail(c, eb, "hipStreamBeginCapture");
  }
  c->capturing = true;
  hipError_t e = enqueue_batch(c);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
  c->capturing = false;
  c->stream = user;
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(c, e, "batched launch sequence");
  }
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  c->batch.graph = graph;
  c->batch.exec = exec;
  c->batch.key = key;
  return run_batch(c);
}

}  // namespace

extern "C" {

int eprl_create(eprl_ctx **out, int device, void *hip_stream) {
  if (!out) return EPRL_EINVAL;
  *out = nullptr;
  eprl_ctx *c = new (std::nothrow) eprl_ctx;
  if (!c) return EPRL_ENOMEM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  bool ok = hipSetDevice(device) == hipSuccess && ring_init_attributes() == hipSuccess &&
            contract_scratch_address(&c->scratch) == hipSuccess;
  for (int k = 0; ok && k < eprl_ctx::kStages; ++k)
    ok = hipEventCreateWithFlags(&c->stage_done[k], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->handoff, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    for (int k = 0; k < eprl_ctx::kStages; ++k)
      if (c->stage_done[k]) (void)hipEventDestroy(c->stage_done[k]);
    if (c->handoff) (void)hipEventDestroy(c->handoff);
    delete c;
    return EPRL_EHIP;
  }
  *out = c;
  return EPRL_OK;
}

void eprl_destroy(eprl_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->ws) (void)hipFree(c->ws);
  for (int k = 0; k < eprl_ctx::kStages; ++k) {
    if (c->stage[k]) (void)hipHostFree(c->stage[k]);
    if (c->stage_done[k]) (void)hipEventDestroy(c->stage_done[k]);
  }
  if (c->handoff) (void)hipEventDestroy(c->handoff);
  if (c->fexp) (void)hipFree(c->fexp);
  if (c->primes) (void)hipFree(c->primes);
  if (c->batch.exec) (void)hipGraphExecDestroy(c->batch.exec);
  if (c->batch.graph) (void)hipGraphDestroy(c->batch.graph);
  if (c->batch.ws) (void)hipFree(c->batch.ws);
  if (c->batch.cap) (void)hipStreamDestroy(c->batch.cap);
  clear_timing(c);
  delete c;
}

const char *eprl_last_error(const eprl_ctx *c) { return c ? c->err.c_str() : "null context"; }

int eprl_set_algorithm(eprl_ctx *c, int algo) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (algo != EPRL_ALGO_AUTO && algo != EPRL_ALGO_SHELL && algo != EPRL_ALGO_RING &&
      algo != EPRL_ALGO_RING_VALU)
    return fail(c, EPRL_EINVAL, "unknown algorithm");
  c->algo = algo;
  return EPRL_OK;
}

int eprl_set_tuning(eprl_ctx *c, int tile_class, int target_workgroups, int staging_level) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (tile_class < 0 || tile_class >= kRingClasses)
    return fail(c, EPRL_EINVAL, "tile class outside 0..8");
  if (target_workgroups != 0 && (target_workgroups < 64 || target_workgroups > (1 << 20)))
    return fail(c, EPRL_EINVAL, "workgroup target must be 0 or in 64..2^20");
  if (staging_level < -1 || staging_level > 2)
    return fail(c, EPRL_EINVAL, "staging level must be -1, 0, 1 or 2");
  c->tune_wg[tile_class] = target_workgroups;
  c->tune_stg[tile_class] = staging_level;
  return EPRL_OK;
}

int eprl_autotune(eprl_ctx *c, const int two_j[10], int dl, const double *B, double *A,
                  int out[3]) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!B || !A || !out) return fail(c, EPRL_EINVAL, "null pointer");
  Plan p;
  int rc = make_plan(two_j, dl, p, c->err);
  if (rc) return rc;
  if (p.ring_cls < 0) return fail(c, EPRL_ERANGE, "no tile class of the factorised order applies");
  const int cls = p.ring_cls;
  int levels[3];
  const int nl = ring_stage_levels(cls, p.nd, levels);
  static const int kTargets[] = {2048, 4096, 8192, 16384};
  const int saved_algo = c->algo, saved_wg = c->tune_wg[cls], saved_stg = c->tune_stg[cls];
  c->algo = EPRL_ALGO_RING;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    c->algo = saved_algo;
    return hip_fail(c, hipGetLastError(), "hipEventCreate");
  }
  float best = 0.0f;
  int best_wg = kRingTargetWG, best_stg = -1;
  for (int li = 0; li < nl && rc == EPRL_OK; ++li) {
    for (int t : kTargets) {
      c->tune_wg[cls] = t;
      c->tune_stg[cls] = levels[li];
      rc = vertex_range_impl(c, two_j, dl, 1.0, B, 0, p.nshell, 0, A);  // warm-up
      if (rc) break;
      // The fastest of three timed calls (single calls vary by a few per cent).
      float ms = 0.0f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep < 3 && rc == EPRL_OK && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess) rc = vertex_range_impl(c, two_j, dl, 1.0, B, 0, p.nshell, 0, A);
        if (rc) break;
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float one = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&one, e0, e1);
        if (e == hipSuccess && (rep == 0 || one < ms)) ms = one;
      }
      if (rc) break;
      if (e != hipSuccess) {
        rc = hip_fail(c, e, "autotune timing");
        break;
      }
      if (best == 0.0f || ms < best) {
        best = ms;
        best_wg = t;
        best_stg = levels[li];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->algo = saved_algo;
  if (rc) {
    c->tune_wg[cls] = saved_wg;
    c->tune_stg[cls] = saved_stg;
    return rc;
  }
  c->tune_wg[cls] = best_wg;
  c->tune_stg[cls] = best_stg;
  out[0] = cls;
  out[1] = best_wg;
  out[2] = best_stg;
  return EPRL_OK;
}

int eprl_set_stream(eprl_ctx *c, void *hip_stream) {
  if (check_ctx(c)) return EPRL_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (s == c->stream) return EPRL_OK;
  // Order the new stream after everything already enqueued on the old one.
  HIP_TRY(c, hipEventRecord(c->handoff, c->stream));
  HIP_TRY(c, hipStreamWaitEvent(s, c->handoff, 0));
  c->stream = s;
  return EPRL_OK;
}

int eprl_layout(const int two_j[10], int dl, int dims_i[5], int two_ilo[5], int64_t *booster_offsets) {
  Plan p;
  std::string err;
  int rc = make_plan(two_j, dl, p, err);
  if (rc) return rc;
  for (int e = 0; e < 5; ++e) {
    if (dims_i) dims_i[e] = p.i[e].n;
    if (two_ilo) two_ilo[e] = p.i[e].lo2;
  }
  if (booster_offsets) std::copy(p.boff.begin(), p.boff.end(), booster_offsets);
  return EPRL_OK;
}

int eprl_count_terms(const int two_j[10], int dl, int64_t *live_shells, double *terms) {
  Plan p;
  std::string err;
  int rc = make_plan(two_j, dl, p, err);
  if (rc) return rc;
  int64_t live;
  double t;
  count_terms(p, live, t);
  if (live_shells) *live_shells = live;
  if (terms) *terms = t;
  return EPRL_OK;
}

int eprl_count_work(const int two_j[10], int dl, double out[5]) {
  if (!out) return EPRL_EINVAL;
  Plan p;
  std::string err;
  int rc = make_plan(two_j, dl, p, err);
  if (rc) return rc;
  count_work(p, out);
  return EPRL_OK;
}

int eprl_vertex_tensor(eprl_ctx *c, const int two_j[10], int dl, double gamma, const double *B,
                       double *A) {
  if (check_ctx(c)) return EPRL_EINVAL;
  Plan probe;
  int rc = make_plan(two_j, dl, probe, c->err);
  if (rc) return rc;
  return vertex_range_impl(c, two_j, dl, gamma, B, 0, probe.nshell, 0, A);
}

int eprl_bf_vertex_tensor(eprl_ctx *c, const int two_j[10], double *A) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!A) return fail(c, EPRL_EINVAL, "null output pointer");
  Prepared prep;
  int rc = prepare(c, two_j, 0, 0, prep, false, nullptr, nullptr, true);
  if (rc) return rc;
  VertexParams vp = vertex_params(prep, nullptr);
  TimedLaunch tl(c, 5);
  HIP_TRY(c, launch_bf_vertex(vp, A, prep.plan.a_size, c->stream));
  return EPRL_OK;
}

int eprl_vertex_tensor_range(eprl_ctx *c, const int two_j[10], int dl, double gamma,
                             const double *B, int64_t shell_begin, int64_t shell_end,
                             int accumulate, double *A) {
  if (check_ctx(c)) return EPRL_EINVAL;
  return vertex_range_impl(c, two_j, dl, gamma, B, shell_begin, shell_end, accumulate ? 1 : 0, A);
}

int eprl_vertex_tensor_cores(eprl_ctx *c, const int two_j[10], int dl, double gamma,
                             const double *B, int64_t core_begin, int64_t core_end, int accumulate,
                             double *A) {
  if (check_ctx(c)) return EPRL_EINVAL;
  return vertex_cores_impl(c, two_j, dl, gamma, B, core_begin, core_end, accumulate ? 1 : 0, A);
}

int eprl_vertex_tensor_batched(eprl_ctx *c, int n, const int *two_j, const int *dl, double gamma,
                               const double *const *boosters, double *const *A) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (n < 0 || (n > 0 && (!two_j || !dl || !boosters || !A)))
    return fail(c, EPRL_EINVAL, "invalid batch arguments");
  if (!(gamma > 0.0) || !std::isfinite(gamma))
    return fail(c, EPRL_EINVAL, "gamma must be finite and positive");
  if (n == 0) return EPRL_OK;
  return batched_impl(c, n, two_j, dl, boosters, A);
}

int eprl_vertex_tensor_scan(eprl_ctx *c, const int two_j[10], int dl_max, double gamma,
                            const double *B, double *A) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!(gamma > 0.0) || !std::isfinite(gamma))
    return fail(c, EPRL_EINVAL, "gamma must be finite and positive");
  if (!two_j || !B || !A) return fail(c, EPRL_EINVAL, "null argument");
  if (dl_max < 0) return fail(c, EPRL_EINVAL, "dl_max must be >= 0");
  const Plan *pp = nullptr;
  int rc = plan_for(c, two_j, dl_max, &pp);
  if (rc) return rc;
  const int64_t a_size = pp->a_size;
  const int n = dl_max + 1;
  std::vector<int> tj((size_t)10 * n), dl(n), lay(n, dl_max);
  std::vector<const double *> bp(n, B);
  std::vector<double *> ap(n);
  for (int d = 0; d < n; ++d) {
    std::copy(two_j, two_j + 10, tj.begin() + 10 * d);
    dl[d] = d;
    ap[d] = A + (size_t)d * a_size;
  }
  return batched_impl(c, n, tj.data(), dl.data(), bp.data(), ap.data(), lay.data());
}

int eprl_contract_boundary(eprl_ctx *c, const int dims_i[5], const double *A,
                           const double *const psi[5], double *F) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!dims_i || !A || !psi || !F) return fail(c, EPRL_EINVAL, "null argument");
  ContractParams cp;
  for (int e = 0; e < 5; ++e) {
    if (dims_i[e] <= 0 || !psi[e]) return fail(c, EPRL_EINVAL, "invalid dimension or vector");
    cp.n[e] = dims_i[e];
    cp.psi[e] = psi[e];
  }
  cp.A = A;
  cp.nblocks = 256;
  int rc = ensure_workspace(c, cp.nblocks * 2 * sizeof(double));
  if (rc) return rc;
  cp.partial = reinterpret_cast<double *>(c->ws);
  HIP_TRY(c, launch_contract(cp, F, c->stream));
  return EPRL_OK;
}

int eprl_contract_boundary_noalloc(eprl_ctx *c, const int dims_i[5], const double *A,
                                   const double *const psi[5], double *F) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!dims_i || !A || !psi || !F) return fail(c, EPRL_EINVAL, "null argument");
  if (!c->scratch) return fail(c, EPRL_EHIP, "contraction scratch address unavailable");
  ContractParams cp;
  for (int e = 0; e < 5; ++e) {
    if (dims_i[e] <= 0 || !psi[e]) return fail(c, EPRL_EINVAL, "invalid dimension or vector");
    cp.n[e] = dims_i[e];
    cp.psi[e] = psi[e];
  }
  cp.A = A;
  cp.nblocks = 256;
  if (cp.nblocks > kContractScratchSlots)
    return fail(c, EPRL_ERANGE, "more partial sums than the fixed scratch holds");
  // Every block writes its own slot before the final kernel reads it: nothing to clear.
  cp.partial = c->scratch;
  HIP_TRY(c, launch_contract(cp, F, c->stream));
  return EPRL_OK;
}

int eprl_contract_boundary_adjoint(eprl_ctx *c, const int two_j[10], int dl, const double *B,
                                   const double *A, const double *const psi[5],
                                   const double grad_F[2], double *const grad_psi[5],
                                   double *grad_boosters) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!psi || !grad_F) return fail(c, EPRL_EINVAL, "null argument");
  for (int e = 0; e < 5; ++e)
    if (!psi[e]) return fail(c, EPRL_EINVAL, "null boundary vector");
  Plan probe;
  int rc = make_plan(two_j, dl, probe, c->err);
  if (rc) return rc;
  if (grad_psi) {
    bool any = false;
    for (int e = 0; e < 5; ++e) any = any || grad_psi[e];
    if (any) {
      if (!A) return fail(c, EPRL_EINVAL, "the vertex tensor is needed for dF/dpsi");
      ContractParams cp;
      for (int e = 0; e < 5; ++e) {
        cp.n[e] = probe.i[e].n;
        cp.psi[e] = psi[e];
      }
      cp.A = A;
      cp.nblocks = 0;
      cp.partial = nullptr;
      HIP_TRY(c, launch_grad_psi(cp, grad_F[0], grad_F[1], grad_psi, c->stream));
    }
  }
  if (!grad_boosters) return EPRL_OK;
  if (!B) return fail(c, EPRL_EINVAL, "null booster pointer");
  if (probe.kmax > 16) return fail(c, EPRL_ERANGE, "intertwiner dimensions above 16 are not supported");
  if (c->algo != EPRL_ALGO_SHELL && probe.ring_KW != 0 && probe.nd <= kAdjRingMaxNd) {
    // Factorised order: per-core G vectors, then a fixed-order sum per booster entry.
    Prepared prep;
    rc = prepare(c, two_j, dl, align_up(adjoint_ring_gbuf_bytes(probe.nd), 256), prep, true, nullptr,
                 &probe);
    if (rc) return rc;
    RingParams rp = ring_params(prep, B);
    TimedLaunch tl(c, 3);
    HIP_TRY(c, launch_adjoint_ring(rp, psi, reinterpret_cast<double *>(prep.tail), prep.plan.boff.back(),
                                   grad_F[0], grad_F[1], grad_boosters, c->stream));
    return EPRL_OK;
  }
  const int kpad = std::max(probe.kmax, 1);
  const size_t gbytes = align_up((size_t)probe.nshell * 4 * kpad * 2 * sizeof(double), 256);
  Prepared prep;
  rc = prepare(c, two_j, dl, gbytes, prep);
  if (rc) return rc;
  AdjointParams ap;
  ap.v = vertex_params(prep, B);
  ap.v.shell_begin = 0;
  ap.v.shell_end = prep.plan.nshell;
  for (int e = 0; e < 5; ++e) ap.psi[e] = psi[e];
  ap.shell_g = reinterpret_cast<double *>(prep.tail);
  ap.kpad = kpad;
  {
    TimedLaunch tl(c, 3);
    HIP_TRY(c, launch_adjoint_shells(ap, c->stream));
  }
  HIP_TRY(c, launch_adjoint_reduce(ap, prep.plan.boff.back(), grad_F[0], grad_F[1], grad_boosters,
                                   c->stream));
  return EPRL_OK;
}

int eprl_sixj_batch(eprl_ctx *c, int n, const int *args, double *out) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (n < 0 || (n > 0 && (!args || !out))) return fail(c, EPRL_EINVAL, "invalid arguments");
  if (n == 0) return EPRL_OK;
  int big = 0;
  for (int q = 0; q < 6 * n; ++q) {
    if (args[q] < 0 || args[q] > kSixjMaxTwo)
      return fail(c, EPRL_ERANGE, "6j argument outside 0..200 (two_j)");
    big = std::max(big, args[q]);
  }
  int rc = ensure_fexp(c, 2 * big + 2);
  if (rc) return rc;
  const size_t bytes = (size_t)n * 6 * sizeof(int);
  rc = ensure_workspace(c, bytes);
  if (rc) return rc;
  char *st;
  rc = staging(c, bytes, &st);
  if (rc) return rc;
  std::memcpy(st, args, bytes);
  rc = upload(c, c->ws, bytes);
  if (rc) return rc;
  HIP_TRY(c, launch_sixj_batch(reinterpret_cast<int *>(c->ws), n, out, c->fexp, c->primes,
                               c->nprime, c->fact_max, c->stream));
  return EPRL_OK;
}

int eprl_shell_fifteenj(eprl_ctx *c, const int two_j[10], int dl, int64_t shell, int kdims[4],
                        double *W, int64_t capacity) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!kdims || !W) return fail(c, EPRL_EINVAL, "null argument");
  Plan probe;
  int rc = make_plan(two_j, dl, probe, c->err);
  if (rc) return rc;
  if (shell < 0 || shell >= probe.nshell) return fail(c, EPRL_EINVAL, "shell index out of range");
  const int nd = probe.nd, nd3 = nd * nd * nd;
  int o[6];
  int64_t r = shell;
  for (int q = 5; q >= 0; --q) {
    o[q] = (int)(r % nd);
    r /= nd;
  }
  const int t[4] = {(o[0] * nd + o[1]) * nd + o[2], (o[3] * nd + o[4]) * nd + o[0],
                    (o[5] * nd + o[1]) * nd + o[3], (o[2] * nd + o[4]) * nd + o[5]};
  int64_t need = probe.i[0].n;
  for (int e = 0; e < 4; ++e) {
    kdims[e] = probe.kr[(e * nd3 + t[e]) * 2 + 1];
    need *= kdims[e];
  }
  if (need > capacity) return fail(c, EPRL_EINVAL, "output capacity too small");
  if (need == 0) return EPRL_OK;
  if (probe.kmax > 16) return fail(c, EPRL_ERANGE, "intertwiner dimensions above 16 are not supported");
  Prepared prep;
  rc = prepare(c, two_j, dl, 0, prep);
  if (rc) return rc;
  VertexParams vp = vertex_params(prep, nullptr);
  HIP_TRY(c, launch_shell_fifteenj(vp, shell, W, c->stream));
  return EPRL_OK;
}

int eprl_timing_enable(eprl_ctx *c, int enable) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (c->stream) HIP_TRY(c, hipStreamSynchronize(c->stream));
  else HIP_TRY(c, hipDeviceSynchronize());
  clear_timing(c);
  c->timing = enable != 0;
  return EPRL_OK;
}

int eprl_timing_read(eprl_ctx *c, int kernel, double *total_ms, int64_t *launches) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (c->stream) HIP_TRY(c, hipStreamSynchronize(c->stream));
  else HIP_TRY(c, hipDeviceSynchronize());
  double total = 0.0;
  int64_t n = 0;
  for (auto &r : c->recs) {
    if (r.kernel != kernel) continue;
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, r.start, r.stop));
    total += ms;
    ++n;
  }
  if (total_ms) *total_ms = total;
  if (launches) *launches = n;
  return EPRL_OK;
}

}  // extern "C"
