// C ABI of the vertex-tensor library: argument checks, workspace management and launch
// sequencing.  All device work is enqueued on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
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
  int towner = -1;              // configuration whose 6j tables this one reads (itself: builds them)
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
  int nring = 0, ncu = 256;
  // One persistent launch per group of items: a tile class and, for the 8-wide classes, one nd
  // (their LDS, and so their occupancy, is sized for the group's nd); items [begin, end) of the
  // work list, estimated cost (sum of item costs), work-queue counter `group index`.
  struct Group {
    int cls, nd, begin, end;
    double cost;
    int xoff;  // wide class: index (in ints, from items_off) of its nine per-XCD list offsets
  };
  std::vector<Group> groups;
  size_t params_off = 0, items_off = 0, counters_off = 0;
};

// Streams beside the capture stream on which the batch's persistent launches run concurrently
// inside the captured graph (all at the default priority).
constexpr int kBatchSide = 3;

struct eprl_ctx {
  int device = 0;
  int ncu = 256;  // compute units of the device
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
  std::vector<int> adj_order_key, adj_order;  // launch order of the factorised adjoint's cores
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
    hipStream_t side[kBatchSide] = {};
    hipEvent_t fork = nullptr, join[kBatchSide] = {};
    BatchSeq seq;
  } batch;
};

namespace {

// Whether the ring tables of plan r hold every entry the factorised kernels read for plan q: the
// same spins, at least as many spin offsets, and virtual-spin and x ranges that contain q's.
bool tables_contain(const Plan &r, const Plan &q) {
  if (r.nd < q.nd) return false;
  for (int t = 0; t < 10; ++t)
    if (r.two_j[t] != q.two_j[t]) return false;
  if (r.i[0].lo2 != q.i[0].lo2 || r.i[0].n != q.i[0].n) return false;
  auto inside = [](int rlo, int rn, int qlo, int qn) {
    if (qn <= 0) return true;
    return rn > 0 && ((qlo - rlo) & 1) == 0 && rlo <= qlo && rlo + 2 * (rn - 1) >= qlo + 2 * (qn - 1);
  };
  for (int e = 0; e < 4; ++e)
    if (!inside(r.K[e].lo2, r.K[e].n, q.K[e].lo2, q.K[e].n)) return false;
  return inside(r.X.lo2, r.X.n, q.X.lo2, q.X.n);
}

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
  rp.tnd = p.nd;
  rp.xlo2 = p.X.lo2;
  rp.xhi2 = p.X.lo2 + 2 * (p.X.n - 1);
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
  // Partial sums, then the eight work-queue counters of the persistent wide kernel.
  int rc = prepare(c, two_j, dl, pbytes + 256, prep, true, &bounds, &probe);
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
      HIP_TRY(c, launch_wide(rp, reinterpret_cast<int *>(prep.tail + pbytes), c->ncu, c->stream));
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

// ---- booster builder (host side) -----------------------------------------------------------

// Gauss-Legendre nodes (ascending) and weights of n points on [-1, 1], by Newton's method on
// the Legendre recurrence in long double.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L)), dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p1 = 1.0L, p2 = 0.0L;
      for (int k = 1; k <= n; ++k) {
        const long double p3 = p2;
        p2 = p1;
        p1 = ((2.0L * k - 1.0L) * z * p2 - (k - 1.0L) * p3) / k;
      }
      dp = n * (z * p1 - p2) / (z * z - 1.0L);
      const long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    x[i] = (double)-z;
    x[n - 1 - i] = (double)z;
    w[i] = w[n - 1 - i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
  }
}

// Jacobi-form constants of d^J_{m' m} (two-unit arguments).
void jacobi_constants(int J2, int mp2, int m2, double &norm, int &mu, int &nu, int &s) {
  mu = std::abs(m2 - mp2) / 2;
  nu = std::abs(m2 + mp2) / 2;
  s = (J2 - std::max(std::abs(m2), std::abs(mp2))) / 2;
  long double f = 1.0L;
  for (int q = 1; q <= nu; ++q) f *= (long double)(s + mu + q) / (long double)(s + q);
  const double xi = (m2 >= mp2 || ((mp2 - m2) / 2) % 2 == 0) ? 1.0 : -1.0;
  norm = xi * (double)std::sqrt(f);
}

// r nodes of the booster quadrature with n subintervals of u = e^{-r} in (0, 1], |I_k| =
// k * 2 / (n (n + 1)): the 30-point rule's nodes, then the 61-point rule's; weights include
// du / u and sinh^2 r / (4 pi).
void booster_r_nodes(int n, const std::vector<double> (&gx)[2], const std::vector<double> (&gw)[2],
                     std::vector<double> &r, std::vector<double> &rw) {
  r.clear();
  rw.clear();
  const double dx = 2.0 / ((double)n * (n + 1));
  const double four_pi = 4.0 * 3.14159265358979323846;
  for (int rule = 0; rule < 2; ++rule) {
    double lo = 0.0;
    for (int k = 1; k <= n; ++k) {
      const double hi = k < n ? lo + k * dx : 1.0;
      for (size_t p = 0; p < gx[rule].size(); ++p) {
        const double u = lo + (hi - lo) * (gx[rule][p] + 1.0) / 2.0;
        const double rr = -std::log(u);
        const double sh = std::sinh(rr);
        r.push_back(rr);
        rw.push_back(gw[rule][p] * (hi - lo) / 2.0 / u * sh * sh / four_pi);
      }
      lo = hi;
    }
  }
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
    if (b.towner != q) continue;  // reads another configuration's tables
    TableParams tp = table_params(b.plan, reinterpret_cast<double *>(ws + b.tables), c);
    TimedLaunch tl(c, 0);
    e = b.ring ? launch_ring_tables(tp, b.plan.toff[5], c->stream)
               : launch_sixj_tables(tp, b.plan.toff[5], c->stream);
  }
  int *counters = reinterpret_cast<int *>(ws + seq.counters_off);
  const int ngroup = (int)seq.groups.size();
  if (e == hipSuccess && ngroup > 0) e = launch_reset_counters(counters, 8 * ngroup, c->stream);
  // Inside a capture the groups run on up to 1 + kBatchSide streams (graph branches), the
  // costliest group first, each on the stream with the least work so far; outside a capture
  // (timed launches) they run one after the other on the context's stream.
  hipStream_t main = c->stream;
  const int nstream = c->capturing ? std::min(ngroup, 1 + kBatchSide) : 1;
  std::vector<hipStream_t> streams(std::max(nstream, 1), main);
  if (e == hipSuccess && nstream > 1) {
    e = hipEventRecord(c->batch.fork, main);
    for (int q = 1; q < nstream && e == hipSuccess; ++q) {
      streams[q] = c->batch.side[q - 1];
      e = hipStreamWaitEvent(streams[q], c->batch.fork, 0);
    }
  }
  std::vector<double> load(streams.size(), 0.0);
  std::vector<int> order(ngroup);
  for (int g = 0; g < ngroup; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return seq.groups[a].cost > seq.groups[b].cost; });
  for (int oi = 0; oi < ngroup && e == hipSuccess; ++oi) {
    const int g = order[oi];
    const BatchSeq::Group &gr = seq.groups[g];
    const int cls = gr.cls, nit = gr.end - gr.begin;
    const int si = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[si] += gr.cost;
    c->stream = streams[si];
    const int *items = reinterpret_cast<const int *>(ws + seq.items_off) + 4 * gr.begin;
    const RingParams *params = reinterpret_cast<const RingParams *>(ws + seq.params_off);
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
      const int *xoff = reinterpret_cast<const int *>(ws + seq.items_off) + gr.xoff;
      e = launch_wide_batch(params, items, xoff, nit, stg ? shm_stg : shm, stg,
                            std::min(nit, seq.ncu), counters + 8 * g, c->stream);
    } else {
      // Enough workgroups to fill the chip at the occupancy the group's LDS allows.
      const size_t shm = ring_smem_bytes(cls, gr.nd, c->tune_stg[cls]);
      const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / std::max<size_t>(shm, 1))));
      const int grid = (int)std::min<int>(nit, seq.ncu * per_cu);
      TimedLaunch tl(c, 6);
      e = launch_ring_batch(params, items, nit, cls, gr.nd, c->tune_stg[cls], grid, counters + 8 * g,
                            c->stream);
    }
  }
  c->stream = main;
  for (int q = 1; q < nstream && e == hipSuccess; ++q) {
    e = hipEventRecord(c->batch.join[q - 1], streams[q]);
    if (e == hipSuccess) e = hipStreamWaitEvent(main, c->batch.join[q - 1], 0);
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
  int fact_max = 0;
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
    b.boff = off;
    off += align_up(p.boff.size() * sizeof(int64_t), 256);
    b.kr = off;
    off += align_up(p.kr.size() * sizeof(int), 256);
    b.sched = off;
    off += align_up(b.bounds.size() * sizeof(int), 256);
    b.partial = off;
    off += align_up((size_t)b.nchunk * p.a_size * sizeof(double), 256);
  }
  // 6j tables: a factorised configuration whose table index ranges (virtual spins, x, spin
  // offsets) lie inside those of another of the same spins reads that one's tables, the one with
  // the most spin offsets (the levels of a shell scan share the tables of the largest dl); the
  // others build their own.
  for (int q = 0; q < n; ++q) {
    ent[q].towner = q;
    if (!ent[q].ring) continue;
    for (int r = 0; r < n; ++r)
      if (r != q && ent[r].ring && ent[r].plan.nd > ent[ent[q].towner].plan.nd &&
          tables_contain(ent[r].plan, ent[q].plan))
        ent[q].towner = r;
  }
  for (int q = 0; q < n; ++q) {  // containment is transitive: follow to a builder
    int t = ent[q].towner;
    while (ent[t].towner != t) t = ent[t].towner;
    ent[q].towner = t;
  }
  for (int q = 0; q < n; ++q)
    if (ent[q].towner == q) {
      ent[q].tables = off;
      off += align_up((size_t)ent[q].plan.toff[5] * sizeof(double), 256);
    }
  for (int q = 0; q < n; ++q) ent[q].tables = ent[ent[q].towner].tables;
  // Work lists of the persistent kernels, one per group: (configuration, chunk, i1, row block),
  // longest first.
  struct Item {
    double cost;
    int cfg, chunk, n1, rb;
  };
  // Groups: (tile class, nd) for the 8-wide classes, the whole wide class as one.
  std::map<std::pair<int, int>, std::vector<Item>> grouped;
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
    std::vector<Item> &dst = grouped[{cls, cls == kWideClass ? 0 : p.nd}];
    for (int ch = 0; ch < nch; ++ch)
      for (int n1 = 0; n1 < p.i[0].n; ++n1) {
        const double cost = ent[q].ccost[(size_t)n1 * nch + ch] * slice;
        for (int rb = 0; rb < nrb; ++rb) dst.push_back({cost, ring_index[q], ch, n1, rb});
      }
  }
  std::vector<Item> items;
  std::vector<BatchSeq::Group> groups;
  std::vector<int> xoffs;  // per wide group: nine per-XCD list offsets
  for (auto &kv : grouped) {
    std::vector<Item> &v = kv.second;
    BatchSeq::Group g{kv.first.first, kv.first.second, (int)items.size(), 0, 0.0, -1};
    for (const Item &it : v) g.cost += it.cost;
    if (g.cls != kWideClass) {
      std::stable_sort(v.begin(), v.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
      items.insert(items.end(), v.begin(), v.end());
    } else {
      // Chunks (configuration, chunk, row block) with all their i1 items, longest first, each to
      // the XCD list with the least work so far; in a list the chunks keep that order and the
      // items of a chunk stay together (longest first).
      std::map<std::tuple<int, int, int>, std::vector<Item>> chunks;
      for (const Item &it : v) chunks[std::make_tuple(it.cfg, it.chunk, it.rb)].push_back(it);
      std::vector<std::pair<double, std::vector<Item> *>> order;
      for (auto &ck : chunks) {
        double cost = 0.0;
        for (const Item &it : ck.second) cost += it.cost;
        std::stable_sort(ck.second.begin(), ck.second.end(),
                         [](const Item &a, const Item &b) { return a.cost > b.cost; });
        order.push_back({cost, &ck.second});
      }
      std::stable_sort(order.begin(), order.end(),
                       [](const std::pair<double, std::vector<Item> *> &a,
                          const std::pair<double, std::vector<Item> *> &b) { return a.first > b.first; });
      std::vector<Item> lists[8];
      double load[8] = {0.0};
      for (auto &o : order) {
        const int x = (int)(std::min_element(load, load + 8) - load);
        load[x] += o.first;
        lists[x].insert(lists[x].end(), o.second->begin(), o.second->end());
      }
      g.xoff = (int)xoffs.size();
      for (int x = 0; x < 8; ++x) {
        xoffs.push_back((int)(items.size() - g.begin));
        items.insert(items.end(), lists[x].begin(), lists[x].end());
      }
      xoffs.push_back((int)(items.size() - g.begin));
    }
    g.end = (int)items.size();
    groups.push_back(g);
  }
  // The per-XCD offsets follow the items in the same device array.
  for (BatchSeq::Group &g : groups)
    if (g.xoff >= 0) g.xoff += 4 * (int)items.size();
  const size_t params_off = off;
  off += align_up((size_t)std::max(nring, 1) * sizeof(RingParams), 256);
  const size_t items_off = off;
  off += align_up((std::max<size_t>(items.size(), 1) * 4 + xoffs.size()) * sizeof(int), 256);
  const size_t counters_off = off;  // eight work-queue counters per group
  off += align_up(std::max<size_t>(groups.size(), 1) * 8 * sizeof(int), 256);
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
    const Plan &tp = ent[ent[q].towner].plan;  // geometry of the tables it reads
    for (int e = 0; e < 4; ++e) {
      rp.K_lo2[e] = tp.K[e].lo2;
      rp.K_n[e] = tp.K[e].n;
    }
    rp.X_lo2 = tp.X.lo2;
    rp.NX = tp.X.n;
    rp.tnd = tp.nd;
    rp.xlo2 = p.X.lo2;
    rp.xhi2 = p.X.lo2 + 2 * (p.X.n - 1);
    const double *tab = reinterpret_cast<const double *>(ws + ent[q].tables);
    rp.U1 = tab + tp.toff[0];
    rp.U2 = tab + tp.toff[1];
    rp.U3 = tab + tp.toff[2];
    rp.U4 = tab + tp.toff[3];
    rp.U5 = tab + tp.toff[4];
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
    std::vector<int> flat(std::max<size_t>(items.size(), 1) * 4 + xoffs.size(), 0);
    for (size_t k = 0; k < items.size(); ++k) {
      flat[4 * k] = items[k].cfg;
      flat[4 * k + 1] = items[k].chunk;
      flat[4 * k + 2] = items[k].n1;
      flat[4 * k + 3] = items[k].rb;
    }
    std::copy(xoffs.begin(), xoffs.end(), flat.begin() + 4 * items.size());
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
  seq.groups = std::move(groups);
  seq.params_off = params_off;
  seq.items_off = items_off;
  seq.counters_off = counters_off;
  seq.ncu = 256;
  (void)hipDeviceGetAttribute(&seq.ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  // Capture the device work on a private stream (the caller's stream may be the null stream,
  // which cannot be captured); the graph is then launched on the caller's stream.
  if (!c->batch.cap) HIP_TRY(c, hipStreamCreateWithFlags(&c->batch.cap, hipStreamNonBlocking));
  if (!c->batch.fork) HIP_TRY(c, hipEventCreateWithFlags(&c->batch.fork, hipEventDisableTiming));
  for (int q = 0; q < kBatchSide; ++q) {
    if (!c->batch.side[q]) HIP_TRY(c, hipStreamCreateWithFlags(&c->batch.side[q], hipStreamNonBlocking));
    if (!c->batch.join[q]) HIP_TRY(c, hipEventCreateWithFlags(&c->batch.join[q], hipEventDisableTiming));
  }
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
            contract_scratch_address(&c->scratch) == hipSuccess &&
            hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess;
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
  for (int q = 0; q < kBatchSide; ++q) {
    if (c->batch.side[q]) (void)hipStreamDestroy(c->batch.side[q]);
    if (c->batch.join[q]) (void)hipEventDestroy(c->batch.join[q]);
  }
  if (c->batch.fork) (void)hipEventDestroy(c->batch.fork);
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

int eprl_contract_vertices(eprl_ctx *c, const int dims_i[5], const double *A, const double *B,
                           double *F) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!dims_i || !A || !B || !F) return fail(c, EPRL_EINVAL, "null argument");
  int64_t total = 1;
  for (int e = 0; e < 5; ++e) {
    if (dims_i[e] <= 0) return fail(c, EPRL_EINVAL, "invalid dimension");
    total *= dims_i[e];
  }
  const int nblocks = (int)std::min<int64_t>(256, (total + 2047) / 2048);
  int rc = ensure_workspace(c, (size_t)nblocks * sizeof(double));
  if (rc) return rc;
  HIP_TRY(c, launch_contract_vertices(A, B, total, nblocks, reinterpret_cast<double *>(c->ws), F,
                                      c->stream));
  return EPRL_OK;
}

int eprl_contract_trailing(eprl_ctx *c, const int dims_i[5], const double *A, int m,
                           const double *const *psi, double *T) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!dims_i || !A || !psi || !T) return fail(c, EPRL_EINVAL, "null argument");
  if (m < 1 || m > 5) return fail(c, EPRL_EINVAL, "between one and five vectors");
  for (int e = 0; e < 5; ++e)
    if (dims_i[e] <= 0) return fail(c, EPRL_EINVAL, "invalid dimension");
  for (int q = 0; q < m; ++q)
    if (!psi[q]) return fail(c, EPRL_EINVAL, "null vector");
  if (m == 5) {  // all five: the boundary contraction
    const double *p5[5] = {psi[0], psi[1], psi[2], psi[3], psi[4]};
    return eprl_contract_boundary(c, dims_i, A, p5, T);
  }
  TrailParams tp;
  std::memset(&tp, 0, sizeof(tp));
  tp.A = A;
  tp.m = m;
  int64_t nlead = 1;
  tp.S = 1;
  for (int e = 0; e < 5 - m; ++e) nlead *= dims_i[e];
  for (int q = 0; q < m; ++q) {
    tp.n[q] = dims_i[5 - m + q];
    tp.psi[q] = psi[q];
    tp.S *= tp.n[q];
  }
  tp.nsplit = trailing_splits(nlead, tp.S);
  tp.T = T;
  if (tp.nsplit > 1) {
    int rc = ensure_workspace(c, (size_t)nlead * tp.nsplit * 2 * sizeof(double));
    if (rc) return rc;
    tp.partial = reinterpret_cast<double *>(c->ws);
  }
  HIP_TRY(c, launch_contract_trailing(tp, nlead, c->stream));
  return EPRL_OK;
}

int eprl_contract_delta3(eprl_ctx *c, int n, int two_klo, int two_x, const double *TA,
                         const double *TB, const double *TC, double *F) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!TA || !TB || !TC || !F) return fail(c, EPRL_EINVAL, "null argument");
  if (n < 1 || n > 256) return fail(c, EPRL_EINVAL, "bulk intertwiner range must hold 1..256 values");
  if (two_klo < 0 || two_x < 0 || (two_klo & 1) || (two_x & 1))
    return fail(c, EPRL_EINVAL, "bulk intertwiners and the internal spin must be integer spins");
  HIP_TRY(c, launch_delta3(n, two_klo, two_x, TA, TB, TC, F, c->stream));
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
  int akl = 0, aiw = 0, akw = 0, ang = 1;
  if (c->algo != EPRL_ALGO_SHELL && probe.ring_KW != 0 && probe.nd <= kAdjRingMaxNd)
    adjoint_ring_dims(probe, akl, aiw, akw, ang);
  if (akl > 0 && adjoint_ring_smem(probe.nd, akl, aiw, akw, ang) <= kAdjRingMaxLds) {
    // Factorised order: per-core G vectors, then a fixed-order sum per booster entry.  The
    // cores' launch order (longest first) is uploaded with the plan.
    std::vector<int> key(two_j, two_j + 10);
    key.push_back(dl);
    if (key != c->adj_order_key) {
      adjoint_ring_order(probe, c->adj_order);
      c->adj_order_key = key;
    }
    Prepared prep;
    rc = prepare(c, two_j, dl, align_up(adjoint_ring_gbuf_bytes(probe.nd, akl), 256), prep, true,
                 &c->adj_order, &probe);
    if (rc) return rc;
    RingParams rp = ring_params(prep, B);
    TimedLaunch tl(c, 3);
    HIP_TRY(c, launch_adjoint_ring(rp, akl, aiw, akw, ang, prep.sched, psi,
                                   reinterpret_cast<double *>(prep.tail), prep.plan.boff.back(),
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

int eprl_threejm_batch(eprl_ctx *c, int n, const int *args, double *out) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (n < 0 || (n > 0 && (!args || !out))) return fail(c, EPRL_EINVAL, "invalid arguments");
  if (n == 0) return EPRL_OK;
  int big = 0;
  for (int q = 0; q < n; ++q)
    for (int a = 0; a < 6; ++a) {
      const int v = args[6 * q + a];
      if ((a < 3 && (v < 0 || v > kSixjMaxTwo)) || (a >= 3 && (v < -kSixjMaxTwo || v > kSixjMaxTwo)))
        return fail(c, EPRL_ERANGE, "3jm argument outside |two_j| <= 200");
      if (a < 3) big = std::max(big, v);
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
  HIP_TRY(c, launch_threejm_batch(reinterpret_cast<int *>(c->ws), n, out, c->fexp, c->primes,
                                  c->nprime, c->fact_max, c->stream));
  return EPRL_OK;
}

int eprl_boosters(eprl_ctx *c, const int two_j[10], int dl, double gamma, double tol, double *B,
                  double info[3]) {
  if (check_ctx(c)) return EPRL_EINVAL;
  if (!two_j || !B) return fail(c, EPRL_EINVAL, "null argument");
  if (!(gamma > 0.0) || !std::isfinite(gamma))
    return fail(c, EPRL_EINVAL, "gamma must be finite and positive");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(c, EPRL_EINVAL, "tol must be finite and positive");
  Plan p;
  int rc = make_plan(two_j, dl, p, c->err);
  if (rc) return rc;
  std::vector<BoosterBlock> blocks;
  booster_blocks(p, blocks);
  const int nb = (int)blocks.size();
  if (info) info[0] = info[1] = info[2] = 0.0;
  if (nb == 0) return EPRL_OK;
  // m-tuples of each edge: m_a in -j_a..j_a (boundary spins), m1 + m2 + m3 + m4 = 0.
  std::vector<int> mtup;
  int mt_edge[4], M_edge[4], jb_edge[4][4];
  for (int e = 0; e < 4; ++e) {
    int jb[4] = {0, 0, 0, 0};
    bool found = false;
    for (const BoosterBlock &b : blocks)
      if (b.edge == e) {
        std::copy(b.jb, b.jb + 4, jb);
        found = true;
        break;
      }
    std::copy(jb, jb + 4, jb_edge[e]);
    mt_edge[e] = (int)mtup.size();
    M_edge[e] = 0;
    if (!found) continue;
    for (int m1 = -jb[0]; m1 <= jb[0]; m1 += 2)
      for (int m2 = -jb[1]; m2 <= jb[1]; m2 += 2)
        for (int m3 = -jb[2]; m3 <= jb[2]; m3 += 2) {
          const int m4 = -(m1 + m2 + m3);
          if (m4 < -jb[3] || m4 > jb[3] || ((jb[3] - m4) & 1)) continue;
          mtup.insert(mtup.end(), {m1, m2, m3, m4});
          ++M_edge[e];
        }
  }
  // d-function keys: for each (j, l) met on a link, the rows m = -j..j.
  std::map<std::pair<int, int>, int> key_base;
  std::vector<DKey> keys;
  auto key_of = [&](int j2, int l2) {
    auto it = key_base.find({j2, l2});
    if (it != key_base.end()) return it->second;
    const int base = (int)keys.size();
    key_base[{j2, l2}] = base;
    const double rho = gamma * (j2 / 2.0 + 1.0);
    double phase = 0.0;
    for (int n2 = j2 + 2; n2 <= l2; n2 += 2) phase += std::atan2(rho, n2 / 2.0);
    phase += 0.5 * 3.14159265358979323846 * ((l2 - j2) / 2);
    for (int m2 = -j2; m2 <= j2; m2 += 2) {
      DKey k;
      k.rho = rho;
      k.ph_re = std::cos(phase);
      k.ph_im = -std::sin(phase);
      k.pre = std::sqrt((j2 + 1.0) * (l2 + 1.0));
      jacobi_constants(j2, j2, m2, k.nj, k.muj, k.nuj, k.sj);
      jacobi_constants(l2, j2, m2, k.nl, k.mul, k.nul, k.sl);
      keys.push_back(k);
    }
    return base;
  };
  // Per block: edge, idim, kdim, M, m-tuple offset, key bases of its four links; packed and
  // 4jm-table offsets.  Coefficient sets: the four edges' boundary tables, then every block's.
  std::vector<int> binfo(9 * (size_t)std::max(nb, 1), 0);
  std::vector<int64_t> boffs(2 * (size_t)std::max(nb, 1), 0);
  std::vector<FourjmSet> sets;
  int64_t ci_edge[4] = {0, 0, 0, 0}, ci_total = 0;
  int fact = 2;
  for (int e = 0; e < 4; ++e) {
    ci_edge[e] = ci_total;
    const int idim = p.i[e + 1].n, ilo = p.i[e + 1].lo2;
    if (M_edge[e] == 0) continue;
    FourjmSet st;
    std::copy(jb_edge[e], jb_edge[e] + 4, st.j);
    st.two_lo = ilo;
    st.n = idim;
    st.M = M_edge[e];
    st.mt = mt_edge[e];
    st.out = ci_total;
    sets.push_back(st);
    ci_total += (int64_t)M_edge[e] * idim;
    const int imax = ilo + 2 * (idim - 1);
    fact = std::max(fact, std::max(jb_edge[e][0] + jb_edge[e][1], jb_edge[e][2] + jb_edge[e][3]) + imax);
  }
  int64_t ck_total = 0, I_total = 0;
  int Mmax = 0, max_entries = 0;
  for (const FourjmSet &st : sets) max_entries = std::max(max_entries, st.M * st.n);
  for (int q = 0; q < nb; ++q) {
    const BoosterBlock &b = blocks[q];
    const int M = M_edge[b.edge];
    int *bi = &binfo[9 * (size_t)q];
    bi[0] = b.edge;
    bi[1] = b.idim;
    bi[2] = b.kdim;
    bi[3] = M;
    bi[4] = (int)I_total;
    for (int a = 0; a < 4; ++a) bi[5 + a] = key_of(b.jb[a], b.lb[a]);
    boffs[2 * q] = b.off;
    boffs[2 * q + 1] = ck_total;
    FourjmSet st;
    std::copy(b.lb, b.lb + 4, st.j);
    st.two_lo = b.two_klo;
    st.n = b.kdim;
    st.M = M;
    st.mt = mt_edge[b.edge];
    st.out = ci_total + ck_total;  // ci and ck share one array
    sets.push_back(st);
    max_entries = std::max(max_entries, M * b.kdim);
    ck_total += (int64_t)M * b.kdim;
    I_total += M;
    Mmax = std::max(Mmax, M);
    const int kmax = b.two_klo + 2 * (b.kdim - 1);
    fact = std::max(fact, std::max(b.lb[0] + b.lb[1], b.lb[2] + b.lb[3]) + kmax);
  }
  if (fact / 2 + 2 > 2 * kSixjMaxTwo + 2) return fail(c, EPRL_ERANGE, "spins beyond the 3jm range");
  rc = ensure_fexp(c, fact / 2 + 2);
  if (rc) return rc;
  const int ns = 256;
  std::vector<double> sx, sw, gx[2], gw[2];
  gauss_legendre(ns, sx, sw);
  gauss_legendre(30, gx[0], gw[0]);
  gauss_legendre(61, gx[1], gw[1]);
  const int nkeys = (int)keys.size();
  // Workspace: the call-independent part first, then the r nodes and the d table (their size
  // grows with n).
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(std::max<size_t>(bytes, 1), 256);
    return o;
  };
  const size_t o_keys = take(keys.size() * sizeof(DKey));
  const size_t o_sx = take(ns * sizeof(double)), o_sw = take(ns * sizeof(double));
  const size_t o_binfo = take(binfo.size() * sizeof(int));
  const size_t o_boffs = take(boffs.size() * sizeof(int64_t));
  const size_t o_mt = take(mtup.size() * sizeof(int));
  const size_t o_sets = take(sets.size() * sizeof(FourjmSet));
  const size_t static_bytes = off;
  const size_t o_coef = take((size_t)(ci_total + ck_total) * sizeof(double));
  const size_t o_I = take((size_t)I_total * 4 * sizeof(double));
  const size_t o_stat = take((size_t)std::max(nb, 1) * 3 * sizeof(double));
  const size_t o_stat3 = take(3 * sizeof(double));
  const size_t o_var = off;
  const int n_max = 512;
  char *ws_seen = nullptr;
  double st3[3] = {0.0, 0.0, 0.0};
  int n = 16;
  for (;;) {
    std::vector<double> r, rw;
    booster_r_nodes(n, gx, gw, r, rw);
    const int nr = (int)r.size(), nr30 = 30 * n;
    off = o_var;
    const size_t o_r = take(nr * sizeof(double)), o_rw = take(nr * sizeof(double));
    const size_t o_dtab = take((size_t)nkeys * nr * 2 * sizeof(double));
    rc = ensure_workspace(c, off);
    if (rc) return rc;
    char *ws = c->ws;
    if (ws != ws_seen) {
      // (Re)load the call-independent data and the 4jm tables.
      char *stg;
      rc = staging(c, static_bytes, &stg);
      if (rc) return rc;
      std::memcpy(stg + o_keys, keys.data(), keys.size() * sizeof(DKey));
      std::memcpy(stg + o_sx, sx.data(), ns * sizeof(double));
      std::memcpy(stg + o_sw, sw.data(), ns * sizeof(double));
      std::memcpy(stg + o_binfo, binfo.data(), binfo.size() * sizeof(int));
      std::memcpy(stg + o_boffs, boffs.data(), boffs.size() * sizeof(int64_t));
      if (!mtup.empty()) std::memcpy(stg + o_mt, mtup.data(), mtup.size() * sizeof(int));
      if (!sets.empty()) std::memcpy(stg + o_sets, sets.data(), sets.size() * sizeof(FourjmSet));
      rc = upload(c, ws, static_bytes);
      if (rc) return rc;
      HIP_TRY(c, launch_fourjm_tables(reinterpret_cast<const FourjmSet *>(ws + o_sets), (int)sets.size(),
                                      max_entries, reinterpret_cast<const int *>(ws + o_mt),
                                      reinterpret_cast<double *>(ws + o_coef), c->fexp, c->primes,
                                      c->nprime, c->stream));
      ws_seen = ws;
    }
    {
      char *stg;
      rc = staging(c, 2 * align_up(nr * sizeof(double), 256), &stg);
      if (rc) return rc;
      std::memcpy(stg, r.data(), nr * sizeof(double));
      std::memcpy(stg + (o_rw - o_r), rw.data(), nr * sizeof(double));
      rc = upload(c, ws + o_r, o_dtab - o_r);
      if (rc) return rc;
    }
    BoosterParams bp;
    std::memset(&bp, 0, sizeof(bp));
    bp.keys = reinterpret_cast<const DKey *>(ws + o_keys);
    bp.nkeys = nkeys;
    bp.sx = reinterpret_cast<const double *>(ws + o_sx);
    bp.sw = reinterpret_cast<const double *>(ws + o_sw);
    bp.ns = ns;
    bp.r = reinterpret_cast<const double *>(ws + o_r);
    bp.rw = reinterpret_cast<const double *>(ws + o_rw);
    bp.nr = nr;
    bp.nr30 = nr30;
    bp.dtab = reinterpret_cast<double *>(ws + o_dtab);
    bp.binfo = reinterpret_cast<const int *>(ws + o_binfo);
    bp.boffs = reinterpret_cast<const int64_t *>(ws + o_boffs);
    bp.mtuples = reinterpret_cast<const int *>(ws + o_mt);
    for (int e = 0; e < 4; ++e) {
      bp.mt_edge[e] = mt_edge[e];
      bp.ci_edge[e] = ci_edge[e];
      for (int a = 0; a < 4; ++a) bp.jb_edge[e][a] = jb_edge[e][a];
    }
    bp.ci = reinterpret_cast<const double *>(ws + o_coef);
    bp.ck = reinterpret_cast<const double *>(ws + o_coef) + ci_total;
    bp.I = reinterpret_cast<double *>(ws + o_I);
    bp.B = B;
    bp.stat = reinterpret_cast<double *>(ws + o_stat);
    bp.nblocks = nb;
    bp.Mmax = Mmax;
    HIP_TRY(c, launch_booster_dfun(bp, c->stream));
    HIP_TRY(c, launch_booster_integrals(bp, c->stream));
    HIP_TRY(c, launch_booster_assemble(bp, reinterpret_cast<double *>(ws + o_stat3), c->stream));
    HIP_TRY(c, hipMemcpyAsync(st3, ws + o_stat3, sizeof(st3), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (st3[0] <= tol * std::max(st3[1], 1e-300) || n >= n_max) break;
    n *= 2;
  }
  if (info) {
    info[0] = st3[0];
    info[1] = st3[2];
    info[2] = n;
  }
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
