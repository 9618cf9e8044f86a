// Host driver and C ABI of liblsba: restarted BFOM / BGMRES on one GPU.
//
// A solve runs restart cycles (Sec. 2.4.2).  Each cycle is queued on the
// context's stream as a fixed sequence of kernels -- IntraOrtho of the
// starting block, then for every loop step the block SpMM, the fused Gram
// product, the small dense step and the fused block update -- followed by the
// cycle-end step and the basis application X += V Xi, U = V [M; -H].  The
// kernels test the device control word and return at once after convergence,
// a Cholesky flag (Sec. 4) or the iteration cap, so the host synchronises
// only once per cycle, to read the control word and the cycle's residual
// estimates.  A cycle's launch sequence depends only on host values fixed for
// the solve (pointers, sizes, method, restart length), so it can also be
// captured once into a hipGraph and replayed with one host call per cycle
// (lsba_context_set_graphs).
//
// The mixed form wraps FP32 inner solves (same cycle machinery with float
// blocks) in FP64 iterative refinement: R = B - A X in FP64, inner solve
// A D = R, X += D.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <type_traits>
#include <type_traits>
#include <vector>

#include "lsba_internal.h"

using namespace lsba;

namespace {
struct EventTimer;
}

// Scratch memory of the no-allocation entry point (lsba_solve_noalloc): a
// file-scope device array, one copy per device, held until the process
// ends.  Host code never uses the array's name as an address: its device
// address is taken once per device by hipGetSymbolAddress (scratch_init, at
// context creation with that device current) and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct lsba_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  Ctl* ctl_host = nullptr;     // pinned
  double* hist_host = nullptr; // pinned, 2 * (kMaxM + 2)
  double* norm_host = nullptr; // pinned, 4
  double* stage_host = nullptr;// pinned, kMaxS * kMaxS (host-to-device staging)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_done = nullptr;   // end of the queued cycle (no timing)
  EventTimer* timer = nullptr;   // non-null while kernel timing is enabled
  hipStream_t side = nullptr;    // second stream: per-column QR updates / convergence tests
  hipStream_t side2 = nullptr;   // third stream: Alg. 7's QR updates, behind its H / J work
  std::vector<hipEvent_t> evs;   // ordering events between the two streams
  bool async_alloc = false;      // serving slots: stream-ordered allocations on `stream`
  // Captured cycles, keyed by every host value their launches read (see
  // CycleRunner::graph_key); dropped whenever a cached buffer is freed.
  struct GraphEnt {
    std::vector<uint8_t> key;
    hipGraphExec_t ex = nullptr;
    uint64_t used = 0;
  };
  std::vector<GraphEnt> graphs;
  uint64_t graph_tick = 0;
  bool graphs_on = false;
  // live operators of this context: destroying the context releases their
  // device memory and detaches them, so that a later lsba_operator_destroy
  // (in any order, e.g. from a garbage collector) never reads a freed context
  std::set<lsba_operator*> ops;
  std::set<lsba_precond*> pcs;   // live preconditioners, released likewise
};


struct lsba_operator {
  lsba_context* ctx = nullptr;
  int64_t n = 0, nnz = 0;
  int64_t* rp = nullptr;
  int* ci = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
};

// Right ILU(0) preconditioner of an operator (factors in device memory).
struct lsba_precond {
  lsba_context* ctx = nullptr;
  IluFactors f;   // holds no reference to the operator it was made from
};

struct lsba_result {
  lsba_status status = LSBA_OK;
  int64_t iters = 0;
  std::vector<double> res, loo;
  std::vector<int32_t> cyc, mafter;
  int64_t a = 0, v = 0, sy = 0;
  double true_relres = NAN;
  double err_vs_ref = NAN;   // set by lsba_result_set_err_vs_ref
  int32_t refine = 0;
  double gpu_ms = 0.0;
  bool have_loo = false;
};

namespace {

thread_local std::string g_create_err;

struct HipError {
  std::string msg;
};

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw HipError{std::string(#expr) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

// HIP-event timer of kernel launches, flushed after every stream synchronisation.
struct EventTimer final : KTimer {
  struct Rec {
    int kind;
    double bytes;
    hipEvent_t a, b;
    int step, phase;
    double flops;
  };
  struct Acc {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0, flops = 0.0;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  hipEvent_t pending = nullptr;
  Acc acc[KK_COUNT];
  int step = 0, phase = 0;   // tag of the launches being queued
  uint32_t mask;             // bit k: time launches of class k
  explicit EventTimer(uint32_t m) : mask(m) {}
  bool on(int kind) const { return (mask >> kind) & 1u; }

  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(hipStream_t st, int kind) override {
    if (!on(kind)) return;
    pending = take();
    HIPCHK(hipEventRecord(pending, st));
  }
  void end(hipStream_t st, int kind, double bytes) override {
    if (!on(kind)) return;
    hipEvent_t b = take();
    HIPCHK(hipEventRecord(b, st));
    recs.push_back({kind, bytes, pending, b, step, phase, 0.0});
  }
  bool kernel_events(int kind, hipEvent_t* a, hipEvent_t* b) override {
    if (!on(kind)) return false;
    *a = take();
    *b = take();
    return true;
  }
  void kernel_done(int kind, hipEvent_t a, hipEvent_t b, double bytes, double flops) override {
    HIPCHK(hipGetLastError());
    recs.push_back({kind, bytes, a, b, step, phase, flops});
  }
  void tag(int st, int ph) {
    step = st;
    phase = ph;
  }
  // Launches of steps after the one that ended the cycle did no algorithmic
  // work (they returned at once, or ran ahead speculatively while the
  // convergence test was pending): keep their durations, drop their bytes.
  // With a Cholesky flag at step k_stop, the updates queued after that step's
  // small kernel (phase 1) did not run either.
  void kill_after(int k_stop, bool flagged) {
    for (auto& r : recs)
      if (r.step > k_stop || (flagged && r.step == k_stop && r.phase == 1)) {
        r.bytes = 0.0;
        r.flops = 0.0;
      }
  }
  void flush() {
    for (auto& r : recs) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
      acc[r.kind].launches += 1;
      acc[r.kind].ms += ms;
      if (r.bytes > 0) acc[r.kind].bytes += r.bytes;
      if (r.flops > 0) acc[r.kind].flops += r.flops;
    }
    recs.clear();
    used = 0;
  }
  ~EventTimer() override {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Counts of one cycle as the paper counts them (Sec. 5): A-calls, basis
// applications and syncs of the loop steps the algorithm executed.
// `ms` is the muscle's syncs per IntraOrtho call (1, or 3 s - 2 for the
// column-wise MGS muscles).
void cycle_counts(int skel, int ms, int j, int status, int flag_step, int64_t& a, int64_t& v,
                  int64_t& sy) {
  const bool delayed = skel == LSBA_BCGSI_LS || skel == LSBA_BMGS_CWY || skel == LSBA_BMGS_ICWY;
  const bool bcgs = skel == LSBA_BCGSI_LS;
  sy += ms;   // IntraOrtho of the starting block
  if (status == ST_FLAGGED && flag_step == 0) return;
  int full, partial = 0;
  if (status == ST_FLAGGED) {
    full = flag_step - 1;
    partial = 1;
  } else {
    full = delayed ? j + 1 : j;
  }
  if (skel == LSBA_BCGS_PIP) {
    // step k: one A-call, one fused inner product (2 applications of the
    // basis), one projection; a flagged step stops before the projection
    a += full + partial;
    sy += full + partial;
    v += 3 * full + 2 * partial;
    return;
  }
  if (skel == LSBA_BCGS_PIO) {
    // step k: one A-call, the inner product and the IntraOrtho (2 syncs),
    // 2 basis applications (inner product, projection); a flagged step
    // stops before its projection
    a += full + partial;
    sy += 2 * (full + partial);
    v += 2 * full + partial;
    return;
  }
  if (skel == LSBA_BMGS) {
    // step k: one A-call, k block inner products and the IntraOrtho
    for (int k = 1; k <= full + partial; ++k) {
      a += 1;
      sy += k + ms;
      v += 2;
    }
    return;
  }
  if (delayed) {
    for (int k = 1; k <= full; ++k) {
      a += 1;
      sy += 1;
      v += (k == 1) ? 1 : (bcgs ? 4 : 3);
    }
    if (partial) {
      a += 1;
      sy += 1;
      v += 2;
    }
  } else {
    // Alg. 5 step: Y, the IntraOrtho, Z; a flagged step stops after the IntraOrtho
    a += full;
    sy += (2 + ms) * full;
    v += 3 * full;
    if (partial) {
      a += 1;
      sy += 1 + ms;
      v += 2;
    }
  }
}

struct ArgError {
  std::string msg;
};
struct Unsupported {
  std::string msg;
};

constexpr size_t kMaxGraphs = 8;
// Stream-ordering events one cycle records: at most two per batch of side
// jobs (about m / 4 + 5 batches) and two to join the side streams.
constexpr int kMaxEvents = kMaxM / 2 + 16;

// Destroy every captured cycle of a context (their launches may still be in
// flight on the context's stream, so it is drained first).
void graphs_clear(lsba_context* c) {
  if (c->graphs.empty()) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.ex);
  c->graphs.clear();
}

hipGraphExec_t graph_find(lsba_context* c, const std::vector<uint8_t>& key) {
  for (auto& g : c->graphs)
    if (g.key == key) {
      g.used = ++c->graph_tick;
      return g.ex;
    }
  return nullptr;
}

void graph_put(lsba_context* c, std::vector<uint8_t> key, hipGraphExec_t ex) {
  if (c->graphs.size() >= kMaxGraphs) {
    auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                [](const lsba_context::GraphEnt& a,
                                   const lsba_context::GraphEnt& b) { return a.used < b.used; });
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    (void)hipGraphExecDestroy(lru->ex);
    c->graphs.erase(lru);
  }
  c->graphs.push_back({std::move(key), ex, ++c->graph_tick});
}

// hipMemcpy2DAsync, or one contiguous copy when both pitches equal the row
// width: a pitched copy to or from pageable host memory moves row by row,
// which for millions of rows takes seconds.
hipError_t copy2d(void* dst, size_t dp, const void* src, size_t sp, size_t w, size_t h,
                  hipMemcpyKind kind, hipStream_t st) {
  if (dp == w && sp == w) return hipMemcpyAsync(dst, src, w * h, kind, st);
  return hipMemcpy2DAsync(dst, dp, src, sp, w, h, kind, st);
}
hipError_t copy2d_sync(void* dst, size_t dp, const void* src, size_t sp, size_t w, size_t h,
                       hipMemcpyKind kind) {
  if (dp == w && sp == w) return hipMemcpy(dst, src, w * h, kind);
  return hipMemcpy2D(dst, dp, src, sp, w, h, kind);
}

void* ctx_buf(lsba_context* c, const std::string& name, size_t bytes) {
  auto& b = c->bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      graphs_clear(c);   // captured launches may point into the old buffer
      if (c->async_alloc) HIPCHK(hipFreeAsync(b.p, c->stream));
      else HIPCHK(hipFree(b.p));
    }
    b.p = nullptr;
    b.bytes = 0;
    const hipError_t e = c->async_alloc ? hipMallocAsync(&b.p, bytes, c->stream)
                                        : hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      b.p = nullptr;
      throw HipError{"allocation of " + std::to_string(bytes) + " bytes for " + name + " failed"};
    }
    b.bytes = bytes;
  }
  return b.p;
}

// Release every cached buffer of a context (stream-ordered for serving slots).
void ctx_release(lsba_context* c) {
  graphs_clear(c);
  for (auto& kv : c->bufs)
    if (kv.second.p) {
      if (c->async_alloc) (void)hipFreeAsync(kv.second.p, c->stream);
      else (void)hipFree(kv.second.p);
    }
  c->bufs.clear();
}

// Device bytes a context's cached buffers hold.
size_t ctx_bytes(const lsba_context* c) {
  size_t t = 0;
  for (const auto& kv : c->bufs) t += kv.second.bytes;
  return t;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device state of one Krylov solve in basis type T.
template <typename T>
struct Krylov {
  int64_t n = 0;
  int s = 0, mmax = 0;
  T* V = nullptr;
  T* U = nullptr;
  T* W = nullptr;
  double* partial = nullptr;
  double* hwork = nullptr;   // HouseQR muscle: TSQR workspace
  Dense d{};
  CoefLayout lay{};
};

// `alloc(name, bytes)` provides device memory (the context's buffer cache, or
// a byte counter for the serving footprint).
template <typename T, typename Alloc>
Krylov<T> make_krylov_with(Alloc&& alloc, int64_t n, int s, int m, const lsba_params& p,
                           const char* tag) {
  Krylov<T> k;
  k.n = n;
  k.s = s;
  k.mmax = m;
  const std::string t(tag);
  const size_t blk = (size_t)n * s * sizeof(T);
  k.V = (T*)alloc(t + "V", blk * (m + 1));
  k.U = (T*)alloc(t + "U", blk);
  k.W = (T*)alloc(t + "W", blk);
  k.partial = (double*)alloc(t + "partial",
                               sizeof(double) * gram_partial_doubles(n, s, m + 2, 2));
  if (p.muscle == LSBA_HOUSEQR)
    k.hwork = (double*)alloc(t + "hwork", sizeof(double) * house_work_doubles(n, s));
  const int ldh = (m + 1) * s;
  const size_t ss = (size_t)s * s;
  const size_t big = (size_t)(m + 2) * ss;
  CoefLayout lay{s, m + 1};
  k.lay = lay;
  // the delayed skeletons keep each loop step's Gram output in its own slot
  const bool per_step = p.skeleton == LSBA_BCGSI_LS || p.skeleton == LSBA_BMGS_CWY ||
                        p.skeleton == LSBA_BMGS_ICWY;
  const size_t gslot = (size_t)(m + 1) * s * 2 * s;
  // carve the small dense state out of one allocation
  struct Item {
    double** dst;
    size_t count;
  };
  Dense& d = k.d;
  std::vector<Item> items = {
      {&d.H, (size_t)(m + 2) * s * ldh},
      {&d.T, (size_t)ldh * ldh},
      {&d.Tt, (size_t)ldh * ldh},
      {&d.J, (size_t)(m + 1) * ss},
      {&d.G, (size_t)(m + 2) * gslot},
      {&d.G2, (size_t)(m + 2) * ss},
      {&d.Beta, ss},
      {&d.C, ss},
      {&d.Qt, (size_t)m * 4 * ss},
      {&d.Rf, (size_t)(m + 1) * s * ldh},
      {&d.g, (size_t)(m + 1) * ss},
      {&d.Dlast, ss},
      {&d.ylast, ss},
      {&d.Xi, (size_t)m * ss},
      {&d.M, (size_t)m * ss},
      {&d.Rinv, ss},
      {&d.P, ss},
      {&d.RiS, (size_t)(m + 2) * ss},
      {&d.PS, (size_t)(m + 2) * ss},
      {&d.Gv, (size_t)ldh * ldh},
      {&d.scratch, 64 * ss + 8 * big},
      {&d.coef64, (size_t)lay.total()},
      {&d.res_hist, (size_t)(m + 2)},
      {&d.loo_hist, (size_t)(m + 2)},
  };
  size_t total = 0;
  for (auto& it : items) total += align256(it.count * sizeof(double));
  const size_t coefT_bytes = align256((size_t)lay.total() * sizeof(T));
  total += coefT_bytes + align256(sizeof(Ctl));
  char* base = (char*)alloc(t + "dense", total);
  size_t off = 0;
  for (auto& it : items) {
    *it.dst = (double*)(base + off);
    off += align256(it.count * sizeof(double));
  }
  if (sizeof(T) == sizeof(double)) {
    d.coefT = d.coef64;
    off += coefT_bytes;
  } else {
    d.coefT = base + off;
    off += coefT_bytes;
  }
  d.ctl = (Ctl*)(base + off);
  d.s = s;
  d.mmax = m;
  d.ldh = ldh;
  d.skel = p.skeleton;
  d.glob = p.muscle == LSBA_GLOBAL ? 1 : 0;
  d.mgs = p.muscle == LSBA_MGS_SVL ? 1 : (p.muscle == LSBA_MGS_LTS ? 2 : 0);
  d.method = p.method;
  d.mixed = sizeof(T) == sizeof(float) ? 1 : 0;
  d.gstride = per_step ? (long long)gslot : 0;
  return k;
}

template <typename T>
Krylov<T> make_krylov(lsba_context* c, int64_t n, int s, int m, const lsba_params& p,
                      const char* tag) {
  return make_krylov_with<T>([c](const std::string& name, size_t bytes) {
    return ctx_buf(c, name, bytes);
  }, n, s, m, p, tag);
}

// Device bytes one FP64 solve holds while it runs: B, X, the basis and
// Krylov state (as make_krylov allocates it) and the norm workspaces.
uint64_t solve_footprint(int64_t n, int s, const lsba_params& p) {
  uint64_t tot = 0;
  auto meas = [&tot](const std::string&, size_t bytes) -> void* {
    tot += bytes;
    return reinterpret_cast<void*>(uintptr_t(4096));   // never dereferenced
  };
  make_krylov_with<double>(meas, n, s, p.m, p, "d_");
  const uint64_t blk64 = (uint64_t)n * s * sizeof(double);
  tot += 2 * blk64;                                                  // B, X
  tot += sizeof(double) * ((uint64_t)n * s / 4096 + 2) + 4 * sizeof(double);   // norm
  if (p.record & LSBA_REC_TRUE_RES) {
    int sh = 0;
    while ((1 << sh) < s) ++sh;
    tot += sizeof(double) * ((((uint64_t)n << sh) + 255) / 256 + 1);   // residual partials
  }
  return tot;
}

struct CycleOut {
  lsba_status status = LSBA_NOT_CONVERGED;
  int64_t iters = 0;
  int64_t a = 0, v = 0, sy = 0;
};

template <typename T>
GramArgs<T> gram_args(const Krylov<T>& k, int nv, std::initializer_list<const T*> xl,
                      std::initializer_list<const T*> xr) {
  GramArgs<T> g{};
  g.n = k.n;
  g.s = k.s;
  g.V = k.V;
  g.nv = nv;
  g.nxl = 0;
  for (const T* p : xl) g.xl[g.nxl++] = p;
  g.nxr = 0;
  for (const T* p : xr) g.xr[g.nxr++] = p;
  g.glob = k.d.glob;
  return g;
}

template <typename T>
UpdateArgs<T> upd_args(const Krylov<T>& k) {
  UpdateArgs<T> u{};
  u.n = k.n;
  u.s = k.s;
  u.V = k.V;
  u.coef = (const T*)k.d.coefT;
  u.lay = k.lay;
  return u;
}

template <typename T>
T* slot(const Krylov<T>& k, int i) {
  return k.V + (int64_t)i * k.n * k.s;
}

// Restart cycles of A X = R for x (zero-initialised by begin) in type T, one
// cycle at a time: begin() queues the set-up, enqueue() queues one whole cycle
// (every kernel reads the device control word and returns once the cycle has
// ended) followed by the copies of the control word and histories to pinned
// host memory and the event c->ev_done; finish(), on the host after that
// event, reads the cycle's outcome and returns true when the solve is over.
template <typename T>
struct CycleRunner {
  lsba_context* c;
  const lsba_operator* op;
  lsba_params p;
  Krylov<T>* kp;
  const T* val;
  const T* rhs;
  T* x;
  double nB, tol;
  lsba_result* res;
  bool delayed = false, bcgs = false, rec_loo = false;
  const T* R0 = nullptr;
  int m = 0, cyc = 0;
  CycleOut out;
  UpdateArgs<T> uapply{};
  // right preconditioning (FP64 only): the cycle's operator is A M^{-1},
  // applied as W = A (M^{-1} V) with M^{-1} V in zpc
  const IluFactors* pc = nullptr;
  double* zpc = nullptr;

  // W = A X, or A M^{-1} X with a preconditioner
  void op_apply(hipStream_t st, const T* X, T* W, const Ctl* ctl, EventTimer* tm) {
    if constexpr (std::is_same_v<T, double>) {
      if (pc) {
        launch_ilu_apply(st, *pc, kp->s, X, zpc, ctl, tm);
        X = zpc;
      }
    }
    launch_spmm<T>(st, kp->n, op->nnz, kp->s, op->rp, op->ci, val, X, W, ctl, tm);
  }

  void begin() {
    Krylov<T>& k = *kp;
    hipStream_t st = c->stream;
    const int s = k.s;
    const int64_t n = k.n;
    Dense& d = k.d;
    Ctl* ctl = d.ctl;
    EventTimer* tm = c->timer;
    (void)s;
    (void)n;
    (void)ctl;
    (void)tm;
    Ctl h{};
    h.stop = 0;
    h.status = ST_RUNNING;
    h.m = p.m;
    h.max_iters = p.max_iters > 0 ? p.max_iters : 0;
    h.nB = nB;
    h.tol = tol;
    h.flag_step = -1;
    // the stream is idle here (every solve ends with a synchronisation), so the
    // pinned staging buffers can be refilled
    *c->ctl_host = h;
    HIPCHK(hipMemcpyAsync(d.ctl, c->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st));
    for (int i = 0; i < s * s; ++i) c->stage_host[i] = (i / s == i % s) ? 1.0 : 0.0;
    HIPCHK(hipMemcpyAsync(d.C, c->stage_host, sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(x, 0, (size_t)n * s * sizeof(T), st));
    delayed = p.skeleton == LSBA_BCGSI_LS || p.skeleton == LSBA_BMGS_CWY ||
              p.skeleton == LSBA_BMGS_ICWY;
    bcgs = p.skeleton == LSBA_BCGSI_LS;
    rec_loo = (p.record & LSBA_REC_LOO) != 0;
    R0 = rhs;
    m = p.m;
  }

  // Host values the launches of cycle cyc_ read: workspace and operator
  // pointers and sizes (the Krylov state holds no padding, so its bytes are
  // its values), the starting block, X, the restart length, the forced flag.
  std::vector<uint8_t> graph_key(int cyc_) const {
    static_assert(std::has_unique_object_representations_v<Krylov<T>>,
                  "the Krylov state must hold no padding bytes");
    std::vector<uint8_t> b;
    auto put = [&](const void* q, size_t nb) {
      const uint8_t* u = (const uint8_t*)q;
      b.insert(b.end(), u, u + nb);
    };
    const int fk = (p.force_flag_cycle == cyc_) ? p.force_flag_step : -1;
    const int64_t ints[] = {(int64_t)sizeof(T), op->n, op->nnz, m, fk, p.muscle, p.skeleton,
                            p.method, rec_loo ? 1 : 0};
    const void* ptrs[] = {op->rp, op->ci, val, R0, x, c->side, c->side2, pc, zpc};
    put(ints, sizeof(ints));
    put(ptrs, sizeof(ptrs));
    put(kp, sizeof(Krylov<T>));
    return b;
  }

  // Queue one cycle: replay its captured graph (capturing it on first use),
  // or launch it kernel by kernel while kernel timing is on; then the
  // read-back of the control word and the residual estimates.
  void enqueue() {
    const int cyc_ = ++cyc;
    hipStream_t st = c->stream;
    Dense& d = kp->d;
    if (c->graphs_on && c->timer == nullptr) {
      std::vector<uint8_t> key = graph_key(cyc_);
      hipGraphExec_t ex = graph_find(c, key);
      if (!ex) {
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        hipGraph_t g = nullptr;
        try {
          record(cyc_);
        } catch (...) {
          (void)hipStreamEndCapture(st, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIPCHK(hipStreamEndCapture(st, &g));
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        graph_put(c, std::move(key), ex);
      }
      HIPCHK(hipGraphLaunch(ex, st));
    } else {
      record(cyc_);
    }
    uapply = upd_args(*kp);
    uapply.in1 = x;
    uapply.out1 = x;
    uapply.out2 = kp->U;
    uapply.nvp = &d.ctl->nv1;
    HIPCHK(hipMemcpyAsync(c->ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(c->hist_host, d.res_hist, sizeof(double) * (m + 1),
                          hipMemcpyDeviceToHost, st));
    if (rec_loo)
      HIPCHK(hipMemcpyAsync(c->hist_host + (kMaxM + 2), d.loo_hist, sizeof(double) * (m + 1),
                            hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(c->ev_done, st));
  }

  // The launches of one cycle, in stream order.
  void record(int cyc_) {
    Krylov<T>& k = *kp;
    hipStream_t st = c->stream;
    const int s = k.s;
    const int64_t n = k.n;
    Dense& d = k.d;
    Ctl* ctl = d.ctl;
    EventTimer* tm = c->timer;
    (void)s;
    (void)n;
    (void)ctl;
    (void)tm;
    hipStream_t side = c->side;
    size_t nev = 0;
    auto event = [&]() -> hipEvent_t {
      if (nev == c->evs.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->evs.push_back(e);
      }
      return c->evs[nev++];
    };
    // the per-column QR update / convergence test of column `col` runs on the
    // side stream, after the skeleton step that made the column final
    // Off-path work (QR update / estimate / convergence test, and for Alg. 7
    // the H column and J recurrence) is queued on the side stream in batches
    // of kSideBatch loop steps behind one event: each step's inputs sit in
    // their own slots, and fewer event records keep the basis-path kernels
    // back to back.
    struct SideJob {
      int kind, arg, mcur;   // 0: finalize column arg; 1: Alg. 7 side step arg
    };
    std::vector<SideJob> pending;
    constexpr int kSideBatch = 4;
    // Alg. 7: the H column / J recurrence (a chain over the steps) runs on
    // `side`, the QR update / convergence test of each finished column on
    // `side2`, one batch behind, so the two chains overlap.
    hipStream_t side2 = c->side2;
    // streams this cycle forked to (under capture only those may be joined)
    bool used_side = false, used_side2 = false;
    auto flush_side = [&]() {
      if (pending.empty()) return;
      hipEvent_t e = event();
      HIPCHK(hipEventRecord(e, st));
      HIPCHK(hipStreamWaitEvent(side, e, 0));
      used_side = true;
      bool any_side = false;
      for (const SideJob& j : pending) {
        if (j.kind == 0) {
          launch_small_finalize(side, d, j.arg, tm);
        } else {
          launch_small_side(side, d, j.arg, j.mcur, tm);
          any_side = true;
        }
      }
      if (any_side) {
        hipEvent_t e2 = event();
        HIPCHK(hipEventRecord(e2, side));
        HIPCHK(hipStreamWaitEvent(side2, e2, 0));
        used_side2 = true;
        for (const SideJob& j : pending)
          if (j.kind == 1) launch_small_finalize(side2, d, j.arg - 1, tm);
      }
      pending.clear();
    };
    // In the last kSideBatch loop steps of the cycle every step is released
    // at once, so that after the last basis kernel only one job of the
    // chain is left to run before the cycle end.
    auto finalize_after = [&](int col, int kk) {
      pending.push_back({0, col, 0});
      if ((int)pending.size() >= kSideBatch || kk > m - kSideBatch) flush_side();
    };
    // Alg. 7: H column, J recurrence and the test of column kk - 1, off the basis path
    auto side_after = [&](int kk, int mcur) {
      pending.push_back({1, kk, mcur});
      if ((int)pending.size() >= kSideBatch || kk > m - kSideBatch) flush_side();
    };
    auto gslot = [&](int kk) { return d.G + (int64_t)kk * d.gstride; };
    auto tag = [&](int step, int phase) {
      if (tm) tm->tag(step, phase);
    };
    nev = 0;
    const int fk = (p.force_flag_cycle == cyc_) ? p.force_flag_step : -1;
    const bool mgs = p.muscle == LSBA_MGS_SVL || p.muscle == LSBA_MGS_LTS;
    // the column-wise muscle on `src` into `dst` (in place when equal): per
    // column j, the syncs are Gram products of the block with itself and the
    // changes in-place updates with the coefficients the phase kernel sets
    auto mgs_muscle = [&](int mode, const T* src, T* dst, int kk, int force) {
      launch_small_mgs(st, d, MGS_INIT, 0, mode, kk, 0, tm);
      auto apply = [&](const T* from) {
        UpdateArgs<T> u = upd_args(k);
        u.in1 = from;
        u.out1 = dst;
        launch_update<T>(st, u, ctl, true, tm);
      };
      if (src != dst) apply(src);
      for (int j = 0; j < s; ++j) {
        if (j > 0) {
          launch_gram<T>(st, gram_args<T>(k, 0, {dst}, {dst}), k.partial, d.G2, ctl, tm);
          launch_small_mgs(st, d, MGS_PROJ, j, mode, kk, 0, tm);
          apply(dst);
        }
        launch_gram<T>(st, gram_args<T>(k, 0, {dst}, {dst}), k.partial, d.G2, ctl, tm);
        launch_small_mgs(st, d, MGS_NORM, j, mode, kk, 0, tm);
        apply(dst);
        if (j > 0) {
          launch_gram<T>(st, gram_args<T>(k, 0, {dst}, {dst}), k.partial, d.G2, ctl, tm);
          launch_small_mgs(st, d, MGS_Z, j, mode, kk, 0, tm);
        }
      }
      launch_small_mgs(st, d, MGS_FINISH, 0, mode, kk, force, tm);
    };
    // IntraOrtho(R0) by CholQR: V_1 = R0 B^{-1} (and U = V_1 for the delayed skeletons)
    tag(0, 0);
    if (p.muscle == LSBA_HOUSEQR) {
      // V_1 (and U) = Q of the TSQR, Beta = R with diag(R) >= 0
      launch_house<T>(st, d, n, s, R0, slot(k, 0), delayed ? k.U : (T*)nullptr, k.hwork,
                      HM_START, 0, fk == 0 ? 1 : 0, tm);
      tag(0, 1);
    } else if (mgs) {
      if (skel_uses_t(d.skel)) launch_t_identity(st, d, tm);
      mgs_muscle(MGS_START, R0, slot(k, 0), 0, fk == 0 ? 1 : 0);
      tag(0, 1);
      if (delayed) {   // U = V_1 (the muscle left C2 = I)
        UpdateArgs<T> u = upd_args(k);
        u.in2 = slot(k, 0);
        u.out2 = k.U;
        launch_update<T>(st, u, ctl, true, tm);
      }
    } else {
      launch_gram<T>(st, gram_args<T>(k, 0, {R0}, {R0}), k.partial, d.G, ctl, tm);
      launch_small_start(st, d, fk == 0 ? 1 : 0, tm);
      tag(0, 1);
      UpdateArgs<T> u = upd_args(k);
      u.in1 = R0;
      u.out1 = slot(k, 0);
      if (delayed) {
        u.in2 = R0;
        u.out2 = k.U;
      }
      launch_update<T>(st, u, ctl, true, tm);
    }
    if (rec_loo) {
      launch_gram<T>(st, gram_args<T>(k, 1, {}, {slot(k, 0)}), k.partial, d.G2, ctl, tm);
      launch_small_loo(st, d, 1, tm);
    }
    if (delayed) {
      for (int kk = 1; kk <= m + 1; ++kk) {
        const int force = fk == kk ? 1 : 0;
        const bool last = kk == m + 1;
        tag(kk, 0);
        if (!last) op_apply(st, k.U, k.W, ctl, tm);
        if (kk == 1)
          launch_gram<T>(st, gram_args<T>(k, 1, {}, {k.W}), k.partial, gslot(kk), ctl, tm);
        else if (!last)
          launch_gram<T>(st, gram_args<T>(k, kk - 1, {k.U}, {k.U, k.W}), k.partial, gslot(kk),
                         ctl, tm);
        else
          launch_gram<T>(st, gram_args<T>(k, kk - 1, {k.U}, {k.U}), k.partial, gslot(kk), ctl,
                         tm);
        launch_small_delayed(st, d, kk, m, force, tm);
        tag(kk, 1);
        if (kk >= 2) {
          if (bcgs) side_after(kk, m);
          else finalize_after(kk - 1, kk);
        }
        UpdateArgs<T> u = upd_args(k);
        if (kk == 1) {
          u.in2 = k.W;
          u.out2 = k.U;
          u.nv2_begin = 0;
          u.nv2 = 1;
        } else {
          u.in1 = k.U;
          u.out1 = slot(k, kk - 1);
          u.nv1 = bcgs ? kk - 1 : 0;
          if (!last) {
            u.in2 = k.W;
            u.out2 = k.U;
            u.nv2_begin = 0;
            u.nv2 = kk - 1;
            u.has_D = 1;
          }
        }
        launch_update<T>(st, u, ctl, true, tm);
        if (rec_loo && kk >= 2) {
          launch_gram<T>(st, gram_args<T>(k, kk, {}, {slot(k, kk - 1)}), k.partial, d.G2, ctl,
                         tm);
          launch_small_loo(st, d, kk, tm);
        }
      }
    } else if (p.skeleton == LSBA_BCGS_PIP) {
      // Alg. 3: SpMM, one fused inner product [V_{1:k} W]^T W, the
      // Pythagorean Cholesky (H column final), one projection
      for (int kk = 1; kk <= m; ++kk) {
        const int force = fk == kk ? 1 : 0;
        tag(kk, 0);
        op_apply(st, slot(k, kk - 1), k.W, ctl, tm);
        launch_gram<T>(st, gram_args<T>(k, kk, {k.W}, {k.W}), k.partial, d.G, ctl, tm);
        launch_small_pip(st, d, kk, force, tm);
        tag(kk, 1);
        finalize_after(kk, kk);
        UpdateArgs<T> u = upd_args(k);
        u.in2 = k.W;
        u.out2 = slot(k, kk);
        u.nv2_begin = 0;
        u.nv2 = kk;
        launch_update<T>(st, u, ctl, true, tm);
        if (rec_loo) {
          launch_gram<T>(st, gram_args<T>(k, kk + 1, {}, {slot(k, kk)}), k.partial, d.G2, ctl,
                         tm);
          launch_small_loo(st, d, kk + 1, tm);
        }
      }
    } else if (p.skeleton == LSBA_BCGS_PIO) {
      // Alg. 4: SpMM, the inner product V_{1:k}^T W, the IntraOrtho of W
      // (CholQR Gram or TSQR, into a scratch block), the Pythagorean
      // Cholesky from the two triangular factors, one projection
      for (int kk = 1; kk <= m; ++kk) {
        const int force = fk == kk ? 1 : 0;
        tag(kk, 0);
        op_apply(st, slot(k, kk - 1), k.W, ctl, tm);
        launch_gram<T>(st, gram_args<T>(k, kk, {}, {k.W}), k.partial, d.G, ctl, tm);
        const int house = p.muscle == LSBA_HOUSEQR ? 1 : 0;
        if (house)
          launch_house<T>(st, d, n, s, k.W, k.U, (T*)nullptr, k.hwork, HM_IO, kk, 0, tm);
        else
          launch_gram<T>(st, gram_args<T>(k, 0, {k.W}, {k.W}), k.partial, d.G2, ctl, tm);
        launch_small_pio(st, d, kk, force, house, tm);
        tag(kk, 1);
        finalize_after(kk, kk);
        UpdateArgs<T> u = upd_args(k);
        u.in2 = k.W;
        u.out2 = slot(k, kk);
        u.nv2_begin = 0;
        u.nv2 = kk;
        launch_update<T>(st, u, ctl, true, tm);
        if (rec_loo) {
          launch_gram<T>(st, gram_args<T>(k, kk + 1, {}, {slot(k, kk)}), k.partial, d.G2, ctl,
                         tm);
          launch_small_loo(st, d, kk + 1, tm);
        }
      }
    } else if (p.skeleton == LSBA_BMGS) {
      // Alg. 2: SpMM, then for i = 1..k one inner product V_i^T W and one
      // subtraction each (in place on W), then the IntraOrtho of W
      for (int kk = 1; kk <= m; ++kk) {
        const int force = fk == kk ? 1 : 0;
        tag(kk, 0);
        op_apply(st, slot(k, kk - 1), k.W, ctl, tm);
        for (int i = 1; i <= kk; ++i) {
          launch_gram<T>(st, gram_args<T>(k, 0, {slot(k, i - 1)}, {k.W}), k.partial, d.G, ctl,
                         tm);
          launch_small_bmgs(st, d, kk, i, tm);
          UpdateArgs<T> u = upd_args(k);
          u.in2 = k.W;
          u.out2 = k.W;
          u.nv2_begin = i - 1;
          u.nv2 = i;
          launch_update<T>(st, u, ctl, true, tm);
        }
        if (p.muscle == LSBA_HOUSEQR) {
          launch_house<T>(st, d, n, s, k.W, slot(k, kk), (T*)nullptr, k.hwork, HM_IO, kk, force,
                          tm);
          tag(kk, 1);
        } else if (mgs) {
          mgs_muscle(MGS_IOB, k.W, slot(k, kk), kk, force);
          tag(kk, 1);
        } else {
          launch_gram<T>(st, gram_args<T>(k, 0, {k.W}, {k.W}), k.partial, d.G2, ctl, tm);
          launch_small_svl_io(st, d, kk, force, tm);
          tag(kk, 1);
          UpdateArgs<T> u = upd_args(k);
          u.in1 = k.W;
          u.out1 = slot(k, kk);
          launch_update<T>(st, u, ctl, true, tm);
        }
        finalize_after(kk, kk);
        if (rec_loo) {
          launch_gram<T>(st, gram_args<T>(k, kk + 1, {}, {slot(k, kk)}), k.partial, d.G2, ctl,
                         tm);
          launch_small_loo(st, d, kk + 1, tm);
        }
      }
    } else {
      for (int kk = 1; kk <= m; ++kk) {
        const int force = fk == kk ? 1 : 0;
        tag(kk, 0);
        op_apply(st, slot(k, kk - 1), k.W, ctl, tm);
        launch_gram<T>(st, gram_args<T>(k, kk, {}, {k.W}), k.partial, d.G, ctl, tm);
        launch_small_svl_y(st, d, kk, tm);
        {
          UpdateArgs<T> u = upd_args(k);
          u.in2 = k.W;
          u.out2 = slot(k, kk);
          u.nv2_begin = 0;
          u.nv2 = kk;
          launch_update<T>(st, u, ctl, true, tm);
        }
        if (p.muscle == LSBA_HOUSEQR) {
          // IntraOrtho of the projected block in place; H_{kk+1,kk} = R
          launch_house<T>(st, d, n, s, slot(k, kk), slot(k, kk), (T*)nullptr, k.hwork, HM_IO, kk,
                          force, tm);
          tag(kk, 1);
        } else if (mgs) {
          // column-wise muscle in place; H_{kk+1,kk} = R, T_{kk+1,kk+1} = its T
          mgs_muscle(MGS_IO5, slot(k, kk), slot(k, kk), kk, force);
          tag(kk, 1);
        } else {
          launch_gram<T>(st, gram_args<T>(k, 0, {slot(k, kk)}, {slot(k, kk)}), k.partial, d.G2,
                         ctl, tm);
          launch_small_svl_io(st, d, kk, force, tm);
          tag(kk, 1);
          UpdateArgs<T> u = upd_args(k);
          u.in1 = slot(k, kk);
          u.out1 = slot(k, kk);
          launch_update<T>(st, u, ctl, true, tm);
        }
        launch_gram<T>(st, gram_args<T>(k, kk, {}, {slot(k, kk)}), k.partial, d.G, ctl, tm);
        launch_small_svl_z(st, d, kk, tm);
        finalize_after(kk, kk);
        if (rec_loo) {
          launch_gram<T>(st, gram_args<T>(k, kk + 1, {}, {slot(k, kk)}), k.partial, d.G2, ctl,
                         tm);
          launch_small_loo(st, d, kk + 1, tm);
        }
      }
    }
    // join the side streams, then end the cycle
    flush_side();
    if (used_side) {
      hipEvent_t e = event();
      HIPCHK(hipEventRecord(e, side));
      HIPCHK(hipStreamWaitEvent(st, e, 0));
    }
    if (used_side2) {
      hipEvent_t e2 = event();
      HIPCHK(hipEventRecord(e2, side2));
      HIPCHK(hipStreamWaitEvent(st, e2, 0));
    }
    tag(1 << 30, 0);
    launch_small_cycle_end(st, d, tm);
    UpdateArgs<T> ua = upd_args(k);
    ua.in1 = x;
    ua.out1 = x;
    ua.out2 = k.U;
    ua.nvp = &ctl->nv1;
    launch_update<T>(st, ua, ctl, false, tm);
  }

  bool finish() {
    Krylov<T>& k = *kp;
    hipStream_t st = c->stream;
    const int s = k.s;
    const int64_t n = k.n;
    Dense& d = k.d;
    Ctl* ctl = d.ctl;
    EventTimer* tm = c->timer;
    (void)s;
    (void)n;
    (void)ctl;
    (void)tm;
    const Ctl& hc = *c->ctl_host;
    const int j = hc.j;
    const int cst = hc.cyc_status;
    if (tm) {
      // bytes of the basis application, known only now
      if (tm->on(KK_UPDATE) && !tm->recs.empty()) {
        tm->recs.back().bytes = update_bytes(uapply, hc.nv1, hc.nv2_begin, hc.nv2);
        tm->recs.back().flops = update_flops(uapply, hc.nv1, hc.nv2_begin, hc.nv2);
      }
      if (cst == ST_CONVERGED || cst == ST_ITERCAP)
        tm->kill_after(delayed ? j + 1 : j, false);
      else if (cst == ST_FLAGGED)
        tm->kill_after(hc.flag_step, true);
      tm->flush();
    }
    const int ms = (p.muscle == LSBA_MGS_SVL || p.muscle == LSBA_MGS_LTS) ? 3 * kp->s - 2 : 1;
    cycle_counts(p.skeleton, ms, j, cst, hc.flag_step, out.a, out.v, out.sy);
    for (int i = 0; i < j; ++i) res->res.push_back(c->hist_host[i]);
    if (rec_loo) {
      for (int i = 0; i < j; ++i) {
        // the loss of orthogonality of the column that ended the solve is not formed
        const bool have = !(i == j - 1 && (cst == ST_CONVERGED || cst == ST_ITERCAP));
        res->loo.push_back(have ? c->hist_host[(kMaxM + 2) + i] : NAN);
      }
    }
    res->cyc.push_back(j);
    res->mafter.push_back(hc.m);
    out.iters = hc.iter;
    if (!hc.cont) {
      if (cst == ST_CONVERGED) out.status = LSBA_OK;
      else if (cst == ST_FLAGGED) out.status = LSBA_BREAKDOWN;
      else out.status = LSBA_NOT_CONVERGED;
      return true;
    }
    m = hc.m;
    R0 = k.U;
    return false;
  }
};

template <typename T>
CycleOut run_cycles(lsba_context* c, const lsba_operator* op, const lsba_params& p,
                    Krylov<T>& k, const T* val, const T* rhs, T* x, double nB, double tol,
                    lsba_result* res, const IluFactors* pc = nullptr, double* zpc = nullptr) {
  CycleRunner<T> r{c, op, p, &k, val, rhs, x, nB, tol, res};
  r.pc = pc;
  r.zpc = zpc;
  r.begin();
  for (;;) {
    if (r.cyc >= p.max_cycles) {
      r.out.status = LSBA_NOT_CONVERGED;
      return r.out;
    }
    r.enqueue();
    HIPCHK(hipEventSynchronize(c->ev_done));
    HIPCHK(hipGetLastError());
    if (r.finish()) return r.out;
  }
}

// ------------------------------------------------------------------ serving

// One request of the serving form: a copy of its right-hand side, its result,
// and host timestamps (steady clock, seconds).
struct SrvRequest {
  uint64_t ticket = 0;
  const lsba_operator* op = nullptr;
  lsba_params p{};
  int s = 0;
  int64_t n = 0;
  uint64_t footprint = 0;
  double* Bh = nullptr;   // pinned host copy of B (n x s), until the request ends
  double* Xh = nullptr;   // pinned host X (n x s), filled when the request ends
  lsba_result* res = nullptr;
  int state = 0;   // 0 queued, 1 running, 2 done
  ~SrvRequest() {
    if (Bh) (void)hipHostFree(Bh);
    if (Xh) (void)hipHostFree(Xh);
  }
};

// A slot runs one admitted request on its own context (streams, events,
// pinned staging, stream-ordered device buffers).
struct SrvSlot {
  lsba_context* c = nullptr;
  SrvRequest* req = nullptr;
  Krylov<double> k{};
  std::unique_ptr<CycleRunner<double>> run;
  double* B64 = nullptr;
  double* X64 = nullptr;
  double nB = 0.0;
  // work queued on the slot's stream and ended by its event ev_done:
  // 0 none, 1 upload of B and its norm, 2 a restart cycle, 3 the end of the
  // request (true residual, download of X)
  int phase = 0;
};

// Workspaces of the norm / residual reductions: taken from the context's
// buffer cache unless the caller passes them (the no-allocation entry point).
struct NormWork {
  double* norm_partial = nullptr;   // norm_partial_doubles(count)
  double* res_partial = nullptr;    // res_partial_doubles(n, s)
  double* out = nullptr;            // 4 doubles
};
size_t norm_partial_doubles(int64_t count) { return (size_t)(count / 4096) + 2; }
size_t res_partial_doubles(int64_t n, int s) {
  int sh = 0;
  while ((1 << sh) < s) ++sh;
  return (size_t)(((n << sh) + 255) / 256) + 1;
}

double device_norm(lsba_context* c, const double* x, int64_t count, const NormWork* w = nullptr) {
  double* partial = w ? w->norm_partial
                      : (double*)ctx_buf(c, "norm_partial",
                                         sizeof(double) * norm_partial_doubles(count));
  int nw = 0;
  launch_sumsq_partial(c->stream, count, x, partial, &nw);
  double* outd = w ? w->out : (double*)ctx_buf(c, "norm_out", sizeof(double) * 4);
  launch_sumsq_final(c->stream, partial, nw, outd);
  HIPCHK(hipMemcpyAsync(c->norm_host, outd, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return c->norm_host[0];
}

// R = B - A X (R may be null) and ||R||_F, FP64.
double device_residual(lsba_context* c, const lsba_operator* op, int s, const double* X,
                       const double* B, double* R, const NormWork* w = nullptr) {
  double* partial = w ? w->res_partial
                      : (double*)ctx_buf(c, "res_partial",
                                         sizeof(double) * res_partial_doubles(op->n, s));
  int nw = 0;
  launch_residual(c->stream, op->n, op->nnz, s, op->rp, op->ci, op->val, X, B, R, partial, &nw,
                  c->timer);
  double* outd = w ? w->out : (double*)ctx_buf(c, "norm_out", sizeof(double) * 4);
  launch_sumsq_final(c->stream, partial, nw, outd);
  HIPCHK(hipMemcpyAsync(c->norm_host, outd, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->timer) c->timer->flush();
  return c->norm_host[0];
}


// Queue ||x||_F (FP64, fixed order) and its copy to the context's pinned
// norm_host[slot] without waiting for it.
void enqueue_norm(lsba_context* c, const double* x, int64_t count, int slot) {
  double* partial = (double*)ctx_buf(c, "norm_partial",
                                     sizeof(double) * norm_partial_doubles(count));
  int nw = 0;
  launch_sumsq_partial(c->stream, count, x, partial, &nw);
  double* outd = (double*)ctx_buf(c, "norm_out", sizeof(double) * 4);
  launch_sumsq_final(c->stream, partial, nw, outd + slot);
  HIPCHK(hipMemcpyAsync(c->norm_host + slot, outd + slot, sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
}

// Queue ||B - A X||_F (FP64) and its copy to norm_host[slot] without waiting.
void enqueue_residual_norm(lsba_context* c, const lsba_operator* op, int s, const double* X,
                           const double* B, int slot) {
  double* partial = (double*)ctx_buf(c, "res_partial",
                                     sizeof(double) * res_partial_doubles(op->n, s));
  int nw = 0;
  launch_residual(c->stream, op->n, op->nnz, s, op->rp, op->ci, op->val, X, B, nullptr, partial,
                  &nw, c->timer);
  double* outd = (double*)ctx_buf(c, "norm_out", sizeof(double) * 4);
  launch_sumsq_final(c->stream, partial, nw, outd + slot);
  HIPCHK(hipMemcpyAsync(c->norm_host + slot, outd + slot, sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
}

void validate_params(const lsba_params* p, int s) {
  if (!p) throw ArgError{"params is NULL"};
  if (p->struct_size != sizeof(lsba_params)) throw ArgError{"params.struct_size mismatch"};
  if (s < 1 || s > kMaxS) throw ArgError{"s must be in [1, 32]"};
  if (p->m < 1 || p->m > kMaxM) throw ArgError{"m must be in [1, 128]"};
  if (p->method != LSBA_FOM && p->method != LSBA_GMRES) throw ArgError{"bad method"};
  if (p->skeleton < LSBA_BCGSI_LS || p->skeleton > LSBA_BCGS_PIO) throw ArgError{"bad skeleton"};
  if (p->muscle < LSBA_CHOLQR || p->muscle > LSBA_MGS_LTS) throw ArgError{"bad muscle"};
  if (p->skeleton == LSBA_BCGS_PIO && p->muscle != LSBA_CHOLQR && p->muscle != LSBA_HOUSEQR)
    throw ArgError{"BCGS-PIO is built with the CholQR and HouseQR muscles only"};
  if (p->precision != LSBA_FP64 && p->precision != LSBA_MIXED) throw ArgError{"bad precision"};
  if (!(p->tol >= 0.0)) throw ArgError{"tol must be >= 0"};
  if (p->max_cycles < 1) throw ArgError{"max_cycles must be >= 1"};
  if (p->precision == LSBA_MIXED && (p->max_refine < 1 || !(p->inner_tol > 0.0)))
    throw ArgError{"mixed form needs max_refine >= 1 and inner_tol > 0"};
}


lsba_status fail(lsba_context* c, lsba_status st, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return st;
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's copy of `scratch` (the current device is
// `device`); taken once per device.
void scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return;   // such devices get no scratch
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch_ptr[device] = p;
}

// Bump allocation of 256-byte aligned pieces of one region (or, with
// base == nullptr, just the bytes such pieces need).
struct Bump {
  char* base;
  size_t used = 0;
  void* take(size_t bytes) {
    void* p = base ? base + used : reinterpret_cast<void*>(uintptr_t(4096));
    used += align256(bytes);
    return p;
  }
};

// Device layout of one FP64 solve carved from a Bump region: B and X
// copies, norm workspaces and the Krylov state.
struct NoallocLayout {
  double* B64 = nullptr;
  double* X64 = nullptr;
  NormWork nw;
  Krylov<double> k{};
};
NoallocLayout noalloc_layout(Bump& b, int64_t n, int s, const lsba_params& p) {
  NoallocLayout L;
  const size_t blk64 = (size_t)n * s * sizeof(double);
  L.B64 = (double*)b.take(blk64);
  L.X64 = (double*)b.take(blk64);
  L.nw.norm_partial = (double*)b.take(sizeof(double) * norm_partial_doubles((int64_t)n * s));
  L.nw.res_partial = (double*)b.take(sizeof(double) * res_partial_doubles(n, s));
  L.nw.out = (double*)b.take(sizeof(double) * 4);
  L.k = make_krylov_with<double>([&b](const std::string&, size_t bytes) { return b.take(bytes); },
                                 n, s, p.m, p, "n_");
  return L;
}

}  // namespace

struct lsba_server {
  lsba_context* ctx = nullptr;
  uint64_t budget = 0, in_use = 0;
  int32_t peak_active = 0;
  uint64_t next_ticket = 1;
  std::vector<SrvSlot> slots;
  std::deque<SrvRequest*> queue;
  std::map<uint64_t, SrvRequest*> reqs;
  std::deque<uint64_t> done;   // completed, not yet reported by poll
};

namespace {

// Admit request r into slot sl: queue the upload of B and ||B||_F (phase 1).
// Nothing here waits for the device: the slot's progress continues in
// srv_progress once the slot's event has completed.
void srv_start(lsba_server* sv, SrvSlot& sl, SrvRequest* r) {
  lsba_context* c = sl.c;
  hipStream_t st = c->stream;
  const size_t blk64 = (size_t)r->n * r->s * sizeof(double);
  sl.req = r;
  r->state = 1;
  sv->in_use += r->footprint;
  sl.B64 = (double*)ctx_buf(c, "B64", blk64);
  sl.X64 = (double*)ctx_buf(c, "X64", blk64);
  r->res->have_loo = (r->p.record & LSBA_REC_LOO) != 0;
  HIPCHK(hipEventRecord(c->ev0, st));
  HIPCHK(hipMemcpyAsync(sl.B64, r->Bh, blk64, hipMemcpyHostToDevice, st));
  enqueue_norm(c, sl.B64, r->n * r->s, 0);
  HIPCHK(hipEventRecord(c->ev_done, st));
  sl.phase = 1;
}

// Queue the end of the request in slot sl (phase 3): its true residual (if
// recorded) and the download of X into pinned host memory.
void srv_finish_enqueue(SrvSlot& sl) {
  lsba_context* c = sl.c;
  SrvRequest* r = sl.req;
  hipStream_t st = c->stream;
  if (sl.run && (r->p.record & LSBA_REC_TRUE_RES))
    enqueue_residual_norm(c, r->op, r->s, sl.X64, sl.B64, 1);
  HIPCHK(hipMemcpyAsync(r->Xh, sl.X64, (size_t)r->n * r->s * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(c->ev1, st));
  HIPCHK(hipEventRecord(c->ev_done, st));
  sl.phase = 3;
}

// The end of the request in slot sl has completed: fill its result, release
// the slot's memory (stream-ordered), report it.
void srv_complete(lsba_server* sv, SrvSlot& sl) {
  lsba_context* c = sl.c;
  SrvRequest* r = sl.req;
  if (sl.run) {
    const CycleOut& o = sl.run->out;
    r->res->status = o.status;
    r->res->iters = o.iters;
    r->res->a = o.a;
    r->res->v = o.v;
    r->res->sy = o.sy;
    if (r->p.record & LSBA_REC_TRUE_RES) r->res->true_relres = c->norm_host[1] / sl.nB;
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  r->res->gpu_ms = ms;
  sl.run.reset();
  ctx_release(c);
  sv->in_use -= r->footprint;
  r->state = 2;   // the pinned copies go with the request at fetch (freeing pinned memory
                  // may wait for the device, which poll never does)
  sv->done.push_back(r->ticket);
  sl.req = nullptr;
  sl.phase = 0;
}

// One pass of the progress engine: advance every slot whose queued work has
// completed (hipEventQuery, never a wait), then admit queued requests in
// arrival order while a slot is free and the byte budget allows.
void srv_progress(lsba_server* sv) {
  for (auto& sl : sv->slots) {
    if (!sl.req || sl.phase == 0) continue;
    const hipError_t q = hipEventQuery(sl.c->ev_done);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();   // HIP records "not ready" as the thread's last error
      continue;
    }
    if (q != hipSuccess) throw HipError{std::string("slot event: ") + hipGetErrorString(q)};
    HIPCHK(hipGetLastError());
    SrvRequest* r = sl.req;
    if (sl.phase == 1) {
      sl.nB = sl.c->norm_host[0];
      if (sl.nB == 0.0) {
        HIPCHK(hipMemsetAsync(sl.X64, 0, (size_t)r->n * r->s * sizeof(double), sl.c->stream));
        r->res->status = LSBA_OK;
        r->res->true_relres = 0.0;
        sl.run.reset();
        srv_finish_enqueue(sl);
        continue;
      }
      sl.k = make_krylov<double>(sl.c, r->n, r->s, r->p.m, r->p, "d_");
      sl.run.reset(new CycleRunner<double>{sl.c, r->op, r->p, &sl.k, r->op->val, sl.B64, sl.X64,
                                           sl.nB, r->p.tol, r->res});
      sl.run->begin();
      sl.run->enqueue();
      sl.phase = 2;
    } else if (sl.phase == 2) {
      bool end = sl.run->finish();
      if (!end && sl.run->cyc >= r->p.max_cycles) {
        sl.run->out.status = LSBA_NOT_CONVERGED;
        end = true;
      }
      if (end) srv_finish_enqueue(sl);
      else sl.run->enqueue();
    } else {
      srv_complete(sv, sl);
    }
  }
  while (!sv->queue.empty()) {
    SrvRequest* r = sv->queue.front();
    if (sv->in_use + r->footprint > sv->budget) break;
    SrvSlot* free_slot = nullptr;
    for (auto& sl : sv->slots)
      if (!sl.req) {
        free_slot = &sl;
        break;
      }
    if (!free_slot) break;
    sv->queue.pop_front();
    srv_start(sv, *free_slot, r);
  }
  int32_t active = 0;
  for (auto& sl : sv->slots) active += sl.req ? 1 : 0;
  if (active > sv->peak_active) sv->peak_active = active;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

lsba_status lsba_params_default(lsba_params* p) {
  if (!p) return LSBA_ERR_ARG;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(lsba_params);
  p->method = LSBA_GMRES;
  p->skeleton = LSBA_BCGSI_LS;
  p->muscle = LSBA_CHOLQR;
  p->precision = LSBA_FP64;
  p->m = 20;
  p->tol = 1e-8;
  p->max_cycles = 50;
  p->max_iters = 0;
  p->max_refine = 20;
  p->inner_tol = 1e-4;
  p->record = 0;
  p->force_flag_cycle = -1;
  p->force_flag_step = -1;
  return LSBA_OK;
}

const char* lsba_status_string(lsba_status st) {
  switch (st) {
    case LSBA_OK: return "converged";
    case LSBA_NOT_CONVERGED: return "not converged";
    case LSBA_BREAKDOWN: return "breakdown (Cholesky flag with no final column)";
    case LSBA_ERR_ARG: return "invalid argument";
    case LSBA_ERR_OOM: return "out of memory";
    case LSBA_ERR_HIP: return "HIP runtime error";
    case LSBA_ERR_UNSUPPORTED: return "unsupported";
    case LSBA_ERR_BUSY: return "busy";
  }
  return "unknown status";
}

const char* lsba_last_error(const lsba_context* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

lsba_status lsba_context_create(int device, void* hip_stream, lsba_context** out) {
  if (!out) return fail(nullptr, LSBA_ERR_ARG, "ctx out pointer is NULL");
  *out = nullptr;
  auto* c = new (std::nothrow) lsba_context();
  if (!c) return fail(nullptr, LSBA_ERR_OOM, "host allocation failed");
  try {
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) {
      delete c;
      return fail(nullptr, LSBA_ERR_ARG, "device index out of range");
    }
    c->device = device;
    HIPCHK(hipSetDevice(device));
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void**)&c->ctl_host, sizeof(Ctl), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->hist_host, sizeof(double) * 2 * (kMaxM + 2),
                         hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->norm_host, sizeof(double) * 4, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->stage_host, sizeof(double) * kMaxS * kMaxS,
                         hipHostMallocDefault));
    HIPCHK(hipEventCreate(&c->ev0));
    HIPCHK(hipEventCreate(&c->ev1));
    HIPCHK(hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming));
    // the stream-ordering events a cycle records (two per batch of side jobs
    // and two at its end: at most kMaxEvents for m <= kMaxM), created here so
    // that solving creates none
    for (int i = 0; i < kMaxEvents; ++i) {
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->evs.push_back(e);
    }
    scratch_init(device);
  } catch (const HipError& e) {
    lsba_context_destroy(c);
    return fail(nullptr, LSBA_ERR_HIP, e.msg);
  }
  *out = c;
  return LSBA_OK;
}

static void operator_release(lsba_operator* op);

void lsba_context_destroy(lsba_context* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (lsba_operator* op : c->ops) {
    operator_release(op);
    op->ctx = nullptr;   // detached: lsba_operator_destroy then frees only the handle
  }
  c->ops.clear();
  for (lsba_precond* pc : c->pcs) {
    ilu_free(pc->f);
    pc->ctx = nullptr;   // detached likewise
  }
  c->pcs.clear();
  ctx_release(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->ctl_host) (void)hipHostFree(c->ctl_host);
  if (c->hist_host) (void)hipHostFree(c->hist_host);
  if (c->norm_host) (void)hipHostFree(c->norm_host);
  if (c->stage_host) (void)hipHostFree(c->stage_host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev_done) (void)hipEventDestroy(c->ev_done);
  delete c->timer;
  for (auto e : c->evs) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->side2) {
    (void)hipStreamSynchronize(c->side2);
    (void)hipStreamDestroy(c->side2);
  }
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

lsba_status lsba_operator_create_csr(lsba_context* c, int64_t n, int64_t nnz,
                                     const int64_t* row_ptr, const int32_t* col_idx,
                                     const double* values, int on_device, lsba_operator** out) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!out || !row_ptr || (nnz > 0 && (!col_idx || !values)))
    return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (n < 1 || nnz < 0) return fail(c, LSBA_ERR_ARG, "n must be >= 1 and nnz >= 0");
  if (n * (int64_t)kMaxS >= ((int64_t)1 << 31) * 64)
    return fail(c, LSBA_ERR_ARG, "n too large");
  *out = nullptr;
  auto* op = new (std::nothrow) lsba_operator();
  if (!op) return fail(c, LSBA_ERR_OOM, "host allocation failed");
  try {
    HIPCHK(hipSetDevice(c->device));
    // validate on the host
    std::vector<int64_t> rp_h;
    std::vector<int32_t> ci_h;
    const int64_t* rp = row_ptr;
    const int32_t* ci = col_idx;
    if (on_device) {
      rp_h.resize(n + 1);
      ci_h.resize(nnz);
      HIPCHK(hipMemcpy(rp_h.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
      if (nnz) HIPCHK(hipMemcpy(ci_h.data(), col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
      rp = rp_h.data();
      ci = ci_h.data();
    }
    if (rp[0] != 0 || rp[n] != nnz) {
      delete op;
      return fail(c, LSBA_ERR_ARG, "row_ptr[0] must be 0 and row_ptr[n] must be nnz");
    }
    for (int64_t i = 0; i < n; ++i)
      if (rp[i + 1] < rp[i]) {
        delete op;
        return fail(c, LSBA_ERR_ARG, "row_ptr is not non-decreasing");
      }
    for (int64_t e = 0; e < nnz; ++e)
      if (ci[e] < 0 || ci[e] >= n) {
        delete op;
        return fail(c, LSBA_ERR_ARG, "column index out of range");
      }
    op->ctx = c;
    op->n = n;
    op->nnz = nnz;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMalloc(&op->rp, sizeof(int64_t) * (n + 1)) != hipSuccess ||
        hipMalloc(&op->ci, sizeof(int) * std::max<int64_t>(nnz, 1)) != hipSuccess ||
        hipMalloc(&op->val, sizeof(double) * std::max<int64_t>(nnz, 1)) != hipSuccess) {
      lsba_operator_destroy(op);
      return fail(c, LSBA_ERR_OOM, "device allocation of the CSR arrays failed");
    }
    HIPCHK(hipMemcpy(op->rp, row_ptr, sizeof(int64_t) * (n + 1), kind));
    if (nnz) {
      HIPCHK(hipMemcpy(op->ci, col_idx, sizeof(int) * nnz, kind));
      HIPCHK(hipMemcpy(op->val, values, sizeof(double) * nnz, kind));
    }
  } catch (const HipError& e) {
    lsba_operator_destroy(op);
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  c->ops.insert(op);
  *out = op;
  return LSBA_OK;
}

// Release an operator's device memory (its context's stream drained first).
static void operator_release(lsba_operator* op) {
  if (op->ctx) {
    (void)hipSetDevice(op->ctx->device);
    if (op->ctx->stream) (void)hipStreamSynchronize(op->ctx->stream);
  }
  if (op->rp) (void)hipFree(op->rp);
  if (op->ci) (void)hipFree(op->ci);
  if (op->val) (void)hipFree(op->val);
  if (op->val32) (void)hipFree(op->val32);
  op->rp = nullptr;
  op->ci = nullptr;
  op->val = nullptr;
  op->val32 = nullptr;
}

void lsba_operator_destroy(lsba_operator* op) {
  if (!op) return;
  operator_release(op);
  if (op->ctx) op->ctx->ops.erase(op);
  delete op;
}

static lsba_status solve_impl(lsba_context* c, const lsba_operator* op, const lsba_precond* pc,
                              const lsba_params* prm, int32_t s, const double* B, int64_t ldb,
                              double* X, int64_t ldx, int on_device, lsba_result** out) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!op || !B || !X || !out) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (op->ctx != c) return fail(c, LSBA_ERR_ARG, "operator belongs to another context");
  *out = nullptr;
  try {
    validate_params(prm, s);
    if (ldb < s || ldx < s) throw ArgError{"ldb and ldx must be >= s"};
    if (pc) {
      if (pc->ctx != c) throw ArgError{"preconditioner belongs to another context"};
      if (pc->f.n != op->n) throw ArgError{"preconditioner and operator differ in size"};
      if (prm->precision != LSBA_FP64)
        throw Unsupported{"preconditioning is available in the FP64 form only"};
    }
  } catch (const ArgError& e) {
    return fail(c, LSBA_ERR_ARG, e.msg);
  } catch (const Unsupported& e) {
    return fail(c, LSBA_ERR_UNSUPPORTED, e.msg);
  }
  const lsba_params p = *prm;
  const int64_t n = op->n;
  auto* r = new (std::nothrow) lsba_result();
  if (!r) return fail(c, LSBA_ERR_OOM, "host allocation failed");
  try {
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const hipMemcpyKind in_kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind out_kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t blk64 = (size_t)n * s * sizeof(double);
    double* B64 = (double*)ctx_buf(c, "B64", blk64);
    double* X64 = (double*)ctx_buf(c, "X64", blk64);
    HIPCHK(hipEventRecord(c->ev0, st));
    HIPCHK(copy2d(B64, s * sizeof(double), B, ldb * sizeof(double), s * sizeof(double),
                            n, in_kind, st));
    const double nB = device_norm(c, B64, n * s);
    r->have_loo = (p.record & LSBA_REC_LOO) != 0;
    if (nB == 0.0) {
      HIPCHK(hipMemsetAsync(X64, 0, blk64, st));
      r->status = LSBA_OK;
      r->true_relres = 0.0;
    } else if (p.precision == LSBA_FP64) {
      Krylov<double> k = make_krylov<double>(c, n, s, p.m, p, "d_");
      double* zpc = pc ? (double*)ctx_buf(c, "Zpc", blk64) : nullptr;
      CycleOut o = run_cycles<double>(c, op, p, k, op->val, B64, X64, nB, p.tol, r,
                                      pc ? &pc->f : nullptr, zpc);
      // right preconditioning: the cycles accumulate Y of A M^{-1} Y = B;
      // X = M^{-1} Y
      if (pc) launch_ilu_apply(st, pc->f, s, X64, X64, nullptr, c->timer);
      r->status = o.status;
      r->iters = o.iters;
      r->a = o.a;
      r->v = o.v;
      r->sy = o.sy;
      if (p.record & LSBA_REC_TRUE_RES)
        r->true_relres = device_residual(c, op, s, X64, B64, nullptr) / nB;
    } else {
      if (!op->val32) {
        auto* mop = const_cast<lsba_operator*>(op);
        if (hipMalloc(&mop->val32, sizeof(float) * std::max<int64_t>(op->nnz, 1)) != hipSuccess)
          throw HipError{"hipMalloc of the FP32 operator values failed"};
        if (op->nnz) launch_cast<float>(st, op->nnz, op->val, mop->val32);
      }
      double* R64 = (double*)ctx_buf(c, "R64", blk64);
      float* Rf = (float*)ctx_buf(c, "Rf32", (size_t)n * s * sizeof(float));
      float* Df = (float*)ctx_buf(c, "Df32", (size_t)n * s * sizeof(float));
      Krylov<float> k = make_krylov<float>(c, n, s, p.m, p, "f_");
      HIPCHK(hipMemsetAsync(X64, 0, blk64, st));
      HIPCHK(hipMemcpyAsync(R64, B64, blk64, hipMemcpyDeviceToDevice, st));
      double rn = nB;
      r->status = LSBA_NOT_CONVERGED;
      for (int it = 0; it < p.max_refine; ++it) {
        if (rn / nB <= p.tol) {
          r->status = LSBA_OK;
          break;
        }
        launch_cast<float>(st, n * s, R64, Rf);
        // each inner solve reduces its residual by inner_tol, but never further
        // than the outer target needs (half of it, for the FP32 estimate's slack)
        const double itol = std::max(p.inner_tol, 0.5 * p.tol * nB / rn);
        CycleOut o = run_cycles<float>(c, op, p, k, op->val32, Rf, Df, rn, itol, r);
        r->iters += o.iters;
        r->a += o.a;
        r->v += o.v;
        r->sy += o.sy;
        r->refine += 1;
        if (o.status == LSBA_BREAKDOWN) {
          r->status = LSBA_BREAKDOWN;
          break;
        }
        launch_add_to_double<float>(st, n * s, Df, X64);
        rn = device_residual(c, op, s, X64, B64, R64);
      }
      if (r->status == LSBA_NOT_CONVERGED && rn / nB <= p.tol) r->status = LSBA_OK;
      r->true_relres = rn / nB;
    }
    HIPCHK(copy2d(X, ldx * sizeof(double), X64, s * sizeof(double), s * sizeof(double),
                            n, out_kind, st));
    HIPCHK(hipEventRecord(c->ev1, st));
    HIPCHK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    r->gpu_ms = ms;
  } catch (const HipError& e) {
    delete r;
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  *out = r;
  return r->status;
}

lsba_status lsba_solve(lsba_context* c, const lsba_operator* op, const lsba_params* prm,
                       int32_t s, const double* B, int64_t ldb, double* X, int64_t ldx,
                       int on_device, lsba_result** out) {
  return solve_impl(c, op, nullptr, prm, s, B, ldb, X, ldx, on_device, out);
}

lsba_status lsba_solve_precond(lsba_context* c, const lsba_operator* op, const lsba_precond* pc,
                               const lsba_params* prm, int32_t s, const double* B, int64_t ldb,
                               double* X, int64_t ldx, int on_device, lsba_result** out) {
  if (c && !pc) return fail(c, LSBA_ERR_ARG, "NULL preconditioner");
  return solve_impl(c, op, pc, prm, s, B, ldb, X, ldx, on_device, out);
}

// ------------------------------------------------------------ ILU(0)

static void precond_release(lsba_precond* pc) {
  if (pc->ctx) {
    (void)hipSetDevice(pc->ctx->device);
    if (pc->ctx->stream) (void)hipStreamSynchronize(pc->ctx->stream);
  }
  ilu_free(pc->f);
}

lsba_status lsba_precond_create_ilu0(lsba_context* c, const lsba_operator* op,
                                     lsba_precond** out) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!op || !out) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (op->ctx != c) return fail(c, LSBA_ERR_ARG, "operator belongs to another context");
  *out = nullptr;
  auto* pc = new (std::nothrow) lsba_precond();
  if (!pc) return fail(c, LSBA_ERR_OOM, "host allocation failed");
  pc->ctx = c;
  try {
    HIPCHK(hipSetDevice(c->device));
    std::vector<int64_t> rp(op->n + 1);
    std::vector<int> ci(op->nnz);
    HIPCHK(hipMemcpy(rp.data(), op->rp, sizeof(int64_t) * (op->n + 1), hipMemcpyDeviceToHost));
    if (op->nnz)
      HIPCHK(hipMemcpy(ci.data(), op->ci, sizeof(int) * op->nnz, hipMemcpyDeviceToHost));
    int64_t bad = -1;
    bool bad_input = false;
    const std::string e = ilu_build(c->stream, op->n, op->nnz, rp.data(), ci.data(), op->val,
                                    pc->f, &bad, &bad_input);
    if (!e.empty()) {
      precond_release(pc);
      delete pc;
      const lsba_status st = bad_input                                  ? LSBA_ERR_ARG
                             : e.find("device allocation") == 0 ? LSBA_ERR_OOM
                                                                : LSBA_ERR_HIP;
      return fail(c, st, e);
    }
  } catch (const HipError& e) {
    precond_release(pc);
    delete pc;
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  c->pcs.insert(pc);
  *out = pc;
  return LSBA_OK;
}

void lsba_precond_destroy(lsba_precond* pc) {
  if (!pc) return;
  precond_release(pc);
  if (pc->ctx) pc->ctx->pcs.erase(pc);
  delete pc;
}

lsba_status lsba_precond_apply(lsba_context* c, const lsba_precond* pc, int32_t s,
                               const double* Y, int64_t ldy, double* Z, int64_t ldz,
                               int on_device) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!pc || !Y || !Z) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (pc->ctx != c) return fail(c, LSBA_ERR_ARG, "preconditioner belongs to another context");
  if (s < 1 || s > kMaxS) return fail(c, LSBA_ERR_ARG, "s must be in [1, 32]");
  if (ldy < s || ldz < s) return fail(c, LSBA_ERR_ARG, "ldy and ldz must be >= s");
  try {
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const int64_t n = pc->f.n;
    const hipMemcpyKind in_kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind out_kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    double* W = (double*)ctx_buf(c, "PcW", (size_t)n * s * sizeof(double));
    HIPCHK(copy2d(W, s * sizeof(double), Y, ldy * sizeof(double), s * sizeof(double),
                            n, in_kind, st));
    launch_ilu_apply(st, pc->f, s, W, W, nullptr, c->timer);
    HIPCHK(hipGetLastError());
    HIPCHK(copy2d(Z, ldz * sizeof(double), W, s * sizeof(double), s * sizeof(double),
                            n, out_kind, st));
    HIPCHK(hipStreamSynchronize(st));
    if (c->timer) c->timer->flush();
  } catch (const HipError& e) {
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  return LSBA_OK;
}

lsba_status lsba_precond_factors(const lsba_precond* pc, int64_t* row_ptr, int32_t* col_idx,
                                 double* values) {
  if (!pc || !row_ptr || (pc->f.nnz > 0 && (!col_idx || !values))) return LSBA_ERR_ARG;
  if (!pc->ctx) return LSBA_ERR_ARG;
  lsba_context* c = pc->ctx;
  try {
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = pc->f.n, nnz = pc->f.nnz;
    HIPCHK(hipMemcpy(row_ptr, pc->f.frp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    if (nnz) {
      HIPCHK(hipMemcpy(col_idx, pc->f.fci, sizeof(int) * nnz, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(values, pc->f.fv, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
  } catch (const HipError& e) {
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  return LSBA_OK;
}

lsba_status lsba_precond_info(const lsba_precond* pc, int64_t* n, int64_t* nnz,
                              int32_t* levels_lower, int32_t* levels_upper) {
  if (!pc) return LSBA_ERR_ARG;
  if (n) *n = pc->f.n;
  if (nnz) *nnz = pc->f.nnz;
  if (levels_lower) *levels_lower = pc->f.lo.nlev;
  if (levels_upper) *levels_upper = pc->f.up.nlev;
  return LSBA_OK;
}

lsba_status lsba_solve_noalloc(lsba_context* c, const lsba_operator* op,
                               const lsba_params* prm, int32_t s, const double* B, int64_t ldb,
                               double* X, int64_t ldx, lsba_result** out) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!op || !B || !X || !out) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (op->ctx != c) return fail(c, LSBA_ERR_ARG, "operator belongs to another context");
  *out = nullptr;
  try {
    validate_params(prm, s);
    if (ldb < s || ldx < s) throw ArgError{"ldb and ldx must be >= s"};
    if (prm->precision != LSBA_FP64)
      throw Unsupported{"lsba_solve_noalloc runs the FP64 form only"};
  } catch (const ArgError& e) {
    return fail(c, LSBA_ERR_ARG, e.msg);
  } catch (const Unsupported& e) {
    return fail(c, LSBA_ERR_UNSUPPORTED, e.msg);
  }
  const lsba_params p = *prm;
  const int64_t n = op->n;
  if (c->device < 0 || c->device >= kScratchDevices || !g_scratch_ptr[c->device])
    return fail(c, LSBA_ERR_UNSUPPORTED, "no scratch memory on this device");
  {
    Bump need{nullptr};
    (void)noalloc_layout(need, n, s, p);
    if (need.used > kScratchBytes)
      return fail(c, LSBA_ERR_ARG,
                  "problem needs " + std::to_string(need.used) +
                      " bytes of workspace; lsba_solve_noalloc has " +
                      std::to_string(kScratchBytes));
  }
  auto* r = new (std::nothrow) lsba_result();
  if (!r) return fail(c, LSBA_ERR_OOM, "host allocation failed");
  // kernel timing (it creates events) and cycle capture (it instantiates
  // graphs) are suspended for this call
  EventTimer* saved_timer = c->timer;
  const bool saved_graphs = c->graphs_on;
  c->timer = nullptr;
  c->graphs_on = false;
  lsba_status ret = LSBA_OK;
  try {
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    Bump b{static_cast<char*>(g_scratch_ptr[c->device])};
    NoallocLayout L = noalloc_layout(b, n, s, p);
    HIPCHK(hipEventRecord(c->ev0, st));
    HIPCHK(copy2d(L.B64, s * sizeof(double), B, ldb * sizeof(double),
                            s * sizeof(double), n, hipMemcpyDeviceToDevice, st));
    const double nB = device_norm(c, L.B64, n * s, &L.nw);
    r->have_loo = (p.record & LSBA_REC_LOO) != 0;
    if (nB == 0.0) {
      HIPCHK(hipMemsetAsync(L.X64, 0, (size_t)n * s * sizeof(double), st));
      r->status = LSBA_OK;
      r->true_relres = 0.0;
    } else {
      CycleOut o = run_cycles<double>(c, op, p, L.k, op->val, L.B64, L.X64, nB, p.tol, r);
      r->status = o.status;
      r->iters = o.iters;
      r->a = o.a;
      r->v = o.v;
      r->sy = o.sy;
      if (p.record & LSBA_REC_TRUE_RES)
        r->true_relres = device_residual(c, op, s, L.X64, L.B64, nullptr, &L.nw) / nB;
    }
    HIPCHK(copy2d(X, ldx * sizeof(double), L.X64, s * sizeof(double),
                            s * sizeof(double), n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipEventRecord(c->ev1, st));
    HIPCHK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    r->gpu_ms = ms;
  } catch (const HipError& e) {
    delete r;
    r = nullptr;
    ret = fail(c, LSBA_ERR_HIP, e.msg);
  }
  c->timer = saved_timer;
  c->graphs_on = saved_graphs;
  if (!r) return ret;
  *out = r;
  return r->status;
}

lsba_status lsba_context_set_timing(lsba_context* c, uint32_t kind_mask) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  try {
    (void)hipSetDevice(c->device);
    if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    delete c->timer;
    c->timer = kind_mask ? new EventTimer(kind_mask) : nullptr;
  } catch (const HipError& e) {
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  return LSBA_OK;
}

lsba_status lsba_context_set_graphs(lsba_context* c, int enable) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  (void)hipSetDevice(c->device);
  graphs_clear(c);
  c->graphs_on = enable != 0;
  return LSBA_OK;
}

lsba_status lsba_context_kernel_stats(const lsba_context* c, int32_t kind, int64_t* launches,
                                      double* total_ms, double* total_bytes) {
  if (!c || kind < 0 || kind >= KK_COUNT) return LSBA_ERR_ARG;
  const EventTimer::Acc a = c->timer ? c->timer->acc[kind] : EventTimer::Acc{};
  if (launches) *launches = a.launches;
  if (total_ms) *total_ms = a.ms;
  if (total_bytes) *total_bytes = a.bytes;
  return LSBA_OK;
}

lsba_status lsba_context_kernel_flops(const lsba_context* c, int32_t kind, double* total_flops) {
  if (!c || kind < 0 || kind >= KK_COUNT || !total_flops) return LSBA_ERR_ARG;
  *total_flops = c->timer ? c->timer->acc[kind].flops : 0.0;
  return LSBA_OK;
}

lsba_status lsba_result_set_err_vs_ref(lsba_context* c, lsba_result* r, int64_t n, int32_t s,
                                       const double* X, int64_t ldx, const double* Xref,
                                       int64_t ldr, int on_device) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!r || !X || !Xref) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (n < 1 || s < 1 || ldx < s || ldr < s) return fail(c, LSBA_ERR_ARG, "bad sizes");
  try {
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const double* Xd = X;
    const double* Rd = Xref;
    int64_t lx = ldx, lr = ldr;
    const size_t blk = (size_t)n * s * sizeof(double);
    if (!on_device) {
      double* a = (double*)ctx_buf(c, "cmp_x", blk);
      double* b = (double*)ctx_buf(c, "cmp_ref", blk);
      HIPCHK(copy2d(a, s * sizeof(double), X, ldx * sizeof(double), s * sizeof(double),
                              n, hipMemcpyHostToDevice, st));
      HIPCHK(copy2d(b, s * sizeof(double), Xref, ldr * sizeof(double),
                              s * sizeof(double), n, hipMemcpyHostToDevice, st));
      Xd = a;
      Rd = b;
      lx = lr = s;
    }
    double* partial = (double*)ctx_buf(c, "cmp_partial",
                                       sizeof(double) * norm_partial_doubles((int64_t)n * s));
    double* outd = (double*)ctx_buf(c, "norm_out", sizeof(double) * 4);
    int nw = 0;
    launch_diff_sumsq_partial(st, n, s, Xd, lx, Rd, lr, partial, &nw);
    launch_sumsq_final(st, partial, nw, outd);
    HIPCHK(hipMemcpyAsync(c->norm_host, outd, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double dn = c->norm_host[0];
    // ||Xref||_F over contiguous rows
    const double* Rc = Rd;
    if (lr != s) {
      double* b = (double*)ctx_buf(c, "cmp_ref", blk);
      HIPCHK(copy2d(b, s * sizeof(double), Rd, lr * sizeof(double), s * sizeof(double),
                              n, hipMemcpyDeviceToDevice, st));
      Rc = b;
    }
    const double rn = device_norm(c, Rc, (int64_t)n * s);
    r->err_vs_ref = rn > 0.0 ? dn / rn : dn;
  } catch (const HipError& e) {
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  return LSBA_OK;
}

double lsba_result_err_vs_ref(const lsba_result* r) { return r ? r->err_vs_ref : NAN; }

lsba_status lsba_result_status(const lsba_result* r) { return r ? r->status : LSBA_ERR_ARG; }
int64_t lsba_result_iters(const lsba_result* r) { return r ? r->iters : 0; }
const double* lsba_result_res_hist(const lsba_result* r) {
  return r && !r->res.empty() ? r->res.data() : nullptr;
}
const double* lsba_result_loo_hist(const lsba_result* r) {
  return r && r->have_loo && !r->loo.empty() ? r->loo.data() : nullptr;
}
int32_t lsba_result_cycles(const lsba_result* r) { return r ? (int32_t)r->cyc.size() : 0; }
const int32_t* lsba_result_cycle_len(const lsba_result* r) {
  return r && !r->cyc.empty() ? r->cyc.data() : nullptr;
}
const int32_t* lsba_result_m_after(const lsba_result* r) {
  return r && !r->mafter.empty() ? r->mafter.data() : nullptr;
}
void lsba_result_counts(const lsba_result* r, int64_t* a, int64_t* v, int64_t* sy) {
  if (a) *a = r ? r->a : 0;
  if (v) *v = r ? r->v : 0;
  if (sy) *sy = r ? r->sy : 0;
}
double lsba_result_true_relres(const lsba_result* r) { return r ? r->true_relres : NAN; }
int32_t lsba_result_refine_steps(const lsba_result* r) { return r ? r->refine : 0; }
double lsba_result_gpu_ms(const lsba_result* r) { return r ? r->gpu_ms : 0.0; }
void lsba_result_destroy(lsba_result* r) { delete r; }

uint64_t lsba_solve_footprint(int64_t n, int32_t s, const lsba_params* p) {
  if (!p || n < 1 || s < 1 || s > kMaxS || p->m < 1 || p->m > kMaxM) return 0;
  return solve_footprint(n, s, *p);
}

lsba_status lsba_server_create(lsba_context* c, uint64_t hbm_budget_bytes, int32_t max_slots,
                               lsba_server** out) {
  if (!c) return fail(nullptr, LSBA_ERR_ARG, "context is NULL");
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes == 0)
    return fail(c, LSBA_ERR_ARG, "need out != NULL, 1 <= max_slots <= 64, budget > 0");
  *out = nullptr;
  auto* sv = new (std::nothrow) lsba_server();
  if (!sv) return fail(c, LSBA_ERR_OOM, "host allocation failed");
  sv->ctx = c;
  sv->budget = hbm_budget_bytes;
  sv->slots.resize(max_slots);
  for (auto& sl : sv->slots) {
    const lsba_status st = lsba_context_create(c->device, nullptr, &sl.c);
    if (st != LSBA_OK) {
      lsba_server_destroy(sv);
      return fail(c, st, "slot context: " + g_create_err);
    }
    sl.c->async_alloc = true;
  }
  *out = sv;
  return LSBA_OK;
}

lsba_status lsba_server_submit(lsba_server* sv, const lsba_operator* op, const lsba_params* prm,
                               int32_t s, const double* B, int64_t ldb, int on_device,
                               uint64_t* ticket) {
  if (!sv) return fail(nullptr, LSBA_ERR_ARG, "server is NULL");
  lsba_context* c = sv->ctx;
  if (!op || !B || !ticket) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  if (op->ctx != c) return fail(c, LSBA_ERR_ARG, "operator belongs to another context");
  try {
    validate_params(prm, s);
    if (ldb < s) throw ArgError{"ldb must be >= s"};
    if (prm->precision != LSBA_FP64) throw Unsupported{"the serving form runs FP64 solves"};
  } catch (const ArgError& e) {
    return fail(c, LSBA_ERR_ARG, e.msg);
  } catch (const Unsupported& e) {
    return fail(c, LSBA_ERR_UNSUPPORTED, e.msg);
  }
  const uint64_t fp = solve_footprint(op->n, s, *prm);
  if (fp > sv->budget) return fail(c, LSBA_ERR_OOM, "request footprint exceeds the server budget");
  auto* r = new (std::nothrow) SrvRequest();
  if (!r) return fail(c, LSBA_ERR_OOM, "host allocation failed");
  r->res = new (std::nothrow) lsba_result();
  if (!r->res) {
    delete r;
    return fail(c, LSBA_ERR_OOM, "host allocation failed");
  }
  r->op = op;
  r->p = *prm;
  r->s = s;
  r->n = op->n;
  r->footprint = fp;
  try {
    HIPCHK(hipSetDevice(c->device));
    const size_t blk = (size_t)r->n * s * sizeof(double);
    if (hipHostMalloc((void**)&r->Bh, blk, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&r->Xh, blk, hipHostMallocDefault) != hipSuccess) {
      delete r->res;
      delete r;
      return fail(c, LSBA_ERR_OOM, "pinned host allocation failed");
    }
    HIPCHK(copy2d_sync(r->Bh, s * sizeof(double), B, ldb * sizeof(double), s * sizeof(double),
                       r->n, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
  } catch (const HipError& e) {
    delete r->res;
    delete r;
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  r->ticket = sv->next_ticket++;
  sv->reqs[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  return LSBA_OK;
}

lsba_status lsba_server_poll(lsba_server* sv, uint64_t* done, int32_t cap, int32_t* n_done) {
  if (!sv) return fail(nullptr, LSBA_ERR_ARG, "server is NULL");
  if (!n_done || cap < 0 || (cap > 0 && !done)) return fail(sv->ctx, LSBA_ERR_ARG, "bad output");
  try {
    HIPCHK(hipSetDevice(sv->ctx->device));
    srv_progress(sv);
  } catch (const HipError& e) {
    return fail(sv->ctx, LSBA_ERR_HIP, e.msg);
  }
  int32_t k = 0;
  while (k < cap && !sv->done.empty()) {
    done[k++] = sv->done.front();
    sv->done.pop_front();
  }
  *n_done = k;
  return LSBA_OK;
}

lsba_status lsba_server_fetch(lsba_server* sv, uint64_t ticket, double* X, int64_t ldx,
                              int on_device, lsba_result** out) {
  if (!sv) return fail(nullptr, LSBA_ERR_ARG, "server is NULL");
  lsba_context* c = sv->ctx;
  if (!X || !out) return fail(c, LSBA_ERR_ARG, "NULL pointer argument");
  *out = nullptr;
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(c, LSBA_ERR_ARG, "unknown ticket");
  SrvRequest* r = it->second;
  if (r->state != 2) return fail(c, LSBA_ERR_BUSY, "request not finished");
  if (ldx < r->s) return fail(c, LSBA_ERR_ARG, "ldx must be >= s");
  try {
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(copy2d_sync(X, ldx * sizeof(double), r->Xh, r->s * sizeof(double),
                       r->s * sizeof(double), r->n,
                       on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
  } catch (const HipError& e) {
    return fail(c, LSBA_ERR_HIP, e.msg);
  }
  *out = r->res;
  sv->reqs.erase(it);
  delete r;
  return (*out)->status;
}

lsba_status lsba_server_stats(const lsba_server* sv, int32_t* active, int32_t* queued,
                              uint64_t* bytes_in_use, int32_t* peak_active) {
  if (!sv) return LSBA_ERR_ARG;
  int32_t a = 0;
  for (const auto& sl : sv->slots) a += sl.req ? 1 : 0;
  if (active) *active = a;
  if (queued) *queued = (int32_t)sv->queue.size();
  if (bytes_in_use) *bytes_in_use = sv->in_use;
  if (peak_active) *peak_active = sv->peak_active;
  return LSBA_OK;
}

void lsba_server_destroy(lsba_server* sv) {
  if (!sv) return;
  for (auto& sl : sv->slots) {
    if (sl.c) {
      (void)hipSetDevice(sl.c->device);
      (void)hipStreamSynchronize(sl.c->side);
      (void)hipStreamSynchronize(sl.c->stream);
      sl.run.reset();
      lsba_context_destroy(sl.c);
      sl.c = nullptr;
    }
  }
  for (auto& kv : sv->reqs) {
    delete kv.second->res;
    delete kv.second;
  }
  delete sv;
}

}  // extern "C"
