// Host runtime and C-ABI of the GCR(k) depth solver (see include/mpgcr.h).
//
// The solve is driven from the host one GCR cycle at a time: every kernel of
// an iteration is enqueued on the solver's stream, the per-member scalars
// (beta, alpha, ||r||, exit decisions) stay on the device, and the host reads
// the members' "done" flags once per cycle.  Finished members make every
// later kernel return at once, so a batch runs until its slowest member.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/mpgcr.h"
#include "cnn_internal.h"
#include "kernels.h"
#include "learned.h"

using namespace mpgcr;

namespace {

thread_local std::string g_create_error;

}  // namespace

// Rows of members with the same points-per-lane M form one contiguous range
// and are processed by one kernel specialisation.
struct RowClass {
  int log2m, row_begin, row_end;
  int flat;   // every member of the range has no orography (set by refresh_flat)
};

namespace {

template <typename T>
T* dalloc(size_t n, hipError_t& err) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess && err == hipSuccess) err = e;
  return (T*)p;
}

}  // namespace

// Stream of the launches the calling thread enqueues: a group's stream inside
// a solve, else the solver's stream.
static thread_local hipStream_t t_stream = nullptr;

struct gcr_solver {
  gcr_params prm{};
  std::vector<int> nx, ny;
  std::vector<MemberGeom> geom_h;
  std::vector<int> have_op;
  std::vector<int> flat_h;            // per member: no orography (mirrors `flat` on the device)
  std::vector<double> scale_h;
  int rows = 0;
  long long npts = 0;
  int nxmax = 0;
  std::vector<RowClass> classes;     // contiguous row ranges of equal points-per-lane
  hipStream_t stream = nullptr;
  // Groups of members with rows contiguous in row order, each solved on a
  // stream of its own, so that one group's kernel boundaries (the drain of
  // the last waves, the start of the next kernel) overlap the others' work.
  // Empty: the whole batch on `stream`.
  struct Group {
    int q0 = 0, q1 = 0;                // members morder[q0 .. q1)
    std::vector<RowClass> classes;     // the group's rows
    hipStream_t st = nullptr;
    hipEvent_t cycle_ev[2] = {};
    int* ring[2] = {};                 // pinned copies of the done flags after a cycle
    hipEvent_t done_ev = nullptr;
  };
  std::vector<Group> groups;
  std::vector<int> morder_h;         // members in row order
  int* morder = nullptr;
  hipEvent_t fork_ev = nullptr;
  // one host thread per group beyond the first enqueues that group's work
  // (one thread cannot enqueue several groups' launches as fast as the GPU runs them)
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_job, cv_done;
  std::function<int(int)> job;       // job(group) of the current solve
  std::vector<int> job_rc;
  long job_gen = 0;
  int job_pending = 0;
  bool quit = false;
  std::mutex err_mu;
  int device = 0;
  std::string err;

  // device memory
  std::vector<void*> allocs;
  MemberGeom* geom = nullptr;
  int* rowmap = nullptr;
  MemberState* state = nullptr;
  Pending* pend = nullptr;            // per member: recorded step-2 updates
  int* done_flag = nullptr;           // per member: the done flag the host polls
  float* split = nullptr;             // split residual: Phi_hat, its NSD differences, Phi_tilde (pooled,
                                      // allocated by the first gcr_set_split_base)
  std::vector<int> have_split;
  double* part = nullptr;
  double* scale = nullptr;
  float* a32[NCOEF] = {};
  __half* a16[NCOEF] = {};
  double* c64 = nullptr;
  float* c32 = nullptr;
  double* phi64 = nullptr;           // depth fields for the on-the-fly coefficients
  double* hs64 = nullptr;
  float* phi32 = nullptr;
  float* hs32 = nullptr;
  int* flat = nullptr;                // per member: no orography (H* = Phi*)
  double* fac64 = nullptr;           // [rows][NFAC] latitude factors
  float* fac32 = nullptr;
  double* x = nullptr;
  double* rhs = nullptr;
  double* r64 = nullptr;
  void* r = nullptr;
  void* e = nullptr;
  void* le = nullptr;
  void* q[2] = {};
  float* qs[2] = {};
  void* p[KMAX + 1] = {};
  void* lp[KMAX + 1] = {};
  float* dx = nullptr;
  double* hist = nullptr;
  int hist_stride = 0;
  // float64 scratch for stand-alone preconditioner calls in the mixed forms
  double* aux_r = nullptr;
  double* aux_e = nullptr;
  double* aux_q[2] = {};
  const double** ptr_rhs = nullptr;  // device tables of caller pointers
  double** ptr_x = nullptr;
  const void** ptr_stage = nullptr;  // pinned host staging for the tables
  MemberState* state_h = nullptr;    // pinned host copy
  int* state_ring[2] = {};           // pinned copies of the done flags after a cycle
  hipEvent_t cycle_ev[2] = {};       // recorded after each copy
  AsmMember* asm_stage = nullptr;    // pinned staging of the assembly table
  hipEvent_t stage_ev[2] = {};       // recorded after the uploads from ptr_stage / asm_stage
  AsmMember* asm_tab = nullptr;      // device assembly table [batch]
  cnn_net* net = nullptr;            // learned preconditioner (GCR_PC_LEARNED), owned
  int* learn_active = nullptr;       // [batch] images the network runs on in one application
  double fallback_ratio = 0.5;

  // optional per-kernel timing with HIP events on the solver's stream
  bool timing = false;
  std::vector<hipEvent_t> ev;        // pool, pairs (start, stop)
  std::vector<int> ev_kind;          // kind of each recorded pair
  size_t ev_used = 0;
  int64_t kt_count[KT_COUNT] = {};
  double kt_ms[KT_COUNT] = {};
  void tm_begin(int kind) {
    if (!timing) return;
    if (ev_used + 2 > ev.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { timing = false; return; }
        ev.push_back(e);
      }
    }
    if (ev_kind.size() < ev.size() / 2) ev_kind.resize(ev.size() / 2);
    ev_kind[ev_used / 2] = kind;
    (void)hipEventRecord(ev[ev_used], t_stream ? t_stream : stream);
  }
  void tm_end() {
    if (!timing) return;
    (void)hipEventRecord(ev[ev_used + 1], t_stream ? t_stream : stream);
    ev_used += 2;
  }
  void tm_collect() {  // after a stream synchronisation
    for (size_t i = 0; i + 1 < ev_used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) {
        kt_count[ev_kind[i / 2]] += 1;
        kt_ms[ev_kind[i / 2]] += ms;
      }
    }
    ev_used = 0;
  }
};

static hipStream_t cur_stream(const gcr_solver* s) { return t_stream ? t_stream : s->stream; }
static void worker_main(gcr_solver* s, int w);
static void stop_workers(gcr_solver* s);

static int fail(gcr_solver* s, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) {
    std::lock_guard<std::mutex> lk(s->err_mu);
    s->err = buf;
  } else {
    g_create_error = buf;
  }
  return code;
}

#define HIPCHK(s, call)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail((s), GCR_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define KLAUNCH(s, kind, ...)   \
  do {                          \
    (s)->tm_begin(kind);        \
    hipLaunchKernelGGL(__VA_ARGS__); \
    (s)->tm_end();              \
  } while (0)

// Launch a kernel through a pointer to its specialisation, timed if enabled.
template <typename... KArgs, typename... Args>
static void launch(gcr_solver* s, int kind, void (*kern)(KArgs...), dim3 grid, dim3 block, Args... args) {
  s->tm_begin(kind);
  hipLaunchKernelGGL(kern, grid, block, 0, cur_stream(s), args...);
  s->tm_end();
}

// One launch of row kernel KNAME<P, M> per row class, each covering that
// class's rows (one wave per row).
static_assert(KT_COUNT == GCR_K_COUNT, "kernel kinds match the header");

#define ROWS_LAUNCH(s, CLASSES, F, KIND, KNAME, P, ...)                                     \
  for (const RowClass& c_ : (CLASSES)) {                                                 \
    Fields f_ = (F);                                                                     \
    f_.row_base = c_.row_begin;                                                          \
    f_.row_end = c_.row_end;                                                             \
    const dim3 g_((c_.row_end - c_.row_begin + WPB - 1) / WPB), b_(WG);                  \
    switch (c_.log2m) {                                                                  \
      case 1: launch(s, KIND, &KNAME<P, 2>, g_, b_, f_, ##__VA_ARGS__); break;            \
      case 2: launch(s, KIND, &KNAME<P, 4>, g_, b_, f_, ##__VA_ARGS__); break;            \
      case 3: launch(s, KIND, &KNAME<P, 8>, g_, b_, f_, ##__VA_ARGS__); break;            \
      default: launch(s, KIND, &KNAME<P, 16>, g_, b_, f_, ##__VA_ARGS__); break;          \
    }                                                                                    \
  }

static std::vector<RowClass> member_class(const gcr_solver* s, int member) {
  const MemberGeom& G = s->geom_h[member];
  return {RowClass{G.log2m, G.row0, G.row0 + G.ny, s->flat_h[member]}};
}

// As ROWS_LAUNCH, for the kernels that evaluate the stencil with coefficients
// formed from the depth fields: a class whose members all lack orography takes
// the variant that reads Phi* only (FL = true), which holds fewer registers.
#define ROWS_LAUNCH_F(s, CLASSES, F, KIND, KNAME, P, ...)                                   \
  for (const RowClass& c_ : (CLASSES)) {                                                 \
    Fields f_ = (F);                                                                     \
    f_.row_base = c_.row_begin;                                                          \
    f_.row_end = c_.row_end;                                                             \
    const dim3 g_((c_.row_end - c_.row_begin + WPB - 1) / WPB), b_(WG);                  \
    switch (std::min(c_.log2m, 4) * 2 + (c_.flat ? 1 : 0)) {                             \
      case 2: launch(s, KIND, &KNAME<P, 2, false>, g_, b_, f_, ##__VA_ARGS__); break;     \
      case 3: launch(s, KIND, &KNAME<P, 2, true>, g_, b_, f_, ##__VA_ARGS__); break;      \
      case 4: launch(s, KIND, &KNAME<P, 4, false>, g_, b_, f_, ##__VA_ARGS__); break;     \
      case 5: launch(s, KIND, &KNAME<P, 4, true>, g_, b_, f_, ##__VA_ARGS__); break;      \
      case 6: launch(s, KIND, &KNAME<P, 8, false>, g_, b_, f_, ##__VA_ARGS__); break;     \
      case 7: launch(s, KIND, &KNAME<P, 8, true>, g_, b_, f_, ##__VA_ARGS__); break;      \
      case 9: launch(s, KIND, &KNAME<P, 16, true>, g_, b_, f_, ##__VA_ARGS__); break;     \
      default: launch(s, KIND, &KNAME<P, 16, false>, g_, b_, f_, ##__VA_ARGS__); break;   \
    }                                                                                    \
  }

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

static Fields make_fields(gcr_solver* s) {
  Fields F{};
  F.geom = s->geom;
  F.rowmap = s->rowmap;
  F.state = s->state;
  F.pend = s->pend;
  F.done_flag = s->done_flag;
  F.part = s->part;
  F.scale = s->scale;
  for (int k = 0; k < NCOEF; ++k) {
    F.cmx.h[k] = s->a16[k];
    F.cmx.f[k] = s->a32[k];
  }
  F.cmx.c = s->c32;
  F.fly64 = FlyPools<double>{s->phi64, s->hs64, s->fac64, s->c64, s->flat};
  F.fly32 = FlyPools<float>{s->phi32, s->hs32, s->fac32, s->c32, s->flat};
  F.x = s->x;
  F.rhs = s->rhs;
  F.rhs_tab = s->ptr_rhs;
  F.x_tab = s->ptr_x;
  F.morder = s->morder;
  F.q0 = 0;
  F.r64 = s->r64;
  F.r = s->r;
  F.e = s->e;
  F.le = s->le;
  for (int i = 0; i < 2; ++i) {
    F.q[i] = s->q[i];
    F.qs[i] = s->qs[i];
  }
  for (int i = 0; i <= s->prm.k; ++i) {
    F.p[i] = s->p[i];
    F.lp[i] = s->lp[i];
  }
  F.dx = s->dx;   // float32 solution increments (GCR_MIXED, GCR_SINGLE), else null
  F.hist = s->hist;
  F.hist_stride = s->hist_stride;
  F.row_base = 0;
  F.row_end = s->rows;
  F.ignore_done = 0;
  F.learned = s->prm.precond == GCR_PC_LEARNED ? 1 : 0;
  F.linf = (s->prm.flags & GCR_F_LINF_EXIT) ? 1 : 0;
  F.fallback_ratio = s->fallback_ratio;
  return F;
}

extern "C" int gcr_default_params(gcr_params* p) {
  if (!p) return GCR_EINVAL;
  std::memset(p, 0, sizeof *p);
  p->batch = 1;
  p->k = 3;
  p->precision = GCR_FP64;
  p->precond = GCR_PC_SEMI_IMPLICIT;
  p->richardson_iters = 2;
  p->polar_rows = -1;
  p->min_iters = -1;
  p->max_iters = 200;
  p->rtol = 1e-8;
  return GCR_OK;
}

static void free_all(gcr_solver* s) {
  stop_workers(s);
  if (s->net) (void)cnn_destroy(s->net);
  s->net = nullptr;
  for (auto& g : s->groups) {
    if (g.st) (void)hipStreamSynchronize(g.st);
    for (int i = 0; i < 2; ++i) {
      if (g.ring[i]) (void)hipHostFree(g.ring[i]);
      if (g.cycle_ev[i]) (void)hipEventDestroy(g.cycle_ev[i]);
    }
    if (g.done_ev) (void)hipEventDestroy(g.done_ev);
    if (g.st && g.st != s->stream) (void)hipStreamDestroy(g.st);
  }
  s->groups.clear();
  if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
  s->fork_ev = nullptr;
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  s->ev.clear();
  for (void* a : s->allocs)
    if (a) (void)hipFree(a);
  s->allocs.clear();
  if (s->ptr_stage) (void)hipHostFree(s->ptr_stage);
  if (s->state_h) (void)hipHostFree(s->state_h);
  if (s->asm_stage) (void)hipHostFree(s->asm_stage);
  for (int i = 0; i < 2; ++i) {
    if (s->state_ring[i]) (void)hipHostFree(s->state_ring[i]);
    if (s->cycle_ev[i]) (void)hipEventDestroy(s->cycle_ev[i]);
    s->state_ring[i] = nullptr;
    s->cycle_ev[i] = nullptr;
  }
  for (int i = 0; i < 2; ++i) {
    if (s->stage_ev[i]) (void)hipEventDestroy(s->stage_ev[i]);
    s->stage_ev[i] = nullptr;
  }
  s->ptr_stage = nullptr;
  s->state_h = nullptr;
  s->asm_stage = nullptr;
}

// Up to GROUPS_MAX groups of members, of about equal point counts, each with
// a stream (group 0: the solver's own; the others: streams of the library,
// default priority), two cycle events and two pinned rings.  Two groups
// overlap one group's kernel drains with the other's work; more groups add
// launches faster than the host enqueues them (three and four measured
// slower on 64 x 512x256), and beyond four streams groups would share the
// process's hardware queues.  Every group launches each kernel once per row
// class it holds, and the host enqueues a launch in a few microseconds
// whatever its size: the batch is split only while each group keeps about
// GROUP_PTS points per class and launch, below which the GPU would wait for
// the host.  The learned preconditioner keeps one group: its network runs
// over the whole batch.
constexpr int GROUPS_MAX = 2;
constexpr long long GROUP_PTS = 1LL << 21;

static hipError_t make_groups(gcr_solver* s) {
  const int B = s->prm.batch;
  long long total = 0;   // groups of about equal points
  for (int m = 0; m < B; ++m) total += (long long)s->geom_h[m].nx * s->geom_h[m].ny;
  const long long fit = total / (GROUP_PTS * (long long)s->classes.size());
  int G = (int)std::min<long long>(std::min(GROUPS_MAX, B), std::max<long long>(fit, 1));
  if (s->prm.precond == GCR_PC_LEARNED || (s->prm.flags & GCR_F_ONE_STREAM)) G = 1;
  if (G < 2) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming);
  int q = 0, row = 0;
  long long pts = 0;
  for (int g = 0; g < G && e == hipSuccess; ++g) {
    gcr_solver::Group grp;
    grp.q0 = q;
    const int r0 = row;
    const long long target = total * (g + 1) / G;
    // at least one member per group, and leave one for each later group
    auto take = [&] {
      const MemberGeom& M = s->geom_h[s->morder_h[q++]];
      row += M.ny;
      pts += (long long)M.nx * M.ny;
    };
    while (q < B - (G - 1 - g) && (q == grp.q0 || pts < target)) take();
    if (g == G - 1)
      while (q < B) take();
    grp.q1 = q;
    for (const RowClass& c : s->classes) {
      const int b = std::max(c.row_begin, r0), en = std::min(c.row_end, row);
      if (en > b) grp.classes.push_back(RowClass{c.log2m, b, en});
    }
    s->groups.push_back(grp);
    gcr_solver::Group& gr = s->groups.back();
    if (g == 0) gr.st = s->stream;
    else e = hipStreamCreateWithFlags(&gr.st, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&gr.cycle_ev[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipHostMalloc((void**)&gr.ring[i], B * sizeof(int), 0);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&gr.done_ev, hipEventDisableTiming);
  }
  if (e == hipSuccess) {
    const int dev = s->device;
    for (int w = 0; w + 1 < G; ++w)
      s->workers.emplace_back([s, w, dev] {
        (void)hipSetDevice(dev);
        worker_main(s, w);
      });
  }
  return e;
}

// Flat bits of the row classes (the solver's and each group's): a class is
// flat when none of its members has orography.
static void refresh_flat(gcr_solver* s) {
  auto mark = [s](std::vector<RowClass>& cls) {
    for (RowClass& c : cls) {
      int all = 1;
      for (int m : s->morder_h) {
        const MemberGeom& G = s->geom_h[m];
        if (G.row0 >= c.row_begin && G.row0 < c.row_end) all &= s->flat_h[m];
      }
      c.flat = all;
    }
  };
  mark(s->classes);
  for (gcr_solver::Group& g : s->groups) mark(g.classes);
}

extern "C" int gcr_create(const gcr_params* prm, gcr_solver** out) {
  if (out) *out = nullptr;
  if (!prm || !out) return fail(nullptr, GCR_EINVAL, "gcr_create: NULL argument");
  const gcr_params& P = *prm;
  if (P.batch < 1 || P.batch > 4096) return fail(nullptr, GCR_EINVAL, "batch must be in [1, 4096], got %d", P.batch);
  if (!P.nx || !P.ny) return fail(nullptr, GCR_EINVAL, "nx/ny arrays must not be NULL");
  if (P.k < 1 || P.k > KMAX) return fail(nullptr, GCR_EINVAL, "k must be in [1, %d], got %d", KMAX, P.k);
  if (P.precision < GCR_FP64 || P.precision > GCR_SINGLE_POLAR64)
    return fail(nullptr, GCR_EINVAL, "unknown precision form %d", P.precision);
  if (P.precond < GCR_PC_NONE || P.precond > GCR_PC_LEARNED)
    return fail(nullptr, GCR_EINVAL, "unsupported preconditioner %d", P.precond);
  if (P.richardson_iters < 1 || P.richardson_iters > 16)
    return fail(nullptr, GCR_EINVAL, "richardson_iters must be in [1, 16], got %d", P.richardson_iters);
  if (P.max_iters < 1 || P.max_iters > 100000) return fail(nullptr, GCR_EINVAL, "max_iters must be in [1, 100000]");
  if (P.min_iters < -1 || P.min_iters > P.max_iters) return fail(nullptr, GCR_EINVAL, "min_iters out of range");
  if (!(P.rtol >= 0.0) || !std::isfinite(P.rtol)) return fail(nullptr, GCR_EINVAL, "rtol must be finite and >= 0");
  if (P.polar_rows < -1) return fail(nullptr, GCR_EINVAL, "polar_rows must be >= -1");
  if (P.flags & ~(GCR_F_RECORD_HISTORY | GCR_F_ONE_STREAM | GCR_F_LINF_EXIT))
    return fail(nullptr, GCR_EINVAL, "unknown flags 0x%x", P.flags);
  for (int m = 0; m < P.batch; ++m) {
    const int nx = P.nx[m], ny = P.ny[m];
    if (!is_pow2(nx) || nx < 8 || nx > NXMAX)
      return fail(nullptr, GCR_EINVAL, "member %d: nx must be a power of two in [8, %d], got %d", m, NXMAX, nx);
    if (ny < 2 || ny > 4096) return fail(nullptr, GCR_EINVAL, "member %d: ny must be in [2, 4096], got %d", m, ny);
    if (P.precond == GCR_PC_LEARNED && (nx != P.nx[0] || ny != P.ny[0] || nx < 64))
      return fail(nullptr, GCR_EINVAL, "the learned preconditioner needs members of one size with nx >= 64");
  }

  gcr_solver* s = new (std::nothrow) gcr_solver();
  if (!s) return fail(nullptr, GCR_ENOMEM, "host allocation failed");
  s->prm = P;
  if (s->prm.min_iters < 0) s->prm.min_iters = std::min(P.k + 1, P.max_iters);
  s->stream = (hipStream_t)P.stream;
  s->prm.nx = nullptr;
  s->prm.ny = nullptr;
  s->nx.assign(P.nx, P.nx + P.batch);
  s->ny.assign(P.ny, P.ny + P.batch);
  s->have_op.assign(P.batch, 0);
  s->have_split.assign(P.batch, 0);
  s->flat_h.assign(P.batch, 0);
  s->scale_h.assign(P.batch, 1.0);
  for (int m = 0; m < P.batch; ++m) {
    MemberGeom G{};
    G.nx = s->nx[m];
    G.ny = s->ny[m];
    G.log2nx = ilog2(G.nx);
    G.log2m = std::max(1, G.log2nx - 6);  // M = max(2, NX/64) points per lane
    int polar = P.polar_rows;
    if (polar < 0) polar = std::max(1, ilog2(std::max(G.ny / 32, 1)));
    G.polar = std::min(polar, G.ny);
    G.off = s->npts;
    s->geom_h.push_back(G);
    s->npts += ((long long)G.nx * G.ny + 63) / 64 * 64;  // member offsets stay 64-element aligned
    s->nxmax = std::max(s->nxmax, G.nx);
  }
  std::vector<int> rowmap_h;
  for (int lm = 1; lm <= 4; ++lm) {
    RowClass c{lm, s->rows, s->rows};
    for (int m = 0; m < P.batch; ++m) {
      MemberGeom& G = s->geom_h[m];
      if (G.log2m != lm) continue;
      G.row0 = s->rows;
      for (int j = 0; j < G.ny; ++j) rowmap_h.push_back(m);
      s->rows += G.ny;
    }
    c.row_end = s->rows;
    if (c.row_end > c.row_begin) s->classes.push_back(c);
  }
  for (int r = 0; r < s->rows; r += s->geom_h[rowmap_h[r]].ny) s->morder_h.push_back(rowmap_h[r]);

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete s;
    return fail(nullptr, GCR_EHIP, "no HIP device available");
  }
  (void)hipGetDevice(&s->device);

  hipError_t herr = hipSuccess;
  auto track = [&](void* a) { s->allocs.push_back(a); return a; };
  const long long N = s->npts;
  const int R = s->rows;
  const bool mixed = P.precision != GCR_FP64;
  const size_t vsz = mixed ? sizeof(float) : sizeof(double);
  const size_t qsz = vsz;  // float16 intermediates (option 3) or Krylov-type ones (options 0-2)
  s->geom = (MemberGeom*)track(dalloc<MemberGeom>(P.batch, herr));
  s->rowmap = (int*)track(dalloc<int>(R, herr));
  s->morder = (int*)track(dalloc<int>(P.batch, herr));
  s->state = (MemberState*)track(dalloc<MemberState>(P.batch, herr));
  s->pend = (Pending*)track(dalloc<Pending>(P.batch, herr));
  s->done_flag = (int*)track(dalloc<int>(P.batch, herr));
  s->part = (double*)track(dalloc<double>((size_t)R * NDOT, herr));
  s->scale = (double*)track(dalloc<double>(P.batch, herr));
  for (int k = 0; k < NCOEF; ++k) {
    s->a32[k] = (float*)track(dalloc<float>(N, herr));
    s->a16[k] = (__half*)track(dalloc<__half>(N, herr));
  }
  s->c64 = (double*)track(dalloc<double>(R, herr));
  s->c32 = (float*)track(dalloc<float>(R, herr));
  s->phi64 = (double*)track(dalloc<double>(N, herr));
  s->hs64 = (double*)track(dalloc<double>(N, herr));
  s->phi32 = (float*)track(dalloc<float>(N, herr));
  s->hs32 = (float*)track(dalloc<float>(N, herr));
  s->flat = (int*)track(dalloc<int>(P.batch, herr));
  s->fac64 = (double*)track(dalloc<double>((size_t)R * NFAC, herr));
  s->fac32 = (float*)track(dalloc<float>((size_t)R * NFAC, herr));
  s->x = (double*)track(dalloc<double>(N, herr));
  s->rhs = (double*)track(dalloc<double>(N, herr));
  s->r64 = (double*)track(dalloc<double>(N, herr));
  s->r = track(dalloc<char>(N * vsz, herr));
  s->e = track(dalloc<char>(N * vsz, herr));
  s->le = track(dalloc<char>(N * vsz, herr));
  for (int i = 0; i < 2; ++i) {
    s->q[i] = track(dalloc<char>(N * qsz, herr));
    s->qs[i] = (float*)track(dalloc<float>(R, herr));
  }
  for (int i = 0; i <= P.k; ++i) {
    s->p[i] = track(dalloc<char>(N * vsz, herr));
    s->lp[i] = track(dalloc<char>(N * vsz, herr));
  }
  if (P.precision == GCR_MIXED || P.precision == GCR_SINGLE || P.precision == GCR_SINGLE_POLAR64)
    s->dx = (float*)track(dalloc<float>(N, herr));
  if (mixed) {
    s->aux_r = (double*)track(dalloc<double>(N, herr));
    s->aux_e = (double*)track(dalloc<double>(N, herr));
    s->aux_q[0] = (double*)track(dalloc<double>(N, herr));
    s->aux_q[1] = (double*)track(dalloc<double>(N, herr));
  }
  s->hist_stride = P.max_iters + 1;
  if (P.flags & GCR_F_RECORD_HISTORY)
    s->hist = (double*)track(dalloc<double>((size_t)P.batch * s->hist_stride, herr));
  s->ptr_rhs = (const double**)track(dalloc<const double*>(P.batch, herr));
  s->ptr_x = (double**)track(dalloc<double*>(P.batch, herr));
  if (herr == hipSuccess) herr = hipHostMalloc((void**)&s->ptr_stage, 2 * P.batch * sizeof(void*), 0);
  s->asm_tab = (AsmMember*)track(dalloc<AsmMember>(P.batch, herr));
  if (herr == hipSuccess) herr = hipHostMalloc((void**)&s->state_h, P.batch * sizeof(MemberState), 0);
  if (herr == hipSuccess) herr = hipHostMalloc((void**)&s->asm_stage, P.batch * sizeof(AsmMember), 0);
  for (int i = 0; i < 2 && herr == hipSuccess; ++i) {
    herr = hipHostMalloc((void**)&s->state_ring[i], P.batch * sizeof(int), 0);
    if (herr == hipSuccess) herr = hipEventCreateWithFlags(&s->cycle_ev[i], hipEventDisableTiming);
    if (herr == hipSuccess) herr = hipEventCreateWithFlags(&s->stage_ev[i], hipEventDisableTiming);
  }
  if (herr != hipSuccess) {
    const bool oom = herr == hipErrorOutOfMemory;
    free_all(s);
    delete s;
    return fail(nullptr, oom ? GCR_ENOMEM : GCR_EHIP, "device allocation failed: %s", hipGetErrorString(herr));
  }
  herr = hipMemcpyAsync(s->geom, s->geom_h.data(), P.batch * sizeof(MemberGeom), hipMemcpyHostToDevice, s->stream);
  if (herr == hipSuccess)
    herr = hipMemcpyAsync(s->rowmap, rowmap_h.data(), R * sizeof(int), hipMemcpyHostToDevice, s->stream);
  if (herr == hipSuccess)
    herr = hipMemcpyAsync(s->morder, s->morder_h.data(), P.batch * sizeof(int), hipMemcpyHostToDevice, s->stream);
  if (herr == hipSuccess) herr = make_groups(s);
  if (herr == hipSuccess) herr = hipMemsetAsync(s->state, 0, P.batch * sizeof(MemberState), s->stream);
  if (herr == hipSuccess) herr = hipMemsetAsync(s->pend, 0, P.batch * sizeof(Pending), s->stream);
  if (herr == hipSuccess) herr = hipMemsetAsync(s->done_flag, 0, P.batch * sizeof(int), s->stream);
  if (herr == hipSuccess) herr = hipMemsetAsync(s->part, 0, (size_t)R * NDOT * sizeof(double), s->stream);
  if (herr == hipSuccess) herr = hipMemsetAsync(s->flat, 0, P.batch * sizeof(int), s->stream);
  for (int i = 0; i < 2 && herr == hipSuccess; ++i) herr = hipEventRecord(s->stage_ev[i], s->stream);
  if (herr == hipSuccess) herr = hipStreamSynchronize(s->stream);
  if (herr != hipSuccess) {
    free_all(s);
    delete s;
    return fail(nullptr, GCR_EHIP, "initialisation failed: %s", hipGetErrorString(herr));
  }
  *out = s;
  return GCR_OK;
}

extern "C" int gcr_destroy(gcr_solver* s) {
  if (!s) return GCR_OK;
  (void)hipStreamSynchronize(s->stream);
  free_all(s);
  delete s;
  return GCR_OK;
}

extern "C" int gcr_set_operators(gcr_solver* s, int32_t count, const int32_t* members, const gcr_operator* ops) {
  if (!s) return GCR_EINVAL;
  if (count < 1 || count > s->prm.batch || !members || !ops)
    return fail(s, GCR_EINVAL, "gcr_set_operators: need 1..batch members and non-NULL tables");
  std::vector<int> seen(s->prm.batch, 0);
  int maxrows = 0;
  for (int t = 0; t < count; ++t) {
    const int member = members[t];
    const gcr_operator* op = &ops[t];
    if (member < 0 || member >= s->prm.batch) return fail(s, GCR_EINVAL, "member %d out of range", member);
    if (seen[member]++) return fail(s, GCR_EINVAL, "member %d listed twice", member);
    if (!op->depth) return fail(s, GCR_EINVAL, "member %d: depth must not be NULL", member);
    if (!(op->dt > 0.0) || !(op->g > 0.0) || !(op->radius > 0.0) || !std::isfinite(op->omega) ||
        !(op->absorber >= 0.0) || !std::isfinite(op->dt * op->g * op->radius * op->absorber))
      return fail(s, GCR_EINVAL, "member %d: dt, g, radius must be > 0, absorber >= 0, all finite", member);
    const MemberGeom& G = s->geom_h[member];
    const long long n = (long long)G.nx * G.ny;
    maxrows = std::max(maxrows, G.ny);
    if (!op->mem_is_device) {
      for (long long k = 0; k < n; ++k)
        if (!(op->depth[k] > 0.0) || !std::isfinite(op->depth[k]))
          return fail(s, GCR_EINVAL, "member %d: depth must be finite and > 0 (point %lld)", member, k);
    }
  }
  // the staging table (pinned) may still feed the previous upload: wait for
  // that copy only, not for the whole stream
  HIPCHK(s, hipEventSynchronize(s->stage_ev[1]));
  for (int t = 0; t < count; ++t) {
    const int member = members[t];
    const gcr_operator* op = &ops[t];
    const MemberGeom& G = s->geom_h[member];
    const long long n = (long long)G.nx * G.ny;
    AsmMember& a = s->asm_stage[t];
    a.member = member;
    a.dt = op->dt;
    a.g = op->g;
    a.omega = op->omega;
    a.radius = op->radius;
    a.absorber = op->absorber;
    a.b_terms = op->b_terms ? 1 : 0;
    if (op->mem_is_device) {
      a.depth = op->depth;
      a.oro = op->orography;
    } else {  // host inputs are staged in the member's x / r64 pool regions
      HIPCHK(s, hipMemcpyAsync(s->x + G.off, op->depth, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
      a.depth = s->x + G.off;
      a.oro = nullptr;
      if (op->orography) {
        HIPCHK(s, hipMemcpyAsync(s->r64 + G.off, op->orography, n * sizeof(double), hipMemcpyHostToDevice,
                                 s->stream));
        a.oro = s->r64 + G.off;
      }
    }
    s->scale_h[member] = op->dt / (2.0 * op->radius * op->radius);
  }
  HIPCHK(s, hipMemcpyAsync(s->asm_tab, s->asm_stage, count * sizeof(AsmMember), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipEventRecord(s->stage_ev[1], s->stream));
  AssembleArgs A{};
  A.tab = s->asm_tab;
  A.geom = s->geom;
  for (int k = 0; k < NCOEF; ++k) {
    A.a32[k] = s->a32[k];
    A.a16[k] = s->a16[k];
  }
  A.c64 = s->c64;
  A.c32 = s->c32;
  A.scale = s->scale;
  A.phi64 = s->phi64;
  A.hs64 = s->hs64;
  A.phi32 = s->phi32;
  A.hs32 = s->hs32;
  A.fac64 = s->fac64;
  A.fac32 = s->fac32;
  A.flat = s->flat;
  bool any_oro = false;
  for (int t = 0; t < count; ++t) any_oro = any_oro || ops[t].orography;
  // rows per workgroup: as many as the staged rows (two halo rows, times two
  // fields with orography) fit in 64 KiB of LDS
  const size_t row_bytes = (any_oro ? 2 : 1) * (size_t)asm_row_lds(s->nxmax) * sizeof(double);
  A.rows = ASM_ROWS;
  while (A.rows > 1 && (A.rows + 2) * row_bytes > 65536) --A.rows;
  const size_t lds = (A.rows + 2) * row_bytes;
  KLAUNCH(s, KT_ASSEMBLE, k_assemble, dim3((maxrows + A.rows - 1) / A.rows, count), dim3(ASM_WG), lds, s->stream,
          A);
  HIPCHK(s, hipGetLastError());
  bool host_inputs = false;
  for (int t = 0; t < count; ++t) host_inputs = host_inputs || !ops[t].mem_is_device;
  if (host_inputs) HIPCHK(s, hipStreamSynchronize(s->stream));  // host arrays are read asynchronously
  for (int t = 0; t < count; ++t) {
    s->have_op[members[t]] = 1;
    s->flat_h[members[t]] = s->asm_stage[t].oro ? 0 : 1;   // as k_assemble sets `flat`
  }
  refresh_flat(s);
  return GCR_OK;
}

extern "C" int gcr_set_operator(gcr_solver* s, int32_t member, const gcr_operator* op) {
  if (!s) return GCR_EINVAL;
  if (!op) return fail(s, GCR_EINVAL, "gcr_set_operator: NULL operator");
  return gcr_set_operators(s, 1, &member, op);
}

// ---------------------------------------------------------------------------
// kernel sequences
// ---------------------------------------------------------------------------
// Learned correction of the preconditioner output F.e (members
// [member0, member0 + count)): residual scale, network input, five
// convolutions over the whole batch of images, update of e.  `use_part`: the
// per-row <r,r> partials of F.r are current (inside a solve).
template <typename P>
static void learned_correction(gcr_solver* s, const std::vector<RowClass>& cls, const Fields& F, int use_part,
                               int member0, int count) {
  LearnArgs A{};
  A.r = F.r;
  A.e = F.e;
  A.feat = s->net->act[0];
  A.feat_stride = s->net->in_stride;
  A.y = s->net->y;
  A.use_part = use_part;
  A.active = s->learn_active;
  KLAUNCH(s, KT_LEARNED, k_learn_sigma<P>, dim3(s->prm.batch), dim3(64), 0, cur_stream(s), F, A, member0, count);
  ROWS_LAUNCH(s, cls, F, KT_LEARNED, k_learn_pack, P, A);
  s->tm_begin(KT_LEARNED);
  (void)cnn_forward_packed(s->net, s->prm.batch, s->net->y, cur_stream(s), s->learn_active);
  s->tm_end();
  ROWS_LAUNCH(s, cls, F, KT_LEARNED, k_learn_apply, P, A);
}

// e = P^{-1}(r) on the rows of `cls`, optionally fused with the step-2
// update along ring slot `slot_nu`.  With the learned preconditioner and
// `learned` >= 0 the network correction follows (learned = 1: partials of
// <r,r> current); members [member0, member0 + count) are corrected.
template <typename P>
static void launch_precond(gcr_solver* s, const std::vector<RowClass>& cls, const Fields& F, int do_update,
                           int slot_nu, int learned = 1, int member0 = 0, int count = -1) {
  const int ri = s->prm.richardson_iters;
  switch (s->prm.precond) {
    case GCR_PC_NONE:
    case GCR_PC_DIAG:
      ROWS_LAUNCH(s, cls, F, KT_SWEEP1, k_update_simple, P, do_update, slot_nu,
                  s->prm.precond == GCR_PC_DIAG ? 1 : 0, -1);
      break;
    case GCR_PC_RICHARDSON: {
      // q_1 = r / diag(L); q_{mu+1} = q_mu - (L q_mu - r) / diag(L)
      ROWS_LAUNCH(s, cls, F, KT_SWEEP1, k_update_simple, P, do_update, slot_nu, 1, ri == 1 ? -1 : 0);
      int cur = 0;
      for (int mu = 1; mu < ri; ++mu) {
        const int nxt = mu + 1 == ri ? -1 : cur ^ 1;
        ROWS_LAUNCH_F(s, cls, F, KT_SWEEP2, k_jacobi, P, cur, nxt);
        cur ^= 1;
      }
      break;
    }
    default: {
      ROWS_LAUNCH(s, cls, F, KT_SWEEP1, k_update_sweep1, P, do_update, slot_nu, ri == 1 ? -1 : 0);
      int cur = 0;
      for (int mu = 1; mu < ri; ++mu) {
        const int nxt = mu + 1 == ri ? -1 : cur ^ 1;
        ROWS_LAUNCH_F(s, cls, F, KT_SWEEP2, k_sweep2, P, cur, nxt);
        cur ^= 1;
      }
      if (s->prm.precond == GCR_PC_LEARNED && learned >= 0 && s->net)
        learned_correction<P>(s, cls, F, learned, member0, count < 0 ? s->prm.batch : count);
    }
  }
}

// The solve of one group of members is enqueued one GCR cycle at a time on
// the group's stream.  After the k iterations of a cycle (and, in the
// residual-replacement forms, the float64 restart) the members' scalars are
// copied to pinned host memory and an event is recorded.  Before waiting for
// that event the host already enqueues the first iteration of the next cycle,
// so the GPU keeps working while the host decides; members that have finished
// make every later kernel return at once, so speculative work on converged
// members costs only empty launches.
template <typename P>
static int run_group(gcr_solver* s, const gcr_solver::Group& g) {
  using A = typename P::A;
  struct StreamScope {   // this thread's launches go to the group's stream
    explicit StreamScope(hipStream_t st) { t_stream = st; }
    ~StreamScope() { t_stream = nullptr; }
  } scope(g.st);
  const int k = s->prm.k, B = s->prm.batch, maxit = s->prm.max_iters;
  Fields F = make_fields(s);
  F.q0 = g.q0;
  const bool replace = s->prm.precision == GCR_MIXED_FP64DOT || s->prm.precision == GCR_MIXED_HALF_PC;
  const dim3 ctl(g.q1 - g.q0), wave(64);
  const std::vector<RowClass>& cls = g.classes;

  // step 1: r_0 = L(x_0) - R (float64), p_0 = P^{-1}(r_0), L(p_0)
  ROWS_LAUNCH_F(s, cls, F, KT_RESIDUAL, k_residual, P, 1, -1, 0, RES_X_IN | RES_RHS_TAB);
  KLAUNCH(s, KT_CONTROL, k_ctrl_init<double>, ctl, wave, 0, g.st, F);
  {
    Fields F0 = F;
    F0.e = s->p[0];   // p_0 = P^{-1}(r_0) written in place
    launch_precond<P>(s, cls, F0, 0, 0);
  }
  Slots sl0{};
  ROWS_LAUNCH_F(s, cls, F, KT_APPLY_L, k_apply_L, P, (const void*)s->p[0], s->lp[0], 1, 0, sl0);
  KLAUNCH(s, KT_CONTROL, k_ctrl_beta<A>, ctl, wave, 0, g.st, F, 0);
  HIPCHK(s, hipGetLastError());

  // iteration `it` (1-based) at window position nu of cycle `cyc`, whose p_0
  // sits in ring slot `base`
  auto iteration = [&](int it, int nu, int base, int cyc) {
    Slots sl{};
    for (int l = 0; l <= k; ++l) sl.s[l] = (base + l) % (k + 1);
    (void)it;
    // step 2 (+ first row solve of step 3)
    launch_precond<P>(s, cls, F, 1, sl.s[nu]);
    // step 3: L(e) with <L e, L p_l>, l = 0..nu
    ROWS_LAUNCH_F(s, cls, F, KT_APPLY_L, k_apply_L, P, (const void*)s->e, s->le, 0, nu + 1, sl);
    KLAUNCH(s, KT_CONTROL, k_ctrl_alpha<A>, ctl, wave, 0, g.st, F, nu + 1, sl, nu == k - 1 ? 1 : 0,
            s->prm.min_iters, maxit, s->prm.rtol, cyc);
    // step 4
    if (nu == k - 1) {   // the cycle's last iteration also applies its solution updates
      ROWS_LAUNCH(s, cls, F, KT_ORTH, k_orth_last, P, nu + 1, sl, sl.s[nu + 1]);
    } else {
      ROWS_LAUNCH(s, cls, F, KT_ORTH, k_orth, P, nu + 1, sl, sl.s[nu + 1]);
    }
    KLAUNCH(s, KT_CONTROL, k_ctrl_beta<A>, ctl, wave, 0, g.st, F, sl.s[nu + 1]);
  };
  // end of cycle `cyc`: its solution updates; (p_0, L p_0) := (p_k, L p_k);
  // residual replacement; flags
  auto cycle_end = [&](int base_next, int ring, int cyc) -> int {
    ROWS_LAUNCH(s, cls, F, KT_SOLUTION, k_apply_pending, P, cyc);
    if (replace) {
      ROWS_LAUNCH_F(s, cls, F, KT_RESIDUAL, k_residual, P, 1, base_next, 1, RES_RHS_TAB);
      KLAUNCH(s, KT_CONTROL, k_ctrl_restart<double>, ctl, wave, 0, g.st, F, base_next);
    }
    // the done flags (a few bytes per member: a small copy); only the group's
    // own members are read from them
    HIPCHK(s, hipMemcpyAsync(g.ring[ring], s->done_flag, B * sizeof(int), hipMemcpyDeviceToHost, g.st));
    HIPCHK(s, hipEventRecord(g.cycle_ev[ring], g.st));
    return GCR_OK;
  };

  int it = 0, base = 0, cycle = 0, rc;
  // cycle 0, complete
  for (int nu = 0; nu < k && it < maxit; ++nu) iteration(++it, nu, base, 0);
  base = (base + k) % (k + 1);
  if ((rc = cycle_end(base, 0, 0)) != GCR_OK) return rc;
  HIPCHK(s, hipGetLastError());
  for (;;) {
    // speculative first iteration of the next cycle
    const bool more = it < maxit;
    if (more) iteration(++it, 0, base, cycle + 1);
    HIPCHK(s, hipEventSynchronize(g.cycle_ev[cycle & 1]));
    bool done = true;
    for (int q = g.q0; q < g.q1; ++q) done = done && g.ring[cycle & 1][s->morder_h[q]] != 0;
    if (done || !more) break;
    for (int nu = 1; nu < k && it < maxit; ++nu) iteration(++it, nu, base, cycle + 1);
    base = (base + k) % (k + 1);
    ++cycle;
    if ((rc = cycle_end(base, cycle & 1, cycle)) != GCR_OK) return rc;
    HIPCHK(s, hipGetLastError());
  }
  // No update is pending here: the loop leaves right after a cycle end, or
  // after a speculative iteration that every member skipped (all were done
  // at that cycle end).  The true residual of the group's members in float64
  // (float32 increments: after they are added, over the whole batch):
  if (!s->dx) {
    ROWS_LAUNCH_F(s, cls, F, KT_RESIDUAL, k_residual, P, 0, -1, 0, RES_X_OUT | RES_RHS_TAB);
    KLAUNCH(s, KT_CONTROL, k_ctrl_true, ctl, wave, 0, g.st, F);
    HIPCHK(s, hipGetLastError());
  }
  return GCR_OK;
}

// Worker thread w enqueues group w + 1 of each solve.
static void worker_main(gcr_solver* s, int w) {
  long seen = 0;
  for (;;) {
    std::function<int(int)> job;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_job.wait(lk, [&] { return s->quit || s->job_gen != seen; });
      if (s->quit) return;
      seen = s->job_gen;
      job = s->job;
    }
    const int rc = job(w + 1);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->job_rc[w + 1] = rc;
      if (--s->job_pending == 0) s->cv_done.notify_all();
    }
  }
}

static void stop_workers(gcr_solver* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->quit = true;
  }
  s->cv_job.notify_all();
  for (std::thread& t : s->workers)
    if (t.joinable()) t.join();
  s->workers.clear();
}

// The whole solve: the groups (forked from the solver's stream, each enqueued
// by its own host thread), joined back on the solver's stream.  Per-kernel
// timing runs one group on the solver's stream (the timing events need one
// stream and one thread).
template <typename P>
static int run_solve(gcr_solver* s) {
  const int B = s->prm.batch;
  const bool split = !s->groups.empty() && !s->timing;
  if (!split) {
    gcr_solver::Group whole;
    whole.q0 = 0;
    whole.q1 = B;
    whole.classes = s->classes;
    whole.st = s->stream;
    for (int i = 0; i < 2; ++i) {
      whole.cycle_ev[i] = s->cycle_ev[i];
      whole.ring[i] = s->state_ring[i];
    }
    const int rc = run_group<P>(s, whole);
    if (rc != GCR_OK) return rc;
  } else {
    HIPCHK(s, hipEventRecord(s->fork_ev, s->stream));
    for (gcr_solver::Group& g : s->groups)
      if (g.st != s->stream) HIPCHK(s, hipStreamWaitEvent(g.st, s->fork_ev, 0));
    const int G = (int)s->groups.size();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->job = [s](int gi) { return run_group<P>(s, s->groups[gi]); };
      s->job_rc.assign(G, GCR_OK);
      s->job_pending = G - 1;
      ++s->job_gen;
    }
    s->cv_job.notify_all();
    const int rc0 = run_group<P>(s, s->groups[0]);
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait(lk, [&] { return s->job_pending == 0; });
    }
    // Every group stream is joined back to the solver's stream, also when a
    // group failed: work already enqueued on it may still read the caller's
    // buffers after this call returns.
    int rc = rc0;
    for (int gi = 1; gi < G && rc == GCR_OK; ++gi) rc = s->job_rc[gi];
    for (gcr_solver::Group& g : s->groups) {
      if (g.st == s->stream) continue;
      const hipError_t e1 = hipEventRecord(g.done_ev, g.st);
      const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s->stream, g.done_ev, 0) : e1;
      if (e2 != hipSuccess && rc == GCR_OK)
        rc = fail(s, GCR_EHIP, "joining member group streams: %s", hipGetErrorString(e2));
    }
    if (rc != GCR_OK) return rc;
  }
  if (s->dx) {
    // float32 increments added to the solution, then the true residual
    const Fields F = make_fields(s);
    const dim3 ctl(B), wave(64);
    const dim3 g((unsigned)std::min<long long>((s->npts + 255) / 256, 65535));
    KLAUNCH(s, KT_COPY, k_apply_increments, g, dim3(256), 0, s->stream, F, s->npts);
    ROWS_LAUNCH_F(s, s->classes, F, KT_RESIDUAL, k_residual, P, 0, -1, 0, RES_X_OUT | RES_RHS_TAB);
    KLAUNCH(s, KT_CONTROL, k_ctrl_true, ctl, wave, 0, s->stream, F);
    HIPCHK(s, hipGetLastError());
  }
  return GCR_OK;
}

extern "C" int gcr_solve(gcr_solver* s, const double* const* rhs, double* const* x, gcr_report* reports) {
  if (!s) return GCR_EINVAL;
  if (!rhs || !x) return fail(s, GCR_EINVAL, "gcr_solve: NULL rhs or x table");
  const int B = s->prm.batch;
  for (int m = 0; m < B; ++m) {
    if (!rhs[m] || !x[m]) return fail(s, GCR_EINVAL, "member %d: NULL field pointer", m);
    if (!s->have_op[m]) return fail(s, GCR_ESTATE, "member %d has no operator (call gcr_set_operator)", m);
  }
  if (s->prm.precond == GCR_PC_LEARNED && !s->net)
    return fail(s, GCR_ESTATE, "learned preconditioner without parameters (call gcr_set_learned)");
  HIPCHK(s, hipEventSynchronize(s->stage_ev[0]));  // staging buffer reuse
  for (int m = 0; m < B; ++m) {
    s->ptr_stage[m] = rhs[m];
    s->ptr_stage[B + m] = x[m];
  }
  HIPCHK(s, hipMemcpyAsync(s->ptr_rhs, s->ptr_stage, B * sizeof(void*), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->ptr_x, s->ptr_stage + B, B * sizeof(void*), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipEventRecord(s->stage_ev[0], s->stream));
  // the caller's rhs and x are read in place by the residual kernels (x is
  // copied into the pool by the first one and back by the last one)
  if (s->dx) HIPCHK(s, hipMemsetAsync(s->dx, 0, s->npts * sizeof(float), s->stream));
  HIPCHK(s, hipGetLastError());
  int rc;
  switch (s->prm.precision) {
    case GCR_FP64: rc = run_solve<PrecF64>(s); break;
    case GCR_MIXED: rc = run_solve<PrecMixed>(s); break;
    case GCR_MIXED_FP64DOT: rc = run_solve<PrecMixedD>(s); break;
    case GCR_SINGLE: rc = run_solve<PrecSingle>(s); break;
    case GCR_SINGLE_POLAR64: rc = run_solve<PrecSingleD>(s); break;
    default: rc = run_solve<PrecMixedP>(s); break;
  }
  if (rc != GCR_OK) return rc;
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, hipMemcpyAsync(s->state_h, s->state, B * sizeof(MemberState), hipMemcpyDeviceToHost, s->stream));
  std::vector<double> hist_h;
  if (s->hist && reports) {
    hist_h.resize((size_t)B * s->hist_stride);
    HIPCHK(s, hipMemcpyAsync(hist_h.data(), s->hist, hist_h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             s->stream));
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->tm_collect();
  // worst soft status: OK < FALLBACK_USED < NOT_CONVERGED < STAGNATED
  auto severity = [](int st) { return st == GCR_FALLBACK_USED ? 1 : st == GCR_OK ? 0 : st + 1; };
  int worst = GCR_OK;
  for (int m = 0; m < B; ++m) {
    const MemberState& S = s->state_h[m];
    const int st = S.status;
    if (severity(st) > severity(worst)) worst = st;
    if (!reports) continue;
    gcr_report& rp = reports[m];
    rp.status = st;
    rp.iterations = S.it;
    rp.restarts = S.restarts;
    rp.fallback_used = S.fallback;
    const double sc = s->prm.precision == GCR_FP64 ? 1.0 : s->scale_h[m];
    rp.r0_norm = S.rho0 / sc;
    rp.rel_res_recursive = S.rho0 > 0 ? S.rn / S.rho0 : 0.0;
    rp.rel_res_true = S.rho0 > 0 ? S.rtrue / S.rho0 : 0.0;
    rp.history_len = 0;
    if (rp.history && rp.history_cap > 0 && s->hist) {
      const int n = std::min(rp.history_cap, std::min(S.it + 1, s->hist_stride));
      std::memcpy(rp.history, hist_h.data() + (size_t)m * s->hist_stride, n * sizeof(double));
      rp.history_len = n;
    }
  }
  return worst;
}

// ---------------------------------------------------------------------------
// stand-alone operator and preconditioner (float64)
// ---------------------------------------------------------------------------
static int check_member(gcr_solver* s, int32_t member, const void* a, const void* b) {
  if (!s) return GCR_EINVAL;
  if (member < 0 || member >= s->prm.batch) return fail(s, GCR_EINVAL, "member %d out of range", member);
  if (!a || !b) return fail(s, GCR_EINVAL, "NULL field pointer");
  if (a == b) return fail(s, GCR_EINVAL, "input and output must not alias");
  if (!s->have_op[member]) return fail(s, GCR_ESTATE, "member %d has no operator", member);
  return GCR_OK;
}

static SplitArgs split_args(const gcr_solver* s) {
  SplitArgs S{};
  S.hat = s->split;
  for (int k = 0; k < NSD; ++k) S.d[k] = s->split + (size_t)(k + 1) * s->npts;
  S.tilde = s->split + (size_t)(NSD + 1) * s->npts;
  return S;
}

extern "C" int gcr_set_split_base(gcr_solver* s, int32_t member, const double* phi0) {
  if (!s) return GCR_EINVAL;
  if (member < 0 || member >= s->prm.batch) return fail(s, GCR_EINVAL, "member %d out of range", member);
  if (!phi0) return fail(s, GCR_EINVAL, "NULL field pointer");
  if (!s->have_op[member]) return fail(s, GCR_ESTATE, "member %d has no operator", member);
  if (!s->split) {
    hipError_t herr = hipSuccess;
    float* buf = dalloc<float>((size_t)(NSD + 2) * s->npts, herr);
    if (herr != hipSuccess) return fail(s, GCR_ENOMEM, "split residual buffers: %s", hipGetErrorString(herr));
    s->allocs.push_back(buf);
    s->split = buf;
  }
  const MemberGeom& G = s->geom_h[member];
  const long long n = (long long)G.nx * G.ny;
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024));
  KLAUNCH(s, KT_COPY, k_to_pool, cg, dim3(256), 0, s->stream, phi0, s->x, G);
  Fields F = make_fields(s);
  F.row_base = G.row0;
  F.row_end = G.row0 + G.ny;
  F.ignore_done = 1;
  ROWS_LAUNCH(s, member_class(s, member), F, KT_RESIDUAL, k_split_base, PrecF64, split_args(s));
  HIPCHK(s, hipGetLastError());
  s->have_split[member] = 1;
  return GCR_OK;
}

extern "C" int gcr_residual_split(gcr_solver* s, int32_t member, const float* phi_tilde, const double* rhs,
                                  double* r) {
  int rc = check_member(s, member, phi_tilde, r);
  if (rc != GCR_OK) return rc;
  if (!rhs) return fail(s, GCR_EINVAL, "NULL rhs");
  if ((const void*)rhs == (const void*)r || (const void*)phi_tilde == (const void*)r)
    return fail(s, GCR_EINVAL, "r must not alias an input");
  if (!s->have_split[member]) return fail(s, GCR_ESTATE, "member %d has no split base (gcr_set_split_base)", member);
  const MemberGeom& G = s->geom_h[member];
  const long long n = (long long)G.nx * G.ny;
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024));
  const SplitArgs S = split_args(s);
  KLAUNCH(s, KT_COPY, k_to_pool_f32, cg, dim3(256), 0, s->stream, phi_tilde, (float*)S.tilde, G);
  KLAUNCH(s, KT_COPY, k_to_pool, cg, dim3(256), 0, s->stream, rhs, s->rhs, G);
  Fields F = make_fields(s);
  F.row_base = G.row0;
  F.row_end = G.row0 + G.ny;
  F.ignore_done = 1;
  ROWS_LAUNCH(s, member_class(s, member), F, KT_RESIDUAL, k_residual_split, PrecF64, S);
  KLAUNCH(s, KT_COPY, k_from_pool, cg, dim3(256), 0, s->stream, (const double*)s->r64, r, G);
  HIPCHK(s, hipGetLastError());
  return GCR_OK;
}

extern "C" int gcr_apply_operator(gcr_solver* s, int32_t member, const double* x, double* y) {
  int rc = check_member(s, member, x, y);
  if (rc != GCR_OK) return rc;
  const MemberGeom& G = s->geom_h[member];
  const long long n = (long long)G.nx * G.ny;
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024));
  KLAUNCH(s, KT_COPY, k_to_pool, cg, dim3(256), 0, s->stream, x, s->x, G);
  Fields F = make_fields(s);
  F.row_base = G.row0;
  F.row_end = G.row0 + G.ny;
  F.ignore_done = 1;
  Slots sl{};
  ROWS_LAUNCH_F(s, member_class(s, member), F, KT_APPLY_L, k_apply_L, PrecF64, (const void*)(s->x), (void*)s->r64, 2,
              0, sl);
  KLAUNCH(s, KT_COPY, k_from_pool, cg, dim3(256), 0, s->stream, (const double*)s->r64, y, G);
  HIPCHK(s, hipGetLastError());
  return GCR_OK;
}

extern "C" int gcr_apply_precond(gcr_solver* s, int32_t member, const double* r, double* e) {
  int rc = check_member(s, member, r, e);
  if (rc != GCR_OK) return rc;
  if (s->prm.precond == GCR_PC_LEARNED && !s->net)
    return fail(s, GCR_ESTATE, "learned preconditioner without parameters (call gcr_set_learned)");
  const MemberGeom& G = s->geom_h[member];
  const long long n = (long long)G.nx * G.ny;
  Fields F = make_fields(s);
  if (s->prm.precision != GCR_FP64) {
    F.r = s->aux_r;
    F.e = s->aux_e;
    F.q[0] = s->aux_q[0];
    F.q[1] = s->aux_q[1];
  }
  F.row_base = G.row0;
  F.row_end = G.row0 + G.ny;
  F.ignore_done = 1;
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024));
  KLAUNCH(s, KT_COPY, k_to_pool, cg, dim3(256), 0, s->stream, r, (double*)F.r, G);
  launch_precond<PrecF64>(s, member_class(s, member), F, 0, 0, 0, member, 1);
  KLAUNCH(s, KT_COPY, k_from_pool, cg, dim3(256), 0, s->stream, (const double*)F.e, e, G);
  HIPCHK(s, hipGetLastError());
  return GCR_OK;
}

// ---------------------------------------------------------------------------
// learned preconditioner
// ---------------------------------------------------------------------------
extern "C" int gcr_set_learned(gcr_solver* s, const float* params, int64_t count, double fallback_ratio) {
  if (!s) return GCR_EINVAL;
  if (s->prm.precond != GCR_PC_LEARNED)
    return fail(s, GCR_EINVAL, "gcr_set_learned needs a solver created with GCR_PC_LEARNED");
  if (!params) return fail(s, GCR_EINVAL, "gcr_set_learned: NULL parameters");
  if (count != cnn_param_count(GCR_LEARNED_CHANNELS))
    return fail(s, GCR_EINVAL, "expected %lld parameters, got %lld",
                (long long)cnn_param_count(GCR_LEARNED_CHANNELS), (long long)count);
  if (!(fallback_ratio > 0.0 && fallback_ratio <= 1.0))
    return fail(s, GCR_EINVAL, "fallback_ratio must be in (0, 1]");
  if (!s->net) {
    hipError_t herr = hipSuccess;
    s->learn_active = dalloc<int>(s->prm.batch, herr);
    if (herr != hipSuccess) return fail(s, GCR_ENOMEM, "learned preconditioner: %s", hipGetErrorString(herr));
    s->allocs.push_back(s->learn_active);
    const int rc = cnn_create(s->nx[0], s->ny[0], s->prm.batch, GCR_LEARNED_CHANNELS, s->stream, &s->net);
    if (rc != GCR_OK) return fail(s, rc, "network: %s", cnn_last_error(nullptr));
  }
  const int rc = cnn_set_params(s->net, params, count);
  if (rc != GCR_OK) return fail(s, rc, "network: %s", cnn_last_error(s->net));
  s->fallback_ratio = fallback_ratio;
  return GCR_OK;
}

extern "C" int gcr_learned_features(gcr_solver* s, int32_t member, const double* x, const double* rhs,
                                    int32_t hi_iters, float* feat, float* target, double* sigma) {
  int rc = check_member(s, member, x, rhs);
  if (rc != GCR_OK) return rc;
  if (!feat) return fail(s, GCR_EINVAL, "gcr_learned_features: NULL feat");
  if (s->prm.precond != GCR_PC_SEMI_IMPLICIT && s->prm.precond != GCR_PC_LEARNED)
    return fail(s, GCR_EINVAL, "features need the semi-implicit preconditioner (option 3)");
  if (hi_iters < 0 || hi_iters > 16) return fail(s, GCR_EINVAL, "hi_iters must be in [0, 16]");
  const MemberGeom& G = s->geom_h[member];
  if (G.nx < 64) return fail(s, GCR_EINVAL, "features need nx >= 64");
  const long long n = (long long)G.nx * G.ny;
  const std::vector<RowClass> cls = member_class(s, member);
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024));
  Fields F = make_fields(s);
  F.row_base = G.row0;
  F.row_end = G.row0 + G.ny;
  F.ignore_done = 1;
  // float64 work buffers: e_lo, e_hi and the two intermediates
  double* elo = s->prm.precision == GCR_FP64 ? (double*)s->e : s->aux_e;
  double* ehi = s->prm.precision == GCR_FP64 ? (double*)s->le : s->aux_r;
  if (s->prm.precision != GCR_FP64) {
    F.q[0] = s->aux_q[0];
    F.q[1] = s->aux_q[1];
  }
  // r = L(x) - rhs and its <r,r> partials
  KLAUNCH(s, KT_COPY, k_to_pool, cg, dim3(256), 0, s->stream, x, s->x, G);
  KLAUNCH(s, KT_COPY, k_to_pool, cg, dim3(256), 0, s->stream, rhs, s->rhs, G);
  ROWS_LAUNCH_F(s, cls, F, KT_RESIDUAL, k_residual, PrecF64, 2, -1, 0, 0);
  F.r = s->r64;
  LearnArgs A{};
  A.r = s->r64;
  A.use_part = 1;
  KLAUNCH(s, KT_LEARNED, k_learn_sigma<PrecF64>, dim3(s->prm.batch), dim3(64), 0, s->stream, F, A, member, 1);
  F.e = elo;
  launch_precond<PrecF64>(s, cls, F, 0, 0, -1);
  if (hi_iters > 0) {
    const int keep = s->prm.richardson_iters;
    s->prm.richardson_iters = hi_iters;
    F.e = ehi;
    launch_precond<PrecF64>(s, cls, F, 0, 0, -1);
    s->prm.richardson_iters = keep;
  }
  for (const RowClass& c : cls) {
    Fields f = F;
    f.row_base = c.row_begin;
    f.row_end = c.row_end;
    const dim3 g((c.row_end - c.row_begin + WPB - 1) / WPB), b(WG);
    float* tg = hi_iters > 0 ? target : nullptr;
    const double* eh = hi_iters > 0 ? ehi : nullptr;
    switch (c.log2m) {
      case 1: launch(s, KT_LEARNED, &k_learn_features<2>, g, b, f, (const double*)s->r64, (const double*)elo, eh, feat, tg); break;
      case 2: launch(s, KT_LEARNED, &k_learn_features<4>, g, b, f, (const double*)s->r64, (const double*)elo, eh, feat, tg); break;
      case 3: launch(s, KT_LEARNED, &k_learn_features<8>, g, b, f, (const double*)s->r64, (const double*)elo, eh, feat, tg); break;
      default: launch(s, KT_LEARNED, &k_learn_features<16>, g, b, f, (const double*)s->r64, (const double*)elo, eh, feat, tg); break;
    }
  }
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, hipMemcpyAsync(s->state_h, s->state, s->prm.batch * sizeof(MemberState), hipMemcpyDeviceToHost,
                           s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  if (sigma) *sigma = s->state_h[member].sigma;
  return GCR_OK;
}

extern "C" const char* gcr_status_string(int code) {
  switch (code) {
    case GCR_OK: return "converged";
    case GCR_NOT_CONVERGED: return "not converged (max_iters reached)";
    case GCR_STAGNATED: return "stagnated (breakdown or no decrease over a cycle)";
    case GCR_FALLBACK_USED: return "converged after falling back to the semi-implicit preconditioner";
    case GCR_EINVAL: return "invalid argument";
    case GCR_ENOMEM: return "out of memory";
    case GCR_EHIP: return "HIP runtime error";
    case GCR_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

extern "C" const char* gcr_last_error(const gcr_solver* s) {
  if (!s) return g_create_error.c_str();
  return s->err.c_str();
}

extern "C" const char* gcr_version(void) { return "mpgcr 0.1.0 gfx950"; }

extern "C" int gcr_set_kernel_timing(gcr_solver* s, int32_t enable) {
  if (!s) return GCR_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->tm_collect();
  s->timing = enable != 0;
  for (int k = 0; k < KT_COUNT; ++k) {
    s->kt_count[k] = 0;
    s->kt_ms[k] = 0.0;
  }
  return GCR_OK;
}

extern "C" int gcr_kernel_time(gcr_solver* s, int32_t kind, int64_t* launches, double* total_ms) {
  if (!s || !launches || !total_ms || kind < 0 || kind >= KT_COUNT) return GCR_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->tm_collect();
  *launches = s->kt_count[kind];
  *total_ms = s->kt_ms[kind];
  return GCR_OK;
}

extern "C" const char* gcr_kernel_name(int32_t kind) {
  static const char* names[KT_COUNT] = {"assemble", "residual", "update_sweep1", "sweep2",  "apply_L",
                                        "orth",     "control",  "copy",          "learned", "solution"};
  return (kind >= 0 && kind < KT_COUNT) ? names[kind] : "unknown";
}
