// Host runtime of the GCR(k) depth solver shared by its translation units:
// the solver object, launch helpers and the kernel sequences of a solve,
// templated on the precision form.  Each form's solve is instantiated in a
// source file of its own (solve_*.hip) so the forms compile in parallel; the
// C-ABI entry points are in solver.hip.
#pragma once
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

// text of the last failed gcr_create on this thread (one variable for every
// translation unit of the library)
inline thread_local std::string g_create_error;

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
inline thread_local hipStream_t t_stream = nullptr;

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
  hipStream_t own_stream = nullptr;  // GCR_F_GRAPH with a NULL stream: the stream used instead
  // Groups of members with rows contiguous in row order, each solved on a
  // stream of its own, so that one group's kernel boundaries (the drain of
  // the last waves, the start of the next kernel) overlap the others' work.
  // Empty: the whole batch on `stream`.
  struct Group {
    int q0 = 0, q1 = 0;                // members morder[q0 .. q1)
    int gi = 0;                        // index of the group's cycle counter
    std::vector<RowClass> classes;     // the group's rows
    hipStream_t st = nullptr;
    hipEvent_t cycle_ev[2] = {};
    int* ring[2] = {};                 // pinned copies of the done flags after a cycle
    hipEvent_t done_ev = nullptr;
    // GCR_F_GRAPH: executable graphs of an iteration [nu][ring base] and of a
    // cycle end [ring base], captured on first use
    mutable std::vector<hipGraphExec_t> g_iter, g_end;
  };
  std::vector<Group> groups;
  Group whole;                       // the whole batch on the solver's stream (no member groups)
  int* cyc_ctr = nullptr;            // per group: the GCR cycle counter (device)
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
  // host copies of the tables last uploaded: a call whose tables equal them
  // (the same caller buffers and operator inputs step after step) uploads
  // nothing, since the device copies already hold them
  std::vector<const void*> ptr_last;
  std::vector<AsmMember> asm_last;
  AsmMember* asm_tab = nullptr;      // device assembly table [batch]
  cnn_net* net = nullptr;            // learned preconditioner (GCR_PC_LEARNED), owned
  int* learn_active = nullptr;       // [batch] images the network runs on in one application
  double fallback_ratio = 0.5;
  double* learn_ref = nullptr;       // [max_iters + 1] reference relative residuals (device), or null
  int learn_ref_n = 0;
  // gcr_si_step: work fields (allocated by its first call) and member tables
  double* si_work = nullptr;
  long long si_wpts = 0;
  void* si_tab = nullptr;
  void* si_stage = nullptr;          // pinned staging of si_tab

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

inline hipStream_t cur_stream(const gcr_solver* s) { return t_stream ? t_stream : s->stream; }

inline int fail(gcr_solver* s, int code, const char* fmt, ...) {
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
void launch(gcr_solver* s, int kind, void (*kern)(KArgs...), dim3 grid, dim3 block, Args... args) {
  s->tm_begin(kind);
  hipLaunchKernelGGL(kern, grid, block, 0, cur_stream(s), args...);
  s->tm_end();
}

// One launch of row kernel KNAME<P, M> per row class, each covering that
// class's rows (one wave per row).
static_assert(KT_COUNT == GCR_K_COUNT, "kernel kinds match the header");

// Several row classes whose points per lane are all <= 8 go in one launch
// of the KNAME<P, 0> variant, which dispatches on each row's class; one
// launch per kernel instead of one per class (an uneven batch would else be
// bound by the host's launch rate).
inline bool merge_classes(const std::vector<RowClass>& cls) {
  if (cls.size() < 2) return false;
  for (const RowClass& c : cls)
    if (c.log2m > 3) return false;
  return true;
}

#define ROWS_LAUNCH(s, CLASSES, F, KIND, KNAME, P, ...)                                     \
  do {                                                                                   \
    const std::vector<RowClass>& cl_ = (CLASSES);                                        \
    if (merge_classes(cl_)) {                                                            \
      Fields f_ = (F);                                                                   \
      f_.row_base = cl_.front().row_begin;                                               \
      f_.row_end = cl_.back().row_end;                                                   \
      const dim3 g_((f_.row_end - f_.row_base + WPB - 1) / WPB), b_(WG);                 \
      launch(s, KIND, &KNAME<P, 0>, g_, b_, f_, ##__VA_ARGS__);                          \
      break;                                                                             \
    }                                                                                    \
    for (const RowClass& c_ : cl_) {                                                     \
      Fields f_ = (F);                                                                   \
      f_.row_base = c_.row_begin;                                                        \
      f_.row_end = c_.row_end;                                                           \
      const dim3 g_((c_.row_end - c_.row_begin + WPB - 1) / WPB), b_(WG);                \
      switch (c_.log2m) {                                                                \
        case 1: launch(s, KIND, &KNAME<P, 2>, g_, b_, f_, ##__VA_ARGS__); break;          \
        case 2: launch(s, KIND, &KNAME<P, 4>, g_, b_, f_, ##__VA_ARGS__); break;          \
        case 3: launch(s, KIND, &KNAME<P, 8>, g_, b_, f_, ##__VA_ARGS__); break;          \
        default: launch(s, KIND, &KNAME<P, 16>, g_, b_, f_, ##__VA_ARGS__); break;        \
      }                                                                                  \
    }                                                                                    \
  } while (0)

inline std::vector<RowClass> member_class(const gcr_solver* s, int member) {
  const MemberGeom& G = s->geom_h[member];
  return {RowClass{G.log2m, G.row0, G.row0 + G.ny, s->flat_h[member]}};
}

// As ROWS_LAUNCH, for the kernels that evaluate the stencil with coefficients
// formed from the depth fields: a class whose members all lack orography takes
// the variant that reads Phi* only (FL = true), which holds fewer registers.
#define ROWS_LAUNCH_F(s, CLASSES, F, KIND, KNAME, P, ...)                                   \
  do {                                                                                   \
    const std::vector<RowClass>& cl_ = (CLASSES);                                        \
    if (merge_classes(cl_)) {                                                            \
      Fields f_ = (F);                                                                   \
      f_.row_base = cl_.front().row_begin;                                               \
      f_.row_end = cl_.back().row_end;                                                   \
      const dim3 g_((f_.row_end - f_.row_base + WPB - 1) / WPB), b_(WG);                 \
      bool fl_ = true;                                                                   \
      for (const RowClass& c_ : cl_) fl_ = fl_ && c_.flat;                               \
      if (fl_) launch(s, KIND, &KNAME<P, 0, true>, g_, b_, f_, ##__VA_ARGS__);           \
      else launch(s, KIND, &KNAME<P, 0, false>, g_, b_, f_, ##__VA_ARGS__);              \
      break;                                                                             \
    }                                                                                    \
    for (const RowClass& c_ : cl_) {                                                     \
      Fields f_ = (F);                                                                   \
      f_.row_base = c_.row_begin;                                                        \
      f_.row_end = c_.row_end;                                                           \
      const dim3 g_((c_.row_end - c_.row_begin + WPB - 1) / WPB), b_(WG);                \
      switch (std::min(c_.log2m, 4) * 2 + (c_.flat ? 1 : 0)) {                           \
        case 2: launch(s, KIND, &KNAME<P, 2, false>, g_, b_, f_, ##__VA_ARGS__); break;   \
        case 3: launch(s, KIND, &KNAME<P, 2, true>, g_, b_, f_, ##__VA_ARGS__); break;    \
        case 4: launch(s, KIND, &KNAME<P, 4, false>, g_, b_, f_, ##__VA_ARGS__); break;   \
        case 5: launch(s, KIND, &KNAME<P, 4, true>, g_, b_, f_, ##__VA_ARGS__); break;    \
        case 6: launch(s, KIND, &KNAME<P, 8, false>, g_, b_, f_, ##__VA_ARGS__); break;   \
        case 7: launch(s, KIND, &KNAME<P, 8, true>, g_, b_, f_, ##__VA_ARGS__); break;    \
        case 9: launch(s, KIND, &KNAME<P, 16, true>, g_, b_, f_, ##__VA_ARGS__); break;   \
        default: launch(s, KIND, &KNAME<P, 16, false>, g_, b_, f_, ##__VA_ARGS__); break; \
      }                                                                                  \
    }                                                                                    \
  } while (0)

inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

inline Fields make_fields(gcr_solver* s) {
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
  F.learn_ref = s->learn_ref_n > 0 ? s->learn_ref : nullptr;
  F.learn_ref_n = s->learn_ref_n;
  F.cyc = s->cyc_ctr;
  return F;
}

// ---------------------------------------------------------------------------
// kernel sequences
// ---------------------------------------------------------------------------
// Learned correction of the preconditioner output F.e (members
// [member0, member0 + count)): residual scale, network input, five
// convolutions over the whole batch of images, update of e.  `use_part`: the
// per-row <r,r> partials of F.r are current (inside a solve).
template <typename P>
void learned_correction(gcr_solver* s, const std::vector<RowClass>& cls, const Fields& F, int use_part,
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
void launch_precond(gcr_solver* s, const std::vector<RowClass>& cls, const Fields& F, int do_update,
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

// the split-residual buffers: Phi_hat, its stored differences, Phi_tilde
inline SplitArgs split_args(const gcr_solver* s) {
  SplitArgs S{};
  S.hat = s->split;
  for (int k = 0; k < NSD; ++k) S.d[k] = s->split + (size_t)(k + 1) * s->npts;
  S.tilde = s->split + (size_t)(NSD + 1) * s->npts;
  return S;
}

// Stand-alone operator (what = 0) or preconditioner (what = 1) of member
// `member` in precision form P, with the kernels a solve of that form runs.
// The form's vectors are the solver's own Krylov buffers (these calls and a
// solve are ordered on the solver's stream).  Directions are held in physical
// units, residuals (and so L applied to a direction) in the form's scaled
// units: x enters as fl(x) in the vector type and y = L_s(x) / s leaves; r
// enters as fl(s r) and e = P^{-1} leaves as held.
template <typename P>
int apply_form(gcr_solver* s, int member, int what, const double* in, double* out) {
  using V = typename P::V;
  const MemberGeom& G = s->geom_h[member];
  const long long n = (long long)G.nx * G.ny;
  const double sc = P::mixed ? s->scale_h[member] : 1.0;
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024)), cb(256);
  Fields F = make_fields(s);
  F.row_base = G.row0;
  F.row_end = G.row0 + G.ny;
  F.ignore_done = 1;
  const std::vector<RowClass> cls = member_class(s, member);
  if (what == 0) {
    KLAUNCH(s, KT_COPY, k_to_pool_v<V>, cg, cb, 0, s->stream, in, (V*)F.e, G, 1.0);
    Slots sl{};
    ROWS_LAUNCH_F(s, cls, F, KT_APPLY_L, k_apply_L, P, (const void*)F.e, F.le, 2, 0, sl);
    KLAUNCH(s, KT_COPY, k_from_pool_v<V>, cg, cb, 0, s->stream, (const V*)F.le, out, G, 1.0 / sc);
  } else {
    KLAUNCH(s, KT_COPY, k_to_pool_v<V>, cg, cb, 0, s->stream, in, (V*)F.r, G, sc);
    launch_precond<P>(s, cls, F, 0, 0, 0, member, 1);
    KLAUNCH(s, KT_COPY, k_from_pool_v<V>, cg, cb, 0, s->stream, (const V*)F.e, out, G, 1.0);
  }
  HIPCHK(s, hipGetLastError());
  return GCR_OK;
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
int run_group(gcr_solver* s, const gcr_solver::Group& g) {
  using A = typename P::A;
  struct StreamScope {   // this thread's launches go to the group's stream
    explicit StreamScope(hipStream_t st) { t_stream = st; }
    ~StreamScope() { t_stream = nullptr; }
  } scope(g.st);
  const int k = s->prm.k, B = s->prm.batch, maxit = s->prm.max_iters;
  Fields F = make_fields(s);
  F.q0 = g.q0;
  F.cyc = s->cyc_ctr + g.gi;
  const bool replace = s->prm.precision == GCR_MIXED_FP64DOT || s->prm.precision == GCR_MIXED_HALF_PC;
  const dim3 ctl(g.q1 - g.q0), wave(64);
  const std::vector<RowClass>& cls = g.classes;
  // GCR_F_GRAPH: the launches of an iteration (per window position and ring
  // base) and of a cycle end (per ring base) are captured once into a HIP
  // graph on the group's stream and replayed; their arguments depend on
  // nothing else (the cycle number lives on the device), and they hold
  // kernel nodes only.
  const bool graphs = (s->prm.flags & GCR_F_GRAPH) && !s->timing && s->prm.precond != GCR_PC_LEARNED;
  if (graphs) {
    g.g_iter.resize((size_t)k * (k + 1), nullptr);
    g.g_end.resize((size_t)k + 1, nullptr);
  }
  auto via_graph = [&](hipGraphExec_t& exec, auto&& enqueue) -> int {
    if (!exec) {
      hipGraph_t graph = nullptr;
      HIPCHK(s, hipStreamBeginCapture(g.st, hipStreamCaptureModeThreadLocal));
      enqueue();
      const hipError_t ec = hipStreamEndCapture(g.st, &graph);
      if (ec != hipSuccess) return fail(s, GCR_EHIP, "graph capture: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        exec = nullptr;
        return fail(s, GCR_EHIP, "graph instantiation: %s", hipGetErrorString(ei));
      }
    }
    HIPCHK(s, hipGraphLaunch(exec, g.st));
    return GCR_OK;
  };

  // step 1: r_0 = L(x_0) - R (float64; or the split single-precision
  // evaluation of paper Section 4.2.1), p_0 = P^{-1}(r_0), L(p_0)
  if (s->prm.flags & GCR_F_SPLIT_R0) {
    ROWS_LAUNCH(s, cls, F, KT_RESIDUAL, k_split_tilde, P, split_args(s));
    ROWS_LAUNCH(s, cls, F, KT_RESIDUAL, k_residual_split, P, split_args(s), 1);
  } else {
    ROWS_LAUNCH_F(s, cls, F, KT_RESIDUAL, k_residual, P, 1, -1, 0, RES_X_IN | RES_RHS_TAB);
  }
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

  // the launches of an iteration at window position nu of a cycle whose p_0
  // sits in ring slot `base`
  auto iteration_launches = [&](int nu, int base) {
    Slots sl{};
    for (int l = 0; l <= k; ++l) sl.s[l] = (base + l) % (k + 1);
    // step 2 (+ first row solve of step 3)
    launch_precond<P>(s, cls, F, 1, sl.s[nu]);
    if (s->prm.flags & (GCR_F_FAULT_NAN_PC | GCR_F_FAULT_ZERO_DIR))
      ROWS_LAUNCH(s, cls, F, KT_SWEEP2, k_fault_e, P, (s->prm.flags & GCR_F_FAULT_NAN_PC) ? 1 : 2, k);
    // step 3: L(e) with <L e, L p_l>, l = 0..nu
    ROWS_LAUNCH_F(s, cls, F, KT_APPLY_L, k_apply_L, P, (const void*)s->e, s->le, 0, nu + 1, sl);
    KLAUNCH(s, KT_CONTROL, k_ctrl_alpha<A>, ctl, wave, 0, g.st, F, nu + 1, sl, nu == k - 1 ? 1 : 0,
            s->prm.min_iters, maxit, s->prm.rtol);
    // step 4
    if (nu == k - 1) {   // the cycle's last iteration also applies its solution updates
      ROWS_LAUNCH(s, cls, F, KT_ORTH, k_orth_last, P, nu + 1, sl, sl.s[nu + 1]);
    } else {
      ROWS_LAUNCH(s, cls, F, KT_ORTH, k_orth, P, nu + 1, sl, sl.s[nu + 1]);
    }
    KLAUNCH(s, KT_CONTROL, k_ctrl_beta<A>, ctl, wave, 0, g.st, F, sl.s[nu + 1]);
  };
  auto iteration = [&](int nu, int base) -> int {
    if (graphs) return via_graph(g.g_iter[(size_t)nu * (k + 1) + base], [&] { iteration_launches(nu, base); });
    iteration_launches(nu, base);
    return GCR_OK;
  };
  // end of a cycle: its solution updates; (p_0, L p_0) := (p_k, L p_k);
  // residual replacement; the next cycle number; the done flags
  auto cycle_end_launches = [&](int base_next) {
    ROWS_LAUNCH(s, cls, F, KT_SOLUTION, k_apply_pending, P);
    if (replace) {
      ROWS_LAUNCH_F(s, cls, F, KT_RESIDUAL, k_residual, P, 1, base_next, 1, RES_RHS_TAB);
      KLAUNCH(s, KT_CONTROL, k_ctrl_restart<double>, ctl, wave, 0, g.st, F, base_next);
    }
    KLAUNCH(s, KT_CONTROL, k_cycle_next, dim3(1), wave, 0, g.st, F.cyc);
  };
  auto cycle_end = [&](int base_next, int ring) -> int {
    if (graphs) {
      const int rc = via_graph(g.g_end[base_next], [&] { cycle_end_launches(base_next); });
      if (rc != GCR_OK) return rc;
    } else {
      cycle_end_launches(base_next);
    }
    // the done flags (a few bytes per member: a small copy); only the group's
    // own members are read from them
    HIPCHK(s, hipMemcpyAsync(g.ring[ring], s->done_flag, B * sizeof(int), hipMemcpyDeviceToHost, g.st));
    HIPCHK(s, hipEventRecord(g.cycle_ev[ring], g.st));
    return GCR_OK;
  };

  int it = 0, base = 0, cycle = 0, rc;
  // cycle 0, complete
  for (int nu = 0; nu < k && it < maxit; ++nu, ++it)
    if ((rc = iteration(nu, base)) != GCR_OK) return rc;
  base = (base + k) % (k + 1);
  if ((rc = cycle_end(base, 0)) != GCR_OK) return rc;
  HIPCHK(s, hipGetLastError());
  for (;;) {
    // speculative first iteration of the next cycle
    const bool more = it < maxit;
    if (more) {
      ++it;
      if ((rc = iteration(0, base)) != GCR_OK) return rc;
    }
    HIPCHK(s, hipEventSynchronize(g.cycle_ev[cycle & 1]));
    bool done = true;
    for (int q = g.q0; q < g.q1; ++q) done = done && g.ring[cycle & 1][s->morder_h[q]] != 0;
    if (done || !more) break;
    for (int nu = 1; nu < k && it < maxit; ++nu, ++it)
      if ((rc = iteration(nu, base)) != GCR_OK) return rc;
    base = (base + k) % (k + 1);
    ++cycle;
    if ((rc = cycle_end(base, cycle & 1)) != GCR_OK) return rc;
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
template <typename P>
int run_solve(gcr_solver* s) {
  const int B = s->prm.batch;
  const bool split = !s->groups.empty() && !s->timing;
  if (!split) {
    const gcr_solver::Group& whole = s->whole;
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

// the solves of the precision forms, each instantiated in its own source file
extern template int run_solve<PrecF64>(gcr_solver*);
extern template int run_solve<PrecMixed>(gcr_solver*);
extern template int run_solve<PrecMixedD>(gcr_solver*);
extern template int run_solve<PrecMixedP>(gcr_solver*);
extern template int run_solve<PrecSingle>(gcr_solver*);
extern template int run_solve<PrecSingleD>(gcr_solver*);
extern template int apply_form<PrecF64>(gcr_solver*, int, int, const double*, double*);
extern template int apply_form<PrecMixed>(gcr_solver*, int, int, const double*, double*);
extern template int apply_form<PrecMixedD>(gcr_solver*, int, int, const double*, double*);
extern template int apply_form<PrecMixedP>(gcr_solver*, int, int, const double*, double*);
extern template int apply_form<PrecSingle>(gcr_solver*, int, int, const double*, double*);
extern template int apply_form<PrecSingleD>(gcr_solver*, int, int, const double*, double*);
