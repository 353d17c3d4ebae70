// C-ABI of the GCR(k) depth solver (see include/mpgcr.h): creation,
// assembly, the solve entry point, stand-alone operator, preconditioner and
// split-residual calls, the learned preconditioner's set-up and timing.
#include "solver_impl.h"

#include <cstdlib>

static void worker_main(gcr_solver* s, int w);
static void stop_workers(gcr_solver* s);

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
  auto drop_graphs = [](gcr_solver::Group& g) {
    for (hipGraphExec_t& e : g.g_iter)
      if (e) (void)hipGraphExecDestroy(e);
    for (hipGraphExec_t& e : g.g_end)
      if (e) (void)hipGraphExecDestroy(e);
    g.g_iter.clear();
    g.g_end.clear();
  };
  drop_graphs(s->whole);
  for (auto& g : s->groups) {
    drop_graphs(g);
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
  if (s->si_stage) (void)hipHostFree(s->si_stage);
  if (s->si_work) (void)hipFree(s->si_work);
  s->si_stage = nullptr;
  s->si_work = nullptr;
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
  if (s->own_stream) {
    (void)hipStreamSynchronize(s->own_stream);
    (void)hipStreamDestroy(s->own_stream);
  }
  s->own_stream = nullptr;
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
  const long long ncls = merge_classes(s->classes) ? 1 : (long long)s->classes.size();   // launches per kernel
  const long long fit = total / (GROUP_PTS * ncls);
  int G = (int)std::min<long long>(std::min(GROUPS_MAX, B), std::max<long long>(fit, 1));
  if (s->prm.precond == GCR_PC_LEARNED || (s->prm.flags & GCR_F_ONE_STREAM)) G = 1;
  // With the runtime's eager code-object loading (HIP_ENABLE_DEFERRED_LOADING=0)
  // a batch split into member groups (several host threads enqueueing) once
  // ended in a host segmentation fault whose cause has not been found; that
  // combination is kept on one stream.
  if (const char* ev = std::getenv("HIP_ENABLE_DEFERRED_LOADING"))
    if (ev[0] == '0' && ev[1] == 0) G = 1;
  if (G < 2) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming);
  int q = 0, row = 0;
  long long pts = 0;
  for (int g = 0; g < G && e == hipSuccess; ++g) {
    gcr_solver::Group grp;
    grp.q0 = q;
    grp.gi = g;
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
    bool changed = false;
    for (RowClass& c : cls) {
      int all = 1;
      for (int m : s->morder_h) {
        const MemberGeom& G = s->geom_h[m];
        if (G.row0 >= c.row_begin && G.row0 < c.row_end) all &= s->flat_h[m];
      }
      changed = changed || c.flat != all;
      c.flat = all;
    }
    return changed;
  };
  // captured graphs hold the kernel variant of each class: a class whose
  // orography status changed drops its group's graphs
  auto drop = [](gcr_solver::Group& g) {
    for (hipGraphExec_t& e : g.g_iter)
      if (e) (void)hipGraphExecDestroy(e);
    for (hipGraphExec_t& e : g.g_end)
      if (e) (void)hipGraphExecDestroy(e);
    g.g_iter.clear();
    g.g_end.clear();
  };
  mark(s->classes);
  if (mark(s->whole.classes)) drop(s->whole);
  for (gcr_solver::Group& g : s->groups)
    if (mark(g.classes)) drop(g);
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
  if (P.flags & ~(GCR_F_RECORD_HISTORY | GCR_F_ONE_STREAM | GCR_F_LINF_EXIT | GCR_F_FAULT_NAN_PC | GCR_F_FAULT_ZERO_DIR |
                  GCR_F_SPLIT_R0 | GCR_F_GRAPH))
    return fail(nullptr, GCR_EINVAL, "unknown flags 0x%x", P.flags);
  if ((P.flags & GCR_F_SPLIT_R0) && P.precision != GCR_SINGLE && P.precision != GCR_SINGLE_POLAR64)
    return fail(nullptr, GCR_EINVAL, "GCR_F_SPLIT_R0 needs GCR_SINGLE or GCR_SINGLE_POLAR64");
  if ((P.flags & GCR_F_FAULT_NAN_PC) && (P.flags & GCR_F_FAULT_ZERO_DIR))
    return fail(nullptr, GCR_EINVAL, "at most one fault-injection flag");
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
  if ((P.flags & GCR_F_GRAPH) && !P.stream) {
    // the null stream cannot be captured: a blocking stream of the solver's
    // own, which the null stream's work stays ordered with
    const hipError_t e = hipStreamCreate(&s->own_stream);
    if (e != hipSuccess) {
      delete s;
      return fail(nullptr, GCR_EHIP, "stream creation: %s", hipGetErrorString(e));
    }
    s->stream = s->own_stream;
  }
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
  s->cyc_ctr = (int*)track(dalloc<int>(GROUPS_MAX + 1, herr));
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
  // the rhs and x tables in one block, uploaded by one copy
  s->ptr_rhs = (const double**)track(dalloc<const double*>(2 * (size_t)P.batch, herr));
  s->ptr_x = s->ptr_rhs ? (double**)(s->ptr_rhs + P.batch) : nullptr;
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
  {   // the whole batch as one group on the solver's stream
    gcr_solver::Group& w = s->whole;
    w.q0 = 0;
    w.q1 = P.batch;
    w.gi = 0;
    w.classes = s->classes;
    w.st = s->stream;
    for (int i = 0; i < 2; ++i) {
      w.cycle_ev[i] = s->cycle_ev[i];
      w.ring[i] = s->state_ring[i];
    }
  }
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
  std::vector<AsmMember> tab(count);
  for (int t = 0; t < count; ++t) {
    const int member = members[t];
    const gcr_operator* op = &ops[t];
    const MemberGeom& G = s->geom_h[member];
    const long long n = (long long)G.nx * G.ny;
    AsmMember& a = tab[t];
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
  if (tab.size() != s->asm_last.size() || std::memcmp(tab.data(), s->asm_last.data(), count * sizeof(AsmMember)) != 0) {
    // the staging table (pinned) may still feed the previous upload: wait
    // for that copy only, not for the whole stream
    HIPCHK(s, hipEventSynchronize(s->stage_ev[1]));
    std::memcpy(s->asm_stage, tab.data(), count * sizeof(AsmMember));
    HIPCHK(s, hipMemcpyAsync(s->asm_tab, s->asm_stage, count * sizeof(AsmMember), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipEventRecord(s->stage_ev[1], s->stream));
    s->asm_last = tab;
  }
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
    s->flat_h[members[t]] = tab[t].oro ? 0 : 1;   // as k_assemble sets `flat`
  }
  refresh_flat(s);
  return GCR_OK;
}

extern "C" int gcr_set_operator(gcr_solver* s, int32_t member, const gcr_operator* op) {
  if (!s) return GCR_EINVAL;
  if (!op) return fail(s, GCR_EINVAL, "gcr_set_operator: NULL operator");
  return gcr_set_operators(s, 1, &member, op);
}

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
  if (s->prm.flags & GCR_F_SPLIT_R0)
    for (int m = 0; m < B; ++m)
      if (!s->have_split[m]) return fail(s, GCR_ESTATE, "member %d has no split base (gcr_set_split_base)", m);
  std::vector<const void*> tab(2 * (size_t)B);
  for (int m = 0; m < B; ++m) {
    tab[m] = rhs[m];
    tab[B + m] = x[m];
  }
  if (tab != s->ptr_last) {
    HIPCHK(s, hipEventSynchronize(s->stage_ev[0]));  // staging buffer reuse
    std::memcpy(s->ptr_stage, tab.data(), tab.size() * sizeof(void*));
    HIPCHK(s, hipMemcpyAsync(s->ptr_rhs, s->ptr_stage, tab.size() * sizeof(void*), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipEventRecord(s->stage_ev[0], s->stream));
    s->ptr_last = tab;
  }
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
  ROWS_LAUNCH(s, member_class(s, member), F, KT_RESIDUAL, k_residual_split, PrecF64, S, 0);
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

// the operator or preconditioner in the solver's precision form
static int apply_in_form(gcr_solver* s, int32_t member, int what, const double* in, double* out) {
  int rc = check_member(s, member, in, out);
  if (rc != GCR_OK) return rc;
  if (what == 1 && s->prm.precond == GCR_PC_LEARNED && !s->net)
    return fail(s, GCR_ESTATE, "learned preconditioner without parameters (call gcr_set_learned)");
  switch (s->prm.precision) {
    case GCR_FP64: return apply_form<PrecF64>(s, member, what, in, out);
    case GCR_MIXED: return apply_form<PrecMixed>(s, member, what, in, out);
    case GCR_MIXED_FP64DOT: return apply_form<PrecMixedD>(s, member, what, in, out);
    case GCR_SINGLE: return apply_form<PrecSingle>(s, member, what, in, out);
    case GCR_SINGLE_POLAR64: return apply_form<PrecSingleD>(s, member, what, in, out);
    default: return apply_form<PrecMixedP>(s, member, what, in, out);
  }
}

extern "C" int gcr_apply_operator_form(gcr_solver* s, int32_t member, const double* x, double* y) {
  return apply_in_form(s, member, 0, x, y);
}

extern "C" int gcr_apply_precond_form(gcr_solver* s, int32_t member, const double* r, double* e) {
  return apply_in_form(s, member, 1, r, e);
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

extern "C" int gcr_set_learned_reference(gcr_solver* s, const double* rel_res, int32_t n) {
  if (!s) return GCR_EINVAL;
  if (s->prm.precond != GCR_PC_LEARNED)
    return fail(s, GCR_EINVAL, "gcr_set_learned_reference needs a solver created with GCR_PC_LEARNED");
  if (n < 0 || n > s->prm.max_iters) return fail(s, GCR_EINVAL, "n must be in [0, max_iters]");
  if (n > 0 && !rel_res) return fail(s, GCR_EINVAL, "NULL reference history");
  for (int i = 1; i <= n; ++i)
    if (!(rel_res[i] > 0.0) || !std::isfinite(rel_res[i]))
      return fail(s, GCR_EINVAL, "reference residual %d must be finite and > 0", i);
  if (n > 0) {
    if (!s->learn_ref) {
      hipError_t herr = hipSuccess;
      s->learn_ref = dalloc<double>((size_t)s->prm.max_iters + 1, herr);
      if (herr != hipSuccess) return fail(s, GCR_ENOMEM, "reference history: %s", hipGetErrorString(herr));
      s->allocs.push_back(s->learn_ref);
    }
    HIPCHK(s, hipMemcpyAsync(s->learn_ref, rel_res, ((size_t)n + 1) * sizeof(double), hipMemcpyHostToDevice,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
  }
  s->learn_ref_n = n;
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
                                        "orth",     "control",  "copy",          "learned", "solution",
                                        "si_step"};
  return (kind >= 0 && kind < KT_COUNT) ? names[kind] : "unknown";
}
