// gcr_apply_precond_static: the float64 semi-implicit Richardson
// preconditioner of one member (as gcr_apply_precond of a GCR_FP64 solver
// with that operator) for callers that cannot allocate device memory.
//
// Every buffer beyond the caller's input and output -- the member's
// geometry, the assembly's depth pools, latitude factors and coefficient
// copies, the pooled residual, the two Richardson intermediates and the
// output before it is written back -- lives in one file-scope device array,
// `scratch`, of SCRATCH_BYTES per GPU.  Its device address is taken once per
// device with hipGetSymbolAddress (the array's name is a host-side stand-in
// in host code) and every kernel gets pointers derived from that address.
// The call launches kernels only (set-up, assembly, copies, row solves): no
// allocation, no host-to-device copy, no memset.  Calls on one GPU share the
// array, so calls that overlap on one GPU (different streams or threads
// without ordering) race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/mpgcr.h"
#include "kernels.h"

using namespace mpgcr;

namespace {

constexpr long long STATIC_MAX_POINTS = GCR_STATIC_MAX_POINTS;
constexpr int STATIC_MAX_ROWS = 4096;
constexpr size_t ALIGN = 256;

constexpr size_t up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

// Layout of the scratch array for a member of at most STATIC_MAX_POINTS
// points and STATIC_MAX_ROWS rows (offsets in bytes, each 256-aligned).
struct Layout {
  size_t geom, asmtab, state, scale, flat, rowmap, part, fac64, fac32, c64, c32, phi64, hs64, phi32, hs32, a16, a32,
      r, e, q0, q1, total;
};

constexpr Layout layout() {
  Layout L{};
  const size_t P = (size_t)STATIC_MAX_POINTS, R = (size_t)STATIC_MAX_ROWS;
  size_t o = 0;
  L.geom = o;   o += up(sizeof(MemberGeom));
  L.asmtab = o; o += up(sizeof(AsmMember));
  L.state = o;  o += up(sizeof(MemberState));
  L.scale = o;  o += up(sizeof(double));
  L.flat = o;   o += up(sizeof(int));
  L.rowmap = o; o += up(R * sizeof(int));
  L.part = o;   o += up(R * NDOT * sizeof(double));
  L.fac64 = o;  o += up(R * NFAC * sizeof(double));
  L.fac32 = o;  o += up(R * NFAC * sizeof(float));
  L.c64 = o;    o += up(R * sizeof(double));
  L.c32 = o;    o += up(R * sizeof(float));
  L.phi64 = o;  o += up(P * sizeof(double));
  L.hs64 = o;   o += up(P * sizeof(double));
  L.phi32 = o;  o += up(P * sizeof(float));
  L.hs32 = o;   o += up(P * sizeof(float));
  L.a16 = o;    o += NCOEF * up(P * sizeof(__half));
  L.a32 = o;    o += NCOEF * up(P * sizeof(float));
  L.r = o;      o += up(P * sizeof(double));
  L.e = o;      o += up(P * sizeof(double));
  L.q0 = o;     o += up(P * sizeof(double));
  L.q1 = o;     o += up(P * sizeof(double));
  L.total = o;
  return L;
}

constexpr Layout LAY = layout();
constexpr size_t SCRATCH_BYTES = LAY.total;

}  // namespace

// The scratch array: one copy per GPU the library runs on, held until the
// process ends.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex g_mu;
constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};   // device address of `scratch` per device (taken once)

}  // namespace

// text of the last failure without a solver on this thread, read by
// gcr_last_error(NULL) (the same variable as the other source files')
inline thread_local std::string g_create_error;

namespace {

int static_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_create_error = buf;
  return code;
}

// the device address of `scratch` on the current device
int scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return static_fail(GCR_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return static_fail(GCR_EHIP, "device %d beyond the supported %d", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return static_fail(GCR_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = (unsigned char*)g_scratch[dev];
  return GCR_OK;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

// the member's geometry, assembly table entry and row map, written from the
// kernel arguments (so the call needs no host-to-device copy)
static __global__ void k_static_setup(MemberGeom G, AsmMember A, MemberGeom* geom, AsmMember* tab, int* rowmap,
                                      MemberState* state) {
  const int t = threadIdx.x;
  if (t == 0) {
    *geom = G;
    *tab = A;
    MemberState S{};
    *state = S;                 // not read with ignore_done set; kept defined
  }
  for (int j = t; j < G.ny; j += blockDim.x) rowmap[j] = 0;
}

template <int M, bool FL>
static void launch_rows(const Fields& F, int ny, int iters, hipStream_t st) {
  const dim3 g((ny + WPB - 1) / WPB), b(WG);
  hipLaunchKernelGGL((k_update_sweep1<PrecF64, M>), g, b, 0, st, F, 0, 0, iters == 1 ? -1 : 0);
  int cur = 0;
  for (int mu = 1; mu < iters; ++mu) {
    const int nxt = mu + 1 == iters ? -1 : cur ^ 1;
    hipLaunchKernelGGL((k_sweep2<PrecF64, M, FL>), g, b, 0, st, F, cur, nxt);
    cur ^= 1;
  }
}

extern "C" int gcr_apply_precond_static(int32_t nx, int32_t ny, const gcr_operator* op, int32_t richardson_iters,
                                        const double* r, double* e, void* stream) {
  if (!op || !r || !e) return static_fail(GCR_EINVAL, "gcr_apply_precond_static: NULL argument");
  if (!pow2(nx) || nx < 8 || nx > NXMAX)
    return static_fail(GCR_EINVAL, "nx must be a power of two in [8, %d], got %d", NXMAX, nx);
  if (ny < 2 || ny > STATIC_MAX_ROWS) return static_fail(GCR_EINVAL, "ny must be in [2, %d], got %d", STATIC_MAX_ROWS, ny);
  if ((long long)nx * ny > STATIC_MAX_POINTS)
    return static_fail(GCR_EINVAL, "nx * ny = %lld exceeds the static work array's %lld points",
                       (long long)nx * ny, STATIC_MAX_POINTS);
  if (richardson_iters < 1 || richardson_iters > 16)
    return static_fail(GCR_EINVAL, "richardson_iters must be in [1, 16], got %d", richardson_iters);
  if (!op->depth || !op->mem_is_device) return static_fail(GCR_EINVAL, "depth must be a device pointer");
  if (op->orography && !op->mem_is_device) return static_fail(GCR_EINVAL, "orography must be a device pointer");
  if (!(op->dt > 0.0) || !(op->g > 0.0) || !(op->radius > 0.0) || !std::isfinite(op->omega) ||
      !(op->absorber >= 0.0) || !std::isfinite(op->dt * op->g * op->radius * op->absorber))
    return static_fail(GCR_EINVAL, "dt, g, radius must be > 0, absorber >= 0, all finite");
  if ((const void*)r == (const void*)e) return static_fail(GCR_EINVAL, "input and output must not alias");
  unsigned char* base = nullptr;
  int rc = scratch_address(&base);
  if (rc != GCR_OK) return rc;
  hipStream_t st = (hipStream_t)stream;

  MemberGeom G{};
  G.nx = nx;
  G.ny = ny;
  G.log2nx = log2i(nx);
  G.log2m = std::max(1, G.log2nx - 6);
  G.polar = std::min(std::max(1, log2i(std::max(ny / 32, 1))), ny);
  G.off = 0;
  G.row0 = 0;
  AsmMember A{};
  A.depth = op->depth;
  A.oro = op->orography;
  A.dt = op->dt;
  A.g = op->g;
  A.omega = op->omega;
  A.radius = op->radius;
  A.absorber = op->absorber;
  A.member = 0;
  A.b_terms = op->b_terms ? 1 : 0;

  MemberGeom* geom = (MemberGeom*)(base + LAY.geom);
  AsmMember* tab = (AsmMember*)(base + LAY.asmtab);
  MemberState* state = (MemberState*)(base + LAY.state);
  int* rowmap = (int*)(base + LAY.rowmap);
  hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(256), 0, st, G, A, geom, tab, rowmap, state);

  AssembleArgs AA{};
  AA.tab = tab;
  AA.geom = geom;
  for (int k = 0; k < NCOEF; ++k) {
    AA.a16[k] = (__half*)(base + LAY.a16 + k * up((size_t)STATIC_MAX_POINTS * sizeof(__half)));
    AA.a32[k] = (float*)(base + LAY.a32 + k * up((size_t)STATIC_MAX_POINTS * sizeof(float)));
  }
  AA.c64 = (double*)(base + LAY.c64);
  AA.c32 = (float*)(base + LAY.c32);
  AA.scale = (double*)(base + LAY.scale);
  AA.phi64 = (double*)(base + LAY.phi64);
  AA.hs64 = (double*)(base + LAY.hs64);
  AA.phi32 = (float*)(base + LAY.phi32);
  AA.hs32 = (float*)(base + LAY.hs32);
  AA.fac64 = (double*)(base + LAY.fac64);
  AA.fac32 = (float*)(base + LAY.fac32);
  AA.flat = (int*)(base + LAY.flat);
  // rows per workgroup: as many as the staged rows fit in 64 KiB of LDS
  const size_t row_bytes = (op->orography ? 2 : 1) * (size_t)asm_row_lds(nx) * sizeof(double);
  AA.rows = ASM_ROWS;
  while (AA.rows > 1 && (AA.rows + 2) * row_bytes > 65536) --AA.rows;
  const size_t lds = (AA.rows + 2) * row_bytes;
  hipLaunchKernelGGL(k_assemble, dim3((ny + AA.rows - 1) / AA.rows, 1), dim3(ASM_WG), lds, st, AA);

  Fields F{};
  F.geom = geom;
  F.rowmap = rowmap;
  F.state = state;
  F.part = (double*)(base + LAY.part);
  F.scale = AA.scale;
  F.fly64 = FlyPools<double>{AA.phi64, AA.hs64, AA.fac64, AA.c64, AA.flat};
  F.fly32 = FlyPools<float>{AA.phi32, AA.hs32, AA.fac32, AA.c32, AA.flat};
  for (int k = 0; k < NCOEF; ++k) {
    F.cmx.h[k] = AA.a16[k];
    F.cmx.f[k] = AA.a32[k];
  }
  F.cmx.c = AA.c32;
  F.r = base + LAY.r;
  F.e = base + LAY.e;
  F.q[0] = base + LAY.q0;
  F.q[1] = base + LAY.q1;
  F.row_base = 0;
  F.row_end = ny;
  F.ignore_done = 1;

  const long long n = (long long)nx * ny;
  const dim3 cg((unsigned)std::min<long long>((n + 255) / 256, 1024)), cb(256);
  hipLaunchKernelGGL(k_to_pool, cg, cb, 0, st, r, (double*)F.r, G);
  const bool flat = op->orography == nullptr;
  switch (G.log2m * 2 + (flat ? 1 : 0)) {
    case 2: launch_rows<2, false>(F, ny, richardson_iters, st); break;
    case 3: launch_rows<2, true>(F, ny, richardson_iters, st); break;
    case 4: launch_rows<4, false>(F, ny, richardson_iters, st); break;
    case 5: launch_rows<4, true>(F, ny, richardson_iters, st); break;
    case 6: launch_rows<8, false>(F, ny, richardson_iters, st); break;
    case 7: launch_rows<8, true>(F, ny, richardson_iters, st); break;
    case 9: launch_rows<16, true>(F, ny, richardson_iters, st); break;
    default: launch_rows<16, false>(F, ny, richardson_iters, st); break;
  }
  hipLaunchKernelGGL(k_from_pool, cg, cb, 0, st, (const double*)F.e, e, G);
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess) return static_fail(GCR_EHIP, "launch: %s", hipGetErrorString(le));
  return GCR_OK;
}
