// Device-side building blocks of the GCR(k) depth solver for gfx950.
//
// Layout of every field: one pooled allocation per field for the whole batch,
// member m occupying [geom.off, geom.off + nx*ny), row-major [NY][NX] with
// longitude fastest (within a row, points are interleaved by lane, see
// below).  Work is distributed one latitude row per wave64 (four rows per
// 256-thread workgroup, no workgroup barriers): the zonal cyclic tridiagonal
// solves of the preconditioner couple a whole row, and the stencil needs rows
// j-1..j+1.  Lane l of a row owns the M = max(2, NX/64) contiguous points
// [l*M, (l+1)*M); the L = NX/M lanes of a row exchange chunk edges with
// cross-lane shuffles.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace mpgcr {

constexpr int WG = 256;             // threads per workgroup
constexpr int WPB = WG / 64;        // rows (waves) per workgroup
constexpr int KMAX = 8;             // largest GCR(k) window
constexpr int NXMAX = 1024;         // longest row (one wave, 16 points per lane)
constexpr int CH = 32;              // channels per pixel of the learned network's tensors

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Slots of the per-row partial inner-product buffer.
constexpr int DOT_RR = 0;               // <r, r> after the step-2 update
constexpr int DOT_LE_LP = 1;            // <L e, L p_l>, l = 0..k-1  -> slots 1..KMAX
constexpr int DOT_R_LP = KMAX + 1;      // <r, L p_new>
constexpr int DOT_LP_LP = KMAX + 2;     // <L p_new, L p_new>
constexpr int DOT_RMAX = KMAX + 3;      // max |r| (maximum-norm exit test only)
constexpr int NDOT = KMAX + 4;

// Face-coefficient arrays, each [NY][NX], pre-divided by the grid factors of
// the difference they multiply, so the stencil is weights x differences:
//   AXX = A^xx_e/dlam^2, AXY = A^xy_e/(4 dlam dphi), BX = B^x_e/(2 dlam)  (east faces)
//   AYY = A^yy_n/dphi^2, AYX = A^yx_n/(4 dlam dphi), BY = B^y_n/(2 dphi)  (north faces;
//   row NY-1 is the pole face and holds zeros)
enum { C_AXX = 0, C_AXY, C_BX, C_AYY, C_AYX, C_BY, NCOEF };

struct MemberGeom {
  int nx, ny, log2nx, polar;  // polar: rows per pole held in float32 (mixed forms)
  long long off;              // first point of the member in pooled fields (multiple of 64)
  int row0;                   // first global row of the member
  int log2m;                  // points per lane M = 1 << log2m
};

// Per-member solver state kept on the device between kernels.
struct MemberState {
  double rho0;                // ||r_0||
  double rn;                  // ||r|| after the last step-2 update
  double rn_cycle;            // ||r|| at the start of the current cycle
  double beta;                // next step-2 coefficient
  double alpha[KMAX];         // step-4 coefficients of the current iteration
  double lpsq[KMAX + 1];      // <L p_l, L p_l> per ring slot
  double rtrue;               // ||L x - R|| recomputed in float64
  double rho0_inf;            // max |r_0| (maximum-norm exit test)
  double sigma;               // RMS of r (learned preconditioner scaling)
  int it, status, done, restarts;
  int fallback, pad1, pad2, pad3;
};

// Step-2 solution updates of the current cycle not yet applied to x, per member.
struct Pending {
  double beta[KMAX];
  int slot[KMAX];             // ring slots of their directions
  int n;
  int cycle;                  // the GCR cycle they belong to
  int by_orth;                // applied by the cycle's last step-4 pass (the member went on)
  int pad;
};

// Quotient a / b: exact in float64; in float32 (the mixed forms' row solves,
// whose inputs are stored in float16) the hardware reciprocal, which is
// within 1 ulp, times a.
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8), and each XCD has its own L2.  Row kernels read the rows above and
// below their own, so the logical block order is remapped to give every XCD
// one contiguous range of blocks: neighbouring rows then meet in the same L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int q = n / NXCD, r = n % NXCD, x = b % NXCD;
  return x * q + (x < r ? x : r) + b / NXCD;
}

// ---------------------------------------------------------------------------
// cross-lane helpers (wave64)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, 64);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// ---------------------------------------------------------------------------
// Row-interleaved storage.  Every internal field stores row point
// i = l*M + k (lane l's k-th point) at offset k*L + l of the row, where
// M = max(2, NX/64) points per lane and L = NX/M lanes (64 for NX >= 128).
// Lane l's loads of row[l + L*k], k = 0..M-1, are then fully coalesced and
// return its contiguous chunk of points [l*M, l*M + M): stencil neighbours
// in longitude are in registers except at chunk edges (one shuffle), and the
// cyclic row solves work on the chunks directly.  Caller-facing fields keep
// the natural [NY][NX] layout; the library permutes on entry and exit.
// Idle lanes (l >= L, only for NX < 128) mirror lane l & (L-1) for loads and
// never store.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int row_slot(int i, int log2m, int L) {   // natural column -> stored offset
  return (i & ((1 << log2m) - 1)) * L + (i >> log2m);
}

// Element k of lane l sits at row + k*L + l.  Rows are read and written with
// raw buffer instructions: the (wave-uniform) row start goes into a scalar
// buffer descriptor, the per-k part k*L into the scalar offset, and the lane
// part is one unsigned vector offset shared by every k -- no per-access
// address arithmetic on the vector ALUs.  The descriptor's extent is the row
// (NX elements), so the hardware drops any access outside it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), (short)0, (int)bytes, 0x00020000);
}

template <typename S>
struct RowIO;
template <>
struct RowIO<float> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
  template <int AUX>
  static __device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, AUX);
  }
};
template <>
struct RowIO<double> {
  typedef unsigned B __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  template <int AUX>
  static __device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, v), r, vo, so, AUX);
  }
};
template <>
struct RowIO<__half> {
  static __device__ __forceinline__ __half ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
  }
  template <int AUX>
  static __device__ __forceinline__ void st(__half v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, vo, so, AUX);
  }
};

template <typename S, typename T>
__device__ __forceinline__ T from_store(S v) { return (T)v; }
template <typename S, typename T>
__device__ __forceinline__ S to_store(T v) { return (S)v; }
template <>
__device__ __forceinline__ float from_store<__half, float>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ double from_store<__half, double>(__half v) { return (double)__half2float(v); }
template <>
__device__ __forceinline__ __half to_store<__half, float>(float v) { return __float2half_rn(v); }
template <>
__device__ __forceinline__ __half to_store<__half, double>(double v) { return __float2half_rn((float)v); }

template <int M, typename S, typename T>
__device__ __forceinline__ void ldr(const S* row, int l, int L, T (&v)[M]) {
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, (unsigned)(M * L) * sizeof(S));
  const unsigned vo = (unsigned)l * sizeof(S);
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = from_store<S, T>(RowIO<S>::ld(r, vo, (unsigned)(k * L) * sizeof(S)));
}
// Row stores are nontemporal (cache policy bit NT) where the rows stream
// through HBM rather than stay in the 256 MB memory-side cache: float64 rows,
// and every row of 1024-point rows (16 points per lane).  Measured on the
// float64 form at 64 x 512x256 (+4%) and at 64 x 1024x512 (+2% in both forms);
// for float32 and float16 rows of the 512-point class, which the next kernel
// reads back from that cache, they measured no gain.
template <int M, int BYTES>
constexpr int row_store_aux() { return (BYTES == 8 || M >= 16) ? 2 : 0; }

template <int M, typename S, typename T>
__device__ __forceinline__ void str(S* row, int l, int L, const T (&v)[M]) {
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, (unsigned)(M * L) * sizeof(S));
  const unsigned vo = (unsigned)l * sizeof(S);
#pragma unroll
  for (int k = 0; k < M; ++k)
    RowIO<S>::template st<row_store_aux<M, (int)sizeof(S)>()>(to_store<S, T>(v[k]), r, vo, (unsigned)(k * L) * sizeof(S));
}

// float16 rows pair their elements: (k, k+1) of lane l (k even) share the
// 32-bit word at half offset (k/2)*2L + 2l, so one load or store moves two
// values of a lane and the wave still touches one contiguous 256-byte span.
__device__ __forceinline__ int half_slot(int l, int k, int L) { return (k >> 1) * 2 * L + 2 * l + (k & 1); }

template <int M, typename T>
__device__ __forceinline__ void ldr(const __half* row, int l, int L, T (&v)[M]) {
  static_assert(M % 2 == 0, "float16 rows hold element pairs");
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, (unsigned)(M * L) * 2u);
  const unsigned vo = (unsigned)l * 4u;
#pragma unroll
  for (int j = 0; j < M / 2; ++j) {
    const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(r, vo, (unsigned)(j * L) * 4u, 0);
    v[2 * j] = (T)__half2float(__builtin_bit_cast(__half, (unsigned short)(w & 0xffffu)));
    v[2 * j + 1] = (T)__half2float(__builtin_bit_cast(__half, (unsigned short)(w >> 16)));
  }
}
template <int M, typename T>
__device__ __forceinline__ void str(__half* row, int l, int L, const T (&v)[M]) {
  static_assert(M % 2 == 0, "float16 rows hold element pairs");
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, (unsigned)(M * L) * 2u);
  const unsigned vo = (unsigned)l * 4u;
#pragma unroll
  for (int j = 0; j < M / 2; ++j) {
    const unsigned lo16 = __builtin_bit_cast(unsigned short, __float2half_rn((float)v[2 * j]));
    const unsigned hi16 = __builtin_bit_cast(unsigned short, __float2half_rn((float)v[2 * j + 1]));
    __builtin_amdgcn_raw_buffer_store_b32(lo16 | (hi16 << 16), r, vo, (unsigned)(j * L) * 4u, row_store_aux<M, 2>());
  }
}

// the same row seen across the pole: longitude shifted by NX/2 = (L/2)*M,
// i.e. the chunk of lane l + L/2
template <int M, typename T>
__device__ __forceinline__ void across_pole(const T (&v)[M], T (&o)[M], int l, int L) {
  const int src = (l + (L >> 1)) & (L - 1);
#pragma unroll
  for (int k = 0; k < M; ++k) o[k] = shfl(v[k], src);
}

// value at longitude i-1 / i+1 for every point of the lane's chunk
template <int M, typename T>
__device__ __forceinline__ void west_of(const T (&v)[M], T (&o)[M], int l, int L) {
  o[0] = shfl(v[M - 1], (l - 1) & (L - 1));
#pragma unroll
  for (int k = 1; k < M; ++k) o[k] = v[k - 1];
}
template <int M, typename T>
__device__ __forceinline__ void east_of(const T (&v)[M], T (&o)[M], int l, int L) {
  o[M - 1] = shfl(v[0], (l + 1) & (L - 1));
#pragma unroll
  for (int k = 0; k < M - 1; ++k) o[k] = v[k + 1];
}

// ---------------------------------------------------------------------------
// Row context of one wave.
// ---------------------------------------------------------------------------
struct RowCtx {
  int m, j, g, nx, ny, lane, L;
  long long rc;           // element offset of the start of row j
  bool south, north;      // row j-1 / row j+1 exist (otherwise: across the pole)
  bool act;               // lane owns points (lane < L)
};

__device__ __forceinline__ RowCtx make_row(const MemberGeom& G, int m, int g, int lane, int M) {
  RowCtx R;
  R.m = m;
  R.g = g;
  R.j = g - G.row0;
  R.nx = G.nx;
  R.ny = G.ny;
  R.L = G.nx / M;
  R.act = lane < R.L;
  R.lane = lane & (R.L - 1);
  R.rc = G.off + (long long)R.j * G.nx;
  R.south = R.j > 0;
  R.north = R.j < G.ny - 1;
  return R;
}

// ---------------------------------------------------------------------------
// Cyclic tridiagonal solve of one latitude row held by one wave.
//   lo_i x_{i-1} + di_i x_i + up_i x_{i+1} = rh_i   (indices mod NX)
// Partition method: lane l owns the M equations of points [lM, lM+M).
// 1. Its first M-1 unknowns are eliminated by a Thomas sweep with the lane's
//    last unknown y_l and the previous lane's last unknown y_{l-1} moved to
//    the right-hand side: x_k = f_k + g_k y_{l-1} + h_k y_l.  The forward
//    sweep runs while the equations are produced (push), so only the sweep's
//    factors are held in registers.
// 2. Substituting into the lane's last equation (which also needs f,g,h of
//    the next lane's first point) leaves one equation per lane coupling
//    y_{l-1}, y_l, y_{l+1}: a cyclic tridiagonal system of size L.
// 3. That system is solved by parallel cyclic reduction across the lanes
//    (shuffles); at stride L every equation reads (A+B+C) y_l = D.
// 4. Back substitution with y_{l-1} from the previous lane.
// The row systems of the preconditioner are strictly diagonally dominant, so
// every elimination step is stable.
// ---------------------------------------------------------------------------
template <typename T, int M>
struct RowSolver {
  static_assert(M >= 2, "at least two points per lane");
  T cp[M - 1], f[M - 1], g[M - 1], h[M - 1];
  T al, bl, cl, dl;   // the lane's last equation

  // equation k of the lane's chunk, in increasing k (k is a compile-time
  // constant after unrolling)
  __device__ __forceinline__ void push(int k, T lo, T di, T up, T rh) {
    if (k == M - 1) {
      al = lo;
      bl = di;
      cl = up;
      dl = rh;
      return;
    }
    // coupling to y_l moves to the right-hand side; it enters at point M-2,
    // so h is zero before it (not held in registers while rows stream in)
    if (k == 0) {
      const T inv = qdiv((T)1, di);
      cp[0] = up * inv;
      f[0] = rh * inv;
      g[0] = -lo * inv;
      h[0] = (k == M - 2) ? -up * inv : (T)0;
    } else {
      const T inv = qdiv((T)1, di - lo * cp[k - 1]);
      cp[k] = up * inv;
      f[k] = (rh - lo * f[k - 1]) * inv;
      g[k] = (-lo * g[k - 1]) * inv;
      h[k] = (k == M - 2) ? -up * inv : (T)0;
    }
  }

  __device__ __forceinline__ void solve(int lane, int L, T (&x)[M]) {
#pragma unroll
    for (int k = M - 3; k >= 0; --k) {
      f[k] -= cp[k] * f[k + 1];
      g[k] -= cp[k] * g[k + 1];
      h[k] -= cp[k] * h[k + 1];
    }
    const int nxt = (lane + 1) & (L - 1), prv = (lane - 1 + L) & (L - 1);
    const T fn = shfl(f[0], nxt), gn = shfl(g[0], nxt), hn = shfl(h[0], nxt);
    T A = al * g[M - 2];
    T B = al * h[M - 2] + bl + cl * gn;
    T C = cl * hn;
    T D = dl - al * f[M - 2] - cl * fn;
    for (int s = 1; s < L; s <<= 1) {
      const int im = (lane - s + L) & (L - 1), ip = (lane + s) & (L - 1);
      const T Am = shfl(A, im), Bm = shfl(B, im), Cm = shfl(C, im), Dm = shfl(D, im);
      const T Ap = shfl(A, ip), Bp = shfl(B, ip), Cp = shfl(C, ip), Dp = shfl(D, ip);
      const T k1 = qdiv(A, Bm), k2 = qdiv(C, Bp);
      B = B - k1 * Cm - k2 * Ap;
      D = D - k1 * Dm - k2 * Dp;
      A = -k1 * Am;
      C = -k2 * Cp;
    }
    const T y = qdiv(D, A + B + C);
    const T ym = shfl(y, prv);
#pragma unroll
    for (int k = 0; k < M - 1; ++k) x[k] = f[k] + g[k] * ym + h[k] * y;
    x[M - 1] = y;
  }
};

}  // namespace mpgcr
