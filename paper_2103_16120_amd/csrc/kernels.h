// Kernels of the GCR(k) depth solver (gfx950).  Row kernels map one latitude
// row to one wave64 (four rows per workgroup); a batch of independent members
// is one flat list of rows, `rowmap[g]` giving the member of global row g.
#pragma once

#include <type_traits>

#include "device.h"

namespace mpgcr {

// kernel kinds for the optional per-kernel timing (values match the header)
enum {
  KT_ASSEMBLE = 0, KT_RESIDUAL, KT_SWEEP1, KT_SWEEP2, KT_APPLY_L, KT_ORTH, KT_CONTROL, KT_COPY, KT_LEARNED,
  KT_SOLUTION, KT_SI_STEP, KT_COUNT
};

// ---------------------------------------------------------------------------
// precision-specific coefficient access (wave-uniform choice per row)
// ---------------------------------------------------------------------------

// float16 storage in the interior, float32 in the polar rows, float32 maths.
struct CoefMixed {
  const __half* h[NCOEF];
  const float* f[NCOEF];
  const float* c;             // scaled Helmholtz coefficient per global row (float32)
};

// Coefficient rows of one storage precision (chosen once per row).
template <typename S, typename T>
struct CoefRow {
  const S* const* a;          // NCOEF arrays
  const T* c;                 // Helmholtz coefficient per global row
  template <int M>
  __device__ __forceinline__ void row(int k, long long start, int l, int L, T (&v)[M]) const {
    ldr<M>(a[k] + start, l, L, v);
  }
  __device__ __forceinline__ T helm(int g) const { return c[g]; }
  // A^xx east faces and A^yy north / south faces of row R (row solves)
  template <int M>
  __device__ __forceinline__ void faces(const RowCtx& R, T (&axe)[M], T (&ayn)[M], T (&ays)[M]) const {
    const int l = R.lane, L = R.L;
    row(C_AXX, R.rc, l, L, axe);
    row(C_AYY, R.rc, l, L, ayn);
    if (R.south) row(C_AYY, R.rc - R.nx, l, L, ays);
    else {
#pragma unroll
      for (int k = 0; k < M; ++k) ays[k] = (T)0;
    }
  }
  // the nine face-coefficient rows the stencil of row R needs
  template <int M>
  __device__ __forceinline__ void load9(const RowCtx& R, T (&axe)[M], T (&axy)[M], T (&bx)[M], T (&ayn)[M],
                                        T (&ayxn)[M], T (&byn)[M], T (&ays)[M], T (&ayxs)[M], T (&bys)[M]) const {
    const int l = R.lane, L = R.L;
    row(C_AXX, R.rc, l, L, axe);
    row(C_AXY, R.rc, l, L, axy);
    row(C_BX, R.rc, l, L, bx);
    row(C_AYY, R.rc, l, L, ayn);
    row(C_AYX, R.rc, l, L, ayxn);
    row(C_BY, R.rc, l, L, byn);
    if (R.south) {
      row(C_AYY, R.rc - R.nx, l, L, ays);
      row(C_AYX, R.rc - R.nx, l, L, ayxs);
      row(C_BY, R.rc - R.nx, l, L, bys);
    } else {           // the south pole face carries no flux
#pragma unroll
      for (int k = 0; k < M; ++k) {   // three stores: a chained assignment left a stack slot
        ays[k] = (T)0;
        ayxs[k] = (T)0;
        bys[k] = (T)0;
      }
    }
  }
};

// Coefficients computed on the fly from the depth fields: Phi* and H* =
// Phi* + H0 in the pooled row layout, and per global row the factors that
// depend on latitude only (written by k_assemble; the expressions below are
// the same as there).  East faces of row j use (FA_KE..FA_BPE), the north face
// j+1/2 uses (FA_KN..FA_BPN), all zero for the last row (no flux through the
// pole face).  Reading two fields instead of six coefficient arrays cuts the
// operator's bytes per point.
enum { FA_KE = 0, FA_FXX, FA_FXY, FA_GBX, FA_BLE, FA_BPE, FA_KN, FA_FYY, FA_FYX, FA_GBY, FA_BLN, FA_BPN, NFAC };

template <typename T>
struct FlyPools {
  const T* phi;               // Phi*, pooled
  const T* hs;                // H* = Phi* + H0, pooled (not written for members without orography)
  const T* fac;               // [rows][NFAC]
  const T* c;                 // Helmholtz coefficient per global row
  const int* flat;            // per member: 1 without orography (H* = Phi*: only Phi* is read)
};

template <typename T, bool FLAT_ONLY = false>
struct CoefFly {             // FLAT_ONLY: every member the launch covers has no orography
  FlyPools<T> P;
  __device__ __forceinline__ T helm(int g) const { return P.c[g]; }
  // A^xx east faces and A^yy north / south faces of row R (row solves)
  template <int M>
  __device__ __forceinline__ void faces(const RowCtx& R, T (&axe)[M], T (&ayn)[M], T (&ays)[M]) const {
    const int l = R.lane, L = R.L;
    T pc[M], pce[M], pn[M];
    ldr<M>(P.phi + R.rc, l, L, pc);
    if (R.north) ldr<M>(P.phi + R.rc + R.nx, l, L, pn);
    else across_pole(pc, pn, l, L);
    east_of(pc, pce, l, L);
    const T* f = P.fac + (long long)R.g * NFAC;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      axe[k] = (f[FA_KE] * (pc[k] + pce[k])) * f[FA_FXX];
      ayn[k] = (f[FA_KN] * (pc[k] + pn[k])) * f[FA_FYY];
    }
    if (R.south) {
      T ps[M];
      ldr<M>(P.phi + R.rc - R.nx, l, L, ps);
      const T* fs = P.fac + (long long)(R.g - 1) * NFAC;
#pragma unroll
      for (int k = 0; k < M; ++k) ays[k] = (fs[FA_KN] * (ps[k] + pc[k])) * fs[FA_FYY];
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) ays[k] = (T)0;
    }
  }
  // the nine face-coefficient rows the stencil of row R needs
  template <int M>
  __device__ __forceinline__ void load9(const RowCtx& R, T (&axe)[M], T (&axy)[M], T (&bx)[M], T (&ayn)[M],
                                        T (&ayxn)[M], T (&byn)[M], T (&ays)[M], T (&ayxs)[M], T (&bys)[M]) const {
    const int l = R.lane, L = R.L;
    T pc[M], ps[M], pn[M], hc[M], hsr[M], hn[M];
    const bool flat = P.flat[R.m] != 0;
    ldr<M>(P.phi + R.rc, l, L, pc);
    if (R.south) ldr<M>(P.phi + R.rc - R.nx, l, L, ps);
    else across_pole(pc, ps, l, L);
    if (R.north) ldr<M>(P.phi + R.rc + R.nx, l, L, pn);
    else across_pole(pc, pn, l, L);
    if (flat) {   // H* = Phi* exactly
#pragma unroll
      for (int k = 0; k < M; ++k) {
        hc[k] = pc[k];
        hsr[k] = ps[k];
        hn[k] = pn[k];
      }
    } else {
      ldr<M>(P.hs + R.rc, l, L, hc);
      if (R.south) ldr<M>(P.hs + R.rc - R.nx, l, L, hsr);
      else across_pole(hc, hsr, l, L);
      if (R.north) ldr<M>(P.hs + R.rc + R.nx, l, L, hn);
      else across_pole(hc, hn, l, L);
    }
    T pce[M], hce[M], hcw[M], hne[M], hnw[M], hse[M], hsw[M];
    east_of(pc, pce, l, L);
    east_of(hc, hce, l, L);
    west_of(hc, hcw, l, L);
    east_of(hn, hne, l, L);
    west_of(hn, hnw, l, L);
    east_of(hsr, hse, l, L);
    west_of(hsr, hsw, l, L);
    const T* f = P.fac + (long long)R.g * NFAC;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const T kap_e = f[FA_KE] * (pc[k] + pce[k]);
      axe[k] = kap_e * f[FA_FXX];
      axy[k] = kap_e * f[FA_FXY];
      bx[k] = f[FA_GBX] * (f[FA_BLE] * (hce[k] - hc[k]) + f[FA_BPE] * ((hn[k] - hsr[k]) + (hne[k] - hse[k])));
      const T kap_n = f[FA_KN] * (pc[k] + pn[k]);
      ayn[k] = kap_n * f[FA_FYY];
      ayxn[k] = kap_n * f[FA_FYX];
      byn[k] = f[FA_GBY] * (f[FA_BLN] * ((hce[k] - hcw[k]) + (hne[k] - hnw[k])) + f[FA_BPN] * (hn[k] - hc[k]));
    }
    if (R.south) {   // the south face is the north face of row j-1
      const T* fs = P.fac + (long long)(R.g - 1) * NFAC;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const T kap = fs[FA_KN] * (ps[k] + pc[k]);
        ays[k] = kap * fs[FA_FYY];
        ayxs[k] = kap * fs[FA_FYX];
        bys[k] = fs[FA_GBY] * (fs[FA_BLN] * ((hse[k] - hsw[k]) + (hce[k] - hcw[k])) + fs[FA_BPN] * (hc[k] - hsr[k]));
      }
    } else {         // the south pole face carries no flux
#pragma unroll
      for (int k = 0; k < M; ++k) {   // three stores: a chained assignment left a stack slot
        ays[k] = (T)0;
        ayxs[k] = (T)0;
        bys[k] = (T)0;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// precision forms
// ---------------------------------------------------------------------------
struct PrecF64 {              // everything float64
  using V = double;           // Krylov vectors
  using A = double;           // inner-product accumulation
  using Q = double;           // preconditioner intermediate storage
  using T = double;           // arithmetic
  static constexpr bool mixed = false;
  static constexpr bool op_f32 = false;   // operator coefficients in float32 (not float16)
  static constexpr bool pc_f32 = false;   // preconditioner coefficients in float32 (not float16)
  static constexpr bool polar64 = false;  // polar rows in float64 (Polar64<P>)
  static constexpr bool coef64 = false;   // scaled float64 coefficients (the polar rows of polar64 forms)
};
struct PrecMixed {            // float32 vectors and inner products, float16 coefficients
  using V = float;
  using A = float;
  using Q = __half;
  using T = float;
  static constexpr bool mixed = true;
  static constexpr bool op_f32 = false;
  static constexpr bool pc_f32 = false;
  static constexpr bool polar64 = false;
  static constexpr bool coef64 = false;
};
struct PrecMixedD {           // as PrecMixed with float64 inner products
  using V = float;
  using A = double;
  using Q = __half;
  using T = float;
  static constexpr bool mixed = true;
  static constexpr bool op_f32 = false;
  static constexpr bool pc_f32 = false;
  static constexpr bool polar64 = false;
  static constexpr bool coef64 = false;
};
struct PrecMixedP {           // as PrecMixedD, float16 only in the preconditioner
  using V = float;
  using A = double;
  using Q = __half;
  using T = float;
  static constexpr bool mixed = true;
  static constexpr bool op_f32 = true;
  static constexpr bool pc_f32 = false;
  static constexpr bool polar64 = false;
  static constexpr bool coef64 = false;
};
struct PrecSingle {           // float32 throughout the solver cycle (paper Section 4.2, option two)
  using V = float;
  using A = float;
  using Q = float;
  using T = float;
  static constexpr bool mixed = true;
  static constexpr bool op_f32 = true;
  static constexpr bool pc_f32 = true;
  static constexpr bool polar64 = false;
  static constexpr bool coef64 = false;
};
struct PrecSingleD : PrecSingle {   // as PrecSingle, float64 in the polar bands (option three)
  static constexpr bool polar64 = true;
};
// The polar rows of a polar64 form: float64 arithmetic on float64
// coefficients (scaled like the float32 ones), the form's storage types.
template <typename P>
struct Polar64 {
  using V = typename P::V;
  using A = double;
  using Q = typename P::Q;
  using T = double;
  static constexpr bool mixed = true;
  static constexpr bool op_f32 = false;
  static constexpr bool pc_f32 = false;
  static constexpr bool polar64 = false;
  static constexpr bool coef64 = true;
};

// float64 coefficients formed from the depth pools, times the member's scale
// dt/(2 a^2) (the mixed forms' units)
struct CoefScaled64 {
  CoefFly<double> cv;
  const double* scale;        // per member
  const int* rowmap;          // global row -> member
  __device__ __forceinline__ double helm(int g) const { return scale[rowmap[g]] * cv.helm(g); }
  template <int M>
  __device__ __forceinline__ void faces(const RowCtx& R, double (&axe)[M], double (&ayn)[M], double (&ays)[M]) const {
    cv.template faces<M>(R, axe, ayn, ays);
    const double s = scale[R.m];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      axe[k] *= s;
      ayn[k] *= s;
      ays[k] *= s;
    }
  }
  template <int M>
  __device__ __forceinline__ void load9(const RowCtx& R, double (&axe)[M], double (&axy)[M], double (&bx)[M],
                                        double (&ayn)[M], double (&ayxn)[M], double (&byn)[M], double (&ays)[M],
                                        double (&ayxs)[M], double (&bys)[M]) const {
    cv.template load9<M>(R, axe, axy, bx, ayn, ayxn, byn, ays, ayxs, bys);
    const double s = scale[R.m];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      axe[k] *= s;
      axy[k] *= s;
      bx[k] *= s;
      ayn[k] *= s;
      ayxn[k] *= s;
      byn[k] *= s;
      ays[k] *= s;
      ayxs[k] *= s;
      bys[k] *= s;
    }
  }
};

// Everything a kernel may touch, passed by value.
struct Fields {
  const MemberGeom* geom;
  const int* rowmap;
  MemberState* state;
  Pending* pend;              // per member: recorded step-2 updates (k_apply_pending)
  int* done_flag;             // per member: copy of state.done, what the host polls
  double* part;               // [rows][NDOT] per-row partial inner products
  const double* scale;        // per member: mixed-form operator scale dt/(2 a^2)
  CoefMixed cmx;
  FlyPools<double> fly64;     // on-the-fly coefficients (float64 operator)
  FlyPools<float> fly32;      // on-the-fly coefficients, scaled (float32 operator)
  double* x;                  // solution, float64 pool
  const double* rhs;          // right-hand side, float64 pool (stand-alone entry points)
  const double* const* rhs_tab;  // caller right-hand sides, natural [NY][NX] order, per member
  double* const* x_tab;       // caller solutions, natural order, per member
  double* r64;                // float64 residual (float64 form, restart scratch)
  void* r;                    // residual in the Krylov type
  void* e;                    // preconditioner output P^{-1}(r)
  void* le;                   // L(e)
  void* q[2];                 // preconditioner intermediates (Q type; V type for options 0-2)
  float* qs[2];               // per-row scales of q when stored as float16
  void* p[KMAX + 1];          // direction ring
  void* lp[KMAX + 1];         // L(direction) ring
  float* dx;                  // float32 solution increments (GCR_MIXED)
  double* hist;               // [batch][hist_stride] recursive residual history, or null
  int hist_stride;
  int row_base;               // global row handled by wave 0 of workgroup 0
  int row_end;                // one past the last global row of the launch
  int ignore_done;            // process finished members too (stand-alone operator calls)
  const int* morder;          // members in row order (control kernels: block b -> morder[q0 + b])
  int q0;
  int learned;                // learned preconditioner active (fallback test at cycle ends)
  int linf;                   // exit test in the maximum norm (max |r| partials kept)
  double fallback_ratio;      // required residual reduction per cycle with it
  const double* learn_ref;    // reference relative residual after iteration i (plain preconditioner), or null
  int learn_ref_n;            // entries 1..learn_ref_n of learn_ref are set
  int* cyc;                   // GCR cycle counter of the launch's member group (device; set to 0 by
                              // k_ctrl_init, advanced by k_cycle_next at every cycle end)
};

// Run fn(coefficient rows) for row j with the storage precision of the
// operator applied inside the Krylov iteration (`op`) or of the
// preconditioner; polar rows always use float32 in the mixed forms.  The
// choice is wave-uniform and made once per row.
template <typename P, bool FL = false, typename Fn>
__device__ __forceinline__ void with_coef(const Fields& F, const MemberGeom& G, int j, bool op, Fn&& fn) {
  if constexpr (!P::mixed) {
    fn(CoefFly<double, FL>{F.fly64});
  } else if constexpr (P::coef64) {
    fn(CoefScaled64{CoefFly<double>{F.fly64}, F.scale, F.rowmap});
  } else if constexpr (P::pc_f32) {   // float32 coefficients formed from the float32 depth, every row
    fn(CoefFly<float, FL>{F.fly32});
  } else {
    const bool f32 = (op && P::op_f32) || (j < G.polar) || (j >= G.ny - G.polar);
    if (f32) fn(CoefRow<float, float>{F.cmx.f, F.cmx.c});
    else fn(CoefRow<__half, float>{F.cmx.h, F.cmx.c});
  }
}

// Wave -> row assignment.  Returns false when the wave has no row or the
// row's member has finished.
__device__ __forceinline__ bool wave_row(const Fields& F, int& g, int& m, MemberGeom& G, int& lane, int& w) {
  lane = threadIdx.x & 63;
  w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  g = F.row_base + xcd_block(blockIdx.x, gridDim.x) * WPB + w;
  if (g >= F.row_end) return false;
  m = F.rowmap[g];
  G = F.geom[m];
  return F.ignore_done || F.state[m].done == 0;
}

// log2 of the points per lane of the wave's row (0 when the wave has no
// row): the row class a launch over several classes dispatches on
__device__ __forceinline__ int row_class(const Fields& F) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = F.row_base + xcd_block(blockIdx.x, gridDim.x) * WPB + w;
  if (g >= F.row_end) return 0;
  return __builtin_amdgcn_readfirstlane(F.geom[F.rowmap[g]].log2m);
}

// Field row readers for the stencil (row-interleaved storage), converted to T.
// Elements k and k+1 (k even) of lane `ln` of a pooled row of n elements: the
// streamed stencil reads rows column pair by column pair (float16 rows hold
// the pair in one word).
template <typename S, typename T>
__device__ __forceinline__ void ld_pair(const S* row, int n, int ln, int k, int L, T& a, T& b) {
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, (unsigned)n * sizeof(S));
  if constexpr (std::is_same<S, __half>::value) {
    const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(r, (unsigned)ln * 4u, (unsigned)((k >> 1) * L) * 4u, 0);
    a = (T)__half2float(__builtin_bit_cast(__half, (unsigned short)(w & 0xffffu)));
    b = (T)__half2float(__builtin_bit_cast(__half, (unsigned short)(w >> 16)));
  } else {
    const unsigned vo = (unsigned)ln * sizeof(S);
    a = from_store<S, T>(RowIO<S>::ld(r, vo, (unsigned)(k * L) * sizeof(S)));
    b = from_store<S, T>(RowIO<S>::ld(r, vo, (unsigned)((k + 1) * L) * sizeof(S)));
  }
}

template <typename T, typename S>
struct RowReader {
  const S* p;
  template <int M>
  __device__ __forceinline__ void row(long long start, int l, int L, T (&v)[M], int /*row_g*/) const {
    ldr<M>(p + start, l, L, v);
  }
  template <int M>
  __device__ __forceinline__ void pair(long long start, int n, int ln, int k, int L, int /*row_g*/, T& a, T& b) const {
    ld_pair<S, T>(p + start, n, ln, k, L, a, b);
  }
};

// Caller fields in natural [NY][NX] order: lane l loads points
// l*M .. l*M + M - 1 of a row, the same points its registers hold in the
// pooled layout, so the stencil code is shared.
template <int M>
__device__ __forceinline__ void ldn(const double* row, int l, double (&v)[M]) {
  const double* q = row + (long long)l * M;
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = q[k];
}

template <int M>
__device__ __forceinline__ void stn(double* row, int l, const double (&v)[M]) {
  double* q = row + (long long)l * M;
#pragma unroll
  for (int k = 0; k < M; ++k) q[k] = v[k];
}

struct NatReader {
  const double* p;            // the member's field, natural order
  long long off;              // pooled offset of the member's first point
  template <int M>
  __device__ __forceinline__ void row(long long start, int l, int /*L*/, double (&v)[M], int /*row_g*/) const {
    ldn<M>(p + (start - off), l, v);
  }
  template <int M>
  __device__ __forceinline__ void pair(long long start, int /*n*/, int ln, int k, int /*L*/, int /*row_g*/, double& a,
                                       double& b) const {
    const double* q = p + (start - off) + (long long)ln * M + k;
    a = q[0];
    b = q[1];
  }
};

// float16 storage with one scale per row
template <typename T>
struct ScaledHalfReader {
  const __half* p;
  const float* qs;
  template <int M>
  __device__ __forceinline__ void row(long long start, int l, int L, T (&v)[M], int row_g) const {
    ldr<M>(p + start, l, L, v);
    const T s = (T)qs[row_g];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] *= s;
  }
  template <int M>
  __device__ __forceinline__ void pair(long long start, int n, int ln, int k, int L, int row_g, T& a, T& b) const {
    ld_pair<__half, T>(p + start, n, ln, k, L, a, b);
    const T s = (T)qs[row_g];
    a *= s;
    b *= s;
  }
};

// ---------------------------------------------------------------------------
// 9-point stencil of the discrete L on one row (each lane: its chunk), split
// into
//   zon  = A^xx zonal second difference          (P^Z)
//   rest = meridional, cross and B terms         (P^M)
//   L    = zon + rest - C x                      (P^H = C x)
// delivered point by point, in chunk order, to emit(k, zon, rest, x, axe,
// axw, ayn, ays) together with the A^xx / A^yy faces the row solves need.
// Rows beyond the poles are the polar row seen across the pole.  The field
// rows are held whole (or streamed, below); the coefficients stream through
// per point.
// ---------------------------------------------------------------------------
template <bool A, typename X>
__device__ __forceinline__ X& pick(X& a, X& b) {
  if constexpr (A) return a;
  else return b;
}

// The stencil with the face coefficients formed point by point from the
// depth rows (on-the-fly coefficients): three rows of the field and three of
// Phi* (and three of H* with orography) instead of nine coefficient rows.
// The per-point expressions are those of CoefFly::load9.  FLAT: H* = Phi*.
template <typename T, int M, bool FLAT, typename CV, typename XR, typename Emit>
__device__ __forceinline__ void stencil_row_fly_whole(const RowCtx& R, const CV& cv, const XR& X, Emit&& emit) {
  const int l = R.lane, L = R.L;
  const int wl = (l - 1) & (L - 1), el = (l + 1) & (L - 1);
  T xc[M], xs[M], xn[M];
  X.row(R.rc, l, L, xc, R.g);
  if (R.south) X.row(R.rc - R.nx, l, L, xs, R.g - 1);
  if (R.north) X.row(R.rc + R.nx, l, L, xn, R.g + 1);
  T pc[M], ps[M], pn[M], hc_[M], hs_[M], hn_[M];
  const T* phi = cv.P.phi;
  ldr<M>(phi + R.rc, l, L, pc);
  if (R.south) ldr<M>(phi + R.rc - R.nx, l, L, ps);
  if (R.north) ldr<M>(phi + R.rc + R.nx, l, L, pn);
  if constexpr (!FLAT) {
    const T* hp = cv.P.hs;
    ldr<M>(hp + R.rc, l, L, hc_);
    if (R.south) ldr<M>(hp + R.rc - R.nx, l, L, hs_);
    if (R.north) ldr<M>(hp + R.rc + R.nx, l, L, hn_);
  }
  T(&hc)[M] = pick<FLAT>(pc, hc_);
  T(&hs)[M] = pick<FLAT>(ps, hs_);
  T(&hn)[M] = pick<FLAT>(pn, hn_);
  if (!R.south) {
    across_pole(xc, xs, l, L);
    across_pole(pc, ps, l, L);
    if constexpr (!FLAT) across_pole(hc_, hs_, l, L);
  }
  if (!R.north) {
    across_pole(xc, xn, l, L);
    across_pole(pc, pn, l, L);
    if constexpr (!FLAT) across_pole(hc_, hn_, l, L);
  }
  // chunk-edge neighbours from the adjacent lanes
  const T cw0 = shfl(xc[M - 1], wl), ceM = shfl(xc[0], el);
  const T sw0 = shfl(xs[M - 1], wl), seM = shfl(xs[0], el);
  const T nw0 = shfl(xn[M - 1], wl), neM = shfl(xn[0], el);
  const T pw0 = shfl(pc[M - 1], wl), peM = shfl(pc[0], el);
  T hcw0 = pw0, hceM = peM, hsw0, hseM, hnw0, hneM;
  if constexpr (!FLAT) {
    hcw0 = shfl(hc[M - 1], wl);
    hceM = shfl(hc[0], el);
  }
  hsw0 = shfl(hs[M - 1], wl);
  hseM = shfl(hs[0], el);
  hnw0 = shfl(hn[M - 1], wl);
  hneM = shfl(hn[0], el);
  // values at chunk index i in -1 .. M (the ends from the adjacent lanes)
  auto at = [](const T (&v)[M], int i, T w, T e) { return i < 0 ? w : (i >= M ? e : v[i]); };
  const T* f = cv.P.fac + (long long)R.g * NFAC;
  const T fKE = f[FA_KE], fXX = f[FA_FXX], fXY = f[FA_FXY], fGBX = f[FA_GBX], fBLE = f[FA_BLE], fBPE = f[FA_BPE];
  const T fKN = f[FA_KN], fYY = f[FA_FYY], fYX = f[FA_FYX], fGBY = f[FA_GBY], fBLN = f[FA_BLN], fBPN = f[FA_BPN];
  // the south face is the north face of row j-1; none at the south pole
  const T* fs = cv.P.fac + (long long)(R.south ? R.g - 1 : R.g) * NFAC;
  const T sKN = R.south ? fs[FA_KN] : (T)0, sYY = R.south ? fs[FA_FYY] : (T)0, sYX = R.south ? fs[FA_FYX] : (T)0;
  const T sGBY = R.south ? fs[FA_GBY] : (T)0, sBLN = R.south ? fs[FA_BLN] : (T)0,
          sBPN = R.south ? fs[FA_BPN] : (T)0;
  // east face of chunk point i (i = -1: the west face of point 0)
  auto east = [&](int i, T& axe, T& axy, T& bx) {
    const T kap_e = fKE * (at(pc, i, pw0, peM) + at(pc, i + 1, pw0, peM));
    axe = kap_e * fXX;
    axy = kap_e * fXY;
    bx = fGBX * (fBLE * (at(hc, i + 1, hcw0, hceM) - at(hc, i, hcw0, hceM)) +
                 fBPE * ((at(hn, i, hnw0, hneM) - at(hs, i, hsw0, hseM)) +
                         (at(hn, i + 1, hnw0, hneM) - at(hs, i + 1, hsw0, hseM))));
  };
  T axe_p, axy_p, bx_p;
  east(-1, axe_p, axy_p, bx_p);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    T axe, axy, bx;
    east(k, axe, axy, bx);
    const T hce = at(hc, k + 1, hcw0, hceM), hcw = at(hc, k - 1, hcw0, hceM);
    const T kap_n = fKN * (pc[k] + pn[k]);
    const T ayn = kap_n * fYY, ayxn = kap_n * fYX;
    const T byn = fGBY * (fBLN * ((hce - hcw) + (at(hn, k + 1, hnw0, hneM) - at(hn, k - 1, hnw0, hneM))) +
                          fBPN * (hn[k] - hc[k]));
    const T kap_s = sKN * (ps[k] + pc[k]);
    const T ays = kap_s * sYY, ayxs = kap_s * sYX;
    const T bys = sGBY * (sBLN * ((at(hs, k + 1, hsw0, hseM) - at(hs, k - 1, hsw0, hseM)) + (hce - hcw)) +
                          sBPN * (hc[k] - hs[k]));
    const T c = xc[k], w = k > 0 ? xc[k - 1] : cw0, e = k < M - 1 ? xc[k + 1] : ceM;
    const T sc = xs[k], sw = k > 0 ? xs[k - 1] : sw0, se = k < M - 1 ? xs[k + 1] : seM;
    const T nc = xn[k], nw = k > 0 ? xn[k - 1] : nw0, ne = k < M - 1 ? xn[k + 1] : neM;
    const T zon = axe * (e - c) - axe_p * (c - w);
    T r = axy * ((nc - sc) + (ne - se)) - axy_p * ((nw - sw) + (nc - sc));
    r += bx * (c + e) - bx_p * (w + c);
    r += ayn * (nc - c) + ayxn * ((e - w) + (ne - nw)) + byn * (c + nc);
    r -= ays * (c - sc) + ayxs * ((se - sw) + (e - w)) + bys * (sc + c);
    emit(k, zon, r, c, axe, axe_p, ayn, ays);
    axe_p = axe;
    axy_p = axy;
    bx_p = bx;
  }
}

// Streamed form: the rows pass column pair by column pair, each pair loaded
// one pair ahead, so a wave holds four columns of every row it reads instead
// of whole rows; the chunk-edge columns come from the adjacent lanes' chunks
// by loads of their own (instead of shuffles of held values).
template <typename T, int M, bool FLAT, typename CV, typename XR, typename Emit>
__device__ __forceinline__ void stencil_row_fly_stream(const RowCtx& R, const CV& cv, const XR& X, Emit&& emit) {
  const int l = R.lane, L = R.L, n = R.nx;
  const int lx = (l + (L >> 1)) & (L - 1);
  // centre, south and north rows: start, lane read by this lane, row index
  // (float16 row scale); a row beyond a pole is the polar row itself read
  // with the lanes shifted by L/2 (longitude + NX/2)
  const long long st[3] = {R.rc, R.south ? R.rc - R.nx : R.rc, R.north ? R.rc + R.nx : R.rc};
  const int lr[3] = {l, R.south ? l : lx, R.north ? l : lx};
  const int gr[3] = {R.g, R.south ? R.g - 1 : R.g, R.north ? R.g + 1 : R.g};
  struct Col {
    T x[3], p[3], h[3];
  };
  // columns k, k+1 (k even) of the lane `dl` lanes away: dl = -1 / +1 give the
  // chunk-edge columns of the adjacent lanes
  auto load_pair = [&](int k, int dl, Col& a, Col& b) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int ln = (lr[r] + dl) & (L - 1);
      X.template pair<M>(st[r], n, ln, k, L, gr[r], a.x[r], b.x[r]);
      ld_pair<T, T>(cv.P.phi + st[r], n, ln, k, L, a.p[r], b.p[r]);
      if constexpr (FLAT) {
        a.h[r] = a.p[r];
        b.h[r] = b.p[r];
      } else {
        ld_pair<T, T>(cv.P.hs + st[r], n, ln, k, L, a.h[r], b.h[r]);
      }
    }
  };
  const T* f = cv.P.fac + (long long)R.g * NFAC;
  const T fKE = f[FA_KE], fXX = f[FA_FXX], fXY = f[FA_FXY], fGBX = f[FA_GBX], fBLE = f[FA_BLE], fBPE = f[FA_BPE];
  const T fKN = f[FA_KN], fYY = f[FA_FYY], fYX = f[FA_FYX], fGBY = f[FA_GBY], fBLN = f[FA_BLN], fBPN = f[FA_BPN];
  // the south face is the north face of row j-1; none at the south pole
  const T* fs = cv.P.fac + (long long)(R.south ? R.g - 1 : R.g) * NFAC;
  const T sKN = R.south ? fs[FA_KN] : (T)0, sYY = R.south ? fs[FA_FYY] : (T)0, sYX = R.south ? fs[FA_FYX] : (T)0;
  const T sGBY = R.south ? fs[FA_GBY] : (T)0, sBLN = R.south ? fs[FA_BLN] : (T)0,
          sBPN = R.south ? fs[FA_BPN] : (T)0;
  // east face of column c (e: the next column)
  auto east = [&](const Col& c, const Col& e, T& axe, T& axy, T& bx) {
    const T kap_e = fKE * (c.p[0] + e.p[0]);
    axe = kap_e * fXX;
    axy = kap_e * fXY;
    bx = fGBX * (fBLE * (e.h[0] - c.h[0]) + fBPE * ((c.h[2] - c.h[1]) + (e.h[2] - e.h[1])));
  };
  T axe_p, axy_p, bx_p;
  auto point = [&](int k, const Col& w, const Col& c, const Col& e) {
    T axe, axy, bx;
    east(c, e, axe, axy, bx);
    const T hce = e.h[0], hcw = w.h[0];
    const T kap_n = fKN * (c.p[0] + c.p[2]);
    const T ayn = kap_n * fYY, ayxn = kap_n * fYX;
    const T byn = fGBY * (fBLN * ((hce - hcw) + (e.h[2] - w.h[2])) + fBPN * (c.h[2] - c.h[0]));
    const T kap_s = sKN * (c.p[1] + c.p[0]);
    const T ays = kap_s * sYY, ayxs = kap_s * sYX;
    const T bys = sGBY * (sBLN * ((e.h[1] - w.h[1]) + (hce - hcw)) + sBPN * (c.h[0] - c.h[1]));
    const T xc = c.x[0], xw = w.x[0], xe = e.x[0];
    const T sc = c.x[1], sw = w.x[1], se = e.x[1];
    const T nc = c.x[2], nw = w.x[2], ne = e.x[2];
    const T zon = axe * (xe - xc) - axe_p * (xc - xw);
    T r = axy * ((nc - sc) + (ne - se)) - axy_p * ((nw - sw) + (nc - sc));
    r += bx * (xc + xe) - bx_p * (xw + xc);
    r += ayn * (nc - xc) + ayxn * ((xe - xw) + (ne - nw)) + byn * (xc + nc);
    r -= ays * (xc - sc) + ayxs * ((se - sw) + (xe - xw)) + bys * (sc + xc);
    emit(k, zon, r, xc, axe, axe_p, ayn, ays);
    axe_p = axe;
    axy_p = axy;
    bx_p = bx;
  };
  // columns k-1, k, k+1 in flight at point k; the next pair is loaded one
  // pair ahead, so a wave holds four columns instead of whole rows
  Col cm, c0, c1;
  {
    Col t;
    load_pair(M - 2, -1, t, cm);   // column -1: the west lane's last column
  }
  load_pair(0, 0, c0, c1);
  east(cm, c0, axe_p, axy_p, bx_p);
#pragma unroll
  for (int kp = 0; kp < M; kp += 2) {
    Col n0, n1;
    if (kp + 2 < M) load_pair(kp + 2, 0, n0, n1);
    else load_pair(0, 1, n0, n1);   // column M: the east lane's first column
    point(kp, cm, c0, c1);
    point(kp + 1, c0, c1, n0);
    cm = c1;
    c0 = n0;
    c1 = n1;
  }
}

// Whole rows or streamed columns: streaming pays where whole float64 rows of
// 16 points per lane would leave one wave per SIMD (measured: the float64
// operator and second sweep at 1024 points per row); elsewhere the whole-row
// form keeps more loads in flight per wave and is faster.
template <typename T, int M>
constexpr bool stream_stencil() { return sizeof(T) == 8 && M >= 16; }

template <typename T, int M, bool FLAT, bool WHOLE, typename CV, typename XR, typename Emit>
__device__ __forceinline__ void stencil_row_fly(const RowCtx& R, const CV& cv, const XR& X, Emit&& emit) {
  if constexpr (!WHOLE && stream_stencil<T, M>()) stencil_row_fly_stream<T, M, FLAT>(R, cv, X, emit);
  else stencil_row_fly_whole<T, M, FLAT>(R, cv, X, emit);
}

template <typename T>
struct is_coef_fly : std::false_type {
  static constexpr bool flat_only = false;
};
template <typename T, bool B>
struct is_coef_fly<CoefFly<T, B>> : std::true_type {
  static constexpr bool flat_only = B;
};

// WHOLE: always hold whole rows (the float64 residual: streaming measured slower)
template <typename T, int M, bool WHOLE = false, typename CV, typename XR, typename Emit>
__device__ __forceinline__ void stencil_row(const RowCtx& R, const CV& cv, const XR& X, Emit&& emit) {
  if constexpr (is_coef_fly<CV>::value) {
    if constexpr (is_coef_fly<CV>::flat_only) stencil_row_fly<T, M, true, WHOLE>(R, cv, X, emit);
    else if (cv.P.flat[R.m] != 0) stencil_row_fly<T, M, true, WHOLE>(R, cv, X, emit);
    else stencil_row_fly<T, M, false, WHOLE>(R, cv, X, emit);
    return;
  }
  const int l = R.lane, L = R.L;
  const int wl = (l - 1) & (L - 1), el = (l + 1) & (L - 1);
  T xc[M], xs[M], xn[M];
  X.row(R.rc, l, L, xc, R.g);
  if (R.south) X.row(R.rc - R.nx, l, L, xs, R.g - 1);
  if (R.north) X.row(R.rc + R.nx, l, L, xn, R.g + 1);
  T axe[M], axy[M], bx[M], ayn[M], ayxn[M], byn[M], ays[M], ayxs[M], bys[M];
  cv.template load9<M>(R, axe, axy, bx, ayn, ayxn, byn, ays, ayxs, bys);
  if (!R.south) across_pole(xc, xs, l, L);
  if (!R.north) across_pole(xc, xn, l, L);
  // chunk-edge neighbours from the adjacent lanes
  const T cw0 = shfl(xc[M - 1], wl), ceM = shfl(xc[0], el);
  const T sw0 = shfl(xs[M - 1], wl), seM = shfl(xs[0], el);
  const T nw0 = shfl(xn[M - 1], wl), neM = shfl(xn[0], el);
  T axe_p = shfl(axe[M - 1], wl), axy_p = shfl(axy[M - 1], wl), bx_p = shfl(bx[M - 1], wl);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const T c = xc[k], w = k > 0 ? xc[k - 1] : cw0, e = k < M - 1 ? xc[k + 1] : ceM;
    const T sc = xs[k], sw = k > 0 ? xs[k - 1] : sw0, se = k < M - 1 ? xs[k + 1] : seM;
    const T nc = xn[k], nw = k > 0 ? xn[k - 1] : nw0, ne = k < M - 1 ? xn[k + 1] : neM;
    const T zon = axe[k] * (e - c) - axe_p * (c - w);
    T r = axy[k] * ((nc - sc) + (ne - se)) - axy_p * ((nw - sw) + (nc - sc));
    r += bx[k] * (c + e) - bx_p * (w + c);
    r += ayn[k] * (nc - c) + ayxn[k] * ((e - w) + (ne - nw)) + byn[k] * (c + nc);
    r -= ays[k] * (c - sc) + ayxs[k] * ((se - sw) + (e - w)) + bys[k] * (sc + c);
    emit(k, zon, r, c, axe[k], axe_p, ayn[k], ays[k]);
    axe_p = axe[k];
    axy_p = axy[k];
    bx_p = bx[k];
  }
}

// A^xx (east, west) and A^yy (north, south) faces of a row, for the row
// systems when no stencil is evaluated.
template <typename T, int M, typename CV>
__device__ __forceinline__ void row_faces(const RowCtx& R, const CV& cv, T (&axe)[M], T (&axw)[M], T (&ayn)[M],
                                          T (&ays)[M]) {
  cv.template faces<M>(R, axe, ayn, ays);
  west_of(axe, axw, R.lane, R.L);
}

// diagonal of L on a row
template <typename T, int M, typename CV>
__device__ __forceinline__ void diag_row(const RowCtx& R, const CV& cv, T (&d)[M]) {
  const int l = R.lane, L = R.L;
  T axe[M], axw[M], axy[M], bx[M], bxw[M], ayn[M], ayxn[M], byn[M], ays[M], ayxs[M], bys[M];
  cv.template load9<M>(R, axe, axy, bx, ayn, ayxn, byn, ays, ayxs, bys);
  west_of(axe, axw, l, L);
  west_of(bx, bxw, l, L);
  const T helm = cv.helm(R.g);
#pragma unroll
  for (int k = 0; k < M; ++k)
    d[k] = -(axe[k] + axw[k]) + (bx[k] - bxw[k]) - ayn[k] + byn[k] - (ays[k] + bys[k]) - helm;
}

// T = I - eta (P^Z - P^H) at one point
template <typename T>
__device__ __forceinline__ void row_system(T eta, T axe, T axw, T helm, T& lo, T& di, T& up) {
  lo = -eta * axw;
  up = -eta * axe;
  di = (T)1 + eta * (axe + axw) + eta * helm;
}

// Solve the row systems (each lane holds its chunk of equations).
template <typename T, int M>
__device__ __forceinline__ void solve_row(const RowCtx& R, const T (&lo)[M], const T (&di)[M], const T (&up)[M],
                                          const T (&rh)[M], T (&x)[M]) {
  RowSolver<T, M> rs;
#pragma unroll
  for (int k = 0; k < M; ++k) rs.push(k, lo[k], di[k], up[k], rh[k]);
  rs.solve(R.lane, R.L, x);
}

// store a preconditioner intermediate (Q type; float16 with a per-row scale)
template <typename P, int M>
__device__ __forceinline__ void store_q(const Fields& F, int qout, const RowCtx& R, const typename P::T (&v)[M]) {
  using T = typename P::T;
  using Q = typename P::Q;
  Q* q = (Q*)F.q[qout] + R.rc;
  if constexpr (std::is_same<Q, __half>::value) {
    float mx = 0.f;
    if (R.act) {
#pragma unroll
      for (int k = 0; k < M; ++k) mx = fmaxf(mx, fabsf((float)v[k]));
    }
    mx = wave_max(mx);
    const float sc = mx > 0.f ? mx : 1.f;
    if (R.lane == 0 && R.act) F.qs[qout][R.g] = sc;
    const float inv = 1.f / sc;
    T t[M];
#pragma unroll
    for (int k = 0; k < M; ++k) t[k] = v[k] * inv;
    if (R.act) str<M>(q, R.lane, R.L, t);
  } else {
    if (R.act) str<M>(q, R.lane, R.L, v);
  }
}

template <typename P, int M>
__device__ __forceinline__ void store_v(void* dst, const RowCtx& R, const typename P::T (&v)[M]) {
  if (R.act) str<M>((typename P::V*)dst + R.rc, R.lane, R.L, v);
}

template <typename A>
__device__ __forceinline__ void write_partial(const Fields& F, const RowCtx& R, int slot, A v) {
  v = wave_sum(v);
  if (R.lane == 0 && R.act) F.part[(long long)R.g * NDOT + slot] = (double)v;
}

// the row's max |v| into slot DOT_RMAX (maximum-norm exit test)
template <int M, typename T>
__device__ __forceinline__ void write_row_max(const Fields& F, const RowCtx& R, const T (&v)[M], double scale) {
  double mx = 0.0;
  if (R.act) {
#pragma unroll
    for (int k = 0; k < M; ++k) mx = fmax(mx, fabs((double)v[k]));
  }
  mx = wave_max(mx);
  if (R.lane == 0 && R.act) F.part[(long long)R.g * NDOT + DOT_RMAX] = mx * scale;
}

// step 2 on one row: r += beta L p_nu ; returns r and <r,r>.  The solution
// update x += beta p_nu of the same step is deferred to k_apply_pending.
template <typename P, int M>
__device__ __forceinline__ typename P::A row_update(const Fields& F, const RowCtx& R, int slot_nu,
                                                    typename P::T (&rv)[M]) {
  using T = typename P::T;
  using V = typename P::V;
  using A = typename P::A;
  const int l = R.lane, L = R.L;
  const double beta = F.state[R.m].beta;
  V* r = (V*)F.r + R.rc;
  T lv[M];
  ldr<M>((const V*)F.lp[slot_nu] + R.rc, l, L, lv);
  A acc = (A)0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    rv[k] = (T)(V)(rv[k] + (T)beta * lv[k]);
    acc += (A)rv[k] * (A)rv[k];
  }
  if (R.act) str<M>(r, l, L, rv);
  if (F.linf) write_row_max<M>(F, R, rv, 1.0);
  return R.act ? acc : (A)0;
}

// ---------------------------------------------------------------------------
// The solution updates of step 2, x += beta p_nu, deferred to the end of the
// GCR cycle: k_ctrl_alpha records each update made (beta and the ring slot
// of p_nu, stamped with the cycle).  A member that goes on past the cycle's
// last iteration has them applied by that iteration's step-4 pass, which
// loads p_0 .. p_{k-1} anyway (k_orth); for the others (finished inside the
// cycle) this pass applies those of the current cycle (the group's counter).
// Either way before anything
// reads x (the restart and final residuals) and before the ring slots are
// reused.
// The float64 operations (GCR_MIXED: float32 increments) and their order are
// those of updating at every iteration; x is read and written once per cycle
// instead of once per iteration.  Finished members apply their last updates
// too.
// ---------------------------------------------------------------------------
template <typename P, int M>
__device__ __forceinline__ void kb_apply_pending(const Fields& F) {
  using T = typename P::T;
  using V = typename P::V;
  const int cycle = *F.cyc;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = F.row_base + xcd_block(blockIdx.x, gridDim.x) * WPB + w;
  if (g >= F.row_end) return;
  const int m = F.rowmap[g];
  const Pending& S = F.pend[m];
  const int n = (S.cycle == cycle && !S.by_orth) ? S.n : 0;
  if (n == 0) return;
  const RowCtx R = make_row(F.geom[m], m, g, lane, M);
  const int l = R.lane, L = R.L;
  if (P::mixed && F.dx) {
    float xv[M];
    ldr<M>(F.dx + R.rc, l, L, xv);
    for (int i = 0; i < n; ++i) {
      const double beta = S.beta[i];
      T pv[M];
      ldr<M>((const V*)F.p[S.slot[i]] + R.rc, l, L, pv);
#pragma unroll
      for (int k = 0; k < M; ++k) xv[k] += (float)beta * (float)pv[k];
    }
    if (R.act) str<M>(F.dx + R.rc, l, L, xv);
  } else {
    double xv[M];
    ldr<M>(F.x + R.rc, l, L, xv);
    for (int i = 0; i < n; ++i) {
      const double beta = S.beta[i];
      T pv[M];
      ldr<M>((const V*)F.p[S.slot[i]] + R.rc, l, L, pv);
#pragma unroll
      for (int k = 0; k < M; ++k) xv[k] += beta * (double)pv[k];
    }
    if (R.act) str<M>(F.x + R.rc, l, L, xv);
  }
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_apply_pending(Fields F) {
  if constexpr (M > 0) {
    kb_apply_pending<P, M>(F);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_apply_pending<P, 2>(F); break;
      case 2: kb_apply_pending<P, 4>(F); break;
      case 3: kb_apply_pending<P, 8>(F); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// step 2 + first semi-implicit Richardson iteration (q_0 = 0, eq. P_Operator):
//   (update)  r += beta L p_nu ; partial <r,r>  (x: k_apply_pending)
//   q1 = T^{-1}(-eta r),  T = I - eta (P^Z - P^H)
// `qout` = -1 writes the result to e (single Richardson iteration).
// ---------------------------------------------------------------------------
template <typename P, int M>
__device__ __forceinline__ void row_update_sweep1(const Fields& F, const RowCtx& R, const MemberGeom& G, int do_update,
                                                  int slot_nu, int qout) {
  using T = typename P::T;
  using V = typename P::V;
  using A = typename P::A;
  with_coef<P>(F, G, R.j, false, [&](const auto& cv) {
    const T helm = cv.helm(R.g);
    T rv[M];
    ldr<M>((const V*)F.r + R.rc, R.lane, R.L, rv);
    if (do_update) {
      const A acc = row_update<P, M>(F, R, slot_nu, rv);
      write_partial<A>(F, R, DOT_RR, acc);
    }
    T axe[M], axw[M], ayn[M], ays[M], lo[M], di[M], up[M], rh[M], xq[M];
    row_faces<T, M>(R, cv, axe, axw, ayn, ays);
  #pragma unroll
    for (int k = 0; k < M; ++k) {
      const T eta = qdiv((T)1, ayn[k] + ays[k]);
      row_system(eta, axe[k], axw[k], helm, lo[k], di[k], up[k]);
      rh[k] = -eta * rv[k];
    }
    solve_row<T, M>(R, lo, di, up, rh, xq);
    if (qout < 0) store_v<P, M>(F.e, R, xq);
    else store_q<P, M>(F, qout, R, xq);
  });
}

template <typename P, int M>
__device__ __forceinline__ void kb_update_sweep1(const Fields& F, int do_update, int slot_nu, int qout) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  if constexpr (P::polar64) {
    if (R.j < G.polar || R.j >= G.ny - G.polar) {
      row_update_sweep1<Polar64<P>, M>(F, R, G, do_update, slot_nu, qout);
      return;
    }
  }
  row_update_sweep1<P, M>(F, R, G, do_update, slot_nu, qout);
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_update_sweep1(Fields F, int do_update, int slot_nu, int qout) {
  if constexpr (M > 0) {
    kb_update_sweep1<P, M>(F, do_update, slot_nu, qout);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_update_sweep1<P, 2>(F, do_update, slot_nu, qout); break;
      case 2: kb_update_sweep1<P, 4>(F, do_update, slot_nu, qout); break;
      case 3: kb_update_sweep1<P, 8>(F, do_update, slot_nu, qout); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// later semi-implicit Richardson iterations (eq. P_Operator):
//   q_out = T^{-1}( q_in + eta (P^M q_in - r) )
// `qout` = -1 writes the final iterate to e.
// ---------------------------------------------------------------------------
template <typename P, int M, bool FL>
__device__ __forceinline__ void row_sweep2(const Fields& F, const RowCtx& R, const MemberGeom& G, int qin,
                                           int qout) {
  using T = typename P::T;
  using V = typename P::V;
  with_coef<P, FL>(F, G, R.j, false, [&](const auto& cv) {
    const T helm = cv.helm(R.g);
    const V* rrow = (const V*)F.r + R.rc;
    RowSolver<T, M> rs;
    // r: the whole row, or (streamed stencil) the current column pair
    T rv[stream_stencil<T, M>() ? 1 : M], r0, r1;
    if constexpr (!stream_stencil<T, M>()) ldr<M>(rrow, R.lane, R.L, rv);
    auto emit = [&](int k, T, T rest, T xc, T axe, T axw, T ayn, T ays) {
      T rk;
      if constexpr (stream_stencil<T, M>()) {
        if ((k & 1) == 0) ld_pair<V, T>(rrow, R.nx, R.lane, k, R.L, r0, r1);
        rk = (k & 1) ? r1 : r0;
      } else {
        rk = rv[k];
      }
      const T eta = qdiv((T)1, ayn + ays);
      T lo, di, up;
      row_system(eta, axe, axw, helm, lo, di, up);
      rs.push(k, lo, di, up, xc + eta * (rest - rk));
    };
    using Q = typename P::Q;
    if constexpr (std::is_same<Q, __half>::value) {
      ScaledHalfReader<T> X{(const __half*)F.q[qin], F.qs[qin]};
      stencil_row<T, M>(R, cv, X, emit);
    } else {
      RowReader<T, Q> X{(const Q*)F.q[qin]};
      stencil_row<T, M>(R, cv, X, emit);
    }
    T xq[M];
    rs.solve(R.lane, R.L, xq);
    if (qout < 0) store_v<P, M>(F.e, R, xq);
    else store_q<P, M>(F, qout, R, xq);
  });
}

template <typename P, int M, bool FL>
__device__ __forceinline__ void kb_sweep2(const Fields& F, int qin, int qout) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  if constexpr (P::polar64) {
    if (R.j < G.polar || R.j >= G.ny - G.polar) {
      row_sweep2<Polar64<P>, M, false>(F, R, G, qin, qout);
      return;
    }
  }
  row_sweep2<P, M, FL>(F, R, G, qin, qout);
}

template <typename P, int M, bool FL>
__global__ __launch_bounds__(WG) void k_sweep2(Fields F, int qin, int qout) {
  if constexpr (M > 0) {
    kb_sweep2<P, M, FL>(F, qin, qout);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_sweep2<P, 2, FL>(F, qin, qout); break;
      case 2: kb_sweep2<P, 4, FL>(F, qin, qout); break;
      case 3: kb_sweep2<P, 8, FL>(F, qin, qout); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// Fault injection for tests of the exit logic (paper Section 2.3: breakdown
// and a non-finite result stop the iteration): every member that has
// completed `at_it` iterations gets a non-finite (mode 1) or an all-zero
// (mode 2) preconditioner output e in place of the computed one.
// ---------------------------------------------------------------------------
template <typename P, int M>
__device__ __forceinline__ void kb_fault_e(const Fields& F, int mode, int at_it) {
  using V = typename P::V;
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  if (F.state[m].it != at_it) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  V v[M];
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = mode == 1 ? (V)__builtin_nan("") : (V)0;
  if (R.act) str<M>((V*)F.e + R.rc, R.lane, R.L, v);
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_fault_e(Fields F, int mode, int at_it) {
  if constexpr (M > 0) {
    kb_fault_e<P, M>(F, mode, at_it);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_fault_e<P, 2>(F, mode, at_it); break;
      case 2: kb_fault_e<P, 4>(F, mode, at_it); break;
      case 3: kb_fault_e<P, 8>(F, mode, at_it); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// preconditioner options 0-2 (paper Section 2.3):
//   first pass  (update as in k_update_sweep1), then q = r or r/diag(L)
//   Richardson  q_out = q_in - (L q_in - r) / diag(L)
// (intermediates in the Krylov type)
// ---------------------------------------------------------------------------
template <typename P, int M>
__device__ __forceinline__ void row_update_simple(const Fields& F, const RowCtx& R, const MemberGeom& G, int do_update,
                                                  int slot_nu, int use_diag, int qout) {
  using T = typename P::T;
  using V = typename P::V;
  using A = typename P::A;
  with_coef<P>(F, G, R.j, false, [&](const auto& cv) {
    T rv[M];
    ldr<M>((const V*)F.r + R.rc, R.lane, R.L, rv);
    if (do_update) {
      const A acc = row_update<P, M>(F, R, slot_nu, rv);
      write_partial<A>(F, R, DOT_RR, acc);
    }
    if (use_diag) {
      T d[M];
      diag_row<T, M>(R, cv, d);
  #pragma unroll
      for (int k = 0; k < M; ++k) rv[k] /= d[k];
    }
    store_v<P, M>(qout < 0 ? F.e : F.q[qout], R, rv);
  });
}

template <typename P, int M>
__device__ __forceinline__ void kb_update_simple(const Fields& F, int do_update, int slot_nu, int use_diag, int qout) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  row_update_simple<P, M>(F, make_row(G, m, g, lane, M), G, do_update, slot_nu, use_diag, qout);
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_update_simple(Fields F, int do_update, int slot_nu, int use_diag, int qout) {
  if constexpr (M > 0) {
    kb_update_simple<P, M>(F, do_update, slot_nu, use_diag, qout);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_update_simple<P, 2>(F, do_update, slot_nu, use_diag, qout); break;
      case 2: kb_update_simple<P, 4>(F, do_update, slot_nu, use_diag, qout); break;
      case 3: kb_update_simple<P, 8>(F, do_update, slot_nu, use_diag, qout); break;
      default: break;
    }
  }
}

template <typename P, int M, bool FL>
__device__ __forceinline__ void row_jacobi(const Fields& F, const RowCtx& R, const MemberGeom& G, int qin, int qout) {
  using T = typename P::T;
  using V = typename P::V;
  // buffer pointers taken before the lambda: indexing F.q inside it made the
  // compiler copy all of F to the stack
  const V* qin_p = (const V*)F.q[qin];
  void* out_p = qout < 0 ? F.e : F.q[qout];
  with_coef<P, FL>(F, G, R.j, false, [&](const auto& cv) {
    const T helm = cv.helm(R.g);
    RowReader<T, V> X{qin_p};
    T rv[M], d[M], o[M];
    diag_row<T, M>(R, cv, d);
    ldr<M>((const V*)F.r + R.rc, R.lane, R.L, rv);
    stencil_row<T, M>(R, cv, X, [&](int k, T zon, T rest, T xc, T, T, T, T) {
      o[k] = xc - ((zon + rest - helm * xc) - rv[k]) / d[k];
    });
    store_v<P, M>(out_p, R, o);
  });
}

template <typename P, int M, bool FL>
__device__ __forceinline__ void kb_jacobi(const Fields& F, int qin, int qout) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  row_jacobi<P, M, FL>(F, make_row(G, m, g, lane, M), G, qin, qout);
}

template <typename P, int M, bool FL>
__global__ __launch_bounds__(WG) void k_jacobi(Fields F, int qin, int qout) {
  if constexpr (M > 0) {
    kb_jacobi<P, M, FL>(F, qin, qout);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_jacobi<P, 2, FL>(F, qin, qout); break;
      case 2: kb_jacobi<P, 4, FL>(F, qin, qout); break;
      case 3: kb_jacobi<P, 8, FL>(F, qin, qout); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// out = L(in) in the Krylov precision, with fused inner products:
//   mode 0: <out, L p_l> for the nl ring slots in `slots`  -> DOT_LE_LP + l
//   mode 1: <r, out>, <out, out>                           -> DOT_R_LP, DOT_LP_LP
//   mode 2: none
// ---------------------------------------------------------------------------
struct Slots {
  int s[KMAX + 1];
};

template <typename P, int M, bool FL>
__device__ __forceinline__ void row_apply_L(const Fields& F, const RowCtx& R, const MemberGeom& G, const void* in,
                                            void* out, int mode, int nl, const Slots& sl) {
  using T = typename P::T;
  using V = typename P::V;
  using A = typename P::A;
  const int l = R.lane, L = R.L;
  auto body = [&](const auto& cv) {
    const T helm = cv.helm(R.g);
    RowReader<T, V> X{(const V*)in};
    T y[M];
    stencil_row<T, M>(R, cv, X, [&](int k, T zon, T rest, T xc, T, T, T, T) {
      y[k] = (T)(V)(zon + rest - helm * xc);
    });
    store_v<P, M>(out, R, y);
    if (mode == 0) {
      for (int li = 0; li < nl; ++li) {
        T lv[M];
        ldr<M>((const V*)F.lp[sl.s[li]] + R.rc, l, L, lv);
        A acc = (A)0;
  #pragma unroll
        for (int k = 0; k < M; ++k) acc += (A)y[k] * (A)lv[k];
        write_partial<A>(F, R, DOT_LE_LP + li, R.act ? acc : (A)0);
      }
    } else if (mode == 1) {
      T rv[M];
      ldr<M>((const V*)F.r + R.rc, l, L, rv);
      A a0 = (A)0, a1 = (A)0;
  #pragma unroll
      for (int k = 0; k < M; ++k) {
        a0 += (A)rv[k] * (A)y[k];
        a1 += (A)y[k] * (A)y[k];
      }
      write_partial<A>(F, R, DOT_R_LP, R.act ? a0 : (A)0);
      write_partial<A>(F, R, DOT_LP_LP, R.act ? a1 : (A)0);
    }
  };
  // float64 and float32 operators: coefficients from the depth fields;
  // float16 operator storage (the paper's mixed form): the stored arrays
  if constexpr (!P::mixed) body(CoefFly<double, FL>{F.fly64});
  else if constexpr (P::coef64) body(CoefScaled64{CoefFly<double>{F.fly64}, F.scale, F.rowmap});
  else if constexpr (P::op_f32) body(CoefFly<float, FL>{F.fly32});
  else with_coef<P>(F, G, R.j, true, body);
}

template <typename P, int M, bool FL>
__device__ __forceinline__ void kb_apply_L(const Fields& F, const void* in, void* out, int mode, int nl, const Slots& sl) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  if constexpr (P::polar64) {
    if (R.j < G.polar || R.j >= G.ny - G.polar) {
      row_apply_L<Polar64<P>, M, false>(F, R, G, in, out, mode, nl, sl);
      return;
    }
  }
  row_apply_L<P, M, FL>(F, R, G, in, out, mode, nl, sl);
}

template <typename P, int M, bool FL>
__global__ __launch_bounds__(WG) void k_apply_L(Fields F, const void* in, void* out, int mode, int nl, Slots sl) {
  if constexpr (M > 0) {
    kb_apply_L<P, M, FL>(F, in, out, mode, nl, sl);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_apply_L<P, 2, FL>(F, in, out, mode, nl, sl); break;
      case 2: kb_apply_L<P, 4, FL>(F, in, out, mode, nl, sl); break;
      case 3: kb_apply_L<P, 8, FL>(F, in, out, mode, nl, sl); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// residual r = L(x) - R in float64 (eq. Residual).  `write_krylov`: 0 writes
// nothing but the partials (final true residual), 1 the Krylov copy
// r = s*r (s = 1 in the float64 form; solve start and restarts), 2 the float64
// r64 (stand-alone use).  Partials: <r,r> (slot DOT_RR, in the Krylov
// scaling); with `lp_slot` >= 0 also <r, L p_slot>.  `respect_done`: skip
// finished members (restart) or not (final check).  `io` moves the caller's
// fields (natural order) in the same pass: RES_RHS_TAB reads R from them,
// RES_X_IN reads x from them and writes the pooled x (solve start), RES_X_OUT
// writes the pooled x back to them (solve end).
// ---------------------------------------------------------------------------
enum { RES_X_IN = 1, RES_X_OUT = 2, RES_RHS_TAB = 4 };

template <typename P, int M, bool FL>
__device__ __forceinline__ void row_residual(const Fields& F, const RowCtx& R, const MemberGeom& G, int write_krylov,
                                             int lp_slot, int io) {
  using V = typename P::V;
  const int l = R.lane, L = R.L;
  const CoefFly<double, FL> cv{F.fly64};
  const double helm = cv.helm(R.g);
  const double s = P::mixed ? F.scale[R.m] : 1.0;
  const long long nat = R.rc - G.off;     // the row's offset in natural order
  double rr[M], b[M], xk[M];
  if (io & RES_RHS_TAB) ldn<M>(F.rhs_tab[R.m] + nat, l, b);
  else ldr<M>(F.rhs + R.rc, l, L, b);
  double acc0 = 0.0, acc1 = 0.0;
  auto body = [&](const auto& X) {
    stencil_row<double, M, true>(R, cv, X, [&](int k, double zon, double rest, double xc, double, double, double, double) {
      rr[k] = zon + rest - helm * xc - b[k];
      acc0 += rr[k] * rr[k];
      xk[k] = xc;
    });
  };
  if (io & RES_X_IN) body(NatReader{F.x_tab[R.m], G.off});
  else body(RowReader<double, double>{F.x});
  if ((io & RES_X_IN) && R.act) str<M>(F.x + R.rc, l, L, xk);
  if ((io & RES_X_OUT) && R.act) stn<M>(F.x_tab[R.m] + nat, l, xk);
  if (write_krylov == 2 && R.act) str<M>(F.r64 + R.rc, l, L, rr);
  if (write_krylov == 1) {
    double rk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) rk[k] = (double)(V)(s * rr[k]);
    if (R.act) str<M>((V*)F.r + R.rc, l, L, rk);
    if (lp_slot >= 0) {
      double lv[M];
      ldr<M>((const V*)F.lp[lp_slot] + R.rc, l, L, lv);
#pragma unroll
      for (int k = 0; k < M; ++k) acc1 += rk[k] * lv[k];
    }
  }
  // the Krylov residual lives in scaled units in the mixed forms
  write_partial<double>(F, R, DOT_RR, R.act ? acc0 * s * s : 0.0);
  if (F.linf) write_row_max<M>(F, R, rr, s);
  write_partial<double>(F, R, DOT_R_LP, R.act ? acc1 : 0.0);
}

template <typename P, int M, bool FL>
__device__ __forceinline__ void kb_residual(const Fields& F, int write_krylov, int lp_slot, int respect_done, int io) {
  int g, m, lane, w;
  MemberGeom G;
  const bool active = wave_row(F, g, m, G, lane, w);
  if (g >= F.row_end || (respect_done && !active)) return;
  row_residual<P, M, FL>(F, make_row(G, m, g, lane, M), G, write_krylov, lp_slot, io);
}

template <typename P, int M, bool FL>
__global__ __launch_bounds__(WG) void k_residual(Fields F, int write_krylov, int lp_slot, int respect_done, int io) {
  if constexpr (M > 0) {
    kb_residual<P, M, FL>(F, write_krylov, lp_slot, respect_done, io);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_residual<P, 2, FL>(F, write_krylov, lp_slot, respect_done, io); break;
      case 2: kb_residual<P, 4, FL>(F, write_krylov, lp_slot, respect_done, io); break;
      case 3: kb_residual<P, 8, FL>(F, write_krylov, lp_slot, respect_done, io); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// Split single-precision residual (paper Section 4.2.1, eq. L_Operator_SP).
// The depth is a float32 base Phi_hat plus a float32 correction Phi_tilde.
// The gradient terms take the stored float32 differences of Phi_hat plus
// those of Phi_tilde; the B and C terms take Phi_SP = Phi_hat + Phi_tilde; all
// in float32, with the face coefficients formed in float64 from the depth
// pools and rounded to float32 (forming them in float32 from float32 depths
// would put the depths' rounding into the B terms' differences of H*, which
// the 1/cos factor amplifies next to the poles).
// The rows within G.polar rows of a pole use the float64 operator on
// Phi_hat + Phi_tilde instead.  The differences are the undivided ones the
// stencil multiplies (zonal and 4-point meridional at east faces, meridional
// and 4-point zonal at north faces).
// ---------------------------------------------------------------------------
enum { SD_LON_E = 0, SD_LAT_E, SD_LAT_N, SD_LON_N, NSD };

struct SplitArgs {
  float* hat;                 // Phi_hat, pooled
  float* d[NSD];              // its stored differences, pooled (north-face ones zero in the last row)
  const float* tilde;         // Phi_tilde, pooled
};

// float32 field rows read as float64 sums hat + tilde (the float64 polar rows)
struct SumReader {
  const float* a;
  const float* b;
  template <int M>
  __device__ __forceinline__ void row(long long start, int l, int L, double (&v)[M], int /*row_g*/) const {
    float x[M], y[M];
    ldr<M>(a + start, l, L, x);
    ldr<M>(b + start, l, L, y);
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = (double)x[k] + (double)y[k];
  }
  template <int M>
  __device__ __forceinline__ void pair(long long start, int n, int ln, int k, int L, int /*row_g*/, double& u,
                                       double& v) const {
    float x0, x1, y0, y1;
    ld_pair<float, float>(a + start, n, ln, k, L, x0, x1);
    ld_pair<float, float>(b + start, n, ln, k, L, y0, y1);
    u = (double)x0 + (double)y0;
    v = (double)x1 + (double)y1;
  }
};

// Phi_hat = fl32(phi) and its float32 differences, from the float64 field in
// the pooled x; differences taken in float64 of the float32 values.
template <typename P, int M>   // P: unused (the row-launch helper's signature)
__device__ __forceinline__ void kb_split_base(const Fields& F, SplitArgs S) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  const int l = R.lane, L = R.L;
  const int wl = (l - 1) & (L - 1), el = (l + 1) & (L - 1);
  double c[M], so[M], no[M];
  ldr<M>(F.x + R.rc, l, L, c);
  if (R.south) ldr<M>(F.x + R.rc - R.nx, l, L, so);
  if (R.north) ldr<M>(F.x + R.rc + R.nx, l, L, no);
  if (!R.south) across_pole(c, so, l, L);
  if (!R.north) across_pole(c, no, l, L);
#pragma unroll
  for (int k = 0; k < M; ++k) {   // the float32 values, as float64
    c[k] = (double)(float)c[k];
    so[k] = (double)(float)so[k];
    no[k] = (double)(float)no[k];
  }
  const double cw0 = shfl(c[M - 1], wl), ceM = shfl(c[0], el);
  const double seM = shfl(so[0], el);
  const double nw0 = shfl(no[M - 1], wl), neM = shfl(no[0], el);
  float h[M], dle[M], dte[M], dtn[M], dln[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double e = k < M - 1 ? c[k + 1] : ceM, wv = k > 0 ? c[k - 1] : cw0;
    const double se = k < M - 1 ? so[k + 1] : seM;
    const double ne = k < M - 1 ? no[k + 1] : neM, nw = k > 0 ? no[k - 1] : nw0;
    h[k] = (float)c[k];
    dle[k] = (float)(e - c[k]);
    dte[k] = (float)((no[k] - so[k]) + (ne - se));
    dtn[k] = R.north ? (float)(no[k] - c[k]) : 0.f;
    dln[k] = R.north ? (float)((e - wv) + (ne - nw)) : 0.f;
  }
  if (R.act) {
    str<M>(S.hat + R.rc, l, L, h);
    str<M>(S.d[SD_LON_E] + R.rc, l, L, dle);
    str<M>(S.d[SD_LAT_E] + R.rc, l, L, dte);
    str<M>(S.d[SD_LAT_N] + R.rc, l, L, dtn);
    str<M>(S.d[SD_LON_N] + R.rc, l, L, dln);
  }
}

template <typename P, int M>   // P: unused (the row-launch helper's signature)
__global__ __launch_bounds__(WG) void k_split_base(Fields F, SplitArgs S) {
  if constexpr (M > 0) {
    kb_split_base<P, M>(F, S);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_split_base<P, 2>(F, S); break;
      case 2: kb_split_base<P, 4>(F, S); break;
      case 3: kb_split_base<P, 8>(F, S); break;
      default: break;
    }
  }
}

// The split of a solve's initial guess (paper Section 4.2.1): Phi_tilde =
// fl32(x_0 - Phi_hat) from the caller's x_0 (natural order) and the stored
// base, and x_0 into the pooled solution, for every member (finished or not).
template <typename P, int M>
__device__ __forceinline__ void kb_split_tilde(const Fields& F, SplitArgs S) {
  int g, m, lane, w;
  MemberGeom G;
  wave_row(F, g, m, G, lane, w);
  if (g >= F.row_end) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  const int l = R.lane, L = R.L;
  double xv[M];
  float hv[M], tv[M];
  ldn<M>(F.x_tab[R.m] + (R.rc - G.off), l, xv);
  ldr<M>(S.hat + R.rc, l, L, hv);
#pragma unroll
  for (int k = 0; k < M; ++k) tv[k] = (float)(xv[k] - (double)hv[k]);
  if (R.act) {
    str<M>((float*)S.tilde + R.rc, l, L, tv);
    str<M>(F.x + R.rc, l, L, xv);
  }
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_split_tilde(Fields F, SplitArgs S) {
  if constexpr (M > 0) {
    kb_split_tilde<P, M>(F, S);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_split_tilde<P, 2>(F, S); break;
      case 2: kb_split_tilde<P, 4>(F, S); break;
      case 3: kb_split_tilde<P, 8>(F, S); break;
      default: break;
    }
  }
}

// r = L_SP(Phi_hat + Phi_tilde) - R.  mode 0 (stand-alone): R from the
// pooled rhs, r into the pooled r64.  mode 1 (a solve's initial residual):
// R from the caller's arrays, r into the Krylov residual in the form's units
// (s r, vector type P::V) with its <r,r> partials (and max |r| with the
// maximum-norm exit), for every member.
template <typename P, int M>
__device__ __forceinline__ void kb_residual_split(const Fields& F, SplitArgs S, int mode) {
  using V = typename P::V;
  int g, m, lane, w;
  MemberGeom G;
  const bool active = wave_row(F, g, m, G, lane, w);
  if (g >= F.row_end || (mode == 0 && !active)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  const int l = R.lane, L = R.L;
  double b[M], out[M];
  if (mode == 1) ldn<M>(F.rhs_tab[R.m] + (R.rc - G.off), l, b);
  else ldr<M>(F.rhs + R.rc, l, L, b);
  if (R.j < G.polar || R.j >= G.ny - G.polar) {   // float64 polar bands
    const CoefFly<double> cv{F.fly64};
    const double helm = cv.helm(R.g);
    stencil_row<double, M, true>(R, cv, SumReader{S.hat, S.tilde},
                           [&](int k, double zon, double rest, double xc, double, double, double, double) {
                             out[k] = zon + rest - helm * xc - b[k];
                           });
  } else {
    const int wl = (l - 1) & (L - 1), el = (l + 1) & (L - 1);
    float axe[M], axy[M], bx[M], ayn[M], ayxn[M], byn[M], ays[M], ayxs[M], bys[M];
    {
      const CoefFly<double> cv{F.fly64};
      double c9[9][M];
      cv.template load9<M>(R, c9[0], c9[1], c9[2], c9[3], c9[4], c9[5], c9[6], c9[7], c9[8]);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        axe[k] = (float)c9[0][k];
        axy[k] = (float)c9[1][k];
        bx[k] = (float)c9[2][k];
        ayn[k] = (float)c9[3][k];
        ayxn[k] = (float)c9[4][k];
        byn[k] = (float)c9[5][k];
        ays[k] = (float)c9[6][k];
        ayxs[k] = (float)c9[7][k];
        bys[k] = (float)c9[8][k];
      }
    }
    const float helm = (float)F.fly64.c[R.g];
    float tc[M], ts[M], tn[M], hc[M], hs[M], hn[M];
    ldr<M>(S.tilde + R.rc, l, L, tc);
    ldr<M>(S.hat + R.rc, l, L, hc);
    if (R.south) {
      ldr<M>(S.tilde + R.rc - R.nx, l, L, ts);
      ldr<M>(S.hat + R.rc - R.nx, l, L, hs);
    } else {
      across_pole(tc, ts, l, L);
      across_pole(hc, hs, l, L);
    }
    if (R.north) {
      ldr<M>(S.tilde + R.rc + R.nx, l, L, tn);
      ldr<M>(S.hat + R.rc + R.nx, l, L, hn);
    } else {
      across_pole(tc, tn, l, L);
      across_pole(hc, hn, l, L);
    }
    float dle[M], dte[M], dtn[M], dln[M], dtns[M], dlns[M];
    ldr<M>(S.d[SD_LON_E] + R.rc, l, L, dle);
    ldr<M>(S.d[SD_LAT_E] + R.rc, l, L, dte);
    ldr<M>(S.d[SD_LAT_N] + R.rc, l, L, dtn);
    ldr<M>(S.d[SD_LON_N] + R.rc, l, L, dln);
    if (R.south) {   // the south face is the north face of row j-1
      ldr<M>(S.d[SD_LAT_N] + R.rc - R.nx, l, L, dtns);
      ldr<M>(S.d[SD_LON_N] + R.rc - R.nx, l, L, dlns);
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        dtns[k] = 0.f;
        dlns[k] = 0.f;
      }
    }
    auto at = [](const float (&v)[M], int i, float w0, float eM) { return i < 0 ? w0 : (i >= M ? eM : v[i]); };
    const float tcw = shfl(tc[M - 1], wl), tce = shfl(tc[0], el);
    const float tsw = shfl(ts[M - 1], wl), tse = shfl(ts[0], el);
    const float tnw = shfl(tn[M - 1], wl), tne = shfl(tn[0], el);
    const float hcw = shfl(hc[M - 1], wl), hce = shfl(hc[0], el);
    const float dlew = shfl(dle[M - 1], wl), dtew = shfl(dte[M - 1], wl);
    float axe_p = shfl(axe[M - 1], wl), axy_p = shfl(axy[M - 1], wl), bx_p = shfl(bx[M - 1], wl);
    // the full east-face differences of chunk point i (i = -1: the west face of point 0)
    auto dlon_e = [&](int i) {
      const float dh = i < 0 ? dlew : dle[i];
      return dh + (at(tc, i + 1, tcw, tce) - at(tc, i, tcw, tce));
    };
    auto dlat_e = [&](int i) {
      const float dh = i < 0 ? dtew : dte[i];
      return dh + ((at(tn, i, tnw, tne) - at(ts, i, tsw, tse)) + (at(tn, i + 1, tnw, tne) - at(ts, i + 1, tsw, tse)));
    };
    float de_p = dlon_e(-1), te_p = dlat_e(-1);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const float de = dlon_e(k), te = dlat_e(k);
      const float dn = dtn[k] + (tn[k] - tc[k]);
      const float ln = dln[k] + ((at(tc, k + 1, tcw, tce) - at(tc, k - 1, tcw, tce)) +
                                 (at(tn, k + 1, tnw, tne) - at(tn, k - 1, tnw, tne)));
      const float dsn = dtns[k] + (tc[k] - ts[k]);
      const float lsn = dlns[k] + ((at(ts, k + 1, tsw, tse) - at(ts, k - 1, tsw, tse)) +
                                   (at(tc, k + 1, tcw, tce) - at(tc, k - 1, tcw, tce)));
      const float csp = hc[k] + tc[k];
      const float esp = at(hc, k + 1, hcw, hce) + at(tc, k + 1, tcw, tce);
      const float wsp = at(hc, k - 1, hcw, hce) + at(tc, k - 1, tcw, tce);
      const float nsp = hn[k] + tn[k], ssp = hs[k] + ts[k];
      const float zon = axe[k] * de - axe_p * de_p;
      float r = axy[k] * te - axy_p * te_p;
      r += bx[k] * (csp + esp) - bx_p * (wsp + csp);
      r += ayn[k] * dn + ayxn[k] * ln + byn[k] * (csp + nsp);
      r -= ays[k] * dsn + ayxs[k] * lsn + bys[k] * (ssp + csp);
      const float lsp = zon + r - helm * csp;
      out[k] = (double)(float)((double)lsp - b[k]);
      axe_p = axe[k];
      axy_p = axy[k];
      bx_p = bx[k];
      de_p = de;
      te_p = te;
    }
  }
  if (mode == 0) {
    if (R.act) str<M>(F.r64 + R.rc, l, L, out);
    return;
  }
  const double s = P::mixed ? F.scale[R.m] : 1.0;
  double rk[M], acc = 0.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    rk[k] = (double)(V)(s * out[k]);
    acc += rk[k] * rk[k];
  }
  if (R.act) str<M>((V*)F.r + R.rc, l, L, rk);
  write_partial<double>(F, R, DOT_RR, R.act ? acc : 0.0);
  if (F.linf) write_row_max<M>(F, R, rk, 1.0);
  write_partial<double>(F, R, DOT_R_LP, 0.0);
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_residual_split(Fields F, SplitArgs S, int mode) {
  if constexpr (M > 0) {
    kb_residual_split<P, M>(F, S, mode);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_residual_split<P, 2>(F, S, mode); break;
      case 2: kb_residual_split<P, 4>(F, S, mode); break;
      case 3: kb_residual_split<P, 8>(F, S, mode); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// step 4: p_{nu+1} = e + sum alpha_l p_l ; L p_{nu+1} = L e + sum alpha_l L p_l,
// with fused <r, L p_{nu+1}> and <L p_{nu+1}, L p_{nu+1}>.  In the last
// iteration of a cycle (`last`) also the cycle's recorded solution updates,
// x += beta_l p_l for l = 0..k-1 in that order, from the directions loaded
// here (k_ctrl_alpha sets by_orth when all k were recorded).
// ---------------------------------------------------------------------------
template <typename P, int M, bool LAST>
__device__ __forceinline__ void row_orth(const Fields& F, const RowCtx& R, int nl, const Slots& sl, int out_slot) {
  using T = typename P::T;
  using V = typename P::V;
  using A = typename P::A;
  const int l = R.lane, L = R.L;
  const Pending& pd = F.pend[R.m];
  const bool upd = LAST && pd.by_orth;
  const bool upd_dx = upd && P::mixed && F.dx;
  const bool upd_x = upd && !upd_dx;
  T pv[M], lv[M], rv[M];
  double xv[M];
  float dxv[M];
  ldr<M>((const V*)F.e + R.rc, l, L, pv);
  ldr<M>((const V*)F.le + R.rc, l, L, lv);
  if (upd_x) ldr<M>(F.x + R.rc, l, L, xv);
  if (upd_dx) ldr<M>(F.dx + R.rc, l, L, dxv);
  for (int li = 0; li < nl; ++li) {
    const T alpha = (T)F.state[R.m].alpha[li];
    T a[M], b[M];
    ldr<M>((const V*)F.p[sl.s[li]] + R.rc, l, L, a);
    ldr<M>((const V*)F.lp[sl.s[li]] + R.rc, l, L, b);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      pv[k] += alpha * a[k];
      lv[k] += alpha * b[k];
    }
    if (upd_x) {
      const double beta = pd.beta[li];
#pragma unroll
      for (int k = 0; k < M; ++k) xv[k] += beta * (double)a[k];
    }
    if (upd_dx) {
      const double beta = pd.beta[li];
#pragma unroll
      for (int k = 0; k < M; ++k) dxv[k] += (float)beta * (float)a[k];
    }
  }
  if (upd_x && R.act) str<M>(F.x + R.rc, l, L, xv);
  if (upd_dx && R.act) str<M>(F.dx + R.rc, l, L, dxv);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    pv[k] = (T)(V)pv[k];
    lv[k] = (T)(V)lv[k];
  }
  if (R.act) {
    str<M>((V*)F.p[out_slot] + R.rc, l, L, pv);
    str<M>((V*)F.lp[out_slot] + R.rc, l, L, lv);
  }
  ldr<M>((const V*)F.r + R.rc, l, L, rv);
  A acc0 = (A)0, acc1 = (A)0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    acc0 += (A)rv[k] * (A)lv[k];
    acc1 += (A)lv[k] * (A)lv[k];
  }
  write_partial<A>(F, R, DOT_R_LP, R.act ? acc0 : (A)0);
  write_partial<A>(F, R, DOT_LP_LP, R.act ? acc1 : (A)0);
}

template <typename P, int M>
__device__ __forceinline__ void kb_orth(const Fields& F, int nl, const Slots& sl, int out_slot) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  row_orth<P, M, false>(F, make_row(G, m, g, lane, M), nl, sl, out_slot);
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_orth(Fields F, int nl, Slots sl, int out_slot) {
  if constexpr (M > 0) {
    kb_orth<P, M>(F, nl, sl, out_slot);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_orth<P, 2>(F, nl, sl, out_slot); break;
      case 2: kb_orth<P, 4>(F, nl, sl, out_slot); break;
      case 3: kb_orth<P, 8>(F, nl, sl, out_slot); break;
      default: break;
    }
  }
}

// the last iteration of a cycle: step 4 and the cycle's solution updates
template <typename P, int M>
__device__ __forceinline__ void kb_orth_last(const Fields& F, int nl, const Slots& sl, int out_slot) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  row_orth<P, M, true>(F, make_row(G, m, g, lane, M), nl, sl, out_slot);
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_orth_last(Fields F, int nl, Slots sl, int out_slot) {
  if constexpr (M > 0) {
    kb_orth_last<P, M>(F, nl, sl, out_slot);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_orth_last<P, 2>(F, nl, sl, out_slot); break;
      case 2: kb_orth_last<P, 4>(F, nl, sl, out_slot); break;
      case 3: kb_orth_last<P, 8>(F, nl, sl, out_slot); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// coefficient assembly (paper eqs. rhslin, Qexpr, L_Operator), one thread per
// point, float64; also writes the scaled float16 / float32 copies.
// ---------------------------------------------------------------------------
struct AsmMember {             // one member of a batched assembly
  const double* depth;        // Phi*, natural [NY][NX] layout (device)
  const double* oro;          // H0 or null
  double dt, g, omega, radius, absorber;
  int member, b_terms;
};

struct AssembleArgs {
  const AsmMember* tab;       // [count]
  const MemberGeom* geom;
  __half* a16[NCOEF];
  float* a32[NCOEF];
  double* c64;                // per global row
  float* c32;
  double* scale;              // per member: mixed-form scale dt/(2 a^2)
  double* phi64;              // Phi* and H* pools (float64, and float32 for the float32 operator)
  double* hs64;
  float* phi32;
  float* hs32;
  double* fac64;              // per global row: NFAC factors (float32: scaled by s)
  float* fac32;
  int* flat;                  // per member: 1 without orography (the H* pools are then not written)
  int rows;                   // rows per workgroup (1..ASM_ROWS; the staged rows must fit the LDS)
};

__device__ __forceinline__ double absorber_at(double lat, double amax) {
  const double kPi = 3.14159265358979323846;
  const double dist = 0.5 * kPi - fabs(lat);
  const double w = 1.0 - dist / (3.0 * kPi / 64.0);
  return amax * (w > 0.0 ? w : 0.0);
}

// One workgroup per (row, table entry).  Rows j-1, j, j+1 of Phi* and of
// H* = Phi* + H0 are staged in LDS with coalesced loads (rows beyond a pole
// are the polar row seen across the pole); the coefficients are then written
// in stored (row-interleaved) order, i.e. coalesced.  The LDS copy of a row is
// itself kept in padded interleaved order, lds(i) = (i mod M)(L+1) + i/M, so
// that the stored-order reads of consecutive threads hit distinct banks.
// Everything that depends on the latitude only is folded into per-row
// factors, leaving no division in the per-point work.
constexpr int ASM_WG = 256;
constexpr int ASM_ROWS = ASM_WG / 64;   // rows per workgroup, one wave each

__host__ __device__ constexpr int asm_row_lds(int nx) { return nx + 16; }   // doubles per staged row (M <= 16)

static __global__ __launch_bounds__(ASM_WG) void k_assemble(AssembleArgs A) {
  // dynamic LDS: Phi* rows j0-1 .. j0+ASM_ROWS, then (with orography) H* rows
  extern __shared__ double asm_lds[];
  const AsmMember P = A.tab[blockIdx.y];
  const MemberGeom G = A.geom[P.member];
  const int nx = G.nx, ny = G.ny, j0 = xcd_block(blockIdx.x, gridDim.x) * A.rows;
  if (j0 >= ny) return;
  const int half = nx >> 1;
  const int lm = G.log2m, Mr = 1 << lm, Lr = nx >> lm;
  const int rs = asm_row_lds(nx);
  auto lidx = [&](int i) { return (i & (Mr - 1)) * (Lr + 1) + (i >> lm); };
  double* sd_all = asm_lds;
  double* sh_all = P.oro ? asm_lds + (A.rows + 2) * rs : asm_lds;
  for (int r = 0; r < A.rows + 2; ++r) {
    int jj = j0 - 1 + r, sh_ = 0;
    if (jj > ny) break;                 // beyond the ghost row of the north pole
    if (jj < 0) { jj = 0; sh_ = half; }
    if (jj >= ny) { jj = ny - 1; sh_ = half; }
    const double* drow = P.depth + (long long)jj * nx;
    const double* orow = P.oro ? P.oro + (long long)jj * nx : nullptr;
    for (int i = threadIdx.x; i < nx; i += ASM_WG) {
      const int src = (i + sh_) & (nx - 1);
      const double d = drow[src];
      sd_all[r * rs + lidx(i)] = d;
      if (orow) sh_all[r * rs + lidx(i)] = d + orow[src];
    }
  }
  __syncthreads();
  // wave w assembles row j = j0 + w from staged rows w, w+1, w+2
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = j0 + w;
  if (w >= A.rows || j >= ny) return;
  const double* sd0 = sd_all + w * rs;
  const double* sh0 = sh_all + w * rs;
  const double kPi = 3.14159265358979323846;
  const double dlam = 2.0 * kPi / nx, dphi = kPi / ny;
  const double delta = 0.5 * P.dt;
  // latitude factors of the row (east faces) and of its north face
  const double lat_c = -0.5 * kPi + (j + 0.5) * dphi, lat_n = -0.5 * kPi + (j + 1.0) * dphi;
  const double cs_c = cos(lat_c), cs_n = cos(lat_n);
  const double gam_c = 1.0 + delta * absorber_at(lat_c, P.absorber);
  const double gam_n = 1.0 + delta * absorber_at(lat_n, P.absorber);
  const double b_c = delta * 2.0 * P.omega * sin(lat_c), b_n = delta * 2.0 * P.omega * sin(lat_n);
  const double D_c = gam_c * gam_c + b_c * b_c, D_n = gam_n * gam_n + b_n * b_n;
  const double s = P.dt / (2.0 * P.radius * P.radius);   // mixed-form scale
  // east faces: kappa = ke * (Phi*_i + Phi*_{i+1}); the differences of H*
  // enter B^x through bl (zonal) and bp (meridional, 4-point average)
  const double ke = delta * P.g * 0.5 / (2.0 * D_c);
  const double fxx = gam_c / cs_c / (dlam * dlam);
  const double fxy = b_c / (4.0 * dlam * dphi);
  const double gbx = delta * P.g / (2.0 * D_c) / (2.0 * dlam);
  const double bl_e = gam_c / cs_c / dlam, bp_e = b_c / (4.0 * dphi);
  // north face
  const double kn = delta * P.g * 0.5 / (2.0 * D_n);
  const double fyy = gam_n * cs_n / (dphi * dphi);
  const double fyx = -b_n / (4.0 * dlam * dphi);
  const double gby = delta * P.g / (2.0 * D_n) / (2.0 * dphi);
  const double bl_n = -b_n / (4.0 * dlam), bp_n = gam_n * cs_n / dphi;
  const bool north = j < ny - 1;   // the pole face carries no flux
  // float32 copies are read by the polar rows (and, as their south face, by
  // the row just below the northern polar rows)
  const bool polar = j < G.polar || j >= ny - G.polar - 1;
  const long long rowoff = G.off + (long long)j * nx;
  const int lL = G.log2nx - lm;   // Lr = 1 << lL lanes hold the row
  // Each pass of a lane covers one element pair (k, k+1) of stored lane l:
  // one 32-bit word of every float16 row, two elements of the others.
  for (int pidx = lane; pidx < half; pidx += 64) {
    const int l = pidx & (Lr - 1), kp = pidx >> lL;
    double out[2][NCOEF], dv[2], hv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = (l << lm) + 2 * kp + h;   // natural column of stored element (l, 2kp + h)
      const int c = lidx(i), ce = lidx((i + 1) & (nx - 1)), cw = lidx((i - 1) & (nx - 1));
      const double d1 = sd0[rs + c];
      dv[h] = d1;
      hv[h] = sh0[rs + c];
      {  // east face (i+1/2, j)
        const double kap = ke * (d1 + sd0[rs + ce]);
        out[h][C_AXX] = kap * fxx;
        out[h][C_AXY] = kap * fxy;
        double bx = 0.0;
        if (P.b_terms) {
          const double dhl = sh0[rs + ce] - sh0[rs + c];
          const double dhp = (sh0[2 * rs + c] - sh0[c]) + (sh0[2 * rs + ce] - sh0[ce]);
          bx = gbx * (bl_e * dhl + bp_e * dhp);
        }
        out[h][C_BX] = bx;
      }
      if (north) {  // north face (i, j+1/2)
        const double kap = kn * (d1 + sd0[2 * rs + c]);
        out[h][C_AYY] = kap * fyy;
        out[h][C_AYX] = kap * fyx;
        double by = 0.0;
        if (P.b_terms) {
          const double dhp = sh0[2 * rs + c] - sh0[rs + c];
          const double dhl = (sh0[rs + ce] - sh0[rs + cw]) + (sh0[2 * rs + ce] - sh0[2 * rs + cw]);
          by = gby * (bl_n * dhl + bp_n * dhp);
        }
        out[h][C_BY] = by;
      } else {
        out[h][C_AYY] = 0.0;
        out[h][C_AYX] = 0.0;
        out[h][C_BY] = 0.0;
      }
    }
    const long long o0 = rowoff + ((long long)(2 * kp) << lL) + l, o1 = o0 + Lr;   // stored slots k*Lr + l
    const long long o16 = rowoff + ((long long)kp << (lL + 1)) + 2 * l;            // the pair's word (in halves)
#pragma unroll
    for (int k = 0; k < NCOEF; ++k) {
      const float v0 = (float)(s * out[0][k]), v1 = (float)(s * out[1][k]);
      if (polar) {
        A.a32[k][o0] = v0;
        A.a32[k][o1] = v1;
      }
      const unsigned lo = __builtin_bit_cast(unsigned short, __float2half_rn(v0));
      const unsigned hi = __builtin_bit_cast(unsigned short, __float2half_rn(v1));
      *(unsigned*)(A.a16[k] + o16) = lo | (hi << 16);
    }
    A.phi64[o0] = dv[0];
    A.phi64[o1] = dv[1];
    A.phi32[o0] = (float)dv[0];
    A.phi32[o1] = (float)dv[1];
    if (P.oro) {
      A.hs64[o0] = hv[0];
      A.hs64[o1] = hv[1];
      A.hs32[o0] = (float)hv[0];
      A.hs32[o1] = (float)hv[1];
    }
  }
  if (lane < NFAC) {   // latitude factors of the on-the-fly coefficients
    const double gb = P.b_terms ? 1.0 : 0.0, nf = north ? 1.0 : 0.0;
    double v;
    switch (lane) {
      case FA_KE: v = ke; break;
      case FA_FXX: v = fxx; break;
      case FA_FXY: v = fxy; break;
      case FA_GBX: v = gb * gbx; break;
      case FA_BLE: v = bl_e; break;
      case FA_BPE: v = bp_e; break;
      case FA_KN: v = nf * kn; break;
      case FA_FYY: v = fyy; break;
      case FA_FYX: v = fyx; break;
      case FA_GBY: v = nf * gb * gby; break;
      case FA_BLN: v = bl_n; break;
      default: v = bp_n; break;
    }
    const bool scaled = lane == FA_KE || lane == FA_GBX || lane == FA_KN || lane == FA_GBY;
    A.fac64[(long long)(G.row0 + j) * NFAC + lane] = v;
    A.fac32[(long long)(G.row0 + j) * NFAC + lane] = (float)(scaled ? s * v : v);
  }
  if (lane == 0) {
    if (j == 0) {
      A.scale[P.member] = s;
      A.flat[P.member] = P.oro ? 0 : 1;
    }
    const double c = 2.0 * P.radius * P.radius * cs_c / P.dt;
    A.c64[G.row0 + j] = c;
    A.c32[G.row0 + j] = (float)(s * c);
  }
}

// ---------------------------------------------------------------------------
// copies between one member's caller field (natural [NY][NX]) and the pools
// (row-interleaved storage), for the stand-alone entry points
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long pool_index(const MemberGeom& G, long long k) {
  const int j = (int)(k >> G.log2nx), i = (int)(k & (G.nx - 1));
  return G.off + ((long long)j << G.log2nx) + row_slot(i, G.log2m, G.nx >> G.log2m);
}

// one member, direct pointers
static __global__ void k_to_pool(const double* src, double* pool, MemberGeom G) {
  const long long n = (long long)G.nx * G.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    pool[pool_index(G, k)] = src[k];
}

static __global__ void k_to_pool_f32(const float* src, float* pool, MemberGeom G) {
  const long long n = (long long)G.nx * G.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    pool[pool_index(G, k)] = src[k];
}

static __global__ void k_from_pool(const double* pool, double* dst, MemberGeom G) {
  const long long n = (long long)G.nx * G.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    dst[k] = pool[pool_index(G, k)];
}

// natural float64 field -> pooled vector type, times `scale` (rounded once)
template <typename V>
__global__ void k_to_pool_v(const double* src, V* pool, MemberGeom G, double scale) {
  const long long n = (long long)G.nx * G.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    pool[pool_index(G, k)] = (V)(scale * src[k]);
}

// pooled vector type -> natural float64 field, times `scale`
template <typename V>
__global__ void k_from_pool_v(const V* pool, double* dst, MemberGeom G, double scale) {
  const long long n = (long long)G.nx * G.ny;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    dst[k] = scale * (double)pool[pool_index(G, k)];
}

// mixed form without float64 accumulator: x += dx at exit, dx = 0
static __global__ void k_apply_increments(Fields F, long long total) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < total;
       k += (long long)gridDim.x * blockDim.x) {
    F.x[k] += (double)F.dx[k];
    F.dx[k] = 0.f;
  }
}

// ---------------------------------------------------------------------------
// control: one wave per member (block b takes member morder[q0 + b], so a
// launch can cover one group of members); sums the member's per-row partials in a
// fixed order (deterministic) and updates the device-resident scalars.
// ---------------------------------------------------------------------------
// Sums of the slots [first, first + ns) (ns <= NS) of the member's per-row
// partials.  Each lane adds its rows in a fixed order (rows lane, lane + 64,
// ...); the loads of MS_UNROLL rows and all slots are issued before the first
// addition, so the wave waits for memory once per chunk, not once per row.
constexpr int MS_UNROLL = 4;

template <typename A, int NS>
__device__ __forceinline__ void member_sums(const Fields& F, const MemberGeom& G, int first, int ns, double* out) {
  const int lane = threadIdx.x;
  A s[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = (A)0;
  const double* base = F.part + (long long)G.row0 * NDOT + first;
  for (int j0 = 0; j0 < G.ny; j0 += 64 * MS_UNROLL) {
    double v[MS_UNROLL][NS];
#pragma unroll
    for (int u = 0; u < MS_UNROLL; ++u) {
      const int jj = j0 + u * 64 + lane;
#pragma unroll
      for (int i = 0; i < NS; ++i) v[u][i] = (jj < G.ny && i < ns) ? base[(long long)jj * NDOT + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < MS_UNROLL; ++u)
#pragma unroll
      for (int i = 0; i < NS; ++i) s[i] += (A)v[u][i];
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) out[i] = (double)wave_sum(s[i]);
}

// max over the member's rows of one partial slot
__device__ __forceinline__ double member_max(const Fields& F, const MemberGeom& G, int slot) {
  double mx = 0.0;
  const double* base = F.part + (long long)G.row0 * NDOT + slot;
  for (int j = threadIdx.x; j < G.ny; j += 64) mx = fmax(mx, base[(long long)j * NDOT]);
  return wave_max(mx);
}

template <typename A>
__device__ __forceinline__ double member_sum(const Fields& F, const MemberGeom& G, int slot) {
  double o[1];
  member_sums<A, 1>(F, G, slot, 1, o);
  return o[0];
}

enum { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_STAGNATED = 2, ST_FALLBACK = 3 };

// the group's cycle counter to the next cycle (one thread; after the cycle's
// last kernel that reads it)
static __global__ void k_cycle_next(int* c) {
  if (threadIdx.x == 0) *c += 1;
}

template <typename A>
__global__ void k_ctrl_init(Fields F) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *F.cyc = 0;
  const int m = F.morder[F.q0 + blockIdx.x];
  const MemberGeom G = F.geom[m];
  const double rr = member_sum<double>(F, G, DOT_RR);
  const double rinf = F.linf ? member_max(F, G, DOT_RMAX) : 0.0;
  if (threadIdx.x == 0) {
    MemberState& S = F.state[m];
    S.rho0 = sqrt(rr);
    S.rho0_inf = rinf;
    S.rn = S.rho0;
    S.rn_cycle = S.rho0;
    S.it = 0;
    S.restarts = 0;
    S.fallback = 0;
    S.beta = 0.0;
    F.pend[m].n = 0;
    F.pend[m].cycle = -1;
    F.pend[m].by_orth = 0;
    S.rtrue = -1.0;
    S.status = ST_NOT_CONVERGED;
    S.done = 0;
    if (!(S.rho0 > 0.0)) {   // zero residual: x_0 solves the problem (NaN: stop too)
      S.status = S.rho0 == 0.0 ? ST_OK : ST_STAGNATED;
      S.done = 1;
    }
    if (F.hist) F.hist[(long long)m * F.hist_stride] = 1.0;
    F.done_flag[m] = S.done;
  }
}

template <typename A>
__global__ void k_ctrl_beta(Fields F, int slot) {
  const int m = F.morder[F.q0 + blockIdx.x];
  MemberState& S = F.state[m];
  if (S.done) return;
  const MemberGeom G = F.geom[m];
  static_assert(DOT_LP_LP == DOT_R_LP + 1, "slot order");
  double d[2];
  member_sums<A, 2>(F, G, DOT_R_LP, 2, d);
  const double num = d[0], lpsq = d[1];
  if (threadIdx.x == 0) {
    S.lpsq[slot] = lpsq;
    const double beta = -num / lpsq;
    if (!(lpsq > 0.0) || !isfinite(beta)) {
      S.status = ST_STAGNATED;
      S.done = 1;
      F.done_flag[m] = 1;
    }
    S.beta = beta;
  }
}

// after step 3: exit test on the updated residual, then step-4 coefficients
template <typename A>
__global__ void k_ctrl_alpha(Fields F, int nl, Slots sl, int cycle_end, int min_iters, int max_iters, double rtol) {
  const int cycle = *F.cyc;
  const int m = F.morder[F.q0 + blockIdx.x];
  MemberState& S = F.state[m];
  if (S.done) return;
  const MemberGeom G = F.geom[m];
  static_assert(DOT_LE_LP == DOT_RR + 1, "slot order");
  double d[KMAX + 1];
  member_sums<A, KMAX + 1>(F, G, DOT_RR, nl + 1, d);
  const double rr = d[0];
  const double* dots = d + 1;
  const double rinf = F.linf ? member_max(F, G, DOT_RMAX) : 0.0;
  if (threadIdx.x == 0) {
    [&] {
      // the step-2 update of this iteration was made: record it for x (the
      // first iteration of a cycle starts the cycle's list)
      Pending& pd = F.pend[m];
      if (pd.cycle != cycle) {
        pd.cycle = cycle;
        pd.n = 0;
        pd.by_orth = 0;
      }
      if (pd.n < KMAX) {
        pd.beta[pd.n] = S.beta;
        pd.slot[pd.n] = sl.s[nl - 1];
        pd.n += 1;
      }
      S.it += 1;
      const double rn = sqrt(rr);
      S.rn = rn;
      if (F.hist && S.it < F.hist_stride) F.hist[(long long)m * F.hist_stride + S.it] = rn / S.rho0;
      if (!isfinite(rn)) {
        S.status = ST_STAGNATED;
        S.done = 1;
        return;
      }
      // learned correction behind the plain preconditioner's reference
      // residual history: drop it from the next preconditioner application on
      if (F.learned && !S.fallback && F.learn_ref && S.it <= F.learn_ref_n && !(rn <= F.learn_ref[S.it] * S.rho0))
        S.fallback = 1;
      const bool small = F.linf ? rinf <= rtol * S.rho0_inf : rn <= rtol * S.rho0;
      if (S.it >= min_iters && small) {
        S.status = S.fallback ? ST_FALLBACK : ST_OK;
        S.done = 1;
        return;
      }
      if (S.it >= max_iters) {
        S.status = ST_NOT_CONVERGED;
        S.done = 1;
        return;
      }
      for (int l = 0; l < nl; ++l) S.alpha[l] = -dots[l] / S.lpsq[sl.s[l]];
      if (cycle_end) {
        // learned correction not reducing the residual enough: drop it
        if (F.learned && !S.fallback && !(rn <= F.fallback_ratio * S.rn_cycle)) {
          S.fallback = 1;
          S.rn_cycle = rn;
          return;
        }
        if (rn >= S.rn_cycle) {
          S.status = ST_STAGNATED;
          S.done = 1;
          return;
        }
        S.rn_cycle = rn;
      }
    }();
    F.done_flag[m] = S.done;
    // going on past the cycle's last iteration: its step-4 pass applies the
    // cycle's recorded solution updates
    Pending& pd = F.pend[m];
    pd.by_orth = (cycle_end && !S.done && pd.n == nl) ? 1 : 0;
  }
}

// after a float64 residual recomputation at a restart: replace ||r|| and beta
template <typename A>
__global__ void k_ctrl_restart(Fields F, int slot0) {
  const int m = F.morder[F.q0 + blockIdx.x];
  MemberState& S = F.state[m];
  if (S.done) return;
  const MemberGeom G = F.geom[m];
  const double rr = member_sum<double>(F, G, DOT_RR);
  const double num = member_sum<double>(F, G, DOT_R_LP);
  if (threadIdx.x == 0) {
    S.restarts += 1;
    S.rn = sqrt(rr);
    S.rn_cycle = S.rn;
    const double beta = -num / S.lpsq[slot0];
    if (!isfinite(beta)) {
      S.status = ST_STAGNATED;
      S.done = 1;
      F.done_flag[m] = 1;
    }
    S.beta = beta;
  }
}

// final float64 true residual of every member
static __global__ void k_ctrl_true(Fields F) {
  const int m = F.morder[F.q0 + blockIdx.x];
  const MemberGeom G = F.geom[m];
  const double rr = member_sum<double>(F, G, DOT_RR);
  if (threadIdx.x == 0) F.state[m].rtrue = sqrt(rr);
}

}  // namespace mpgcr
