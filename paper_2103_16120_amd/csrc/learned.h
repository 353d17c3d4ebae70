// Solver-side kernels of the learned preconditioner: scale of the residual,
// feature packing into the network's input tensor, and the correction
//   e <- e + T^{-1}( s sigma N(r / sigma, e / (s sigma), cos(lat)) )
// in physical units (s = dt / (2 a^2); L is of size 1/s, so e = P^{-1} r is of
// size s r and both network inputs are of order one).  T = I - eta (P^Z - P^H)
// is the row operator of the semi-implicit preconditioner: the network's
// output passes through the same implicit zonal solve as the Richardson
// iterates, which keeps its pixel-scale errors out of the stiff zonal part of
// L near the poles.  In the mixed forms r is held scaled by s, so there
// sigma_held = s sigma.
#pragma once

#include "kernels.h"

namespace mpgcr {

constexpr int LEARN_CIN = 3;

struct LearnArgs {
  const void* r;         // residual in the form's vector type (pooled, row-interleaved)
  void* e;               // preconditioner output to correct (same type and layout)
  __bf16* feat;          // network input [batch][ny][nx][feat_stride] (bf16, NHWC)
  int feat_stride;       // channels stored per pixel (8 or 32)
  const float* y;        // network output [batch][ny][nx]
  int use_part;          // sigma from the per-row <r,r> partials (1) or from r (0)
  int* active;           // [batch]: members corrected by this application (network input mask), or null
};

// cosine of the cell-centre latitude of row j (rows from the south pole)
__device__ __forceinline__ double learn_cos(int j, int ny) { return sin(M_PI * (j + 0.5) / ny); }

__device__ __forceinline__ bool learn_skip(const Fields& F, const MemberState& S) {
  return !F.ignore_done && (S.done || S.fallback);
}

// sigma of each member: RMS of its residual in the form's units.  One block
// per member of the batch; members outside [member0, member0 + count) or
// skipped are marked inactive, so the network does not run on their images.
template <typename P>
__global__ void k_learn_sigma(Fields F, LearnArgs A, int member0, int count) {
  using V = typename P::V;
  const int m = blockIdx.x;
  MemberState& S = F.state[m];
  const bool act = m >= member0 && m < member0 + count && !learn_skip(F, S);
  if (A.active && threadIdx.x == 0) A.active[m] = act ? 1 : 0;
  if (!act) return;
  const MemberGeom G = F.geom[m];
  double rr;
  if (A.use_part) {
    rr = member_sum<double>(F, G, DOT_RR);
  } else {
    const V* r = (const V*)A.r + G.off;
    const long long n = (long long)G.nx * G.ny;
    double acc = 0.0;
    for (long long k = threadIdx.x; k < n; k += 64) {
      const double v = (double)r[k];
      acc += v * v;
    }
    rr = wave_sum(acc);
  }
  if (threadIdx.x == 0) S.sigma = sqrt(rr / ((double)G.nx * G.ny));
}

// per-member factors: features (r * fr, e * fe); correction y * fc.  `sigma`
// is the RMS of r as held, u * sigma_physical.
template <typename P>
__device__ __forceinline__ void learn_factors(const Fields& F, int m, double sigma, double& fr, double& fe,
                                              double& fc) {
  const double s = F.scale[m];
  const double u = P::mixed ? s : 1.0;    // r held as u * r_physical
  if (sigma > 0.0) {
    fr = 1.0 / sigma;
    fe = u / (s * sigma);
    fc = s * sigma / u;
  } else {
    fr = fe = fc = 0.0;
  }
}

// one wave per row: write the row's pixels of the network input
template <typename P, int M>
__device__ __forceinline__ void kb_learn_pack(const Fields& F, LearnArgs A) {
  using V = typename P::V;
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const MemberState& S = F.state[m];
  if (learn_skip(F, S)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  double fr, fe, fc;
  learn_factors<P>(F, m, S.sigma, fr, fe, fc);
  double rv[M], ev[M];
  ldr<M>((const V*)A.r + R.rc, R.lane, R.L, rv);
  ldr<M>((const V*)A.e + R.rc, R.lane, R.L, ev);
  if (!R.act) return;
  const __bf16 cz = (__bf16)(float)learn_cos(R.j, G.ny);
  const long long row_pix = ((long long)m * G.ny + R.j) * G.nx;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int i = R.lane * M + k;
    bf16x8 v0;
#pragma unroll
    for (int c = 0; c < 8; ++c) v0[c] = (__bf16)0.f;
    v0[0] = (__bf16)(float)(rv[k] * fr);
    v0[1] = (__bf16)(float)(ev[k] * fe);
    v0[2] = cz;
    bf16x8* dst = (bf16x8*)(A.feat + (row_pix + i) * A.feat_stride);
    dst[0] = v0;
    for (int q = 1; q < A.feat_stride / 8; ++q) dst[q] = bf16x8{};
  }
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_learn_pack(Fields F, LearnArgs A) {
  if constexpr (M > 0) {
    kb_learn_pack<P, M>(F, A);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_learn_pack<P, 2>(F, A); break;
      case 2: kb_learn_pack<P, 4>(F, A); break;
      case 3: kb_learn_pack<P, 8>(F, A); break;
      default: break;
    }
  }
}

// T = I - eta (P^Z - P^H) of the lane's points of one row
template <typename T, int M, typename CV>
__device__ __forceinline__ void learn_row_system(const RowCtx& R, const CV& cv, T (&lo)[M], T (&di)[M],
                                                 T (&up)[M]) {
  const T helm = cv.helm(R.g);
  T axe[M], axw[M], ayn[M], ays[M];
  row_faces<T, M>(R, cv, axe, axw, ayn, ays);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const T eta = qdiv((T)1, ayn[k] + ays[k]);
    row_system(eta, axe[k], axw[k], helm, lo[k], di[k], up[k]);
  }
}

// one wave per row: e += T^{-1}(fc * y)
template <typename P, int M>
__device__ __forceinline__ void kb_learn_apply(const Fields& F, LearnArgs A) {
  using T = typename P::T;
  using V = typename P::V;
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const MemberState& S = F.state[m];
  if (learn_skip(F, S)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  double fr, fe, fc;
  learn_factors<P>(F, m, S.sigma, fr, fe, fc);
  const float* yrow = A.y + ((long long)m * G.ny + R.j) * G.nx + R.lane * M;
  with_coef<P>(F, G, R.j, false, [&](const auto& cv) {
    T lo[M], di[M], up[M], rh[M], z[M], ev[M];
    learn_row_system<T, M>(R, cv, lo, di, up);
#pragma unroll
    for (int k = 0; k < M; ++k) rh[k] = (T)(fc * (double)yrow[k]);
    solve_row<T, M>(R, lo, di, up, rh, z);
    ldr<M>((const V*)A.e + R.rc, R.lane, R.L, ev);
#pragma unroll
    for (int k = 0; k < M; ++k) ev[k] += z[k];
    if (R.act) str<M>((V*)A.e + R.rc, R.lane, R.L, ev);
  });
}

template <typename P, int M>
__global__ __launch_bounds__(WG) void k_learn_apply(Fields F, LearnArgs A) {
  if constexpr (M > 0) {
    kb_learn_apply<P, M>(F, A);
  } else {   // rows of several row classes (M = 2, 4, 8) in one launch
    switch (row_class(F)) {
      case 1: kb_learn_apply<P, 2>(F, A); break;
      case 2: kb_learn_apply<P, 4>(F, A); break;
      case 3: kb_learn_apply<P, 8>(F, A); break;
      default: break;
    }
  }
}

// training data, natural [NY][NX] order: features and target T(e_hi - e_lo)
// (scaled) of one member from float64 pooled r, e_lo and (optionally) e_hi
template <int M>
__global__ __launch_bounds__(WG) void k_learn_features(Fields F, const double* r, const double* elo,
                                                       const double* ehi, float* feat, float* target) {
  int g, m, lane, w;
  MemberGeom G;
  if (!wave_row(F, g, m, G, lane, w)) return;
  const RowCtx R = make_row(G, m, g, lane, M);
  double fr, fe, fc;
  learn_factors<PrecF64>(F, m, F.state[m].sigma, fr, fe, fc);
  const long long np = (long long)G.nx * G.ny;
  const float cz = (float)learn_cos(R.j, G.ny);
  double lo[M], di[M], up[M];
  learn_row_system<double, M>(R, CoefFly<double>{F.fly64}, lo, di, up);
  if (!R.act) return;
  // stored position of natural point i of the row: (i mod M) * L + i / M
  auto at = [&](const double* v, int i) {
    i &= G.nx - 1;
    return v[R.rc + (long long)(i & (M - 1)) * R.L + (i / M)];
  };
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int i = R.lane * M + k;
    const long long dst = (long long)R.j * G.nx + i;
    feat[dst] = (float)(at(r, i) * fr);
    feat[np + dst] = (float)(at(elo, i) * fe);
    feat[2 * np + dst] = cz;
    if (target) {
      const double dc = at(ehi, i) - at(elo, i);
      const double dw = at(ehi, i - 1) - at(elo, i - 1);
      const double de = at(ehi, i + 1) - at(elo, i + 1);
      target[dst] = (float)((lo[k] * dw + di[k] * dc + up[k] * de) * fe);
    }
  }
}

}  // namespace mpgcr
