// One semi-implicit time step of the shallow-water model around the elliptic
// solve (paper Sections 2.1-2.2: eqs. SWE1-SWE3, RSWE2-RSWE3, MPDATA, rhslin,
// Qexpr, Elliptic, vadv), for every member of a solver's batch:
//   1. the forcings R^n at the cell centres and Q~ = Q^n + dt/2 R^n;
//   2. face Courant numbers of the advective velocity extrapolated to
//      n + 1/2 from n and n-1;
//   3. MPDATA (donor cell + one corrective pass) of Phi^n, Q~_x, Q~_y:
//      Phi* and Qhat;
//   4. the implicit momentum inverted pointwise (eq. Qexpr): Qhathat, the
//      part of Q^{n+1} known before the solve (inside the corrective pass
//      of 3, from its Phi* and Qhat in registers);
//   5. the right-hand side R = D(F^n) + D(Fhathat) - C Phi^n of the elliptic
//      problem L(Phi^{n+1}) = R, with the operator assembled from Phi* and
//      H0 and solved by the solver's own precision form, warm-started from
//      Phi^n;
//   6. Q^{n+1} = Qhathat + A grad Phi^{n+1} + B Phi^{n+1} (eq. Qexpr).
// Fields are natural [NY][NX] float64 arrays; the kernels take one thread per
// column and band of four rows and one workgroup row (blockIdx.y) per member.
// Work arrays are the solver's, allocated on the first call.
#include "solver_impl.h"

namespace {

struct SiMember {
  const double *phi, *qx, *qy;         // state at n
  const double *phi0, *qx0, *qy0;      // state at n-1
  const double *oro, *qbx, *qby;       // H0, relaxation target (null: zero)
  double *phi1, *qx1, *qy1;            // state at n+1
  double dt, g, omega, radius, absorber;
  int nx, ny, log2nx;
  long long w;                         // offset of the member's work fields
};

// work fields per member, each wpts (>= nx * (ny + 1)) values; W_LAT holds
// the latitude table: per row j, cos(lat_j), sin(lat_j), cos(lat_{j+1/2}),
// alpha(lat_j)
enum { W_CX = 0, W_CY, W_P1, W_Q1X, W_Q1Y, W_AXP, W_AYP, W_AXQX, W_AYQX, W_AXQY, W_AYQY, W_PHIS,
       W_QTX, W_QTY, W_QHHX, W_QHHY, W_RHS, W_LAT, W_COUNT };
enum { LT_COS = 0, LT_SIN, LT_COSN, LT_ALPHA, LT_N };

struct SiArgs {
  const SiMember* tab;
  double* work;
  long long wpts;                      // values per work field and member
};

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double lat_of(int j, int ny) { return -0.5 * kPi + (j + 0.5) * (kPi / ny); }

__device__ __forceinline__ double alpha_at(double lat, double amax) {
  const double dist = 0.5 * kPi - fabs(lat);
  const double w = 1.0 - dist / (3.0 * kPi / 64.0);
  return amax * (w > 0.0 ? w : 0.0);
}

// value of field f at row jj (may be -1 or ny: the row across the pole,
// shifted by nx/2, times `sign`) and column ii (periodic)
__device__ __forceinline__ double at(const double* f, int jj, int ii, int nx, int ny, double sign) {
  double s = 1.0;
  if (jj < 0) {
    jj = 0;
    ii += nx >> 1;
    s = sign;
  } else if (jj >= ny) {
    jj = ny - 1;
    ii += nx >> 1;
    s = sign;
  }
  return s * f[(long long)jj * nx + (ii & (nx - 1))];
}

__device__ __forceinline__ double* wf(const SiArgs& A, const SiMember& M, int k) {
  return A.work + M.w + (long long)k * A.wpts;
}

// One thread per column i and band of SI_BAND consecutive rows j0 .. j1-1 of
// member blockIdx.y: a stencil's neighbour rows are loaded once per band
// row and rolled down in registers instead of loaded once per point.  Bands
// are numbered row-major over (band, column).  gridDim.x is a multiple of the
// XCD count, so block x of every member runs on XCD x mod 8; xcd_block gives
// each XCD a contiguous range of bands, and the neighbour rows a stencil
// reads come from that XCD's own L2.
constexpr int SI_BAND = 4;
#define SI_BANDS(A, M)                                                                        \
  const SiMember M = (A).tab[blockIdx.y];                                                     \
  const int nb_ = ((M.ny + SI_BAND - 1) / SI_BAND) * M.nx;                                    \
  for (int t_ = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; t_ < nb_;        \
       t_ += gridDim.x * blockDim.x)                                                          \
    for (int i_ = t_ & (M.nx - 1), j0_ = (t_ >> M.log2nx) * SI_BAND, j1_ = min(j0_ + SI_BAND, M.ny), once_ = 1; \
         once_; once_ = 0)

// the latitude table of every member
// Field stores are nontemporal: a step's work fields (18 float64 fields per
// point over the batch) stream through HBM, far beyond the memory-side cache.
__device__ __forceinline__ void nts(double* p, double v) { __builtin_nontemporal_store(v, p); }

__global__ void k_si_lat(SiArgs A) {
  const SiMember M = A.tab[blockIdx.y];
  double* t = wf(A, M, W_LAT);
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M.ny; j += gridDim.x * blockDim.x) {
    const double lat = lat_of(j, M.ny);
    t[LT_N * j + LT_COS] = cos(lat);
    t[LT_N * j + LT_SIN] = sin(lat);
    t[LT_N * j + LT_COSN] = cos(-0.5 * kPi + (j + 1.0) * (kPi / M.ny));
    t[LT_N * j + LT_ALPHA] = alpha_at(lat, M.absorber);
  }
}

// velocity of eq. vadv over a^2 at a cell: (Q_x / (a Phi), cos Q_y / (a Phi))
__device__ __forceinline__ void vel(const double* phi, const double* qx, const double* qy, long long k, double cs,
                                    double a, double& vx, double& vy) {
  vx = qx[k] / (a * phi[k]);
  vy = cs * qy[k] / (a * phi[k]);
}

// 1-2: forcings, Q~ = Q + dt/2 R^n, and the face Courant numbers at n + 1/2
__global__ void k_si_prepare(SiArgs A) {
  SI_BANDS(A, M) {
    const int nx = M.nx, ny = M.ny;
    const double* lt = wf(A, M, W_LAT);
    const double a = M.radius, d = 0.5 * M.dt;
    const double dlam = 2.0 * kPi / nx, dphi = kPi / ny;
    // Phi + H0 (across-pole rows as in the operator)
    auto hs = [&](int jj, int ii) {
      return at(M.phi, jj, ii, nx, ny, 1.0) + (M.oro ? at(M.oro, jj, ii, nx, ny, 1.0) : 0.0);
    };
    // advective velocity at n + 1/2 = 1.5 v^n - 0.5 v^{n-1} at a cell
    auto vext = [&](int jj, int ii, double& vx, double& vy) {
      const long long kk = (long long)jj * nx + (ii & (nx - 1));
      const double c = lt[LT_N * jj + LT_COS];
      double x1, y1, x0, y0;
      vel(M.phi, M.qx, M.qy, kk, c, a, x1, y1);
      vel(M.phi0, M.qx0, M.qy0, kk, c, a, x0, y0);
      vx = 1.5 * x1 - 0.5 * x0;
      vy = 1.5 * y1 - 0.5 * y0;
    };
    // column i rolled down the band: Phi + H0 at rows j-1, j; v at row j
    double hs_m = hs(j0_ - 1, i_), hs_c = hs(j0_, i_);
    double vx, vy;
    vext(j0_, i_, vx, vy);
    double* __restrict__ qtx = wf(A, M, W_QTX);
    double* __restrict__ qty = wf(A, M, W_QTY);
    double* __restrict__ ocx = wf(A, M, W_CX);
    double* __restrict__ ocy = wf(A, M, W_CY);
#pragma unroll
    for (int r = 0; r < SI_BAND; ++r) {
      const int j = j0_ + r;
      if (j >= j1_) break;
      const long long k = (long long)j * nx + i_;
      const double cs = lt[LT_N * j + LT_COS], sn = lt[LT_N * j + LT_SIN];
      const double hs_n = hs(j + 1, i_);
      // gradient of Phi + H0 (central differences)
      const double hx = (hs(j, i_ + 1) - hs(j, i_ - 1)) / (2.0 * dlam);
      const double hy = (hs_n - hs_m) / (2.0 * dphi);
      const double ph = M.phi[k], qx = M.qx[k], qy = M.qy[k];
      const double f = 2.0 * M.omega * sn, al = lt[LT_N * j + LT_ALPHA], t = sn / cs;
      const double qbx = M.qbx ? M.qbx[k] : 0.0, qby = M.qby ? M.qby[k] : 0.0;
      const double rx = -M.g / (a * cs) * ph * hx + f * qy + t * qx * qy / (a * ph) - al * (qx - qbx);
      const double ry = -M.g / a * ph * hy - f * qx - t * qx * qx / (a * ph) - al * (qy - qby);
      nts(qtx + k, qx + d * rx);
      nts(qty + k, qy + d * ry);
      // Courant numbers at the east face and the north face j + 1/2 (zero at the north pole)
      double vxe, vye;
      vext(j, i_ + 1, vxe, vye);
      nts(ocx + k, 0.5 * (vx + vxe) * M.dt / dlam);
      double cyn = 0.0, vxn = 0.0, vyn = 0.0;
      if (j < ny - 1) {
        vext(j + 1, i_, vxn, vyn);
        cyn = 0.5 * (vy + vyn) * M.dt / dphi;
      }
      nts(ocy + k, cyn);
      hs_m = hs_c;
      hs_c = hs_n;
      vx = vxn;
      vy = vyn;
    }
  }
}

// 4: Qhathat at point (j, i) from the corrective pass's Phi* (ps) and
// Qhat (qhx, qhy), and the initial guess of the solve (Phi^n)
__device__ __forceinline__ void si_qhh_point(const SiArgs& A, const SiMember& M, int j, int i, double ps, double qhx,
                                             double qhy) {
  const int nx = M.nx, ny = M.ny;
  const long long k = (long long)j * nx + i;
  const double* lt = wf(A, M, W_LAT);
  const double cs = lt[LT_N * j + LT_COS], sn = lt[LT_N * j + LT_SIN], t = sn / cs;
  const double a = M.radius, d = 0.5 * M.dt;
  const double dlam = 2.0 * kPi / nx, dphi = kPi / ny;
  const double al = lt[LT_N * j + LT_ALPHA], gam = 1.0 + d * al, b = d * 2.0 * M.omega * sn;
  const double D = gam * gam + b * b;
  double h0x = 0.0, h0y = 0.0;
  if (M.oro) {
    h0x = (at(M.oro, j, i + 1, nx, ny, 1.0) - at(M.oro, j, i - 1, nx, ny, 1.0)) / (2.0 * dlam);
    h0y = (at(M.oro, j + 1, i, nx, ny, 1.0) - at(M.oro, j - 1, i, nx, ny, 1.0)) / (2.0 * dphi);
  }
  const double mx = t * M.qx[k] * M.qy[k] / (a * M.phi[k]), my = -t * M.qx[k] * M.qx[k] / (a * M.phi[k]);
  const double mx0 = t * M.qx0[k] * M.qy0[k] / (a * M.phi0[k]), my0 = -t * M.qx0[k] * M.qx0[k] / (a * M.phi0[k]);
  const double qbx = M.qbx ? M.qbx[k] : 0.0, qby = M.qby ? M.qby[k] : 0.0;
  const double ex = qhx + d * (al * qbx + 2.0 * mx - mx0) - d * M.g / (a * cs) * 0.5 * ps * h0x;
  const double ey = qhy + d * (al * qby + 2.0 * my - my0) - d * M.g / a * 0.5 * ps * h0y;
  nts(wf(A, M, W_QHHX) + k, (gam * ex + b * ey) / D);
  nts(wf(A, M, W_QHHY) + k, (-b * ex + gam * ey) / D);
  nts(M.phi1 + k, M.phi[k]);
}

// donor-cell pass of the three advected fields: out = in - (div of upwind
// fluxes) / cos(lat); `ax*` / `ay*`: the Courant numbers of each field
struct UpwindSet {
  int in[3], out[3], cx[3], cy[3];     // work fields; in[0] < 0: Phi^n (the first pass); out[f] < 0: not stored
};

// SHARED: the three fields move with the same Courant numbers (the first
// pass), which are then read once per point.  QHH (the corrective pass):
// the implicit inversion of step 4 follows at each point, from the pass's
// Phi* and Qhat in registers; only Phi* of the three fields is stored.
template <bool SHARED, bool QHH>
__global__ void k_si_upwind(SiArgs A, UpwindSet U) {
  SI_BANDS(A, M) {
    const int nx = M.nx, ny = M.ny;
    const double* lt = wf(A, M, W_LAT);
    const int ie = (i_ + 1) & (nx - 1), iw = (i_ - 1) & (nx - 1);
    auto flux = [](double c, double l, double r) { return fmax(c, 0.0) * l + fmin(c, 0.0) * r; };
    const double* psi[3];
    const double* cxa[3];
    const double* cya[3];
    // the outputs are never read by this pass (restrict lets the next rows'
    // loads be issued before this row's stores)
    double* __restrict__ out[3];
    for (int f = 0; f < 3; ++f) {
      psi[f] = U.in[f] < 0 ? M.phi : wf(A, M, U.in[f]);
      cxa[f] = wf(A, M, U.cx[SHARED ? 0 : f]);
      cya[f] = wf(A, M, U.cy[SHARED ? 0 : f]);
      out[f] = U.out[f] < 0 ? nullptr : wf(A, M, U.out[f]);   // < 0: not stored (the fused inversion)
    }
    // column i rolled down the band: psi at rows j-1, j and C^y at face j-1/2
    const long long k0 = (long long)j0_ * nx + i_;
    double ps_m[3], ps_c[3], cy_s[3];
    for (int f = 0; f < 3; ++f) {
      ps_m[f] = j0_ > 0 ? psi[f][k0 - nx] : 0.0;
      ps_c[f] = psi[f][k0];
      cy_s[f] = (j0_ > 0 && (!SHARED || f == 0)) ? cya[f][k0 - nx] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < SI_BAND; ++r) {
      const int j = j0_ + r;
      if (j >= j1_) break;
      const long long row = (long long)j * nx, k = row + i_;
      const double g = lt[LT_N * j + LT_COS];
      double ce = 0.0, cw = 0.0, cn = 0.0;
      double nv[3];
      const double cs0 = cy_s[0];   // face j-1/2 of the shared Courant numbers
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        if (!SHARED || f == 0) {
          ce = cxa[f][k];
          cw = cxa[f][row + iw];
          cn = j < ny - 1 ? cya[f][k] : 0.0;
        }
        const double cs = SHARED ? cs0 : cy_s[f];
        const double ps_n = j < ny - 1 ? psi[f][k + nx] : 0.0;
        const double fe = flux(ce, ps_c[f], psi[f][row + ie]);
        const double fw = flux(cw, psi[f][row + iw], ps_c[f]);
        const double fn = j < ny - 1 ? flux(cn, ps_c[f], ps_n) : 0.0;
        const double fs = j > 0 ? flux(cs, ps_m[f], ps_c[f]) : 0.0;
        nv[f] = ps_c[f] - ((fe - fw) + (fn - fs)) / g;
        if (!QHH || f == 0) nts(out[f] + k, nv[f]);
        ps_m[f] = ps_c[f];
        ps_c[f] = ps_n;
        if (!SHARED || f == 0) cy_s[f] = cn;
      }
      if constexpr (QHH) si_qhh_point(A, M, j, i_, nv[0], nv[1], nv[2]);
    }
  }
}

// antidiffusive Courant numbers of the corrective pass for the three fields
// (|psi| in the ratios; momenta change sign across a pole)
__global__ void k_si_antidiff(SiArgs A) {
  SI_BANDS(A, M) {
    const int nx = M.nx, ny = M.ny;
    const double* lt = wf(A, M, W_LAT);
    const double* cx = wf(A, M, W_CX);
    const double* cy = wf(A, M, W_CY);
    const int ins[3] = {W_P1, W_Q1X, W_Q1Y};
    const int oxs[3] = {W_AXP, W_AXQX, W_AXQY};
    const int oys[3] = {W_AYP, W_AYQX, W_AYQY};
    const double tiny = 1e-300;
    // |psi| of the three fields at rows j-1 .. j+1, columns i-1 .. i+1 (the
    // rows beyond a pole seen across it; the momenta change sign there, which
    // |psi| does not see), rolled down the band
    double w[3][3][3];   // [field][row j-1, j, j+1][column i-1, i, i+1]
    auto load_row = [&](int fdx, int jj, double (&r)[3]) {
      const double* psi = wf(A, M, ins[fdx]);
      const double sg = fdx == 0 ? 1.0 : -1.0;
      r[0] = fabs(at(psi, jj, i_ - 1, nx, ny, sg));
      r[1] = fabs(at(psi, jj, i_, nx, ny, sg));
      r[2] = fabs(at(psi, jj, i_ + 1, nx, ny, sg));
    };
    // face Courant numbers: C^x at columns i-1, i of rows j, j+1; C^y (face
    // jj + 1/2, zero at the poles) at columns i, i+1 of rows j-1, j
    auto cxr = [&](int jj, double (&r)[2]) {
      r[0] = cx[(long long)jj * nx + ((i_ - 1) & (nx - 1))];
      r[1] = cx[(long long)jj * nx + i_];
    };
    auto cyr = [&](int jj, double (&r)[2]) {
      const bool in = jj >= 0 && jj < ny - 1;
      r[0] = in ? cy[(long long)jj * nx + i_] : 0.0;
      r[1] = in ? cy[(long long)jj * nx + ((i_ + 1) & (nx - 1))] : 0.0;
    };
    for (int fdx = 0; fdx < 3; ++fdx) {
      load_row(fdx, j0_ - 1, w[fdx][0]);
      load_row(fdx, j0_, w[fdx][1]);
    }
    double cxw[2][2], cyw[2][2];   // C^x rows j, j+1; C^y rows j-1, j
    cxr(j0_, cxw[0]);
    cyr(j0_ - 1, cyw[0]);
    cyr(j0_, cyw[1]);
    // the six outputs are written through restrict pointers: the next rows'
    // loads may be issued before this row's stores
    double* __restrict__ ox[3] = {wf(A, M, oxs[0]), wf(A, M, oxs[1]), wf(A, M, oxs[2])};
    double* __restrict__ oy[3] = {wf(A, M, oys[0]), wf(A, M, oys[1]), wf(A, M, oys[2])};
#pragma unroll
    for (int r = 0; r < SI_BAND; ++r) {
      const int j = j0_ + r;
      if (j >= j1_) break;
      const long long k = (long long)j * nx + i_;
      for (int fdx = 0; fdx < 3; ++fdx) load_row(fdx, j + 1, w[fdx][2]);
      if (j < ny - 1) cxr(j + 1, cxw[1]);
      const double gx = lt[LT_N * j + LT_COS];
      const double cyb = 0.25 * (cyw[1][0] + cyw[1][1] + cyw[0][0] + cyw[0][1]);
      const double c = cxw[0][1];
      double cxb = 0.0;
      if (j < ny - 1) cxb = 0.25 * (cxw[0][1] + cxw[0][0] + cxw[1][1] + cxw[1][0]);
      const double cyn = cyw[1][0];
      const double gy = lt[LT_N * j + LT_COSN];
      for (int fdx = 0; fdx < 3; ++fdx) {
        const double(&u)[3][3] = w[fdx];   // u[row][column]: rows j-1, j, j+1; columns i-1, i, i+1
        // east face
        const double pc = u[1][1], pe = u[1][2];
        const double axr = (pe - pc) / (pe + pc + tiny);
        const double num = (u[2][2] + u[2][1]) - (u[0][2] + u[0][1]);
        const double den = (u[2][2] + u[2][1]) + (u[0][2] + u[0][1]);
        const double bxr = 0.5 * num / (den + tiny);
        nts(ox[fdx] + k, (fabs(c) - c * c / gx) * axr - c * cyb / gx * bxr);
        // north face (interior faces only)
        double ay = 0.0;
        if (j < ny - 1) {
          const double pn = u[2][1];
          const double ayr = (pn - pc) / (pn + pc + tiny);
          const double nm = (u[2][2] + u[1][2]) - (u[2][0] + u[1][0]);
          const double dn = (u[2][2] + u[1][2]) + (u[2][0] + u[1][0]);
          const double byr = 0.5 * nm / (dn + tiny);
          ay = (fabs(cyn) - cyn * cyn / gy) * ayr - cyn * cxb / gy * byr;
        }
        nts(oy[fdx] + k, ay);
      }
      // roll the windows down one row
      for (int fdx = 0; fdx < 3; ++fdx)
        for (int r = 0; r < 2; ++r)
          for (int q = 0; q < 3; ++q) w[fdx][r][q] = w[fdx][r + 1][q];
      cxw[0][0] = cxw[1][0];
      cxw[0][1] = cxw[1][1];
      cyw[0][0] = cyw[1][0];
      cyw[0][1] = cyw[1][1];
      cyr(j + 1, cyw[1]);
    }
  }
}

// 5: R = D(F^n) + D(Fhathat) - C Phi^n, F = (a Q_x, a cos Q_y) at the faces
// (means of the two cells; no flux through the poles)
__global__ void k_si_rhs(SiArgs A) {
  SI_BANDS(A, M) {
    const int nx = M.nx, ny = M.ny;
    const double a = M.radius;
    const double dlam = 2.0 * kPi / nx, dphi = kPi / ny;
    const double* lt = wf(A, M, W_LAT);
    const double* hx = wf(A, M, W_QHHX);
    const double* hy = wf(A, M, W_QHHY);
    double* __restrict__ out = wf(A, M, W_RHS);
    const int ie = (i_ + 1) & (nx - 1), iw = (i_ - 1) & (nx - 1);
    auto qsx = [&](long long kk) { return M.qx[kk] + hx[kk]; };
    auto qsy = [&](long long kk) { return M.qy[kk] + hy[kk]; };
    // column i rolled down the band: Q_y + Qhathat_y at rows j-1, j
    const long long k0 = (long long)j0_ * nx + i_;
    double ys_m = j0_ > 0 ? qsy(k0 - nx) : 0.0, ys_c = qsy(k0);
#pragma unroll
    for (int r = 0; r < SI_BAND; ++r) {
      const int j = j0_ + r;
      if (j >= j1_) break;
      const long long row = (long long)j * nx, k = row + i_;
      const double ys_n = j < ny - 1 ? qsy(k + nx) : 0.0;
      const double xs_c = qsx(k);
      const double fe = a * 0.5 * (xs_c + qsx(row + ie)), fw = a * 0.5 * (qsx(row + iw) + xs_c);
      const double cn = lt[LT_N * j + LT_COSN], csf = j > 0 ? lt[LT_N * (j - 1) + LT_COSN] : 0.0;
      const double fn = j < ny - 1 ? a * cn * 0.5 * (ys_c + ys_n) : 0.0;
      const double fs = j > 0 ? a * csf * 0.5 * (ys_m + ys_c) : 0.0;
      const double C = 2.0 * a * a * lt[LT_N * j + LT_COS] / M.dt;
      nts(out + k, (fe - fw) / dlam + (fn - fs) / dphi - C * M.phi[k]);
      ys_m = ys_c;
      ys_c = ys_n;
    }
  }
}

// 6: Q^{n+1} = Qhathat + A grad Phi^{n+1} + B Phi^{n+1}
__global__ void k_si_recover(SiArgs A) {
  SI_BANDS(A, M) {
    const int nx = M.nx, ny = M.ny;
    const double* lt = wf(A, M, W_LAT);
    const double a = M.radius, d = 0.5 * M.dt;
    const double dlam = 2.0 * kPi / nx, dphi = kPi / ny;
    const double* ps = wf(A, M, W_PHIS);
    const double* p1 = M.phi1;
    auto hs = [&](int jj, int ii) { return at(ps, jj, ii, nx, ny, 1.0) + (M.oro ? at(M.oro, jj, ii, nx, ny, 1.0) : 0.0); };
    // column i rolled down the band: Phi^{n+1} and Phi* + H0 at rows j-1, j
    double p1_m = at(p1, j0_ - 1, i_, nx, ny, 1.0), p1_c = at(p1, j0_, i_, nx, ny, 1.0);
    double hs_m = hs(j0_ - 1, i_), hs_c = hs(j0_, i_);
    double* __restrict__ qx1 = M.qx1;
    double* __restrict__ qy1 = M.qy1;
#pragma unroll
    for (int r = 0; r < SI_BAND; ++r) {
      const int j = j0_ + r;
      if (j >= j1_) break;
      const long long k = (long long)j * nx + i_;
      const double cs = lt[LT_N * j + LT_COS], sn = lt[LT_N * j + LT_SIN];
      const double al = lt[LT_N * j + LT_ALPHA], gam = 1.0 + d * al, b = d * 2.0 * M.omega * sn;
      const double D = gam * gam + b * b;
      const double p1_n = at(p1, j + 1, i_, nx, ny, 1.0), hs_n = hs(j + 1, i_);
      const double px = (at(p1, j, i_ + 1, nx, ny, 1.0) - at(p1, j, i_ - 1, nx, ny, 1.0)) / (2.0 * dlam);
      const double py = (p1_n - p1_m) / (2.0 * dphi);
      const double hx = (hs(j, i_ + 1) - hs(j, i_ - 1)) / (2.0 * dlam);
      const double hy = (hs_n - hs_m) / (2.0 * dphi);
      const double ux = -d * M.g / (a * cs) * 0.5 * (p1_c * hx + ps[k] * px);
      const double uy = -d * M.g / a * 0.5 * (p1_c * hy + ps[k] * py);
      nts(qx1 + k, wf(A, M, W_QHHX)[k] + (gam * ux + b * uy) / D);
      nts(qy1 + k, wf(A, M, W_QHHY)[k] + (-b * ux + gam * uy) / D);
      p1_m = p1_c;
      p1_c = p1_n;
      hs_m = hs_c;
      hs_c = hs_n;
    }
  }
}

}  // namespace

extern "C" int gcr_si_step(gcr_solver* s, const gcr_si_member* members, gcr_report* reports) {
  if (!s) return GCR_EINVAL;
  if (!members) return fail(s, GCR_EINVAL, "gcr_si_step: NULL member table");
  const int B = s->prm.batch;
  long long wpts = 0;
  for (int m = 0; m < B; ++m) {
    const gcr_si_member& q = members[m];
    if (!q.phi || !q.qx || !q.qy || !q.phi_old || !q.qx_old || !q.qy_old || !q.phi_new || !q.qx_new || !q.qy_new)
      return fail(s, GCR_EINVAL, "member %d: NULL state field", m);
    if (!(q.dt > 0.0) || !(q.g > 0.0) || !(q.radius > 0.0) || !std::isfinite(q.omega) || !(q.absorber >= 0.0))
      return fail(s, GCR_EINVAL, "member %d: dt, g, radius must be > 0, absorber >= 0", m);
    {   // the new fields are written while every other field is read
      const void* outs[3] = {q.phi_new, q.qx_new, q.qy_new};
      const void* ins[9] = {q.phi, q.qx, q.qy, q.phi_old, q.qx_old, q.qy_old, q.orography, q.qbar_x, q.qbar_y};
      for (int a = 0; a < 3; ++a) {
        for (int b = a + 1; b < 3; ++b)
          if (outs[a] == outs[b]) return fail(s, GCR_EINVAL, "member %d: the new fields must be distinct", m);
        for (const void* in : ins)
          if (outs[a] == in) return fail(s, GCR_EINVAL, "member %d: the new state must not alias an input field", m);
      }
    }
    wpts = std::max(wpts, (long long)s->nx[m] * (s->ny[m] + 1));
  }
  wpts = (wpts + 63) / 64 * 64;
  if (!s->si_work || s->si_wpts < wpts) {
    hipError_t herr = hipSuccess;
    if (s->si_work) (void)hipFree(s->si_work);
    s->si_work = dalloc<double>((size_t)wpts * W_COUNT * B, herr);
    if (herr != hipSuccess) {
      s->si_work = nullptr;
      return fail(s, GCR_ENOMEM, "semi-implicit step work arrays: %s", hipGetErrorString(herr));
    }
    s->si_wpts = wpts;
    if (!s->si_tab) {
      s->si_tab = dalloc<SiMember>(B, herr);
      if (herr == hipSuccess) herr = hipHostMalloc(&s->si_stage, (size_t)B * sizeof(SiMember), 0);
      if (herr != hipSuccess) return fail(s, GCR_ENOMEM, "semi-implicit step tables: %s", hipGetErrorString(herr));
      s->allocs.push_back(s->si_tab);
    }
  }
  // the staged table may still feed the previous upload
  HIPCHK(s, hipStreamSynchronize(s->stream));
  SiMember* tab_h = (SiMember*)s->si_stage;
  int nymax = 0, nbandmax = 0;
  for (int m = 0; m < B; ++m) {
    const gcr_si_member& q = members[m];
    SiMember& t = tab_h[m];
    t.phi = q.phi;
    t.qx = q.qx;
    t.qy = q.qy;
    t.phi0 = q.phi_old;
    t.qx0 = q.qx_old;
    t.qy0 = q.qy_old;
    t.oro = q.orography;
    t.qbx = q.qbar_x;
    t.qby = q.qbar_y;
    t.phi1 = q.phi_new;
    t.qx1 = q.qx_new;
    t.qy1 = q.qy_new;
    t.dt = q.dt;
    t.g = q.g;
    t.omega = q.omega;
    t.radius = q.radius;
    t.absorber = q.absorber;
    t.nx = s->nx[m];
    t.ny = s->ny[m];
    t.log2nx = ilog2(t.nx);
    t.w = (long long)m * W_COUNT * wpts;
    nymax = std::max(nymax, t.ny);
    nbandmax = std::max(nbandmax, t.nx * ((t.ny + SI_BAND - 1) / SI_BAND));
  }
  HIPCHK(s, hipMemcpyAsync(s->si_tab, tab_h, (size_t)B * sizeof(SiMember), hipMemcpyHostToDevice, s->stream));
  SiArgs A{(const SiMember*)s->si_tab, s->si_work, wpts};
  const dim3 blk(256);
  const int nblk_b = (std::min((nbandmax + 255) / 256, 4096) + NXCD - 1) / NXCD * NXCD;
  const dim3 grid_b((unsigned)nblk_b, (unsigned)B);   // the band kernels
  KLAUNCH(s, KT_SI_STEP, k_si_lat, dim3((unsigned)((nymax + 255) / 256), (unsigned)B), blk, 0, s->stream, A);
  KLAUNCH(s, KT_SI_STEP, k_si_prepare, grid_b, blk, 0, s->stream, A);
  UpwindSet U1{{-1, W_QTX, W_QTY}, {W_P1, W_Q1X, W_Q1Y}, {W_CX, W_CX, W_CX}, {W_CY, W_CY, W_CY}};
  KLAUNCH(s, KT_SI_STEP, (k_si_upwind<true, false>), grid_b, blk, 0, s->stream, A, U1);
  KLAUNCH(s, KT_SI_STEP, k_si_antidiff, grid_b, blk, 0, s->stream, A);
  // the corrective pass stores Phi*; its Qhat goes straight into the implicit inversion
  UpwindSet U2{{W_P1, W_Q1X, W_Q1Y}, {W_PHIS, -1, -1}, {W_AXP, W_AXQX, W_AXQY}, {W_AYP, W_AYQX, W_AYQY}};
  KLAUNCH(s, KT_SI_STEP, (k_si_upwind<false, true>), grid_b, blk, 0, s->stream, A, U2);
  KLAUNCH(s, KT_SI_STEP, k_si_rhs, grid_b, blk, 0, s->stream, A);
  HIPCHK(s, hipGetLastError());
  // the elliptic problem: the operator from Phi* and H0, solved from Phi^n
  std::vector<gcr_operator> ops(B);
  std::vector<int32_t> mem(B);
  std::vector<const double*> rhs(B);
  std::vector<double*> xs(B);
  for (int m = 0; m < B; ++m) {
    const gcr_si_member& q = members[m];
    gcr_operator& o = ops[m];
    o.dt = q.dt;
    o.g = q.g;
    o.omega = q.omega;
    o.radius = q.radius;
    o.absorber = q.absorber;
    o.depth = s->si_work + (long long)m * W_COUNT * wpts + (long long)W_PHIS * wpts;
    o.orography = q.orography;
    o.b_terms = 1;
    o.mem_is_device = 1;
    mem[m] = m;
    rhs[m] = s->si_work + (long long)m * W_COUNT * wpts + (long long)W_RHS * wpts;
    xs[m] = q.phi_new;
  }
  int rc = gcr_set_operators(s, B, mem.data(), ops.data());
  if (rc < 0) return rc;
  const int st = gcr_solve(s, rhs.data(), xs.data(), reports);
  if (st < 0) return st;
  KLAUNCH(s, KT_SI_STEP, k_si_recover, grid_b, blk, 0, s->stream, A);
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return st;
}
