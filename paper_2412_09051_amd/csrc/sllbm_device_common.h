// Device helpers shared by the HIP kernels of libsllbm: closed-form Hermite
// equilibrium and the per-node gather of one streamed population on tensor meshes.
#pragma once

#include <hip/hip_runtime.h>

#include "sllbm_kernels.h"

namespace sllbm {

// ------------------------------------------------------------------ equilibrium
// Closed form of the 4th-order Hermite expansion (f^eq display, N = 4) in the scaled
// variables xi = zeta/sqrt(T0), ut = u/sqrt(T0), t = T/T0 - 1, s = xi.ut, q = |xi|^2:
//   f^eq / (w rho) = c0 + c1 s + c2 s^2 + s^3/6 + s^4/24
// with c0 = A0 + A1 q + A2 q^2, c1 = B0 + B1 q, c2 = C0 + C1 q (per-node constants).
struct EqNode {
  double rho, ux, uy, uz;
  double A0, A1, A2, B0, B1, C0, C1;
};

__device__ __forceinline__ EqNode eq_prepare(double rho, double u0, double u1, double u2, double T,
                                             const StepArgs &a, int D) {
  EqNode e;
  e.rho = rho;
  e.ux = u0 * a.inv_sqrtT0;
  e.uy = u1 * a.inv_sqrtT0;
  e.uz = u2 * a.inv_sqrtT0;
  double U = e.ux * e.ux + e.uy * e.uy + e.uz * e.uz;
  double t = T / a.T0 - 1.0;
  double Dd = (double)D;
  e.A0 = 1.0 - 0.5 * U - 0.5 * t * Dd + 0.125 * U * U + 0.25 * t * U * (Dd + 2.0) + 0.125 * t * t * Dd * (Dd + 2.0);
  e.A1 = 0.5 * t - 0.25 * t * U - 0.25 * t * t * (Dd + 2.0);
  e.A2 = 0.125 * t * t;
  e.B0 = 1.0 - 0.5 * U - 0.5 * t * (Dd + 2.0);
  e.B1 = 0.5 * t;
  e.C0 = 0.5 - 0.25 * U - 0.25 * t * (Dd + 4.0);
  e.C1 = 0.25 * t;
  return e;
}

// Equilibrium at the forced velocity u + F dt / rho (Kupershtokh's exact difference,
// Sec. 4.3): F is the step's constant force, or the plan's controlled device value.
__device__ __forceinline__ EqNode eq_forced(double rho, double u0, double u1, double u2, double T,
                                            const StepArgs &a, int D) {
  double F0 = a.force[0], F1 = a.force[1], F2 = a.force[2];
  if (a.force_dev) {
    F0 = a.force_dev[0];
    F1 = a.force_dev[1];
    F2 = a.force_dev[2];
  }
  const double r = a.dt / rho;
  return eq_prepare(rho, u0 + F0 * r, u1 + F1 * r, u2 + F2 * r, T, a, D);
}

// vel: [zeta x,y,z, xi x,y,z, |xi|^2, w] of one velocity
__device__ __forceinline__ double eq_f(const EqNode &e, const double *vel) {
  double s = vel[3] * e.ux + vel[4] * e.uy + vel[5] * e.uz;
  double q = vel[6];
  double c0 = e.A0 + q * (e.A1 + q * e.A2);
  double c1 = e.B0 + e.B1 * q;
  double c2 = e.C0 + e.C1 * q;
  double poly = c0 + s * (c1 + s * (c2 + s * (1.0 / 6.0 + s * (1.0 / 24.0))));
  return vel[7] * e.rho * poly;
}

// ------------------------------------------------------------------ Prandtl-number term
// The collision of Sec. 3.1 adds (1/tau - 1/tau_Pr) h*_i with tau_Pr = (tau - 1/2)/Pr + 1/2.
// h* (deferred to the paper's references; this library's reading) is the lowest-order
// Hermite part that carries the node's heat flux and no moment of order <= 2:
//   f*_i = w_i (q_f . zeta_i)(|zeta_i|^2 - (D+2) T0) / ((D+2) T0^3),  g*_i = 2 w_i (q_g . zeta_i) / T0,
// with c = zeta - u, q_f = 1/2 sum_i c |c|^2 f_i, q_g = 1/2 sum_i c g_i over the streamed
// values.  The equilibria carry no heat flux, so the isothermal-wall correction leaves q as it is.
struct HeatFlux {
  double f0, f1, f2, g0, g1, g2;
};

__device__ __forceinline__ void heat_flux_add(HeatFlux &q, const double *vel, double u0, double u1, double u2,
                                              double f, double g) {
  const double c0 = vel[0] - u0, c1 = vel[1] - u1, c2 = vel[2] - u2;
  const double hf = 0.5 * (c0 * c0 + c1 * c1 + c2 * c2) * f, hg = 0.5 * g;
  q.f0 += c0 * hf;
  q.f1 += c1 * hf;
  q.f2 += c2 * hf;
  q.g0 += c0 * hg;
  q.g1 += c1 * hg;
  q.g2 += c2 * hg;
}

// Per-node coefficients of the term: af = coef q_f / ((D+2) T0^2), ag = 2 coef q_g / T0, so
// that coef f*_i = w_i (af . zeta_i)(|xi_i|^2 - (D+2)) and coef g*_i = w_i (ag . zeta_i).
struct PrTerm {
  double af0, af1, af2, ag0, ag1, ag2, dp2;
};

__device__ __forceinline__ PrTerm pr_term(const HeatFlux &q, double inv_tau, const StepArgs &a, int D) {
  const double tpr = (1.0 / inv_tau - 0.5) / a.Pr + 0.5;
  const double coef = inv_tau - 1.0 / tpr;
  const double cf = coef / ((D + 2) * a.T0 * a.T0), cg = 2.0 * coef / a.T0;
  PrTerm p;
  p.af0 = cf * q.f0;
  p.af1 = cf * q.f1;
  p.af2 = cf * q.f2;
  p.ag0 = cg * q.g0;
  p.ag1 = cg * q.g1;
  p.ag2 = cg * q.g2;
  p.dp2 = (double)(D + 2);
  return p;
}

// vel: [zeta x,y,z, xi x,y,z, |xi|^2, w] of one velocity
__device__ __forceinline__ void pr_add(const PrTerm &p, const double *vel, double &fo, double &go) {
  const double zf = p.af0 * vel[0] + p.af1 * vel[1] + p.af2 * vel[2];
  const double zg = p.ag0 * vel[0] + p.ag1 * vel[1] + p.ag2 * vel[2];
  fo += vel[7] * zf * (vel[6] - p.dp2);
  go += vel[7] * zg;
}

// ------------------------------------------------------------------ tensor streaming
template <typename T> struct WeightSel;
template <> struct WeightSel<double> {
  __device__ static const double *get(const DevAxis &ax) { return ax.w64; }
  __device__ static double exc(const ExcEntry &e, int j) { return e.w[j]; }
};
template <> struct WeightSel<float> {
  __device__ static const float *get(const DevAxis &ax) { return ax.w32; }
  __device__ static float exc(const ExcEntry &e, int j) { return e.w32[j]; }
};

// Streamed value of velocity i at node n (tensor mesh): the departure point's
// interpolant (eq:intf) evaluated sum-factorised with per-axis 1D weights; boundary
// layers use their face entries (bounce-back / outlet stencil, or inlet equilibrium).
template <typename T, int D, int P>
__device__ __forceinline__ void stream_tp(const DevTensorPlan &pl, const StepArgs &sa, const T *__restrict__ pin,
                                          const int (&n)[3], int i, const ExcEntry *e0, const ExcEntry *e1,
                                          int fax0, int fax1, double scale, double &fv, double &gv) {
  const ExcEntry *ex = nullptr;
  int fax = -1;
  if (e0 && e0[i].kind != EXC_NONE) { ex = &e0[i]; fax = fax0; }
  else if (e1 && e1[i].kind != EXC_NONE) { ex = &e1[i]; fax = fax1; }
  const int Q = pl.Q;
  if (ex && ex->kind == EXC_INLET) {
    const double *st = sa.inlet + 5 * ex->src;
    EqNode e = eq_prepare(st[0], st[1], st[2], st[3], st[4], sa, D);
    fv = eq_f(e, pl.vel + 8 * i);
    gv = st[4] * sa.gbase * fv;
    return;
  }
  int src = ex ? ex->src : i;
  int st[3];
  int len[3];
  T w[3][P + 1];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    len[a] = 1;
    st[a] = 0;
#pragma unroll
    for (int j = 0; j <= P; j++) w[a][j] = (j == 0) ? T(1) : T(0);
  }
#pragma unroll
  for (int a = 0; a < D; a++) {
    const DevAxis &ax = pl.ax[a];
    if (a == fax) {
      st[a] = ex->start;
      len[a] = P + 1;
#pragma unroll
      for (int j = 0; j <= P; j++) w[a][j] = WeightSel<T>::exc(*ex, j);
    } else {
      int tb = ex ? ex->tab[a] : pl.tab_reg[a * Q + i];
      if (ax.ident[tb]) {
        st[a] = n[a];
        len[a] = 1;
      } else {
        size_t r = (size_t)tb * ax.N + n[a];
        st[a] = ax.start[r];
        len[a] = P + 1;
        const T *wp = WeightSel<T>::get(ax) + r * (P + 1);
#pragma unroll
        for (int j = 0; j <= P; j++) w[a][j] = wp[j];
      }
    }
  }
  const int N0 = pl.ax[0].N, N1 = pl.ax[1].N, N2 = pl.ax[2].N;
  const T *F = pin + (size_t)src * pl.N;
  const T *G = pin + ((size_t)Q + src) * pl.N;
  T fz = 0, gz = 0;
#pragma unroll
  for (int jz = 0; jz <= P; jz++) {
    if (jz >= len[2]) break;
    int mz = st[2] + jz;
    if (mz >= N2) mz -= N2;
    T fy = 0, gy = 0;
#pragma unroll
    for (int jy = 0; jy <= P; jy++) {
      if (jy >= len[1]) break;
      int my = st[1] + jy;
      if (my >= N1) my -= N1;
      size_t row = ((size_t)mz * N1 + my) * N0;
      T fx = 0, gx = 0;
#pragma unroll
      for (int jx = 0; jx <= P; jx++) {
        if (jx >= len[0]) break;
        int mx = st[0] + jx;
        if (mx >= N0) mx -= N0;
        fx += w[0][jx] * F[row + mx];
        gx += w[0][jx] * G[row + mx];
      }
      fy += w[1][jy] * fx;
      gy += w[1][jy] * gx;
    }
    fz += w[2][jz] * fy;
    gz += w[2][jz] * gy;
  }
  fv = scale * (double)fz;
  gv = scale * (double)gz;
}

}  // namespace sllbm
