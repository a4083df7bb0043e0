// CSR step kernel for curvilinear meshes (gfx950): one node per lane; every
// (velocity, node) row names the cell holding the departure point and the source
// population (bounce-back: the opposite one) in one word, and the departure point's
// reference coordinates in that cell, from which the kernel evaluates the (p+1)^2 weights
// of eq:intf; or an inlet state (Sec. 3.3.1).  Interpolation accumulates in FP64 for both
// storage precisions.  For Q = 25 (D2V25) the 50 streamed values stay in registers
// between the moments and the relaxation, so every row is read once per step.
#include <hip/hip_runtime.h>

#include "sllbm_device_common.h"
#include "sllbm_kernels.h"

namespace sllbm {

// Lagrange basis of the cell's support points at t (eq:intf): l_a = lam_a prod_{b != a} (t - x_b),
// by prefix and suffix products (no division; exact 0/1 at a support point).
template <int P>
__device__ __forceinline__ void basis_at(const DevCsrPlan &pl, double t, double (&l)[P + 1]) {
  double d[P + 1], pre[P + 1];
#pragma unroll
  for (int b = 0; b <= P; b++) d[b] = t - pl.xref[b];
  pre[0] = 1.0;
#pragma unroll
  for (int a = 1; a <= P; a++) pre[a] = pre[a - 1] * d[a - 1];
  double suf = 1.0;
#pragma unroll
  for (int a = P; a >= 0; a--) {
    l[a] = pl.lam[a] * pre[a] * suf;
    suf *= d[a];
  }
}

// The reference coordinates (xi, eta) of row (i, k): FP64 plans store them as two FP64
// planes per velocity, FP32 plans as one interleaved FP32 pair per row (8 B per row
// instead of 16; the coordinate's rounding moves the interpolated value by at most about 1e-7
// of its change across the cell, far below the FP32 storage rounding).
template <typename T> struct RowXi;
template <> struct RowXi<double> {
  __device__ static void get(const DevCsrPlan &pl, int i, int64_t k, double &x, double &y) {
    x = pl.row_xi[(size_t)(2 * i) * pl.N + k];
    y = pl.row_xi[(size_t)(2 * i + 1) * pl.N + k];
  }
};
template <> struct RowXi<float> {
  __device__ static void get(const DevCsrPlan &pl, int i, int64_t k, double &x, double &y) {
    const float2 r = ((const float2 *)pl.row_xf)[(size_t)i * pl.N + k];
    x = r.x;
    y = r.y;
  }
};

// The plan row of (velocity i, node k): the cell holding the departure point (-1: inlet),
// the source population (or the inlet's bc index) and the reference coordinates.
struct CsrRow {
  int c, src;
  double xi, eta;
};
template <typename T>
__device__ __forceinline__ CsrRow load_row(const DevCsrPlan &pl, int64_t k, int i) {
  CsrRow r;
  const int code = pl.row_code[(size_t)i * pl.N + k];
  // the opposite velocity through the scalar cache (i is the same for the whole wave)
  const int op = ((const int32_t __attribute__((address_space(4))) *)pl.opp)[i];
  r.c = code < 0 ? -1 : (code & (kCsrOpp - 1));
  r.src = code < 0 ? -1 - code : ((code & kCsrOpp) ? op : i);
  RowXi<T>::get(pl, i, k, r.xi, r.eta);
  return r;
}

template <typename T, int P>
__device__ __forceinline__ void stream_row(const DevCsrPlan &pl, const StepArgs &sa, const T *__restrict__ pin,
                                           int i, const CsrRow &r, double scale, double &fv, double &gv) {
  constexpr int NPC = (P + 1) * (P + 1);
  const int64_t N = pl.N;
  const int c = r.c, src = r.src;
  if (c < 0) {  // equilibrium inlet (Sec. 3.3.1)
    const double *st = sa.inlet + 5 * src;
    EqNode e = eq_prepare(st[0], st[1], st[2], st[3], st[4], sa, 2);
    fv = eq_f(e, pl.vel + 8 * i);
    gv = st[4] * sa.gbase * fv;
    return;
  }
  // the (p+1)^2 weights are products of the 1D bases at the departure point's reference
  // coordinates, evaluated here instead of being read from the plan
  double lx[P + 1], ly[P + 1];
  basis_at<P>(pl, r.xi, lx);
  basis_at<P>(pl, r.eta, ly);
  const int32_t *cn = pl.cell_nodes + (size_t)c * NPC;
  const T *F = pin + (size_t)src * N;
  const T *G = pin + ((size_t)pl.Q + src) * N;
  double a = 0, b = 0;
#pragma unroll
  for (int jy = 0; jy <= P; jy++) {
    double ax = 0, bx = 0;
#pragma unroll
    for (int jx = 0; jx <= P; jx++) {
      const int n = cn[jx + (P + 1) * jy];
      ax += lx[jx] * (double)F[n];
      bx += lx[jx] * (double)G[n];
    }
    a += ly[jy] * ax;
    b += ly[jy] * bx;
  }
  fv = scale * a;
  gv = scale * b;
}

template <typename T, int P>
__device__ __forceinline__ void stream_csr(const DevCsrPlan &pl, const StepArgs &sa, const T *__restrict__ pin,
                                           int64_t k, int i, double scale, double &fv, double &gv) {
  stream_row<T, P>(pl, sa, pin, i, load_row<T>(pl, k, i), scale, fv, gv);
}

// relaxation of one node given its streamed populations (thermal wall, BGK, force)
struct NodeRelax {
  EqNode eq, eqp, eqf;
  bool thermal, force;
  double Tpre, gT, itau, u0, u1;
  PrTerm pt;   // the quasi-equilibrium term (kernels instantiated for Pr != 1)
};

__device__ __forceinline__ NodeRelax node_relax(const StepArgs &sa, double rho, double j0, double j1, double E,
                                                double Tw) {
  NodeRelax s;
  double u0 = j0 / rho, u1 = j1 / rho;
  s.u0 = u0;
  s.u1 = u1;
  s.Tpre = (E - rho * (u0 * u0 + u1 * u1)) / (2.0 * rho * sa.cv);
  s.thermal = (Tw == Tw);
  double Tn = s.thermal ? Tw : s.Tpre;
  s.eq = eq_prepare(rho, u0, u1, 0.0, Tn, sa, 2);
  if (s.thermal) s.eqp = eq_prepare(rho, u0, u1, 0.0, s.Tpre, sa, 2);
  s.force = sa.has_force;
  if (s.force) s.eqf = eq_forced(rho, u0, u1, 0.0, Tn, sa, 2);
  s.itau = 0.0;
  if (sa.relax_mode == 0) s.itau = 1.0 / sa.tau_bar;
  if (sa.relax_mode == 1) s.itau = 1.0 / (sa.mu_ref * pow(Tn / sa.T_ref, sa.mu_exp) / (rho * Tn * sa.dt) + 0.5);
  s.gT = Tn * sa.gbase;
  return s;
}

template <int PR>
__device__ __forceinline__ void relax_one(const NodeRelax &s, const StepArgs &sa, const double *vi, double f, double g,
                                          double &fo, double &go) {
  double fe = eq_f(s.eq, vi);
  if (s.thermal) {  // eq:thermalBC
    double fp = eq_f(s.eqp, vi);
    f += fe - fp;
    g += s.gT * fe - s.Tpre * sa.gbase * fp;
  }
  fo = f;
  go = g;
  if (sa.relax_mode != 2) {
    fo = f - (f - fe) * s.itau;
    go = g - (g - s.gT * fe) * s.itau;
    if constexpr (PR) pr_add(s.pt, vi, fo, go);
    if (s.force) {
      double df = eq_f(s.eqf, vi) - fe;
      fo += df;
      go += s.gT * df;
    }
  }
}

template <typename T, int P, int QS, int PR>
__global__ void __launch_bounds__(kBlock) k_step_csr(const DevCsrPlan pl, const StepArgs sa, const T *__restrict__ pin,
                                                      T *__restrict__ pout) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= pl.N) return;
  const int64_t N = pl.N;
  const double scale = sa.scale ? *sa.scale : 1.0;
  const double Tw = pl.node_Tw[k];
  double rho = 0, j0 = 0, j1 = 0, E = 0;
  if constexpr (QS > 0) {
    double fs[QS], gs[QS];
    // the plan row of the next velocity is loaded while this one's gathers are in flight
    // (its cell, source and coordinates then start the next velocity's chain of loads)
    CsrRow nx = load_row<T>(pl, k, 0);
#pragma unroll
    for (int i = 0; i < QS; i++) {
      const CsrRow cur = nx;
      if (i + 1 < QS) nx = load_row<T>(pl, k, i + 1);
      stream_row<T, P>(pl, sa, pin, i, cur, scale, fs[i], gs[i]);
      const double *vi = pl.vel + 8 * i;
      rho += fs[i];
      j0 += vi[0] * fs[i];
      j1 += vi[1] * fs[i];
      E += (vi[0] * vi[0] + vi[1] * vi[1]) * fs[i] + gs[i];
    }
    NodeRelax s = node_relax(sa, rho, j0, j1, E, Tw);
    if constexpr (PR) {
      HeatFlux q = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < QS; i++) heat_flux_add(q, pl.vel + 8 * i, s.u0, s.u1, 0.0, fs[i], gs[i]);
      s.pt = pr_term(q, s.itau, sa, 2);
    }
#pragma unroll
    for (int i = 0; i < QS; i++) {
      double fo, go;
      relax_one<PR>(s, sa, pl.vel + 8 * i, fs[i], gs[i], fo, go);
      pout[(size_t)i * N + k] = (T)fo;
      pout[((size_t)QS + i) * N + k] = (T)go;
    }
  } else {
    const int Q = pl.Q;
    for (int i = 0; i < Q; i++) {
      double f, g;
      stream_csr<T, P>(pl, sa, pin, k, i, scale, f, g);
      const double *vi = pl.vel + 8 * i;
      rho += f;
      j0 += vi[0] * f;
      j1 += vi[1] * f;
      E += (vi[0] * vi[0] + vi[1] * vi[1]) * f + g;
    }
    NodeRelax s = node_relax(sa, rho, j0, j1, E, Tw);
    if constexpr (PR) {  // the heat flux needs u: one more streaming pass
      HeatFlux q = {0, 0, 0, 0, 0, 0};
      for (int i = 0; i < Q; i++) {
        double f, g;
        stream_csr<T, P>(pl, sa, pin, k, i, scale, f, g);
        heat_flux_add(q, pl.vel + 8 * i, s.u0, s.u1, 0.0, f, g);
      }
      s.pt = pr_term(q, s.itau, sa, 2);
    }
    for (int i = 0; i < Q; i++) {
      double f, g, fo, go;
      stream_csr<T, P>(pl, sa, pin, k, i, scale, f, g);
      relax_one<PR>(s, sa, pl.vel + 8 * i, f, g, fo, go);
      pout[(size_t)i * N + k] = (T)fo;
      pout[((size_t)Q + i) * N + k] = (T)go;
    }
  }
}

namespace {
// D2V25 and D2Q19 keep a node's streamed values in registers between moments and relaxation;
// PR = 1 instantiates the Prandtl-number term (Pr != 1), PR = 0 leaves it out
template <typename T, int P, int PR>
void launch_csr_q(sllbm_plan_s *Pl, dim3 grid, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  if (Pl->cp.Q == 25)
    hipLaunchKernelGGL((k_step_csr<T, P, 25, PR>), grid, dim3(kBlock), 0, s, Pl->cp, a, (const T *)pin, (T *)pout);
  else if (Pl->cp.Q == 19)
    hipLaunchKernelGGL((k_step_csr<T, P, 19, PR>), grid, dim3(kBlock), 0, s, Pl->cp, a, (const T *)pin, (T *)pout);
  else
    hipLaunchKernelGGL((k_step_csr<T, P, 0, PR>), grid, dim3(kBlock), 0, s, Pl->cp, a, (const T *)pin, (T *)pout);
}

template <typename T, int P>
void launch_csr_t(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  dim3 grid((unsigned)((Pl->cp.N + kBlock - 1) / kBlock));
  ProfScope ps(Pl, "k_step_csr", s);
  if (a.pr_on) {
    launch_csr_q<T, P, 1>(Pl, grid, a, pin, pout, s);
  } else {
    launch_csr_q<T, P, 0>(Pl, grid, a, pin, pout, s);
  }
}
}  // namespace

int launch_step_csr(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  int p = Pl->mesh.p;
  bool f32 = Pl->prec == SLLBM_F32;
#define CCASE(PP)                                                         \
  if (p == PP) {                                                          \
    if (f32) launch_csr_t<float, PP>(Pl, a, pin, pout, s);                \
    else launch_csr_t<double, PP>(Pl, a, pin, pout, s);                   \
    return SLLBM_OK;                                                      \
  }
  CCASE(1) CCASE(2) CCASE(3) CCASE(4)
#undef CCASE
  return fail(SLLBM_EUNSUPPORTED, "no curvilinear GPU kernel for order %d (p must be 1..4)", p);
}

}  // namespace sllbm
