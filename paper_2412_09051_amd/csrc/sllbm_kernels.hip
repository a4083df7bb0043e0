// HIP kernels of libsllbm for gfx950 (CDNA4, wave64).
//
//   k_init          populations from nodal (rho, u, T): f = f^eq, g = g^eq
//   k_step_gather   fused stream + boundary + moments + thermal wall + BGK + force, one
//                   node per lane; per-axis interpolation tables on tensor meshes,
//                   sum-factorised in registers (two sweeps over the velocities: the
//                   first accumulates the conserved moments, the second re-streams and
//                   relaxes, so no per-node stash is needed)
//   k_moments       nodal rho, u, T and block partials of the totals
//   k_reduce_final  deterministic second pass of every FP64 reduction
//
// FP32 plans store and interpolate populations in float with float accumulation;
// moments, the temperature solve, the equilibrium and all reductions are FP64.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sllbm_kernels.h"

namespace sllbm {

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) return fail(SLLBM_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

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

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-reduce kRedWidth doubles (fixed tree: wave shuffles, then wave 0 sums the
// four wave results in order) and store one partial per block.
__device__ void block_partial(double (&v)[kRedWidth], double *out) {
  __shared__ double red[kBlock / 64][kRedWidth];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kRedWidth; q++) {
    double s = wave_sum(v[q]);
    if (lane == 0) red[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kRedWidth) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; w++) s += red[w][threadIdx.x];
    out[(size_t)blockIdx.x * kRedWidth + threadIdx.x] = s;
  }
}

// Second pass: one block sums nblk partials in a fixed order.  mode 1 additionally
// turns the mass into the rescale factor mass_ref / M.
__global__ void __launch_bounds__(kBlock) k_reduce_final(const double *__restrict__ part, int64_t nblk,
                                                         double *__restrict__ dst, int mode, double mass_ref,
                                                         double *__restrict__ scale_out) {
  double v[kRedWidth];
#pragma unroll
  for (int q = 0; q < kRedWidth; q++) v[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
    for (int q = 0; q < kRedWidth; q++) v[q] += part[b * kRedWidth + q];
  __shared__ double red[kBlock / 64][kRedWidth];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kRedWidth; q++) {
    double s = wave_sum(v[q]);
    if (lane == 0) red[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kRedWidth) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; w++) s += red[w][threadIdx.x];
    dst[threadIdx.x] = s;
    if (mode == 1 && threadIdx.x == 0) *scale_out = mass_ref / s;
  }
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

template <typename T, int D, int P>
__global__ void __launch_bounds__(kBlock) k_step_gather(const DevTensorPlan pl, const StepArgs sa,
                                                         const T *__restrict__ pin, T *__restrict__ pout) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= pl.N) return;
  const int Q = pl.Q;
  int n[3];
  {
    int64_t r = k;
    n[0] = (int)(r % pl.ax[0].N);
    r /= pl.ax[0].N;
    n[1] = (int)(r % pl.ax[1].N);
    n[2] = (int)(r / pl.ax[1].N);
  }
  const ExcEntry *er[2] = {nullptr, nullptr};
  int fax[2] = {-1, -1};
  double Tw = __builtin_nan("");
  for (int f = 0; f < pl.nfaces; f++) {
    const DevFace &F = pl.face[f];
    int l = F.side == 0 ? n[F.axis] : pl.ax[F.axis].N - 1 - n[F.axis];
    if (l < F.depth) {
      er[f] = F.e + (size_t)l * Q;
      fax[f] = F.axis;
      double t = F.Tw[l];
      if (t == t) Tw = t;
    }
  }
  const double scale = sa.scale ? *sa.scale : 1.0;

  // sweep 1: conserved moments of the streamed populations (eq:density, eq:momentum,
  // total energy)
  double rho = 0, j0 = 0, j1 = 0, j2 = 0, E = 0;
  for (int i = 0; i < Q; i++) {
    double fv, gv;
    stream_tp<T, D, P>(pl, sa, pin, n, i, er[0], er[1], fax[0], fax[1], scale, fv, gv);
    const double *vi = pl.vel + 8 * i;
    rho += fv;
    j0 += vi[0] * fv;
    j1 += vi[1] * fv;
    j2 += vi[2] * fv;
    E += (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]) * fv + gv;
  }
  const double u0 = j0 / rho, u1 = j1 / rho, u2 = j2 / rho;
  const double Tpre = (E - rho * (u0 * u0 + u1 * u1 + u2 * u2)) / (2.0 * rho * sa.cv);
  const bool thermal = (Tw == Tw);
  const double Tn = thermal ? Tw : Tpre;
  EqNode eq = eq_prepare(rho, u0, u1, u2, Tn, sa, D);
  EqNode eqp;
  if (thermal) eqp = eq_prepare(rho, u0, u1, u2, Tpre, sa, D);
  EqNode eqf;
  if (sa.has_force) {
    double r = sa.dt / rho;
    eqf = eq_prepare(rho, u0 + sa.force[0] * r, u1 + sa.force[1] * r, u2 + sa.force[2] * r, Tn, sa, D);
  }
  double inv_tau = 0.0;
  if (sa.relax_mode == 0) inv_tau = 1.0 / sa.tau_bar;
  if (sa.relax_mode == 1) {
    double mu = sa.mu_ref * pow(Tn / sa.T_ref, sa.mu_exp);
    inv_tau = 1.0 / (mu / (rho * Tn * sa.dt) + 0.5);
  }
  const double gT = Tn * sa.gbase;

  // sweep 2: re-stream, isothermal-wall correction (eq:thermalBC), BGK relaxation,
  // Kupershtokh forcing, store
  for (int i = 0; i < Q; i++) {
    double fv, gv;
    stream_tp<T, D, P>(pl, sa, pin, n, i, er[0], er[1], fax[0], fax[1], scale, fv, gv);
    const double *vi = pl.vel + 8 * i;
    double fe = eq_f(eq, vi);
    if (thermal) {
      double fp = eq_f(eqp, vi);
      fv += fe - fp;
      gv += gT * fe - Tpre * sa.gbase * fp;
    }
    double fo = fv, go = gv;
    if (sa.relax_mode != 2) {
      fo = fv - (fv - fe) * inv_tau;
      go = gv - (gv - gT * fe) * inv_tau;
      if (sa.has_force) {
        double df = eq_f(eqf, vi) - fe;
        fo += df;
        go += gT * df;
      }
    }
    pout[(size_t)i * pl.N + k] = (T)fo;
    pout[((size_t)Q + i) * pl.N + k] = (T)go;
  }
}

// ------------------------------------------------------------------ init / moments
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init(int64_t N, int Q, int D, const double *__restrict__ vel,
                                                  const StepArgs sa, const double *__restrict__ rho,
                                                  const double *__restrict__ u, const double *__restrict__ Tf,
                                                  T *__restrict__ pop) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= N) return;
  double uu[3] = {0, 0, 0};
  for (int a = 0; a < D; a++) uu[a] = u[(size_t)a * N + k];
  double Tk = Tf[k];
  EqNode e = eq_prepare(rho[k], uu[0], uu[1], uu[2], Tk, sa, D);
  for (int i = 0; i < Q; i++) {
    double fe = eq_f(e, vel + 8 * i);
    pop[(size_t)i * N + k] = (T)fe;
    pop[((size_t)Q + i) * N + k] = (T)(Tk * sa.gbase * fe);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_moments(int64_t N, int Q, int D, const double *__restrict__ vel,
                                                     const double *__restrict__ vol, const StepArgs sa,
                                                     const T *__restrict__ pop, double *__restrict__ rho_o,
                                                     double *__restrict__ u_o, double *__restrict__ T_o,
                                                     double *__restrict__ part, int do_part) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v[kRedWidth];
#pragma unroll
  for (int q = 0; q < kRedWidth; q++) v[q] = 0.0;
  if (k < N) {
    double r = 0, j[3] = {0, 0, 0}, E = 0;
    for (int i = 0; i < Q; i++) {
      const double *vi = vel + 8 * i;
      double f = (double)pop[(size_t)i * N + k];
      double g = (double)pop[((size_t)Q + i) * N + k];
      r += f;
      j[0] += vi[0] * f;
      j[1] += vi[1] * f;
      j[2] += vi[2] * f;
      E += (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]) * f + g;
    }
    double uu = 0;
    for (int a = 0; a < 3; a++) uu += (j[a] / r) * (j[a] / r);
    double Tk = (E - r * uu) / (2.0 * r * sa.cv);
    if (rho_o) rho_o[k] = r;
    if (u_o)
      for (int a = 0; a < D; a++) u_o[(size_t)a * N + k] = j[a] / r;
    if (T_o) T_o[k] = Tk;
    double V = vol[k];
    v[0] = V * r;
    for (int a = 0; a < D; a++) v[1 + a] = V * j[a];
    v[1 + D] = V * E;
    bool bad = !(r > 0.0) || !(Tk > 0.0) || !isfinite(r) || !isfinite(Tk) || !isfinite(E);
    v[kRedWidth - 1] = bad ? 1.0 : 0.0;
  }
  if (do_part) block_partial(v, part);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_mass_partial(int64_t N, int Q, const double *__restrict__ vol,
                                                          const T *__restrict__ pop, double *__restrict__ part) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v[kRedWidth];
#pragma unroll
  for (int q = 0; q < kRedWidth; q++) v[q] = 0.0;
  if (k < N) {
    double r = 0;
    for (int i = 0; i < Q; i++) r += (double)pop[(size_t)i * N + k];
    v[0] = vol[k] * r;
  }
  block_partial(v, part);
}

// ------------------------------------------------------------------ launchers
namespace {
int64_t nblocks(int64_t N) { return (N + kBlock - 1) / kBlock; }

template <typename T, int D, int P>
void launch_gather_t(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  hipLaunchKernelGGL((k_step_gather<T, D, P>), dim3((unsigned)nblocks(Pl->tp.N)), dim3(kBlock), 0, s, Pl->tp, a,
                     (const T *)pin, (T *)pout);
}

template <typename T>
int dispatch_gather(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  int D = Pl->mesh.dim, p = Pl->mesh.p;
#define CASE(DD, PP) \
  if (D == DD && p == PP) { launch_gather_t<T, DD, PP>(Pl, a, pin, pout, s); return SLLBM_OK; }
  CASE(2, 1) CASE(2, 2) CASE(2, 3) CASE(2, 4) CASE(3, 1) CASE(3, 2) CASE(3, 3) CASE(3, 4)
#undef CASE
  return fail(SLLBM_EUNSUPPORTED, "no GPU kernel for dim %d order %d (p must be 1..4)", D, p);
}
}  // namespace

int launch_step(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  if (Pl->kernel != 0) return fail(SLLBM_EUNSUPPORTED, "curvilinear step kernel not available");
  int rc = Pl->prec == SLLBM_F32 ? dispatch_gather<float>(Pl, a, pin, pout, s)
                                 : dispatch_gather<double>(Pl, a, pin, pout, s);
  if (rc) return rc;
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

int launch_init(sllbm_plan_s *Pl, const StepArgs &a, const double *rho, const double *u, const double *T, void *pop,
                hipStream_t s) {
  int64_t N = Pl->mesh.n_nodes;
  const double *vel = Pl->kernel == 0 ? Pl->tp.vel : Pl->cp.vel;
  if (Pl->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_init<float>, dim3((unsigned)nblocks(N)), dim3(kBlock), 0, s, N, Pl->vel.Q, Pl->mesh.dim, vel,
                       a, rho, u, T, (float *)pop);
  else
    hipLaunchKernelGGL(k_init<double>, dim3((unsigned)nblocks(N)), dim3(kBlock), 0, s, N, Pl->vel.Q, Pl->mesh.dim,
                       vel, a, rho, u, T, (double *)pop);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

int launch_moments(sllbm_plan_s *Pl, const StepArgs &a, const void *pop, double *rho, double *u, double *T,
                   bool totals, hipStream_t s) {
  int64_t N = Pl->mesh.n_nodes, nb = nblocks(N);
  const double *vel = Pl->kernel == 0 ? Pl->tp.vel : Pl->cp.vel;
  const double *vol = Pl->kernel == 0 ? Pl->tp.vol : Pl->cp.vol;
  double *part = Pl->scratch + kScratchHead;
  if (Pl->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_moments<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Pl->vel.Q, Pl->mesh.dim, vel, vol,
                       a, (const float *)pop, rho, u, T, part, totals ? 1 : 0);
  else
    hipLaunchKernelGGL(k_moments<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Pl->vel.Q, Pl->mesh.dim, vel,
                       vol, a, (const double *)pop, rho, u, T, part, totals ? 1 : 0);
  HIP_TRY(hipGetLastError());
  if (totals) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, nb,
                       Pl->scratch + kSlotTotals, 0, 0.0, (double *)nullptr);
    HIP_TRY(hipGetLastError());
  }
  return SLLBM_OK;
}

int launch_mass_scale(sllbm_plan_s *Pl, const void *pop, double mass_ref, hipStream_t s) {
  int64_t N = Pl->mesh.n_nodes, nb = nblocks(N);
  const double *vol = Pl->kernel == 0 ? Pl->tp.vol : Pl->cp.vol;
  double *part = Pl->scratch + kScratchHead;
  if (Pl->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_mass_partial<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Pl->vel.Q, vol,
                       (const float *)pop, part);
  else
    hipLaunchKernelGGL(k_mass_partial<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Pl->vel.Q, vol,
                       (const double *)pop, part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, nb,
                     Pl->scratch + kSlotMass, 1, mass_ref, Pl->scratch + kSlotScale);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

}  // namespace sllbm
