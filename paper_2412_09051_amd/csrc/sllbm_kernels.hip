// HIP kernels of libsllbm for gfx950 (CDNA4, wave64).
//
//   k_init          populations from nodal (rho, u, T): f = f^eq, g = g^eq
//   k_step_gather   fused stream + boundary + moments + thermal wall + BGK + force, one
//                   node per lane; per-axis interpolation tables on tensor meshes,
//                   sum-factorised in registers (two sweeps over the velocities: the
//                   first streams, stores the streamed values in the node's output slots
//                   and sums the conserved moments; the second reads them back and
//                   relaxes them in place)
//   k_moments       nodal rho, u, T and block partials of the totals
//   k_reduce_final  deterministic second pass of every FP64 reduction
//
// FP32 plans store and interpolate populations in float with float accumulation;
// moments, the temperature solve, the equilibrium and all reductions are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>

#include "sllbm_device_common.h"
#include "sllbm_kernels.h"

namespace sllbm {

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) return fail(SLLBM_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

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

// Nodes with n[axis] < lo_cnt or n[axis] >= N_axis - hi_cnt: the boundary layers of both
// faces of the bounded axis in one launch (the whole mesh: axis 0, lo_cnt N_x, hi_cnt 0).
struct Slab {
  int axis, lo_cnt, hi_cnt;
  int64_t total;   // nodes in the slab
  int lanes;       // lanes per node: 1, 2 or 4 (set by the launcher)
};

// Lanes per node of the gather kernel (Slab::lanes, at most kGatherLanes): a node's
// velocities are dealt round-robin to an aligned group of lanes, whose partial moments are
// summed by shuffles within the group (a group is either all inside the slab or all past it,
// so the lanes a shuffle reads are active).  Small slabs take 4 lanes per node so that the
// launch still fills the chip; large ones 1, so that a load instruction covers 64 nodes of
// one population rather than 16 nodes of four.
constexpr int kGatherLanes = 4;

template <typename T, int D, int P, int PR>
__global__ void __launch_bounds__(kBlock) k_step_gather(const DevTensorPlan pl, const StepArgs sa, const Slab sl,
                                                         const T *__restrict__ pin, T *__restrict__ pout) {
  static_assert(kBlock % kGatherLanes == 0 && 64 % kGatherLanes == 0, "lane groups must not straddle a wave");
  const int lanes = sl.lanes;
  const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t q = gt / lanes;
  const int sub = (int)(gt % lanes);
  if (q >= sl.total) return;
  const int Q = pl.Q;
  auto group_sum = [lanes](double v) __attribute__((always_inline)) {
    for (int o = 1; o < lanes; o <<= 1) v += __shfl_xor(v, o, lanes);
    return v;
  };
  int n[3];
  {
    // slab axis fastest (low layers, then high layers), then the remaining axes in x, y, z order
    const int span = sl.lo_cnt + sl.hi_cnt;
    int64_t r = q / span;
    const int l = (int)(q % span);
    n[sl.axis] = l < sl.lo_cnt ? l : pl.ax[sl.axis].N - sl.hi_cnt + (l - sl.lo_cnt);
    for (int a = 0; a < 3; a++) {
      if (a == sl.axis) continue;
      n[a] = (int)(r % pl.ax[a].N);
      r /= pl.ax[a].N;
    }
  }
  const int64_t k = (int64_t)n[0] + (int64_t)pl.ax[0].N * ((int64_t)n[1] + (int64_t)pl.ax[1].N * n[2]);
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

  // sweep 1: stream every velocity, store the streamed value in this node's output slot
  // and sum the conserved moments (eq:density, eq:momentum, total energy)
  double rho = 0, j0 = 0, j1 = 0, j2 = 0, E = 0;
  for (int i = sub; i < Q; i += lanes) {
    double fv, gv;
    stream_tp<T, D, P>(pl, sa, pin, n, i, er[0], er[1], fax[0], fax[1], scale, fv, gv);
    pout[(size_t)i * pl.N + k] = (T)fv;
    pout[((size_t)Q + i) * pl.N + k] = (T)gv;
    const double *vi = pl.vel + 8 * i;
    rho += fv;
    j0 += vi[0] * fv;
    j1 += vi[1] * fv;
    j2 += vi[2] * fv;
    E += (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]) * fv + gv;
  }
  rho = group_sum(rho);
  j0 = group_sum(j0);
  j1 = group_sum(j1);
  j2 = group_sum(j2);
  E = group_sum(E);
  const double u0 = j0 / rho, u1 = j1 / rho, u2 = j2 / rho;
  const double Tpre = (E - rho * (u0 * u0 + u1 * u1 + u2 * u2)) / (2.0 * rho * sa.cv);
  const bool thermal = (Tw == Tw);
  const double Tn = thermal ? Tw : Tpre;
  EqNode eq = eq_prepare(rho, u0, u1, u2, Tn, sa, D);
  EqNode eqp;
  if (thermal) eqp = eq_prepare(rho, u0, u1, u2, Tpre, sa, D);
  EqNode eqf;
  if (sa.has_force) eqf = eq_forced(rho, u0, u1, u2, Tn, sa, D);
  double inv_tau = 0.0;
  if (sa.relax_mode == 0) inv_tau = 1.0 / sa.tau_bar;
  if (sa.relax_mode == 1) {
    double mu = sa.mu_ref * pow(Tn / sa.T_ref, sa.mu_exp);
    inv_tau = 1.0 / (mu / (rho * Tn * sa.dt) + 0.5);
  }
  const double gT = Tn * sa.gbase;
  PrTerm pt;
  if constexpr (PR) {  // Pr != 1: the heat flux of the stored streamed values (it needs u)
    HeatFlux hq = {0, 0, 0, 0, 0, 0};
    for (int i = sub; i < Q; i += lanes)
      heat_flux_add(hq, pl.vel + 8 * i, u0, u1, u2, (double)pout[(size_t)i * pl.N + k],
                    (double)pout[((size_t)Q + i) * pl.N + k]);
    hq.f0 = group_sum(hq.f0);
    hq.f1 = group_sum(hq.f1);
    hq.f2 = group_sum(hq.f2);
    hq.g0 = group_sum(hq.g0);
    hq.g1 = group_sum(hq.g1);
    hq.g2 = group_sum(hq.g2);
    pt = pr_term(hq, inv_tau, sa, D);
  }

  // sweep 2: read the stored streamed values back (this thread wrote them), isothermal-wall
  // correction (eq:thermalBC), BGK relaxation, quasi-equilibrium term, Kupershtokh forcing,
  // store
  for (int i = sub; i < Q; i += lanes) {
    double fv = (double)pout[(size_t)i * pl.N + k];
    double gv = (double)pout[((size_t)Q + i) * pl.N + k];
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
      if constexpr (PR) pr_add(pt, vi, fo, go);
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

// f-only totals of a population set: mass, momentum[3] (both from f alone, eq:density and
// eq:momentum) and the volume, weighted by the nodal quadrature volumes.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mass_partial(int64_t N, int Q, int D, const double *__restrict__ vel,
                                                          const double *__restrict__ vol, const T *__restrict__ pop,
                                                          double *__restrict__ part) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v[kRedWidth];
#pragma unroll
  for (int q = 0; q < kRedWidth; q++) v[q] = 0.0;
  if (k < N) {
    double r = 0, j0 = 0, j1 = 0, j2 = 0;
    constexpr int RB = 5;   // loads issued per batch, ahead of their use
    for (int i0 = 0; i0 < Q; i0 += RB) {
      T fb[RB];
#pragma unroll
      for (int b = 0; b < RB; b++)
        if (i0 + b < Q) fb[b] = pop[(size_t)(i0 + b) * N + k];
#pragma unroll
      for (int b = 0; b < RB; b++) {
        if (i0 + b >= Q) break;
        const double f = (double)fb[b];
        const double *vi = vel + 8 * (i0 + b);
        r += f;
        j0 += vi[0] * f;
        j1 += vi[1] * f;
        j2 += vi[2] * f;
      }
    }
    const double V = vol[k];
    v[0] = V * r;
    v[1] = V * j0;
    v[2] = V * j1;
    v[3] = D == 3 ? V * j2 : 0.0;
    v[4] = V;
  }
  block_partial(v, part);
}

// Force controller (Sec. 4.3: the force is adjusted by a PI controller that holds the
// mean momentum): e = target - M_a / V, I += e dt, F_a = F0_a + kp e + ki I.  One thread.
__global__ void k_force_update(const double *__restrict__ tot, double *__restrict__ force,
                               const double *__restrict__ force0, double *__restrict__ ctl, int axis, double target,
                               double kp, double ki, double dt) {
  if (threadIdx.x != 0) return;
  const double mean = tot[1 + axis] / tot[4];
  const double e = target - mean;
  const double I = ctl[0] + e * dt;
  force[axis] = force0[axis] + kp * e + ki * I;
  ctl[0] = I;
  ctl[1] = e;
  ctl[2] = mean;
  ctl[3] += 1.0;
}

__global__ void k_force_reset(double *__restrict__ force, double *__restrict__ force0, double *__restrict__ ctl,
                              double F0, double F1, double F2) {
  if (threadIdx.x != 0) return;
  force[0] = force0[0] = F0;
  force[1] = force0[1] = F1;
  force[2] = force0[2] = F2;
  ctl[0] = ctl[1] = ctl[2] = ctl[3] = 0.0;
}

// ------------------------------------------------------------------ launchers
namespace {
int64_t nblocks(int64_t N) { return (N + kBlock - 1) / kBlock; }

// lanes per node for a gather launch over `nodes` nodes: enough lanes for about 4096 waves
// (256 CUs at 4 waves per SIMD), at most kGatherLanes
int gather_lanes(int64_t nodes) {
  int lanes = 1;
  while (lanes < kGatherLanes && nodes * lanes < 4096 * 64) lanes *= 2;
  return lanes;
}

template <typename T, int D, int P>
void launch_gather_t(sllbm_plan_s *Pl, const StepArgs &a, const Slab &sl, const void *pin, void *pout,
                     hipStream_t s) {
  if (sl.total <= 0) return;
  ProfScope ps(Pl, "k_step_gather", s);
  const dim3 grid((unsigned)nblocks(sl.total * sl.lanes));
  if (a.pr_on)
    hipLaunchKernelGGL((k_step_gather<T, D, P, 1>), grid, dim3(kBlock), 0, s, Pl->tp, a, sl, (const T *)pin,
                       (T *)pout);
  else
    hipLaunchKernelGGL((k_step_gather<T, D, P, 0>), grid, dim3(kBlock), 0, s, Pl->tp, a, sl, (const T *)pin,
                       (T *)pout);
}

template <typename T>
int dispatch_gather(sllbm_plan_s *Pl, const StepArgs &a, const Slab &sl, const void *pin, void *pout, hipStream_t s) {
  int D = Pl->mesh.dim, p = Pl->mesh.p;
#define CASE(DD, PP) \
  if (D == DD && p == PP) { launch_gather_t<T, DD, PP>(Pl, a, sl, pin, pout, s); return SLLBM_OK; }
  CASE(2, 1) CASE(2, 2) CASE(2, 3) CASE(2, 4) CASE(3, 1) CASE(3, 2) CASE(3, 3) CASE(3, 4)
#undef CASE
  return fail(SLLBM_EUNSUPPORTED, "no GPU kernel for dim %d order %d (p must be 1..4)", D, p);
}
}  // namespace

bool step_has_relax_launch(const sllbm_plan_s *P) { return P->kernel == 0 && P->use_tile() && P->mesh.dim == 3; }

int launch_step(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s, bool relax) {
  if (Pl->kernel == 1) {
    int rc = launch_step_csr(Pl, a, pin, pout, s);
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    return SLLBM_OK;
  }
  const DevTensorPlan &tp = Pl->tp;
  auto gather = [&](const Slab &sl) {
    return Pl->prec == SLLBM_F32 ? dispatch_gather<float>(Pl, a, sl, pin, pout, s)
                                 : dispatch_gather<double>(Pl, a, sl, pin, pout, s);
  };
  int rc;
  if (Pl->use_tile()) {
    // interior nodes: LDS-tiled kernel; boundary-layer slabs: per-node gather
    rc = launch_step_tile(Pl, a, pin, pout, s, relax);
    if (rc) return rc;
    // the faces with boundary layers all lie on the one bounded axis: one launch covers both
    Slab sl{-1, 0, 0, 0, 1};
    for (int f = 0; f < tp.nfaces; f++) {
      const DevFace &F = tp.face[f];
      if (F.depth <= 0) continue;
      if (sl.axis >= 0 && sl.axis != F.axis)
        return fail(SLLBM_EUNSUPPORTED, "boundary layers on two axes of a tensor plan");
      sl.axis = F.axis;
      (F.side == 0 ? sl.lo_cnt : sl.hi_cnt) = F.depth;
    }
    if (sl.axis >= 0) {
      const int Na = tp.ax[sl.axis].N;
      sl.lo_cnt = std::min(sl.lo_cnt, Na);
      sl.hi_cnt = std::min(sl.hi_cnt, Na - sl.lo_cnt);   // layers of both faces overlap on a thin mesh
      sl.total = (int64_t)(sl.lo_cnt + sl.hi_cnt) * (tp.N / Na);
      sl.lanes = gather_lanes(sl.total);
      if ((rc = gather(sl))) return rc;
    }
  } else {
    Slab sl{0, tp.ax[0].N, 0, tp.N, gather_lanes(tp.N)};
    rc = gather(sl);
  }
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

int launch_moments_to(sllbm_plan_s *Pl, const StepArgs &a, const void *pop, double *rho, double *u, double *T,
                      double *part, double *totals, hipStream_t s) {
  int64_t N = Pl->mesh.n_nodes, nb = nblocks(N);
  const double *vel = Pl->kernel == 0 ? Pl->tp.vel : Pl->cp.vel;
  const double *vol = Pl->kernel == 0 ? Pl->tp.vol : Pl->cp.vol;
  const int do_part = totals ? 1 : 0;
  if (Pl->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_moments<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Pl->vel.Q, Pl->mesh.dim, vel, vol,
                       a, (const float *)pop, rho, u, T, part, do_part);
  else
    hipLaunchKernelGGL(k_moments<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Pl->vel.Q, Pl->mesh.dim, vel,
                       vol, a, (const double *)pop, rho, u, T, part, do_part);
  HIP_TRY(hipGetLastError());
  if (totals) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, nb, totals, 0, 0.0,
                       (double *)nullptr);
    HIP_TRY(hipGetLastError());
  }
  return SLLBM_OK;
}

int launch_moments(sllbm_plan_s *Pl, const StepArgs &a, const void *pop, double *rho, double *u, double *T,
                   bool totals, hipStream_t s) {
  return launch_moments_to(Pl, a, pop, rho, u, T, Pl->scratch + kScratchHead,
                           totals ? Pl->scratch + kSlotTotals : nullptr, s);
}

namespace {
// f-only totals of pop into scratch[kSlotMass..]; mode 1 also writes the rescale factor
int launch_f_totals(sllbm_plan_s *Pl, const void *pop, int mode, double mass_ref, hipStream_t s) {
  int64_t N = Pl->mesh.n_nodes, nb = nblocks(N);
  const double *vel = Pl->kernel == 0 ? Pl->tp.vel : Pl->cp.vel;
  const double *vol = Pl->kernel == 0 ? Pl->tp.vol : Pl->cp.vol;
  double *part = Pl->scratch + kScratchHead;
  const int Q = Pl->vel.Q, D = Pl->mesh.dim;
  if (Pl->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_mass_partial<float>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Q, D, vel, vol,
                       (const float *)pop, part);
  else
    hipLaunchKernelGGL(k_mass_partial<double>, dim3((unsigned)nb), dim3(kBlock), 0, s, N, Q, D, vel, vol,
                       (const double *)pop, part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, nb,
                     Pl->scratch + kSlotMass, mode, mass_ref, Pl->scratch + kSlotScale);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}
}  // namespace

int launch_mass_scale(sllbm_plan_s *Pl, const void *pop, double mass_ref, hipStream_t s) {
  ProfScope ps(Pl, "k_mass_scale", s);
  return launch_f_totals(Pl, pop, 1, mass_ref, s);
}

int launch_force_reset(sllbm_plan_s *Pl, const double *force0, hipStream_t s) {
  double *sc = Pl->scratch;
  hipLaunchKernelGGL(k_force_reset, dim3(1), dim3(64), 0, s, sc + kSlotForce, sc + kSlotForce0, sc + kSlotCtl,
                     force0[0], force0[1], force0[2]);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

int launch_force_update(sllbm_plan_s *Pl, int axis, double target, double kp, double ki, double dt, const void *pop,
                        hipStream_t s) {
  ProfScope ps(Pl, "k_force_update", s);
  int rc = launch_f_totals(Pl, pop, 0, 0.0, s);
  if (rc) return rc;
  double *sc = Pl->scratch;
  hipLaunchKernelGGL(k_force_update, dim3(1), dim3(64), 0, s, (const double *)(sc + kSlotMass), sc + kSlotForce,
                     (const double *)(sc + kSlotForce0), sc + kSlotCtl, axis, target, kp, ki, dt);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

}  // namespace sllbm
