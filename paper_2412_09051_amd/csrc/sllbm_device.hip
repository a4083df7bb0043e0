// Device half of libsllbm (gfx950): plan upload, the fused stream + collide step,
// equilibrium initialisation, moments and deterministic FP64 reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>

#include "sllbm_internal.h"
#include "sllbm_kernels.h"

using namespace sllbm;

namespace {

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) return fail(SLLBM_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

template <typename V>
int upload(sllbm_plan_s *P, const std::vector<V> &h, const V **dptr) {
  if (h.empty()) { *dptr = nullptr; return SLLBM_OK; }
  void *d = nullptr;
  size_t bytes = sizeof(V) * h.size();
  hipError_t e = P->dalloc.get(&d, bytes);
  if (e != hipSuccess) return fail(SLLBM_ENOMEM, "device allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
  P->dev_allocs.push_back(d);
  e = hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(SLLBM_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
  P->table_bytes += (int64_t)bytes;
  *dptr = (const V *)d;
  return SLLBM_OK;
}

int check_params(const sllbm_plan_s *P, const sllbm_params *prm) {
  if (!prm) return fail(SLLBM_EINVAL, "params is NULL");
  if (!(prm->gamma > 1.0)) return fail(SLLBM_EINVAL, "gamma must be > 1");
  if (!(prm->Pr > 0.0) || !std::isfinite(prm->Pr))
    return fail(SLLBM_EINVAL, "Pr must be a positive finite number (got %g)", prm->Pr);
  if (prm->relax_mode < 0 || prm->relax_mode > 2) return fail(SLLBM_EINVAL, "relax_mode must be 0, 1 or 2");
  if (prm->relax_mode == 0 && !(prm->tau_bar > 0.5))
    return fail(SLLBM_EINVAL, "tau_bar must be > 1/2 (got %g)", prm->tau_bar);
  if (prm->relax_mode == 1 && !(prm->mu_ref > 0 && prm->T_ref > 0))
    return fail(SLLBM_EINVAL, "relax_mode 1 needs mu_ref > 0 and T_ref > 0");
  if (prm->mass_fix && !(prm->mass_ref > 0)) return fail(SLLBM_EINVAL, "mass_fix needs mass_ref > 0");
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(prm->force[a])) return fail(SLLBM_EINVAL, "force must be finite");
  if (prm->force_device != 0 && prm->force_device != 1) return fail(SLLBM_EINVAL, "force_device must be 0 or 1");
  if (prm->force_device && !P->force_ready)
    return fail(SLLBM_EINVAL, "force_device = 1 before sllbm_force_reset set the plan's force");
  return SLLBM_OK;
}

StepArgs make_args(const sllbm_plan_s *P, const sllbm_params *prm) {
  StepArgs a{};
  int D = P->mesh.dim;
  a.gamma = prm->gamma;
  a.cv = 1.0 / (prm->gamma - 1.0);
  a.gbase = 2.0 * a.cv - D;
  a.dt = P->dt;
  a.T0 = P->vel.T0;
  a.inv_sqrtT0 = 1.0 / std::sqrt(P->vel.T0);
  a.relax_mode = prm->relax_mode;
  a.tau_bar = prm->tau_bar;
  a.mu_ref = prm->mu_ref;
  a.T_ref = prm->T_ref;
  a.mu_exp = prm->mu_exp;
  a.has_force = 0;
  for (int d = 0; d < 3; d++) {
    a.force[d] = d < D ? prm->force[d] : 0.0;
    if (a.force[d] != 0.0) a.has_force = 1;
  }
  a.Pr = prm->Pr;
  a.pr_on = (prm->Pr != 1.0 && prm->relax_mode != 2) ? 1 : 0;
  a.force_dev = nullptr;
  if (prm->force_device) {
    a.force_dev = P->scratch + kSlotForce;
    a.has_force = 1;
  }
  a.scale = nullptr;
  a.inlet = P->inlet_dev;
  return a;
}

size_t elem_size(const sllbm_plan_s *P) { return P->prec == SLLBM_F32 ? 4 : 8; }

int check_pop(const sllbm_plan_s *P, const void *pop, const char *what) {
  if (!pop) return fail(SLLBM_EINVAL, "%s is NULL", what);
  if (((uintptr_t)pop) % 16) return fail(SLLBM_EINVAL, "%s must be 16-byte aligned", what);
  return SLLBM_OK;
}

int require_device(const sllbm_plan_s *P) {
  if (!P->has_device) return fail(SLLBM_EHIP, "plan has no GPU tables (no device was available when it was built)");
  HIP_TRY(hipSetDevice(P->device));
  return SLLBM_OK;
}

// z chunk (cells) of the velocity-split 3D step: the axis is cut into nzc equal chunks, as
// few as give at least two rounds of work items (x-y tiles x chunks x velocities) over two
// workgroups per compute unit: longer chunks re-read fewer departure planes beyond their own
// and fill and drain their pipelines less often.  (Measured on the 96^3 Taylor-Green mesh
// and the 128 x 96 x 64 channel: chunks of a smaller count than this, or chunks much shorter,
// were slower; a tiny last chunk beside long ones too.)
int col_chunk_cells(const Mesh &m, int Q, int tx, int ty, const int org[2], const int end[2]) {
  const int P = m.p, ncz = m.N[2] / P;
  const int64_t tiles = (int64_t)((end[0] - org[0] + tx - 1) / tx) * ((end[1] - org[1] + ty - 1) / ty);
  const int64_t slots = 256 * 2;
  int last = 0;
  for (int nzc = 1; nzc <= ncz; nzc++) {
    const int zc = (ncz + nzc - 1) / nzc;
    // (a periodic axis must be longer than a chunk and its halo)
    if (zc > ncz - 2 || zc * P > kColZMax || (ncz + zc - 1) / zc != nzc) continue;
    last = zc;
    if (tiles * Q * nzc >= 2 * slots) return zc;
  }
  return last;
}

}  // namespace

namespace sllbm {
namespace {
std::mutex g_alloc_mu;
DevAllocator g_alloc;
}  // namespace
DevAllocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}
}  // namespace sllbm

extern "C" int sllbm_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*release)(void *ptr, void *ctx),
                                   void *ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(SLLBM_EINVAL, "set_allocator: give both functions, or neither (back to hipMalloc/hipFree)");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.release = release;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return SLLBM_OK;
}

// ------------------------------------------------------------------ plan

extern "C" int sllbm_interp_plan(sllbm_mesh ms, const sllbm_velset *v, double dt, int prec, sllbm_plan *out) {
  if (!ms || !v || !out) return fail(SLLBM_EINVAL, "interp_plan: NULL argument");
  *out = nullptr;
  const Mesh &m = ms->m;
  if (v->dim != m.dim) return fail(SLLBM_EINVAL, "interp_plan: velocity set dim %d != mesh dim %d", v->dim, m.dim);
  if (v->Q < 1 || v->Q > kMaxQ || !v->zeta || !v->w || !v->opposite || !(v->T0 > 0))
    return fail(SLLBM_EINVAL, "interp_plan: velocity set needs 1 <= Q <= %d, T0 > 0, non-NULL arrays", kMaxQ);
  for (int i = 0; i < v->Q; i++)
    if (v->opposite[i] < 0 || v->opposite[i] >= v->Q)
      return fail(SLLBM_EINVAL, "interp_plan: opposite[%d] out of range", i);
  if (!(dt > 0) || !std::isfinite(dt)) return fail(SLLBM_EINVAL, "interp_plan: dt must be > 0");
  if (prec != SLLBM_F64 && prec != SLLBM_F32) return fail(SLLBM_EINVAL, "interp_plan: prec must be F64 or F32");

  sllbm_plan_s *P = new (std::nothrow) sllbm_plan_s();
  if (!P) return fail(SLLBM_ENOMEM, "interp_plan: out of host memory");
  P->dalloc = current_allocator();
  P->mesh = m;
  P->dt = dt;
  P->prec = prec;
  VelSet &V = P->vel;
  V.dim = v->dim;
  V.Q = v->Q;
  V.T0 = v->T0;
  V.zeta.assign(v->zeta, v->zeta + v->Q * v->dim);
  V.w.assign(v->w, v->w + v->Q);
  V.opp.assign(v->opposite, v->opposite + v->Q);

  HostTables t;
  int rc;
  if (m.kind == SLLBM_MESH_TENSOR) {
    P->kernel = 0;
    rc = build_tensor_tables(m, V, dt, t, &P->n_exceptions, &P->n_thermal);
  } else {
    P->kernel = 1;
    rc = build_csr_tables(m, V, dt, t, &P->n_exceptions, &P->n_thermal);
  }
  if (rc != SLLBM_OK) { delete P; return rc; }
  P->vol = node_volumes(m);
  if (P->kernel == 0) {
    int c[3];
    // (the tiled kernels address a population plane through 32-bit byte offsets)
    const int64_t plane_bytes = m.n_nodes * (prec == SLLBM_F32 ? 4 : 8);
    P->tile_ok = tile_cells(m.dim, m.p, c) && tile_eligible(m, t, c) && plane_bytes <= kBufMaxBytes ? 1 : 0;
    if (P->tile_ok) {
      int64_t ntiles = 1;
      for (int a = 0; a < m.dim; a++) ntiles *= (m.N[a] + c[a] * m.p - 1) / (c[a] * m.p);
      P->tile_auto = ntiles >= kTileMinTiles ? 1 : 0;
    }
    for (int id : t.tab_reg) P->tile_tabs = std::max(P->tile_tabs, id + 1);
    if (P->tile_ok && m.dim == 3 && col_q_supported(V.Q)) {
      // the x-y tiles cover the nodes between the bounded faces' boundary layers (which the
      // gather kernel steps), from and to the nearest cell boundaries outside them
      int org[2] = {0, 0}, end[2] = {(int)m.N[0], (int)m.N[1]};
      for (int f = 0; f < t.nfaces; f++) {
        const int a = t.face_axis[f];
        if (a > 1) continue;
        const int whole = t.face_depth[f] / m.p * m.p;   // whole cells inside the layers
        if (t.face_side[f] == 0) org[a] = whole;
        else end[a] = (int)m.N[a] - whole;
      }
      // the widest tile that applies (two columns per thread where that pays, else one)
      for (int cpt = col_cpt(prec == SLLBM_F32 ? 4 : 8, m.p, V.Q); cpt >= 1 && !P->col_ok; cpt--) {
        int cx = 0, cy = 0, L = 0;
        if (m.p == 2) cx = ColShape<2>::CX, cy = cpt * ColShape<2>::CY, L = kColWin<2>;
        if (m.p == 3) cx = ColShape<3>::CX, cy = cpt * ColShape<3>::CY, L = kColWin<3>;
        if (m.p == 4) cx = ColShape<4>::CX, cy = cpt * ColShape<4>::CY, L = kColWin<4>;
        const int zc = cx > 0 && end[0] > org[0] && end[1] > org[1] ? col_chunk_cells(m, V.Q, cx * m.p, cy * m.p, org, end) : 0;
        if (zc > 0 && L > 0 && col_eligible(m, t, cx, cy, zc, L, org, end)) {
          P->col_ok = 1;
          P->col_zc = zc;
          P->col_cpt = cpt;
          for (int a = 0; a < 2; a++) {
            P->col_org[a] = org[a];
            P->col_end[a] = end[a];
          }
        }
      }
    }
  }

  // velocity constants: zeta x,y,z, xi = zeta/sqrt(T0), |xi|^2, w
  t.vel.assign(8 * (size_t)V.Q, 0.0);
  for (int i = 0; i < V.Q; i++) {
    double q = 0;
    for (int d = 0; d < V.dim; d++) {
      double z = V.zeta[i * V.dim + d];
      t.vel[8 * i + d] = z;
      t.vel[8 * i + 3 + d] = z / std::sqrt(V.T0);
      q += (z / std::sqrt(V.T0)) * (z / std::sqrt(V.T0));
    }
    t.vel[8 * i + 6] = q;
    t.vel[8 * i + 7] = V.w[i];
  }
  std::vector<double> inlet(5 * (size_t)std::max<size_t>(1, m.bcs.size()), 0.0);
  for (size_t b = 0; b < m.bcs.size(); b++) {
    inlet[5 * b + 0] = m.bcs[b].rho;
    for (int d = 0; d < 3; d++) inlet[5 * b + 1 + d] = d < m.dim ? m.bcs[b].u[d] : 0.0;
    inlet[5 * b + 4] = m.bcs[b].T;
  }

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    P->has_device = 0;
    *out = P;
    return SLLBM_OK;
  }
  (void)hipGetDevice(&P->device);
  P->has_device = 1;

#define UP(vec, dst)                                  \
  do {                                                \
    int _rc = upload(P, vec, &(dst));                 \
    if (_rc != SLLBM_OK) { sllbm_plan_destroy(P); return _rc; } \
  } while (0)

  const double *vel_d = nullptr, *inlet_d = nullptr, *vol_d = nullptr;
  UP(t.vel, vel_d);
  UP(inlet, inlet_d);
  UP(P->vol, vol_d);
  P->inlet_dev = inlet_d;
  if (P->kernel == 0) {
    DevTensorPlan &tp = P->tp;
    tp.dim = m.dim;
    tp.p = m.p;
    tp.Q = V.Q;
    tp.N = m.n_nodes;
    for (int a = 0; a < 3; a++) {
      DevAxis &ax = tp.ax[a];
      ax.N = m.N[a];
      ax.periodic = a < m.dim ? (m.periodic(a) ? 1 : 0) : 1;
      ax.ntab = t.ntab[a];
      std::vector<float> w32(t.w[a].size());
      for (size_t r = 0; r < t.w[a].size(); r += m.p + 1) round_weights_f32(&t.w[a][r], m.p + 1, &w32[r]);
      UP(t.start[a], ax.start);
      UP(t.w[a], ax.w64);
      UP(w32, ax.w32);
      UP(t.ident[a], ax.ident);
    }
    UP(t.tab_reg, tp.tab_reg);
    tp.nfaces = t.nfaces;
    for (int f = 0; f < t.nfaces; f++) {
      DevFace &F = tp.face[f];
      F.axis = t.face_axis[f];
      F.side = t.face_side[f];
      F.depth = t.face_depth[f];
      UP(t.face_e[f], F.e);
      UP(t.face_Tw[f], F.Tw);
    }
    tp.vel = vel_d;
    tp.vol = vol_d;
  } else {
    DevCsrPlan &cp = P->cp;
    cp.dim = m.dim;
    cp.p = m.p;
    cp.Q = V.Q;
    cp.N = m.n_nodes;
    cp.npc = 1;
    for (int d = 0; d < m.dim; d++) cp.npc *= (m.p + 1);
    std::vector<int32_t> cn32(m.cell_nodes.begin(), m.cell_nodes.end());
    UP(cn32, cp.cell_nodes);
    if (m.n_cells >= kCsrOpp) {
      sllbm_plan_destroy(P);
      return fail(SLLBM_EUNSUPPORTED, "curvilinear plans hold at most %d cells", (int)kCsrOpp - 1);
    }
    std::vector<int32_t> code(t.row_cell.size());
    for (size_t i = 0; i < (size_t)V.Q; i++)
      for (size_t k = 0; k < (size_t)m.n_nodes; k++) {
        const size_t r = i * (size_t)m.n_nodes + k;
        const int32_t c = t.row_cell[r], src = t.row_src[r];
        if (c >= 0 && src != (int32_t)i && src != V.opp[i]) {
          sllbm_plan_destroy(P);
          return fail(SLLBM_EGEOM, "curvilinear row (%zu, %zu): source %d is neither the velocity nor its opposite", i,
                      k, (int)src);
        }
        code[r] = c < 0 ? -1 - src : (c | (src != (int32_t)i ? kCsrOpp : 0));
      }
    UP(code, cp.row_code);
    UP(V.opp, cp.opp);
    cp.row_xi = nullptr;
    cp.row_xf = nullptr;
    if (P->prec == SLLBM_F32) {
      std::vector<float> xf(t.row_xi.size());
      const size_t N = (size_t)m.n_nodes;
      for (size_t i = 0; i < (size_t)V.Q; i++)
        for (size_t k = 0; k < N; k++) {
          xf[2 * (i * N + k)] = (float)t.row_xi[(2 * i) * N + k];
          xf[2 * (i * N + k) + 1] = (float)t.row_xi[(2 * i + 1) * N + k];
        }
      UP(xf, cp.row_xf);
    } else {
      UP(t.row_xi, cp.row_xi);
    }
    for (int a = 0; a <= m.p; a++) {
      cp.xref[a] = m.xref[a];
      double l = 1.0;
      for (int b = 0; b <= m.p; b++)
        if (b != a) l *= m.xref[a] - m.xref[b];
      cp.lam[a] = 1.0 / l;
    }
    UP(t.node_Tw, cp.node_Tw);
    cp.vel = vel_d;
    cp.vol = vol_d;
  }
#undef UP
  int64_t nblk = (m.n_nodes + kBlock - 1) / kBlock;
  P->scratch_len = kScratchHead + kRedWidth * nblk;
  hipError_t e = P->dalloc.get((void **)&P->scratch, sizeof(double) * P->scratch_len);
  if (e != hipSuccess) {
    sllbm_plan_destroy(P);
    return fail(SLLBM_ENOMEM, "device allocation (scratch): %s", hipGetErrorString(e));
  }
  if (P->tile_ok) {
    e = P->dalloc.get((void **)&P->nstate, sizeof(double) * 6 * (size_t)m.n_nodes);
    if (e != hipSuccess) {
      sllbm_plan_destroy(P);
      return fail(SLLBM_ENOMEM, "device allocation (node state): %s", hipGetErrorString(e));
    }
  }
  *out = P;
  return SLLBM_OK;
}

extern "C" int sllbm_plan_info(sllbm_plan P, sllbm_plan_info_t *info) {
  if (!P || !info) return fail(SLLBM_EINVAL, "plan_info: NULL argument");
  info->n_nodes = P->mesh.n_nodes;
  info->Q = P->vel.Q;
  info->dim = P->mesh.dim;
  info->order_p = P->mesh.p;
  info->prec = P->prec;
  info->n_exceptions = P->n_exceptions;
  info->n_thermal_nodes = P->n_thermal;
  info->table_bytes = P->table_bytes;
  info->has_device = P->has_device;
  info->kernel = P->kernel == 1 ? 1 : (P->use_col() ? 3 : (P->use_tile() ? 2 : 0));
  return SLLBM_OK;
}

extern "C" int sllbm_plan_select_kernel(sllbm_plan P, int kernel) {
  if (!P) return fail(SLLBM_EINVAL, "plan_select_kernel: plan is NULL");
  if (kernel < 0 || kernel > 3) return fail(SLLBM_EINVAL, "plan_select_kernel: kernel must be 0, 1, 2 or 3");
  if (kernel == 2 && !P->tile_ok)
    return fail(SLLBM_EUNSUPPORTED, "plan_select_kernel: the tiled kernel does not apply to this plan");
  if (kernel == 3 && !P->col_ok)
    return fail(SLLBM_EUNSUPPORTED, "plan_select_kernel: the velocity-split 3D step does not apply to this plan");
  P->kernel_choice = kernel;
  return SLLBM_OK;
}

// ------------------------------------------------------------------ per-kernel timing

namespace sllbm {
namespace {
hipEvent_t prof_event(Profiler &pr) {
  if (!pr.pool.empty()) {
    hipEvent_t e = pr.pool.back();
    pr.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// wait for the recorded launches, add their times, recycle the events
void prof_flush(Profiler &pr) {
  for (const auto &r : pr.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      pr.total_ms[r.id] += ms;
      pr.launches[r.id] += 1;
    }
    pr.pool.push_back(r.a);
    pr.pool.push_back(r.b);
  }
  pr.pending.clear();
}
}  // namespace

void prof_begin(sllbm_plan_s *P, const char *name, hipStream_t s, int *id, hipEvent_t *a) {
  *id = -1;
  *a = nullptr;
  Profiler &pr = P->prof;
  if (!pr.on) return;
  int k = 0;
  while (k < (int)pr.names.size() && pr.names[k] != name) k++;
  if (k == (int)pr.names.size()) {
    pr.names.push_back(name);
    pr.total_ms.push_back(0.0);
    pr.launches.push_back(0);
  }
  hipEvent_t e = prof_event(pr);
  if (!e || hipEventRecord(e, s) != hipSuccess) return;
  *id = k;
  *a = e;
}

void prof_end(sllbm_plan_s *P, int id, hipEvent_t a, hipStream_t s) {
  if (id < 0) return;
  Profiler &pr = P->prof;
  hipEvent_t b = prof_event(pr);
  if (!b || hipEventRecord(b, s) != hipSuccess) return;
  pr.pending.push_back({id, a, b});
  if (pr.pending.size() > 8192) prof_flush(pr);
}
}  // namespace sllbm

extern "C" int sllbm_plan_profile(sllbm_plan P, int enable) {
  if (!P) return fail(SLLBM_EINVAL, "plan_profile: plan is NULL");
  if (!P->has_device) return fail(SLLBM_EHIP, "plan_profile: the plan has no device");
  HIP_TRY(hipSetDevice(P->device));
  prof_flush(P->prof);
  if (enable) {
    P->prof.names.clear();
    P->prof.total_ms.clear();
    P->prof.launches.clear();
  }
  P->prof.on = enable != 0;
  return SLLBM_OK;
}

extern "C" int sllbm_plan_profile_read(sllbm_plan P, int max, char (*names)[32], double *total_ms, int64_t *launches) {
  if (!P) return fail(SLLBM_EINVAL, "plan_profile_read: plan is NULL");
  if (max < 0 || (max > 0 && (!names || !total_ms || !launches)))
    return fail(SLLBM_EINVAL, "plan_profile_read: NULL output with max > 0");
  if (P->has_device) {
    HIP_TRY(hipSetDevice(P->device));
    prof_flush(P->prof);
  }
  int n = (int)P->prof.names.size();
  for (int k = 0; k < n && k < max; k++) {
    std::snprintf(names[k], 32, "%s", P->prof.names[k].c_str());
    total_ms[k] = P->prof.total_ms[k];
    launches[k] = P->prof.launches[k];
  }
  return n;
}

extern "C" void sllbm_plan_destroy(sllbm_plan P) {
  if (!P) return;
  if (P->has_device) {
    (void)hipSetDevice(P->device);
    prof_flush(P->prof);
    for (hipEvent_t e : P->prof.pool) (void)hipEventDestroy(e);
    for (void *d : P->dev_allocs) P->dalloc.put(d);
    P->dalloc.put(P->scratch);
    P->dalloc.put(P->nstate);
  }
  delete P;
}

// ------------------------------------------------------------------ launches

extern "C" int sllbm_init_equilibrium(sllbm_plan P, const sllbm_params *prm, const double *rho, const double *u,
                                      const double *T, void *pop, void *stream) {
  if (!P) return fail(SLLBM_EINVAL, "init_equilibrium: plan is NULL");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if (!rho || !u || !T) return fail(SLLBM_EINVAL, "init_equilibrium: rho, u and T are required");
  if ((rc = check_pop(P, pop, "pop"))) return rc;
  if ((rc = require_device(P))) return rc;
  StepArgs a = make_args(P, prm);
  return launch_init(P, a, rho, u, T, pop, (hipStream_t)stream);
}

extern "C" int sllbm_step(sllbm_plan P, const sllbm_params *prm, const void *pin, void *pout, void *stream) {
  if (!P) return fail(SLLBM_EINVAL, "step: plan is NULL");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if ((rc = check_pop(P, pin, "pop_in")) || (rc = check_pop(P, pout, "pop_out"))) return rc;
  size_t bytes = 2 * (size_t)P->vel.Q * (size_t)P->mesh.n_nodes * elem_size(P);
  const char *a0 = (const char *)pin, *b0 = (const char *)pout;
  if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(SLLBM_EINVAL, "step: pop_in and pop_out overlap");
  if ((rc = require_device(P))) return rc;
  StepArgs a = make_args(P, prm);
  hipStream_t s = (hipStream_t)stream;
  if (prm->mass_fix) {
    rc = launch_mass_scale(P, pin, prm->mass_ref, s);
    if (rc) return rc;
    a.scale = P->scratch + kSlotScale;
  }
  return launch_step(P, a, pin, pout, s);
}

extern "C" int sllbm_step_learned(sllbm_plan P, const sllbm_params *prm, sllbm_mlp m, const void *pin, void *pout,
                                  void *stream) {
  if (!P) return fail(SLLBM_EINVAL, "step_learned: plan is NULL");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if ((rc = check_pop(P, pin, "pop_in")) || (rc = check_pop(P, pout, "pop_out"))) return rc;
  size_t bytes = 2 * (size_t)P->vel.Q * (size_t)P->mesh.n_nodes * elem_size(P);
  const char *a0 = (const char *)pin, *b0 = (const char *)pout;
  if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(SLLBM_EINVAL, "step_learned: pop_in and pop_out overlap");
  if ((rc = require_device(P))) return rc;
  if ((rc = learned_check(P, m))) return rc;
  StepArgs a = make_args(P, prm);
  hipStream_t s = (hipStream_t)stream;
  if (prm->mass_fix) {
    rc = launch_mass_scale(P, pin, prm->mass_ref, s);
    if (rc) return rc;
    a.scale = P->scratch + kSlotScale;
  }
  if (!step_has_relax_launch(P)) {
    // kernels that relax as they stream: the step, then the correction on its result
    if ((rc = launch_step(P, a, pin, pout, s))) return rc;
    return launch_mlp_correct(P, prm, m, pout, s);
  }
  if ((rc = launch_step(P, a, pin, pout, s, false))) return rc;
  return launch_relax_correct(P, a, m, pout, s);
}

extern "C" int sllbm_force_reset(sllbm_plan P, const double *force0, void *stream) {
  if (!P || !force0) return fail(SLLBM_EINVAL, "force_reset: NULL argument");
  double F[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < P->mesh.dim; a++) {
    if (!std::isfinite(force0[a])) return fail(SLLBM_EINVAL, "force_reset: force must be finite");
    F[a] = force0[a];
  }
  int rc;
  if ((rc = require_device(P))) return rc;
  if ((rc = launch_force_reset(P, F, (hipStream_t)stream))) return rc;
  P->force_ready = true;
  return SLLBM_OK;
}

extern "C" int sllbm_force_update(sllbm_plan P, const sllbm_force_ctl *c, const void *pop, void *stream) {
  if (!P || !c) return fail(SLLBM_EINVAL, "force_update: NULL argument");
  if (!P->force_ready) return fail(SLLBM_EINVAL, "force_update: call sllbm_force_reset first");
  if (c->axis < 0 || c->axis >= P->mesh.dim)
    return fail(SLLBM_EINVAL, "force_update: axis %d outside 0..%d", c->axis, P->mesh.dim - 1);
  if (!std::isfinite(c->target) || !std::isfinite(c->kp) || !std::isfinite(c->ki) || !(c->dt >= 0) ||
      !std::isfinite(c->dt))
    return fail(SLLBM_EINVAL, "force_update: target, gains must be finite and dt >= 0");
  int rc;
  if ((rc = check_pop(P, pop, "pop"))) return rc;
  if ((rc = require_device(P))) return rc;
  return launch_force_update(P, c->axis, c->target, c->kp, c->ki, c->dt, pop, (hipStream_t)stream);
}

extern "C" int sllbm_force_read(sllbm_plan P, double *state_host, void *stream) {
  if (!P || !state_host) return fail(SLLBM_EINVAL, "force_read: NULL argument");
  if (!P->force_ready) return fail(SLLBM_EINVAL, "force_read: call sllbm_force_reset first");
  int rc;
  if ((rc = require_device(P))) return rc;
  hipStream_t s = (hipStream_t)stream;
  double h[12];
  HIP_TRY(hipMemcpyAsync(h, P->scratch + kSlotForce, sizeof(double) * 12, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int q = 0; q < 3; q++) state_host[q] = h[q];
  for (int q = 0; q < 4; q++) state_host[3 + q] = h[kSlotCtl - kSlotForce + q];
  return SLLBM_OK;
}

namespace {
// Fixed device scratch of sllbm_moments_noalloc: kRedWidth doubles of final totals, then the
// block partials of the totals reduction (kRedWidth doubles per block of kBlock nodes) for
// up to kNoAllocMaxNodes nodes: 8 MiB plus 64 bytes.  Each GPU the library runs on holds its
// own copy until the process ends; every call on that GPU shares it.
constexpr int64_t kNoAllocMaxNodes = int64_t(1) << 25;
constexpr size_t kNoAllocDoubles = (size_t)kRedWidth * (size_t)(1 + kNoAllocMaxNodes / kBlock);
__device__ __align__(256) double scratch[kNoAllocDoubles];

// Device address of `scratch` on each GPU, looked up once per device (with that device
// current) on its first call; host code uses only these addresses.
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kNoAllocMaxDevices] = {};

int noalloc_scratch(int device, double **out) {
  if (device < 0 || device >= kNoAllocMaxDevices)
    return fail(SLLBM_EUNSUPPORTED, "moments_noalloc: device %d beyond the %d it keeps scratch for", device,
                kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SLLBM_EHIP, "moments_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[device] = (double *)p;
  }
  *out = g_scratch_dev[device];
  return SLLBM_OK;
}

// Totals [2 + dim] from the kRedWidth reduced doubles; SLLBM_EUNSTABLE if any node was bad.
int totals_out(const sllbm_plan_s *P, const double *h, double *totals_host, const char *who) {
  int D = P->mesh.dim;
  for (int q = 0; q < 2 + D; q++) totals_host[q] = h[q];
  if (h[kRedWidth - 1] > 0)
    return fail(SLLBM_EUNSTABLE, "%s: %.0f nodes with non-finite values, rho <= 0 or T <= 0", who, h[kRedWidth - 1]);
  return SLLBM_OK;
}
}  // namespace

extern "C" int sllbm_moments_noalloc(sllbm_plan P, const sllbm_params *prm, const void *pop, double *rho, double *u,
                                     double *T, double *totals_host, void *stream) {
  if (!P) return fail(SLLBM_EINVAL, "moments_noalloc: plan is NULL");
  if (P->mesh.n_nodes > kNoAllocMaxNodes)
    return fail(SLLBM_EINVAL, "moments_noalloc: %lld nodes exceed the %lld its fixed scratch holds",
                (long long)P->mesh.n_nodes, (long long)kNoAllocMaxNodes);
  int rc = check_params(P, prm);
  if (rc) return rc;
  if ((rc = check_pop(P, pop, "pop"))) return rc;
  if ((rc = require_device(P))) return rc;
  double *scr = nullptr;
  if ((rc = noalloc_scratch(P->device, &scr))) return rc;
  StepArgs a = make_args(P, prm);
  hipStream_t s = (hipStream_t)stream;
  // every block writes its partial and the final pass overwrites the totals, so nothing
  // left in the scratch by an earlier call is read
  rc = launch_moments_to(P, a, pop, rho, u, T, scr + kRedWidth, totals_host ? scr : nullptr, s);
  if (rc) return rc;
  if (totals_host) {
    double h[kRedWidth];
    HIP_TRY(hipMemcpyAsync(h, scr, sizeof(double) * kRedWidth, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return totals_out(P, h, totals_host, "moments_noalloc");
  }
  return SLLBM_OK;
}

extern "C" int sllbm_moments(sllbm_plan P, const sllbm_params *prm, const void *pop, double *rho, double *u,
                             double *T, double *totals_host, void *stream) {
  if (!P) return fail(SLLBM_EINVAL, "moments: plan is NULL");
  int rc = check_params(P, prm);
  if (rc) return rc;
  if ((rc = check_pop(P, pop, "pop"))) return rc;
  if ((rc = require_device(P))) return rc;
  StepArgs a = make_args(P, prm);
  hipStream_t s = (hipStream_t)stream;
  rc = launch_moments(P, a, pop, rho, u, T, totals_host != nullptr, s);
  if (rc) return rc;
  if (totals_host) {
    double h[kRedWidth];
    HIP_TRY(hipMemcpyAsync(h, P->scratch + kSlotTotals, sizeof(double) * kRedWidth, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return totals_out(P, h, totals_host, "moments");
  }
  return SLLBM_OK;
}
