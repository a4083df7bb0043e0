// LDS-tiled fused SLLBM step on tensor-product meshes (gfx950, wave64).
//
// One workgroup owns a cell-aligned tile of TX x TY x TZ nodes.  For every velocity i
// it stages the departure region of f_i and g_i (the tile shifted by the velocity's
// displacement, at most one cell of halo on one side per axis) from HBM into LDS, then
// applies the separable interpolant of eq:intf as three 1D passes (x, y, z) in LDS:
// the cost per streamed value is 3(p+1) multiply-adds instead of (p+1)^3 gathers.
// Two launches per step: the first streams every velocity, stores the streamed f_i, g_i
// and reduces their conserved moments per node into a small node-state array (6 doubles
// per node); the second relaxes the stored populations in place, one node per lane.
// (Built with TILE_STORE=0, the second launch re-streams instead of reading the stored
// values: half the HBM writes, twice the interpolation.)  Nodes in the boundary layers of a bounded
// face (where some departure point leaves the domain, and where the isothermal-wall
// correction acts) are left to the per-node gather kernel, launched on those slabs.
#include <hip/hip_runtime.h>

#include "sllbm_device_common.h"
#include "sllbm_kernels.h"

namespace sllbm {

#ifndef TILE_WPE
#define TILE_WPE 4
#endif
#ifndef TILE_WPE2
#define TILE_WPE2 2
#endif
#ifndef PASS_UNROLL
#define PASS_UNROLL 1
#endif
// 1: the moments launch also stores the streamed populations and a per-node kernel
// relaxes them in place; 0: the second launch re-streams them instead
#ifndef TILE_STORE
#define TILE_STORE 1
#endif

struct TileGrid {
  int nt[3];   // tiles per axis
  int q, r;    // ntiles = 8 q + r (XCD remap)
};

// Stencil start of node n0 + t along one axis relative to the tile origin n0, brought
// into [-P, T] across the periodic seam (the plan guarantees a unique such value).
template <int P>
__device__ __forceinline__ int rel_start(int s, int n0, int N, int T) {
  int r = s - n0;
  if (r > T) r -= N;
  else if (r < -P) r += N;
  return r;
}

struct AxGeo {
  int tb;      // table id
  int ident;   // zero displacement along this axis
  int rs;      // region start relative to the tile origin
  int R;       // region extent
};

template <int P>
__device__ __forceinline__ AxGeo axis_geo(const DevAxis &ax, int tb, int n0, int vt, int T) {
  AxGeo g;
  g.tb = tb;
  g.ident = ax.ident[tb];
  if (g.ident) {
    g.rs = 0;
    g.R = vt;
  } else {
    const int32_t *st = ax.start + (size_t)tb * ax.N + n0;
    int sf = rel_start<P>(st[0], n0, ax.N, T);
    int sl = rel_start<P>(st[vt - 1], n0, ax.N, T);
    g.rs = sf;
    g.R = sl + P - sf + 1;
  }
  return g;
}

template <typename T, int P>
__device__ __forceinline__ void axis_weights(const DevAxis &ax, const AxGeo &g, int n0, int t, int T_, int &off,
                                             int &len, T (&w)[P + 1]) {
  if (g.ident) {
    off = t;
    len = 1;
    w[0] = T(1);
#pragma unroll
    for (int j = 1; j <= P; j++) w[j] = T(0);
    return;
  }
  size_t row = (size_t)g.tb * ax.N + n0 + t;
  off = rel_start<P>(ax.start[row], n0, ax.N, T_) - g.rs;
  len = P + 1;
  const T *wp = WeightSel<T>::get(ax) + row * (P + 1);
#pragma unroll
  for (int j = 0; j <= P; j++) w[j] = wp[j];
}

__device__ __forceinline__ int wrap_idx(int g, int N) {
  if (g < 0) g += N;
  else if (g >= N) g -= N;
  return g;
}

// MODE 1: streamed moments -> node state (rho, u, T, 1/tau_bar as [6][N] doubles), and
// with TILE_STORE the streamed populations -> pout;
// MODE 2: re-stream, relax against the node state, store.
template <typename T, int D, int P, int CX, int CY, int CZ, int BS, int WPE, int MODE>
__global__ void __launch_bounds__(BS, WPE) k_step_tile(const DevTensorPlan pl, const StepArgs sa, const TileGrid tg,
                                                    const T *__restrict__ pin, T *__restrict__ pout,
                                                    double *__restrict__ nstate) {
  constexpr int TX = CX * P, TY = CY * P, TZ = (D == 3) ? CZ * P : 1;
  constexpr int RX = TX + P + 1, RY = TY + P + 1, RZ = (D == 3) ? TZ + P + 1 : 1;
  constexpr int NT = TX * TY * TZ;
  constexpr int NPT = (NT + BS - 1) / BS;
  constexpr int SS = RZ * RY * RX;           // one population's staging size
  constexpr int XS = RZ * RY * TX;           // one population's x-pass output
  constexpr int YS = RZ * TY * TX;           // one population's y-pass output (3D)
  constexpr int NST = (SS + BS - 1) / BS;      // staged elements per thread and population
  constexpr int NW = TX + TY + TZ;           // weight rows: one per tile position and axis
  static_assert(NW <= BS, "weight rows exceed the workgroup");
  __shared__ T S[2 * SS];
  __shared__ T X[2 * XS];
  __shared__ T WT[NW * (P + 1)];
  __shared__ int OT[NW];
  T *Yb = S;

  const int Q = pl.Q;
  const int tid = threadIdx.x;
  const int64_t N = pl.N;
  const int Nx = pl.ax[0].N, Ny = pl.ax[1].N, Nz = pl.ax[2].N;

  // XCD-aware tile index: consecutive workgroups go round-robin to the 8 XCDs; give each
  // XCD a contiguous range of tiles so that neighbouring tiles share its L2.
  const int bid = blockIdx.x;
  const int xcd = bid & 7, jj = bid >> 3;
  const int tile = xcd * tg.q + min(xcd, tg.r) + jj;
  const int b0 = tile % tg.nt[0];
  const int b1 = (tile / tg.nt[0]) % tg.nt[1];
  const int b2 = tile / (tg.nt[0] * tg.nt[1]);
  const int n0x = b0 * TX, n0y = b1 * TY, n0z = b2 * TZ;
  const int vx = min(TX, Nx - n0x), vy = min(TY, Ny - n0y), vz = (D == 3) ? min(TZ, Nz - n0z) : 1;

  // owned nodes: flat tile index tid + BS m, x fastest
  int otx[NPT], oty[NPT], otz[NPT];
  bool own[NPT];
#pragma unroll
  for (int m = 0; m < NPT; m++) {
    int f = tid + BS * m;
    otx[m] = f % TX;
    oty[m] = (f / TX) % TY;
    otz[m] = f / (TX * TY);
    own[m] = (f < NT) && otx[m] < vx && oty[m] < vy && otz[m] < vz;
    // nodes in the boundary layers of a bounded face are computed by the per-node
    // gather kernel (launched on those slabs); this kernel leaves them alone
    for (int fc = 0; fc < pl.nfaces; fc++) {
      const DevFace &F = pl.face[fc];
      int n3 = F.axis == 0 ? n0x + otx[m] : (F.axis == 1 ? n0y + oty[m] : n0z + otz[m]);
      int l = F.side == 0 ? n3 : pl.ax[F.axis].N - 1 - n3;
      if (l < F.depth) own[m] = false;
    }
  }
  const double scale = sa.scale ? *sa.scale : 1.0;

  auto node_index = [&](int m) __attribute__((always_inline)) -> int64_t {
    return (int64_t)(n0x + otx[m]) + (int64_t)Nx * ((int64_t)(n0y + oty[m]) + (int64_t)Ny * (n0z + otz[m]));
  };
  // ---- software pipeline: the departure region of velocity i+1 is loaded into
  // registers while velocity i is interpolated out of LDS
  T pf[NST], pg[NST];
  T pw[P + 1];
  int poff = 0;
  AxGeo ng[3], cg[3];
  auto prefetch = [&](int i) __attribute__((always_inline)) {
    ng[0] = axis_geo<P>(pl.ax[0], pl.tab_reg[i], n0x, vx, TX);
    ng[1] = axis_geo<P>(pl.ax[1], pl.tab_reg[Q + i], n0y, vy, TY);
    if (D == 3) {
      ng[2] = axis_geo<P>(pl.ax[2], pl.tab_reg[2 * Q + i], n0z, vz, TZ);
    } else {
      ng[2].tb = 0; ng[2].ident = 1; ng[2].rs = 0; ng[2].R = 1;
    }
    const T *F = pin + (size_t)i * N;
    const T *G = pin + ((size_t)Q + i) * N;
#pragma unroll
    for (int s = 0; s < NST; s++) {
      int e = tid + BS * s;
      int rx = e % RX, ry = (e / RX) % RY, rz = e / (RX * RY);
      if (e < SS && rx < ng[0].R && ry < ng[1].R && rz < ng[2].R) {
        int gxx = wrap_idx(n0x + ng[0].rs + rx, Nx);
        int gyy = wrap_idx(n0y + ng[1].rs + ry, Ny);
        int gzz = (D == 3) ? wrap_idx(n0z + ng[2].rs + rz, Nz) : 0;
        size_t k = (size_t)gxx + (size_t)Nx * ((size_t)gyy + (size_t)Ny * gzz);
        pf[s] = F[k];
        pg[s] = G[k];
      }
    }
    if (tid < NW) {
      int ax = tid < TX ? 0 : (tid < TX + TY ? 1 : 2);
      int q = tid - (ax == 0 ? 0 : (ax == 1 ? TX : TX + TY));
      int vt = ax == 0 ? vx : (ax == 1 ? vy : vz);
      int n0a = ax == 0 ? n0x : (ax == 1 ? n0y : n0z);
      int Ta = ax == 0 ? TX : (ax == 1 ? TY : TZ);
      int len;
      const AxGeo &ga = ax == 0 ? ng[0] : (ax == 1 ? ng[1] : ng[2]);
      const DevAxis &da = ax == 0 ? pl.ax[0] : (ax == 1 ? pl.ax[1] : pl.ax[2]);
      if (ax < D && q < vt) axis_weights<T, P>(da, ga, n0a, q, Ta, poff, len, pw);
    }
  };
  auto commit = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NST; s++) {
      int e = tid + BS * s;
      int rx = e % RX, ry = (e / RX) % RY, rz = e / (RX * RY);
      if (e < SS && rx < ng[0].R && ry < ng[1].R && rz < ng[2].R) {
        S[e] = pf[s];
        S[SS + e] = pg[s];
      }
    }
    if (tid < NW) {
#pragma unroll
      for (int j = 0; j <= P; j++) WT[tid * (P + 1) + j] = pw[j];
      OT[tid] = poff;
    }
    cg[0] = ng[0];
    cg[1] = ng[1];
    cg[2] = ng[2];
  };

  // Streamed f_i, g_i of every owned node out of the committed LDS region: three 1D
  // passes (two in 2D), then the boundary-layer pairs by per-node gather.
  auto interpolate = [&](double (&fv)[NPT], double (&gv)[NPT]) __attribute__((always_inline)) {
    const int Ry = cg[1].R, Rz = cg[2].R;
    {  // x-pass: S[rz][ry][*] -> X[rz][ry][tx]; each thread keeps one tx (and its
       // weights) and walks the rows
      constexpr int NRX = BS / TX;          // rows in flight per sweep of the workgroup
      const int len = cg[0].ident ? 1 : P + 1;
      const int tx = tid % TX, r0 = tid / TX;
      if (r0 < NRX && tx < vx) {
        const int off = OT[tx];
        T w[P + 1];
#pragma unroll
        for (int j = 0; j <= P; j++) w[j] = WT[tx * (P + 1) + j];
        const int nrows = Ry * Rz;
#pragma unroll PASS_UNROLL
        for (int rr = r0; rr < RY * RZ; rr += NRX) {
          int ry = rr % Ry, rz = rr / Ry;
          if (rr >= nrows) break;
          const T *sf = S + (rz * RY + ry) * RX + off;
          T a = 0, b = 0;
#pragma unroll
          for (int j = 0; j <= P; j++) {
            if (j >= len) break;
            a += w[j] * sf[j];
            b += w[j] * sf[SS + j];
          }
          int l = (rz * RY + ry) * TX + tx;
          X[l] = a;
          X[XS + l] = b;
        }
      }
    }
    __syncthreads();
    if constexpr (D == 3) {
      {  // y-pass: X[rz][*][tx] -> Yb[rz][ty][tx]; each thread keeps one (tx, ty)
        constexpr int NRY = BS / (TX * TY);
        static_assert(NRY >= 1, "tile cross-section exceeds the workgroup");
        const int len = cg[1].ident ? 1 : P + 1;
        const int tx = tid % TX, ty = (tid / TX) % TY, z0 = tid / (TX * TY);
        if (z0 < NRY && tx < vx && ty < vy) {
          const int off = OT[TX + ty];
          T w[P + 1];
#pragma unroll
          for (int j = 0; j <= P; j++) w[j] = WT[(TX + ty) * (P + 1) + j];
#pragma unroll PASS_UNROLL
          for (int rz = z0; rz < RZ; rz += NRY) {
            if (rz >= Rz) break;
            const T *xf = X + (rz * RY + off) * TX + tx;
            T a = 0, b = 0;
#pragma unroll
            for (int j = 0; j <= P; j++) {
              if (j >= len) break;
              a += w[j] * xf[j * TX];
              b += w[j] * xf[XS + j * TX];
            }
            int l = (rz * TY + ty) * TX + tx;
            Yb[l] = a;
            Yb[YS + l] = b;
          }
        }
      }
      __syncthreads();
      const int len = cg[2].ident ? 1 : P + 1;
#pragma unroll
      for (int m = 0; m < NPT; m++) {  // z-pass for the owned nodes
        fv[m] = gv[m] = 0.0;
        if (!own[m]) continue;
        const T *yf = Yb + (OT[TX + TY + otz[m]] * TY + oty[m]) * TX + otx[m];
        const T *w = WT + (TX + TY + otz[m]) * (P + 1);
        T a = 0, b = 0;
#pragma unroll
        for (int j = 0; j <= P; j++) {
          if (j >= len) break;
          a += w[j] * yf[j * TY * TX];
          b += w[j] * yf[YS + j * TY * TX];
        }
        fv[m] = scale * (double)a;
        gv[m] = scale * (double)b;
      }
    } else {
      const int len = cg[1].ident ? 1 : P + 1;
#pragma unroll
      for (int m = 0; m < NPT; m++) {  // y-pass (last in 2D) for the owned nodes
        fv[m] = gv[m] = 0.0;
        if (!own[m]) continue;
        const T *xf = X + OT[TX + oty[m]] * TX + otx[m];
        const T *w = WT + (TX + oty[m]) * (P + 1);
        T a = 0, b = 0;
#pragma unroll
        for (int j = 0; j <= P; j++) {
          if (j >= len) break;
          a += w[j] * xf[j * TX];
          b += w[j] * xf[XS + j * TX];
        }
        fv[m] = scale * (double)a;
        gv[m] = scale * (double)b;
      }
    }
  };
  // one pipeline stage: velocity i is committed to LDS, velocity `next` (or -1) is
  // prefetched, and i is interpolated
  auto stream_velocity = [&](int i, int next, double (&fv)[NPT], double (&gv)[NPT]) __attribute__((always_inline)) {
    __syncthreads();  // everyone is done reading the previous velocity out of LDS
    commit();
    if (next >= 0) prefetch(next);
    __syncthreads();
    interpolate(fv, gv);
  };

  prefetch(0);
  if (MODE == 1) {
    // -------- sweep 1: conserved moments of the streamed populations -> node state
    double rho[NPT], j0[NPT], j1[NPT], j2[NPT], E[NPT];
#pragma unroll
    for (int m = 0; m < NPT; m++) rho[m] = j0[m] = j1[m] = j2[m] = E[m] = 0.0;
    for (int i = 0; i < Q; i++) {
      double fv[NPT], gv[NPT];
      stream_velocity(i, i + 1 < Q ? i + 1 : -1, fv, gv);
      const double *vi = pl.vel + 8 * i;
      const double z2 = vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2];
      if (TILE_STORE) {
#pragma unroll
        for (int m = 0; m < NPT; m++) {
          if (!own[m]) continue;
          const int64_t k = node_index(m);
          pout[(size_t)i * N + k] = (T)fv[m];
          pout[((size_t)Q + i) * N + k] = (T)gv[m];
        }
      }
#pragma unroll
      for (int m = 0; m < NPT; m++) {
        rho[m] += fv[m];
        j0[m] += vi[0] * fv[m];
        j1[m] += vi[1] * fv[m];
        j2[m] += vi[2] * fv[m];
        E[m] += z2 * fv[m] + gv[m];
      }
    }
    // node state: rho, u, T, 1/tau_bar (isothermal walls act only inside the boundary
    // layers, which the gather kernel handles)
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      if (!own[m]) continue;
      double r = rho[m];
      double u0 = j0[m] / r, u1 = j1[m] / r, u2 = j2[m] / r;
      double Tn = (E[m] - r * (u0 * u0 + u1 * u1 + u2 * u2)) / (2.0 * r * sa.cv);
      double it = 0.0;
      if (sa.relax_mode == 0) it = 1.0 / sa.tau_bar;
      if (sa.relax_mode == 1) {
        double mu = sa.mu_ref * pow(Tn / sa.T_ref, sa.mu_exp);
        it = 1.0 / (mu / (r * Tn * sa.dt) + 0.5);
      }
      const int64_t k = node_index(m);
      nstate[k] = r;
      nstate[N + k] = u0;
      nstate[2 * N + k] = u1;
      nstate[3 * N + k] = u2;
      nstate[4 * N + k] = Tn;
      nstate[5 * N + k] = it;
    }
  } else {
    // -------- sweep 2: re-stream, BGK relaxation, forcing, store
    double rho[NPT], nu0[NPT], nu1[NPT], nu2[NPT], Tn[NPT], itau[NPT];
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      const int64_t k = own[m] ? node_index(m) : 0;
      rho[m] = nstate[k];
      nu0[m] = nstate[N + k];
      nu1[m] = nstate[2 * N + k];
      nu2[m] = nstate[3 * N + k];
      Tn[m] = nstate[4 * N + k];
      itau[m] = nstate[5 * N + k];
    }
    for (int i = 0; i < Q; i++) {
      double fv[NPT], gv[NPT];
      stream_velocity(i, i + 1 < Q ? i + 1 : -1, fv, gv);
      const double *vi = pl.vel + 8 * i;
#pragma unroll
      for (int m = 0; m < NPT; m++) {
        if (!own[m]) continue;
        double f = fv[m], g = gv[m];
        // the node's equilibrium coefficients are rebuilt per velocity on purpose:
        // "+ 0 * w_i" keeps them inside the loop (hoisting them costs ~40 registers
        // per node and halves the occupancy)
        const double r_m = rho[m] + 0.0 * vi[7];
        EqNode e = eq_prepare(r_m, nu0[m], nu1[m], nu2[m], Tn[m], sa, D);
        double fe = eq_f(e, vi);
        const double gT = Tn[m] * sa.gbase;
        double fo = f, go = g;
        if (sa.relax_mode != 2) {
          fo = f - (f - fe) * itau[m];
          go = g - (g - gT * fe) * itau[m];
          if (sa.has_force) {
            EqNode ef = eq_forced(r_m, nu0[m], nu1[m], nu2[m], Tn[m], sa, D);
            double df = eq_f(ef, vi) - fe;
            fo += df;
            go += gT * df;
          }
        }
        const int64_t k = node_index(m);
        pout[(size_t)i * N + k] = (T)fo;
        pout[((size_t)Q + i) * N + k] = (T)go;
      }
    }
  }
}

// In-place BGK relaxation and forcing of the streamed populations the moments launch
// stored, one node per lane (its equilibrium coefficients built once); nodes in the
// boundary layers of a bounded face belong to the gather kernel and are skipped.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_relax_nodes(const DevTensorPlan pl, const StepArgs sa,
                                                        T *__restrict__ pop, const double *__restrict__ nstate) {
  const int64_t N = pl.N;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= N) return;
  const int Nx = pl.ax[0].N, Ny = pl.ax[1].N;
  for (int fc = 0; fc < pl.nfaces; fc++) {
    const DevFace &F = pl.face[fc];
    int64_t n3 = F.axis == 0 ? k % Nx : (F.axis == 1 ? (k / Nx) % Ny : k / ((int64_t)Nx * Ny));
    int64_t l = F.side == 0 ? n3 : pl.ax[F.axis].N - 1 - n3;
    if (l < F.depth) return;
  }
  if (sa.relax_mode == 2) return;   // pure streaming: the stored values are final
  const int Q = pl.Q;
  const double rho = nstate[k], u0 = nstate[N + k], u1 = nstate[2 * N + k], u2 = nstate[3 * N + k];
  const double Tn = nstate[4 * N + k], itau = nstate[5 * N + k];
  const EqNode e = eq_prepare(rho, u0, u1, u2, Tn, sa, D);
  EqNode ef = e;
  if (sa.has_force) ef = eq_forced(rho, u0, u1, u2, Tn, sa, D);
  const double gT = Tn * sa.gbase;
  for (int i = 0; i < Q; i++) {
    const double *vi = pl.vel + 8 * i;
    T *pf = pop + (size_t)i * N + k;
    T *pg = pop + ((size_t)Q + i) * N + k;
    double f = (double)*pf, g = (double)*pg;
    double fe = eq_f(e, vi);
    double fo = f - (f - fe) * itau;
    double go = g - (g - gT * fe) * itau;
    if (sa.has_force) {
      double df = eq_f(ef, vi) - fe;
      fo += df;
      go += gT * df;
    }
    *pf = (T)fo;
    *pg = (T)go;
  }
}

// ------------------------------------------------------------------ launcher

namespace {
template <typename T, int D, int P, int CX, int CY, int CZ>
int launch_tile_t(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  constexpr int BS = D == 3 ? 512 : 256;   // threads per workgroup
  // minimum waves per SIMD the register budget must allow, per launch
  constexpr int WPE = TILE_WPE, WPE2 = TILE_WPE2;
  constexpr int TX = CX * P, TY = CY * P, TZ = (D == 3) ? CZ * P : 1;
  const DevTensorPlan &tp = Pl->tp;
  TileGrid tg;
  tg.nt[0] = (tp.ax[0].N + TX - 1) / TX;
  tg.nt[1] = (tp.ax[1].N + TY - 1) / TY;
  tg.nt[2] = D == 3 ? (tp.ax[2].N + TZ - 1) / TZ : 1;
  int ntiles = tg.nt[0] * tg.nt[1] * tg.nt[2];
  tg.q = ntiles / 8;
  tg.r = ntiles % 8;
  {
    ProfScope ps(Pl, "k_step_tile", s);
    hipLaunchKernelGGL((k_step_tile<T, D, P, CX, CY, CZ, BS, WPE, 1>), dim3(ntiles), dim3(BS), 0, s, tp, a, tg,
                       (const T *)pin, (T *)pout, Pl->nstate);
  }
  if (TILE_STORE) {
    (void)WPE2;
    ProfScope ps(Pl, "k_relax_nodes", s);
    hipLaunchKernelGGL((k_relax_nodes<T, D>), dim3((unsigned)((tp.N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, tp,
                       a, (T *)pout, (const double *)Pl->nstate);
  } else {
    ProfScope ps(Pl, "k_step_tile_restream", s);
    hipLaunchKernelGGL((k_step_tile<T, D, P, CX, CY, CZ, BS, WPE2, 2>), dim3(ntiles), dim3(BS), 0, s, tp, a, tg,
                       (const T *)pin, (T *)pout, Pl->nstate);
  }
  return SLLBM_OK;
}
}  // namespace

int launch_step_tile(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s) {
  int D = Pl->mesh.dim, p = Pl->mesh.p;
  bool f32 = Pl->prec == SLLBM_F32;
#define TCASE(DD, PP)                                                                                  \
  if (D == DD && p == PP) {                                                                            \
    constexpr int CX = TileShape<DD, PP>::CX, CY = TileShape<DD, PP>::CY, CZ = TileShape<DD, PP>::CZ; \
    return f32 ? launch_tile_t<float, DD, PP, CX, CY, CZ>(Pl, a, pin, pout, s)                          \
               : launch_tile_t<double, DD, PP, CX, CY, CZ>(Pl, a, pin, pout, s);                        \
  }
  TCASE(2, 2) TCASE(2, 3) TCASE(2, 4) TCASE(3, 2) TCASE(3, 3) TCASE(3, 4)
#undef TCASE
  return fail(SLLBM_EUNSUPPORTED, "no tiled kernel for dim %d order %d", D, p);
}

}  // namespace sllbm
