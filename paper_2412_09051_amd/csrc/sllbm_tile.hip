// LDS-tiled fused SLLBM step on tensor-product meshes (gfx950, wave64).
//
// One workgroup owns a cell-aligned tile of nodes.  For a velocity i it stages the
// departure region of f_i and g_i (the tile shifted by the velocity's displacement, at most
// one cell of halo on one side per axis) from HBM into LDS, then applies the separable
// interpolant of eq:intf as 1D passes: (p+1) multiply-adds per pass and streamed value
// instead of (p+1)^d gathers.  Nodes in the boundary layers of a bounded face (where some
// departure point leaves the domain, and where the isothermal-wall correction acts) are left
// to the per-node gather kernel, launched on those slabs.  Three schedules, each measured on
// MI355X as the faster one where it applies:
//  * 2D (k_step_tile2d): every velocity of a tile of at most 256 nodes, the weight rows of
//    every table in LDS for the whole tile, buffer-load staging, the y contraction per node
//    straight out of the x-pass buffer (two barriers per velocity).  With Q = 25 or 19 a
//    node's streamed values stay in registers and the node is relaxed in the same launch.
//  * 3D tile (k_step_tile3d): every velocity of a 3D tile, x, y and z passes through LDS
//    (four barriers per velocity, or two with the passes of consecutive velocities skewed);
//    it stores the streamed values and the node state, and a second launch relaxes.
//  * velocity-split 3D (k_stream_col3d, then k_relax_moments): one velocity per workgroup
//    on a column of output nodes walked once along z (one barrier per source plane), then a
//    launch that forms each node's moments from its stored streamed values and relaxes them.
#include <hip/hip_runtime.h>

#include "sllbm_device_common.h"
#include "sllbm_kernels.h"

namespace sllbm {

#ifndef TILE_WPE
#define TILE_WPE 4
#endif
#ifndef COL_WPE64
#define COL_WPE64 5
#endif
#ifndef COL_WPE32
#define COL_WPE32 5
#endif
#ifndef COL_PADS
#define COL_PADS 0
#endif
#ifndef COL_PADX
#define COL_PADX 0
#endif
#ifndef COL_PD64
#define COL_PD64 2
#endif
#ifndef COL_PD32
#define COL_PD32 2
#endif

// 2D plans with this many velocities (D2V25) run the single-pass tile kernel, at 3 waves
// per SIMD (FP64: 168 VGPRs and a 36-byte spill, which beats 2 waves without one); so do
// plans on the reduced set D2Q19 (with the wide table count)
constexpr int kStashQ = 25;
constexpr int kStashQ19 = 19;

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

// Loads through a buffer resource: the base address stays in scalar registers and each
// lane supplies a 32-bit byte offset; the hardware returns 0 past num_records bytes.
template <typename T> struct BufLoad;
template <> struct BufLoad<double> {
  __device__ static double get(__amdgpu_buffer_rsrc_t r, int off) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return __builtin_bit_cast(double, v);
  }
};
template <> struct BufLoad<float> {
  __device__ static float get(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
};
template <typename T> struct BufStore;
template <> struct BufStore<double> {
  __device__ static void put(__amdgpu_buffer_rsrc_t r, int off, double v) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
  }
};
template <> struct BufStore<float> {
  __device__ static void put(__amdgpu_buffer_rsrc_t r, int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
  }
};
// A byte offset past every buffer this file builds (they hold at most kBufMaxBytes): loads
// at it return 0 and stores are dropped, so a lane without an element needs no branch.
// Memory accesses under divergent branches make the compiler wait for every access in
// flight (vmcnt(0)) before the next use of any of them, which serialises the prefetch
// with the passes it is meant to overlap.
constexpr int kBufOutOfRange = (int)kBufMaxBytes;
// the offset through an empty asm: the compiler keeps one offset register per access instead
// of turning the choice between a real and the out-of-range offset back into branches
__device__ __forceinline__ int opaque_off(int off) {
  asm volatile("" : "+v"(off));
  return off;
}
// The 8 constants of velocity i (zeta, xi, |xi|^2, w) through the scalar cache: the step
// never writes the velocity table, and scalar loads stay out of the vector-memory counter
// that the population loads and stores are waited on with.
__device__ __forceinline__ void vel_consts(const double *vel, int i, double (&v)[8]) {
  const double __attribute__((address_space(4))) *c = (const double __attribute__((address_space(4))) *)(vel + 8 * i);
#pragma unroll
  for (int j = 0; j < 8; j++) v[j] = c[j];
}
// one of three values by a runtime index, taken by value: a conditional expression over
// lvalues selects their addresses, which pins the arrays or the plan they live in to scratch
template <typename V>
__device__ __forceinline__ V sel3(int k, V a, V b, V c) {
  return k == 0 ? a : (k == 1 ? b : c);
}
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const T *base, int64_t elems) {
  const int64_t bytes = elems * (int64_t)sizeof(T);
  return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff),
                                           0x00020000);
}

__device__ __forceinline__ int wrap_idx(int g, int N) {
  if (g < 0) g += N;
  else if (g >= N) g -= N;
  return g;
}

// 2D: streams every velocity of one tile and stores the streamed f_i, g_i of the owned
// nodes and their node state (rho, u0, u1, u2, T, 1/tau_bar as [6][N] doubles).  The
// weight rows of every table are staged in LDS once per tile.  Per velocity i the
// workgroup passes two barriers:
//   barrier; x-pass of i (staging S -> X); barrier;
//   commit i+1 (registers -> S) and issue the loads of i+2; y contraction of i per owned
//   node straight out of X; store; moments.
// So the loads of a velocity are in flight for a whole iteration, and the y work of
// velocity i overlaps the staging of i+1.
template <typename T, int D, int P, int CX, int CY, int CZ, int BS, int WPE, int QR, int PR, int NTAB>
__global__ void __launch_bounds__(BS, WPE) k_step_tile2d(const DevTensorPlan pl, const StepArgs sa, const TileGrid tg,
                                                    const T *__restrict__ pin, T *__restrict__ pout,
                                                    double *__restrict__ nstate) {
  constexpr int TX = CX * P, TY = CY * P, TZ = (D == 3) ? CZ * P : 1;
  constexpr int RX = TX + P + 1, RY = TY + P + 1, RZ = (D == 3) ? TZ + P + 1 : 1;
  constexpr int NT = TX * TY * TZ;
  constexpr int NPT = (NT + BS - 1) / BS;
  static_assert(D == 2, "the 2D tile kernel");
  constexpr int SS = RZ * RY * RX;           // one population's staging size
  constexpr int XS = RZ * RY * TX;           // one population's x-pass output
  constexpr int NST = (SS + BS - 1) / BS;    // staged elements per thread and population
  constexpr int NW = TX + TY + TZ;           // weight rows of one table: one per tile position and axis
  __shared__ T S[2 * SS];
  __shared__ T X[2 * XS];
  __shared__ T WT[NTAB * NW * (P + 1)];   // row tb * NW + (axis base) + t
  __shared__ int OT[NTAB * NW];           // stencil start relative to the table's region
  __shared__ int GEO[2 * kMaxQ];          // per axis and velocity: region start rs | extent R << 16
  __shared__ int GTB[2 * kMaxQ];          // table id | identity flag << 30

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

  // weight rows and stencil offsets of every table of every axis, for this tile (read
  // by the passes of all velocities; the loop's first barrier publishes them)
  for (int r = tid; r < NTAB * NW; r += BS) {
    const int tb = r / NW, q0 = r % NW;
    const int ax = q0 < TX ? 0 : (q0 < TX + TY ? 1 : 2);
    const int t = q0 - (ax == 0 ? 0 : (ax == 1 ? TX : TX + TY));
    const int vt = ax == 0 ? vx : (ax == 1 ? vy : vz);
    const int n0a = ax == 0 ? n0x : (ax == 1 ? n0y : n0z);
    const int Ta = ax == 0 ? TX : (ax == 1 ? TY : TZ);
    const DevAxis &da = ax == 0 ? pl.ax[0] : (ax == 1 ? pl.ax[1] : pl.ax[2]);
    if (ax >= D || tb >= da.ntab || t >= vt) continue;
    const AxGeo g = axis_geo<P>(da, tb, n0a, vt, Ta);
    int off, len;
    T w[P + 1];
    axis_weights<T, P>(da, g, n0a, t, Ta, off, len, w);
#pragma unroll
    for (int j = 0; j <= P; j++) WT[r * (P + 1) + j] = w[j];
    OT[r] = off;
  }
  // the departure-region geometry of every velocity along x and y, once per tile
  for (int e = tid; e < 2 * Q; e += BS) {
    const int a = e / Q, i = e - a * Q;
    const int tb = pl.tab_reg[a * Q + i];
    const AxGeo g = a == 0 ? axis_geo<P>(pl.ax[0], tb, n0x, vx, TX) : axis_geo<P>(pl.ax[1], tb, n0y, vy, TY);
    GEO[a * kMaxQ + i] = (g.rs & 0xffff) | (g.R << 16);
    GTB[a * kMaxQ + i] = g.tb | (g.ident << 30);
  }
  __syncthreads();

  // staging elements of this thread: region coordinates, independent of the velocity
  // (packed 10 bits each: x | y << 10 | z << 20; x = RX marks no element)
  int epk[NST];
#pragma unroll
  for (int s = 0; s < NST; s++) {
    const int e = tid + BS * s;
    const int rx = e < SS ? e % RX : RX, ry = e < SS ? (e / RX) % RY : 0, rz = e < SS ? e / (RX * RY) : 0;
    epk[s] = rx | (ry << 10) | (rz << 20);
  }
  static_assert(RX < 1024 && RY < 1024 && RZ < 1024, "staging coordinates are packed in 10 bits");
  auto staged = [&](int s, const AxGeo (&g)[3]) __attribute__((always_inline)) -> bool {
    return (epk[s] & 1023) < g[0].R && ((epk[s] >> 10) & 1023) < g[1].R && (epk[s] >> 20) < g[2].R;
  };

  // ---- software pipeline: registers hold the departure region of the velocity after
  // the one in LDS.  The loads are issued by every lane (out-of-range offsets for lanes
  // without an element), so that the compiler counts the loads in flight exactly instead of
  // waiting for all of them at the next use of any.
  T pf[NST], pg[NST];
  AxGeo ng[3], cg[3];
  auto geo = [&](int a, int i) __attribute__((always_inline)) {
    AxGeo g;   // the same for the whole workgroup: held in scalar registers
    const int v = __builtin_amdgcn_readfirstlane(GEO[a * kMaxQ + i]);
    const int t = __builtin_amdgcn_readfirstlane(GTB[a * kMaxQ + i]);
    g.rs = (int)(short)(v & 0xffff);
    g.R = v >> 16;
    g.tb = t & 0x3fffffff;
    g.ident = t >> 30;
    return g;
  };
  // velocity i (i >= Q: nothing, every offset out of range)
  auto prefetch = [&](int i) __attribute__((always_inline)) {
    const bool real = i < Q;
    const int iv = real ? i : Q - 1;
    ng[0] = geo(0, iv);
    ng[1] = geo(1, iv);
    ng[2].tb = 0; ng[2].ident = 1; ng[2].rs = 0; ng[2].R = 1;
    const __amdgpu_buffer_rsrc_t rf = buf_rsrc(pin + (size_t)iv * N, N);
    const __amdgpu_buffer_rsrc_t rg = buf_rsrc(pin + ((size_t)Q + iv) * N, N);
    const int sx = n0x + ng[0].rs, sy = n0y + ng[1].rs;
#pragma unroll
    for (int s = 0; s < NST; s++) {
      const bool in = real && staged(s, ng);
      const int gxx = wrap_idx(sx + (epk[s] & 1023), Nx);
      const int gyy = wrap_idx(sy + ((epk[s] >> 10) & 1023), Ny);
      const int off = opaque_off(in ? (gxx + Nx * gyy) * (int)sizeof(T) : kBufOutOfRange);
      pf[s] = BufLoad<T>::get(rf, off);
      pg[s] = BufLoad<T>::get(rg, off);
    }
  };
  auto commit = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NST; s++) {
      if (staged(s, ng)) {
        const int e = tid + BS * s;
        S[e] = pf[s];
        S[SS + e] = pg[s];
      }
    }
    cg[0] = ng[0];
    cg[1] = ng[1];
    cg[2] = ng[2];
  };

  // x-pass: S[rz][ry][*] -> X[rz][ry][tx]; each thread keeps one tx (and its weights)
  // and walks the rows of the committed region
  auto xpass = [&](int off) __attribute__((always_inline)) {
    constexpr int NRX = BS / TX;          // rows in flight per sweep of the workgroup
    const int Ry = cg[1].R;   // one plane in 2D: the row counter is ry itself
    const int len = cg[0].ident ? 1 : P + 1;
    const int tx = tid % TX, r0 = tid / TX;
    if (r0 < NRX && tx < vx) {
      const int row = cg[0].tb * NW + tx;
      T w[P + 1];
#pragma unroll
      for (int j = 0; j <= P; j++) w[j] = WT[row * (P + 1) + j];
      constexpr int MR = (RY * RZ + NRX - 1) / NRX;   // rows per thread at most
#pragma unroll 4
      for (int q = 0; q < MR; q++) {
        const int rr = r0 + q * NRX;
        if (rr >= Ry) break;
        const T *sf = S + rr * RX + off;
        T a = 0, b = 0;
#pragma unroll
        for (int j = 0; j <= P; j++) {
          if (j >= len) break;
          a += w[j] * sf[j];
          b += w[j] * sf[SS + j];
        }
        const int l = rr * TX + tx;
        X[l] = a;
        X[XS + l] = b;
      }
    }
  };

  // y contraction for the owned nodes straight out of X
  auto ypass_nodes = [&](int tby, int leny, const int (&yo)[NPT], double (&fv)[NPT], double (&gv)[NPT])
                         __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      fv[m] = gv[m] = 0.0;
      if (!own[m]) continue;
      const int ry = tby * NW + TX + oty[m];
      const T *wy = WT + ry * (P + 1);
      const T *xr = X + yo[m] * TX + otx[m];
      T a = 0, b = 0;
#pragma unroll
      for (int jy = 0; jy <= P; jy++) {
        if (jy >= leny) break;
        a += wy[jy] * xr[jy * TX];
        b += wy[jy] * xr[XS + jy * TX];
      }
      fv[m] = scale * (double)a;
      gv[m] = scale * (double)b;
    }
  };

  double rho[NPT], j0[NPT], j1[NPT], j2[NPT], E[NPT];
#pragma unroll
  for (int m = 0; m < NPT; m++) rho[m] = j0[m] = j1[m] = j2[m] = E[m] = 0.0;
  // one velocity: x-pass, commit of the next one, y contraction, moments
  auto velocity = [&](int i, double (&fv)[NPT], double (&gv)[NPT]) __attribute__((always_inline)) {
    // the stencil starts of this thread's x-pass row and y-pass nodes (the tables are
    // constant): read before the barrier, they take an LDS round trip off each pass
    const int xo = OT[cg[0].tb * NW + tid % TX];
    int yo[NPT];
#pragma unroll
    for (int m = 0; m < NPT; m++) yo[m] = OT[cg[1].tb * NW + TX + oty[m]];
    __syncthreads();   // velocity i is in S; X is free
    xpass(xo);
    __syncthreads();   // X holds velocity i; S is free
    const int tby = cg[1].tb, leny = cg[1].ident ? 1 : P + 1;
    if (i + 1 < Q) commit();
    prefetch(i + 2);
    ypass_nodes(tby, leny, yo, fv, gv);
    // the velocity table is never written by the step: read through the scalar cache
    const double __attribute__((address_space(4))) *vi =
        (const double __attribute__((address_space(4))) *)(pl.vel + 8 * i);
    const double z2 = vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2];
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      rho[m] += fv[m];
      j0[m] += vi[0] * fv[m];
      j1[m] += vi[1] * fv[m];
      j2[m] += vi[2] * fv[m];
      E[m] += z2 * fv[m] + gv[m];
    }
  };
  // QR > 0 (Q = QR): the streamed values stay in registers and every owned node is
  // relaxed and stored at the end, a single pass over the populations; QR = 0: the
  // streamed values are stored and a second launch relaxes them
  constexpr int QL = QR > 0 ? QR : 1;
  T fs[NPT][QL], gs[NPT][QL];
  prefetch(0);
  commit();
  prefetch(1);
  if constexpr (QR > 0) {
#pragma unroll
    for (int i = 0; i < QR; i++) {
      double fv[NPT], gv[NPT];
      velocity(i, fv, gv);
#pragma unroll
      for (int m = 0; m < NPT; m++) {
        fs[m][i] = (T)fv[m];
        gs[m][i] = (T)gv[m];
      }
    }
  } else {
    for (int i = 0; i < Q; i++) {
      double fv[NPT], gv[NPT];
      velocity(i, fv, gv);
      const __amdgpu_buffer_rsrc_t of = buf_rsrc(pout + (size_t)i * N, N);
      const __amdgpu_buffer_rsrc_t og = buf_rsrc(pout + ((size_t)Q + i) * N, N);
#pragma unroll
      for (int m = 0; m < NPT; m++) {
        const int off = opaque_off(own[m] ? (int)node_index(m) * (int)sizeof(T) : kBufOutOfRange);
        BufStore<T>::put(of, off, (T)fv[m]);
        BufStore<T>::put(og, off, (T)gv[m]);
      }
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
    if constexpr (QR > 0) {
      // BGK relaxation and Kupershtokh forcing of the stored (rounded) streamed values,
      // as the relaxation launch does for the two-launch path
      if (sa.relax_mode == 2) {
#pragma unroll
        for (int i = 0; i < QR; i++) {
          pout[(size_t)i * N + k] = fs[m][i];
          pout[((size_t)QR + i) * N + k] = gs[m][i];
        }
        continue;
      }
      const EqNode e = eq_prepare(r, u0, u1, u2, Tn, sa, D);
      EqNode ef = e;
      if (sa.has_force) ef = eq_forced(r, u0, u1, u2, Tn, sa, D);
      const double gT = Tn * sa.gbase;
      PrTerm pt;
      if constexpr (PR) {  // Pr != 1
        HeatFlux hq = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < QR; i++) {
          double vi[8];
          vel_consts(pl.vel, i, vi);
          heat_flux_add(hq, vi, u0, u1, u2, (double)fs[m][i], (double)gs[m][i]);
        }
        pt = pr_term(hq, it, sa, D);
      }
#pragma unroll
      for (int i = 0; i < QR; i++) {
        double vi[8];
        vel_consts(pl.vel, i, vi);
        const double f = (double)fs[m][i], g = (double)gs[m][i];
        const double fe = eq_f(e, vi);
        double fo = f - (f - fe) * it;
        double go = g - (g - gT * fe) * it;
        if constexpr (PR) pr_add(pt, vi, fo, go);
        if (sa.has_force) {
          const double df = eq_f(ef, vi) - fe;
          fo += df;
          go += gT * df;
        }
        pout[(size_t)i * N + k] = (T)fo;
        pout[((size_t)QR + i) * N + k] = (T)go;
      }
    } else {
      nstate[k] = r;
      nstate[N + k] = u0;
      nstate[2 * N + k] = u1;
      nstate[3 * N + k] = u2;
      nstate[4 * N + k] = Tn;
      nstate[5 * N + k] = it;
    }
  }
}

// 3D: streams every velocity of one tile through LDS in three 1D passes (x, y, z) and
// stores the streamed f_i, g_i of the owned nodes and their node state (rho, u0, u1,
// u2, T, 1/tau_bar as [6][N] doubles).  Two schedules:
//  SK = 0: per velocity, barrier; commit velocity i from registers to LDS (with its weight
//    rows) and issue the loads of i+1; barrier; x-pass (S -> X); barrier; y-pass (X -> Y,
//    Y aliasing S); barrier; z contraction per owned node.  Four barriers per velocity.
//  SK = 1: the passes of consecutive velocities are skewed so that a velocity costs two
//    barriers: phase A contracts velocity i-1 along z (Y -> the owned nodes) and runs the
//    x-pass of velocity i; phase B runs the y-pass of i and commits velocity i+1 into S,
//    then issues the loads of i+2.  Every LDS buffer is written in one phase and read in
//    the other, so Y needs its own buffer and the weight rows are double-buffered (velocity
//    i's z rows are still read after i+1 is committed).
template <typename T, int D, int P, int CX, int CY, int CZ, int BS, int WPE, int SK>
__global__ void __launch_bounds__(BS, WPE) k_step_tile3d(const DevTensorPlan pl, const StepArgs sa, const TileGrid tg,
                                                    const T *__restrict__ pin, T *__restrict__ pout,
                                                    double *__restrict__ nstate) {
  static_assert(D == 3, "the 2D tiles have a kernel of their own");
  constexpr int TX = CX * P, TY = CY * P, TZ = CZ * P;
  constexpr int RX = TX + P + 1, RY = TY + P + 1, RZ = TZ + P + 1;
  constexpr int NT = TX * TY * TZ;
  constexpr int NPT = (NT + BS - 1) / BS;
  constexpr int SS = RZ * RY * RX;           // one population's staging size
  constexpr int XS = RZ * RY * TX;           // one population's x-pass output
  constexpr int YS = RZ * TY * TX;           // one population's y-pass output
  constexpr int NST = (SS + BS - 1) / BS;    // staged elements per thread and population
  constexpr int NW = TX + TY + TZ;           // weight rows: one per tile position and axis
  constexpr int WS = NW * (P + 1);
  static_assert(NW <= 64, "the weight rows are loaded by the first wave");
  static_assert(BS >= TX * TY, "tile cross-section exceeds the workgroup");
  constexpr int NB = SK ? 2 : 1;             // weight-row buffers
  __shared__ T S[2 * SS];
  __shared__ T X[2 * XS];
  __shared__ T Ys[SK ? 2 * YS : 1];
  __shared__ T WT[NB * WS];
  __shared__ int OT[NB * NW];
  __shared__ int GEO[3 * kMaxQ];             // per axis and velocity: region start rs | extent R << 16
  __shared__ int GTB[3 * kMaxQ];             // table id | identity flag << 30
  static_assert(SK || YS <= SS, "the y-pass output must fit the staging buffer it reuses");
  T *const Y = SK ? Ys : S;

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
  const int vx = min(TX, Nx - n0x), vy = min(TY, Ny - n0y), vz = min(TZ, Nz - n0z);

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
  // the departure-region geometry of every velocity along every axis, once per tile (a
  // chain of dependent table loads each; per velocity it is then an LDS read)
  for (int e = tid; e < 3 * Q; e += BS) {
    const int a = e / Q, i = e - a * Q;
    const int vt = sel3(a, vx, vy, vz), n0 = sel3(a, n0x, n0y, n0z), Ta = sel3(a, TX, TY, TZ);
    const int tb = pl.tab_reg[a * Q + i];
    AxGeo g;   // (one call per axis: a runtime index into the plan would copy it to scratch)
    if (a == 0) g = axis_geo<P>(pl.ax[0], tb, n0, vt, Ta);
    else if (a == 1) g = axis_geo<P>(pl.ax[1], tb, n0, vt, Ta);
    else g = axis_geo<P>(pl.ax[2], tb, n0, vt, Ta);
    GEO[a * kMaxQ + i] = (g.rs & 0xffff) | (g.R << 16);
    GTB[a * kMaxQ + i] = g.tb | (g.ident << 30);
  }
  __syncthreads();

  auto node_index = [&](int m) __attribute__((always_inline)) -> int64_t {
    return (int64_t)(n0x + otx[m]) + (int64_t)Nx * ((int64_t)(n0y + oty[m]) + (int64_t)Ny * (n0z + otz[m]));
  };
  // ---- software pipeline: the departure region of velocity i+2 is loaded into
  // registers while velocities i and i+1 are interpolated out of LDS.  The per-velocity
  // geometry comes from LDS (built once per tile), the weight rows are loaded by the first
  // wave without a divergent branch, every lane issues the stores of the streamed values
  // (out-of-range offsets for lanes without a node) and the velocity constants come through
  // the scalar cache: none of these makes the compiler wait for all memory accesses in
  // flight, which the per-velocity table loads and branchy stores used to do.
  T pf[NST], pg[NST];
  T pw[P + 1];
  int pst = 0;       // raw stencil start of this thread's weight row
#pragma unroll
  for (int s = 0; s < NST; s++) pf[s] = pg[s] = T(0);
#pragma unroll
  for (int j = 0; j <= P; j++) pw[j] = T(0);
  AxGeo ng[3], cg[3];
  auto geo = [&](int a, int i) __attribute__((always_inline)) {
    AxGeo g;   // the same for the whole workgroup: held in scalar registers
    const int v = __builtin_amdgcn_readfirstlane(GEO[a * kMaxQ + i]);
    const int t = __builtin_amdgcn_readfirstlane(GTB[a * kMaxQ + i]);
    g.rs = (int)(short)(v & 0xffff);
    g.R = v >> 16;
    g.tb = t & 0x3fffffff;
    g.ident = t >> 30;
    return g;
  };
  // velocity i's departure region and this thread's weight row (thread t < NW: row t, for
  // axis ax and tile position q); i >= Q loads nothing (every offset out of range)
  auto prefetch = [&](int i) __attribute__((always_inline)) {
    const bool real = i < Q;
    const int iv = real ? i : Q - 1;
    ng[0] = geo(0, iv);
    ng[1] = geo(1, iv);
    ng[2] = geo(2, iv);
    const T *F = pin + (size_t)iv * N, *G = pin + ((size_t)Q + iv) * N;
#pragma unroll
    for (int s = 0; s < NST; s++) {
      int e = tid + BS * s;
      int rx = e % RX, ry = (e / RX) % RY, rz = e / (RX * RY);
      const bool in = real && e < SS && rx < ng[0].R && ry < ng[1].R && rz < ng[2].R;
      const int gxx = wrap_idx(n0x + ng[0].rs + rx, Nx);
      const int gyy = wrap_idx(n0y + ng[1].rs + ry, Ny);
      const int gzz = wrap_idx(n0z + ng[2].rs + rz, Nz);
      // Conditional loads here (unlike the weight rows, stores and the 2D kernel): the
      // compiler then waits for them before the passes of the current velocity, which keeps
      // the workgroups of an XCD close in velocity, so that neighbouring tiles still find each
      // other's departure regions in L2.  Fully pipelined loads (every lane, out-of-range
      // offsets) drift the workgroups apart: on the 128 x 96 x 64 channel (D3V125, p = 2, FP32,
      // 8^3-node tiles) the launch then fetches 29 GB instead of 9 GB and takes 10.6 ms against
      // 8.3 ms, while the larger p = 3 tiles of the Taylor-Green vortex gain at most 2 %.
      if (in) {
        pf[s] = F[gxx + (size_t)Nx * (gyy + (size_t)Ny * gzz)];
        pg[s] = G[gxx + (size_t)Nx * (gyy + (size_t)Ny * gzz)];
      }
    }
    if (tid < 64) {   // the wave holding the NW row threads (a wave-uniform branch)
      const int tt = opaque_off(tid), t = tt < NW ? tt : 0;
      const int ax = t < TX ? 0 : (t < TX + TY ? 1 : 2);
      const int q = t - sel3(ax, 0, TX, TX + TY);
      const int n0a = sel3(ax, n0x, n0y, n0z), axN = sel3(ax, Nx, Ny, Nz);
      const int tb = sel3(ax, ng[0].tb, ng[1].tb, ng[2].tb);
      const int32_t *st = sel3(ax, pl.ax[0].start, pl.ax[1].start, pl.ax[2].start);
      const T *wt = sel3(ax, WeightSel<T>::get(pl.ax[0]), WeightSel<T>::get(pl.ax[1]), WeightSel<T>::get(pl.ax[2]));
      // positions past a partial tile read the axis's last row (their weights are not used)
      const int row = opaque_off(tb * axN + min(n0a + q, axN - 1));
      pst = st[row];
#pragma unroll
      for (int j = 0; j <= P; j++) pw[j] = wt[(size_t)row * (P + 1) + j];
    }
  };
  // the prefetched velocity into S and weight buffer wb (placeholder: offsets 0, so that the
  // passes over it stay inside the buffers)
  auto commit = [&](int wb, bool placeholder = false) __attribute__((always_inline)) {
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
      // (derived from an opaque copy of tid: recomputed here each velocity rather than held
      // across the loop, where the register budget would spill them and the reload would
      // wait on every access in flight)
      const int t = opaque_off(tid);
      const int ax = t < TX ? 0 : (t < TX + TY ? 1 : 2);
      const int q = t - sel3(ax, 0, TX, TX + TY);
      const int n0a = sel3(ax, n0x, n0y, n0z), axN = sel3(ax, Nx, Ny, Nz), Ta = sel3(ax, TX, TY, TZ);
      const int ident = sel3(ax, ng[0].ident, ng[1].ident, ng[2].ident);
      const int rs = sel3(ax, ng[0].rs, ng[1].rs, ng[2].rs);
#pragma unroll
      for (int j = 0; j <= P; j++) WT[wb * WS + t * (P + 1) + j] = ident ? T(j == 0 ? 1 : 0) : pw[j];
      OT[wb * NW + t] = placeholder ? 0 : (ident ? q : rel_start<P>(pst, n0a, axN, Ta) - rs);
    }
    cg[0] = ng[0];
    cg[1] = ng[1];
    cg[2] = ng[2];
  };
  // x-pass of the committed velocity: S[rz][ry][*] -> X[rz][ry][tx]; each thread keeps one
  // tx (and its weights) and walks the rows
  auto xpass = [&](int wb) __attribute__((always_inline)) {
    constexpr int NRX = BS / TX;          // rows in flight per sweep of the workgroup
    const int Ry = cg[1].R, Rz = cg[2].R;
    const int len = cg[0].ident ? 1 : P + 1;
    const int tx = tid % TX, r0 = tid / TX;
    if (r0 < NRX && tx < vx) {
      const int off = OT[wb * NW + tx];
      T w[P + 1];
#pragma unroll
      for (int j = 0; j <= P; j++) w[j] = WT[wb * WS + tx * (P + 1) + j];
      // rows rz RY + ry of the staging grid: the compile-time stride RY splits the counter
      // (a runtime divisor would cost an emulated division per row); rows beyond the
      // region's Ry are skipped
      const int nrows = RY * Rz;
#pragma unroll 1
      for (int rr = r0; rr < nrows; rr += NRX) {
        if (rr % RY >= Ry) continue;
        const T *sf = S + rr * RX + off;
        T a = 0, b = 0;
#pragma unroll
        for (int j = 0; j <= P; j++) {
          if (j >= len) break;
          a += w[j] * sf[j];
          b += w[j] * sf[SS + j];
        }
        const int l = rr * TX + tx;
        X[l] = a;
        X[XS + l] = b;
      }
    }
  };
  // y-pass: X[rz][*][tx] -> Y[rz][ty][tx]; each thread keeps one (tx, ty)
  auto ypass = [&](int wb) __attribute__((always_inline)) {
    constexpr int NRY = BS / (TX * TY);
    const int Rz = cg[2].R;
    const int len = cg[1].ident ? 1 : P + 1;
    const int tx = tid % TX, ty = (tid / TX) % TY, z0 = tid / (TX * TY);
    if (z0 < NRY && tx < vx && ty < vy) {
      const int off = OT[wb * NW + TX + ty];
      T w[P + 1];
#pragma unroll
      for (int j = 0; j <= P; j++) w[j] = WT[wb * WS + (TX + ty) * (P + 1) + j];
#pragma unroll 1
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
        Y[l] = a;
        Y[YS + l] = b;
      }
    }
  };
  // z contraction for the owned nodes, with the weight buffer and row length of the
  // velocity the y-pass left in Y
  auto zpass = [&](int wb, int len, double (&fv)[NPT], double (&gv)[NPT]) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      fv[m] = gv[m] = 0.0;
      if (!own[m]) continue;
      const T *yf = Y + (OT[wb * NW + TX + TY + otz[m]] * TY + oty[m]) * TX + otx[m];
      const T *w = WT + wb * WS + (TX + TY + otz[m]) * (P + 1);
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
  };

  double rho[NPT], j0[NPT], j1[NPT], j2[NPT], E[NPT];
#pragma unroll
  for (int m = 0; m < NPT; m++) rho[m] = j0[m] = j1[m] = j2[m] = E[m] = 0.0;
  // store the streamed values of velocity i and add them to the moments
  // (i < 0: a placeholder velocity, every store out of range and no moments)
  auto accumulate = [&](int i, const double (&fv)[NPT], const double (&gv)[NPT]) __attribute__((always_inline)) {
    const int iv = i < 0 ? 0 : i;
    // the velocity table is never written by the step: read through the scalar cache, so
    // that these loads do not join the vector-memory counter the prefetch waits on
    const double __attribute__((address_space(4))) *vi =
        (const double __attribute__((address_space(4))) *)(pl.vel + 8 * iv);
    const double z2 = vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2];
    const __amdgpu_buffer_rsrc_t of = buf_rsrc(pout + (size_t)iv * N, N);
    const __amdgpu_buffer_rsrc_t og = buf_rsrc(pout + ((size_t)Q + iv) * N, N);
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      const int off = opaque_off(own[m] && i >= 0 ? (int)node_index(m) * (int)sizeof(T) : kBufOutOfRange);
      BufStore<T>::put(of, off, (T)fv[m]);
      BufStore<T>::put(og, off, (T)gv[m]);
    }
    if (i < 0) return;
#pragma unroll
    for (int m = 0; m < NPT; m++) {
      rho[m] += fv[m];
      j0[m] += vi[0] * fv[m];
      j1[m] += vi[1] * fv[m];
      j2[m] += vi[2] * fv[m];
      E[m] += z2 * fv[m] + gv[m];
    }
  };

  if constexpr (!SK) {
    // iteration -1 only issues the loads of velocity 0: its commit, passes and stores run on
    // placeholder values (a valid geometry, offsets 0, every store out of range), so that every
    // iteration issues the same memory operations in the same order and the compiler's
    // counts of those in flight stay exact around the loop
    ng[0] = geo(0, 0);
    ng[1] = geo(1, 0);
    ng[2] = geo(2, 0);
    for (int i = -1; i < Q; i++) {
      __syncthreads();  // everyone is done reading the previous velocity out of LDS
      commit(0, i < 0);
      prefetch(i + 1);
      __syncthreads();
      xpass(0);
      __syncthreads();
      ypass(0);
      __syncthreads();
      double fv[NPT], gv[NPT];
      zpass(0, cg[2].ident ? 1 : P + 1, fv, gv);
      accumulate(i, fv, gv);
    }
  } else {
  prefetch(0);
  commit(0);
  prefetch(1);
  __syncthreads();
  int zlen = 0;
  for (int i = 0; i < Q; i++) {
    const int wb = i & 1;
    // phase A: z of velocity i-1, x of velocity i (at i = 0 a placeholder with no rows and
    // every store out of range, so that each iteration issues the same memory operations)
    {
      double fv[NPT], gv[NPT];
      zpass(wb ^ 1, zlen, fv, gv);
      accumulate(i - 1, fv, gv);
    }
    xpass(wb);
    __syncthreads();
    // phase B: y of velocity i, commit of velocity i+1, loads of i+2
    ypass(wb);
    zlen = cg[2].ident ? 1 : P + 1;
    if (i + 1 < Q) commit(wb ^ 1);
    prefetch(i + 2);
    __syncthreads();
  }
  {
    double fv[NPT], gv[NPT];
    zpass((Q - 1) & 1, zlen, fv, gv);
    accumulate(Q - 1, fv, gv);
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
}

// In-place BGK relaxation and forcing of the streamed populations the moments launch
// stored, V adjacent nodes per lane (their equilibrium coefficients built once; V = 2 turns
// every population access into one vector load or store of V elements when N is even);
// nodes in the boundary layers of a bounded face belong to the gather kernel and are left
// as they are.
template <typename T, int V> struct VecOf;
template <typename T> struct VecOf<T, 1> { typedef T type; };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };

template <typename T, int D, int V, int PR>
__global__ void __launch_bounds__(kBlock) k_relax_nodes(const DevTensorPlan pl, const StepArgs sa,
                                                        T *__restrict__ pop, const double *__restrict__ nstate) {
  typedef typename VecOf<T, V>::type VT;
  const int64_t N = pl.N;
  const int64_t k0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * V;
  if (k0 >= N) return;
  if (sa.relax_mode == 2) return;   // pure streaming: the stored values are final
  const int Nx = pl.ax[0].N, Ny = pl.ax[1].N;
  bool act[V];
  EqNode e[V], ef[V];
  double itau[V], gT[V];
#pragma unroll
  for (int v = 0; v < V; v++) {
    const int64_t k = k0 + v;
    act[v] = k < N;
    for (int fc = 0; fc < pl.nfaces; fc++) {
      const DevFace &F = pl.face[fc];
      int64_t n3 = F.axis == 0 ? k % Nx : (F.axis == 1 ? (k / Nx) % Ny : k / ((int64_t)Nx * Ny));
      int64_t l = F.side == 0 ? n3 : pl.ax[F.axis].N - 1 - n3;
      if (l < F.depth) act[v] = false;
    }
    const int64_t kk = act[v] ? k : k0;
    const double rho = nstate[kk], u0 = nstate[N + kk], u1 = nstate[2 * N + kk], u2 = nstate[3 * N + kk];
    const double Tn = nstate[4 * N + kk];
    itau[v] = nstate[5 * N + kk];
    e[v] = eq_prepare(rho, u0, u1, u2, Tn, sa, D);
    ef[v] = e[v];
    if (sa.has_force) ef[v] = eq_forced(rho, u0, u1, u2, Tn, sa, D);
    gT[v] = Tn * sa.gbase;
  }
  bool any = false;
#pragma unroll
  for (int v = 0; v < V; v++) any = any || act[v];
  if (!any) return;   // all in a boundary layer (or past N): nothing to read or write
  const int Q = pl.Q;
  PrTerm pt[V];
  if constexpr (PR) {  // Pr != 1: a first pass over the populations for the heat flux
    HeatFlux hq[V];
    double uu[V][3];
#pragma unroll
    for (int v = 0; v < V; v++) {
      hq[v] = {0, 0, 0, 0, 0, 0};
      const int64_t kk = act[v] ? k0 + v : k0;
      uu[v][0] = nstate[N + kk];
      uu[v][1] = nstate[2 * N + kk];
      uu[v][2] = nstate[3 * N + kk];
    }
    for (int i = 0; i < Q; i++) {
      double vi[8];
      vel_consts(pl.vel, i, vi);
      VT fvec = *(const VT *)(pop + (size_t)i * N + k0), gvec = *(const VT *)(pop + ((size_t)Q + i) * N + k0);
#pragma unroll
      for (int v = 0; v < V; v++)
        if (act[v]) heat_flux_add(hq[v], vi, uu[v][0], uu[v][1], uu[v][2], (double)((T *)&fvec)[v], (double)((T *)&gvec)[v]);
    }
#pragma unroll
    for (int v = 0; v < V; v++) pt[v] = pr_term(hq[v], itau[v], sa, D);
  }
  for (int i = 0; i < Q; i++) {
    double vi[8];
    vel_consts(pl.vel, i, vi);
    VT *pf = (VT *)(pop + (size_t)i * N + k0);
    VT *pg = (VT *)(pop + ((size_t)Q + i) * N + k0);
    VT fvec = *pf, gvec = *pg;
#pragma unroll
    for (int v = 0; v < V; v++) {
      if (!act[v]) continue;
      T &fr = ((T *)&fvec)[v];
      T &gr = ((T *)&gvec)[v];
      const double f = (double)fr, g = (double)gr;
      const double fe = eq_f(e[v], vi);
      double fo = f - (f - fe) * itau[v];
      double go = g - (g - gT[v] * fe) * itau[v];
      if constexpr (PR) pr_add(pt[v], vi, fo, go);
      if (sa.has_force) {
        const double df = eq_f(ef[v], vi) - fe;
        fo += df;
        go += gT[v] * df;
      }
      fr = (T)fo;
      gr = (T)go;
    }
    *pf = fvec;
    *pg = gvec;
  }
}

// ------------------------------------------------------ velocity-split 3D step
// A second schedule of the 3D step for plans whose node's 2Q streamed values fit in a lane's
// registers (D3Q45): velocities are independent until the relaxation, so the streaming
// launch takes one velocity per workgroup, on a column of output nodes (an x-y tile of
// TX x TY nodes and a chunk of consecutive z planes).  The workgroup walks the departure
// region's source planes along z once each: per plane it stages the x-y departure region
// into LDS, contracts it along x (LDS) and along y (into a register per owned column), and
// keeps the last L y-contracted planes of its column in registers; each output plane is
// emitted from that window a fixed number of planes D after its own index (D set per
// workgroup so that every stencil plane has arrived), so that every iteration issues the
// same loads and stores.  The stored streamed values are then relaxed by a launch that
// reads a node's 2Q values into the registers of a few waves, forms the moments and relaxes
// them: the step reads and writes each population twice, with no node-state array and no
// re-staging of a departure region per velocity and tile.
//
// Along x and y the tile is cell-aligned (48 x 12 nodes at p = 2, 3, 4); along z a chunk of
// whole cells.  The separable contraction (x, then y, then z, each in the order of its
// stencil) is the tiled kernel's: the streamed values are the same numbers.

struct ColGrid {
  int nt0, nt1;   // x-y tiles
  int ox, oy;     // the first tile's origin (a cell boundary; 0 unless a bounded face's layers come first)
  int ex, ey;     // the tiles cover the nodes below these
  int zc;         // output planes per z chunk (whole cells)
  int nzc;        // chunks along z
  int q, r;       // work items (tiles x chunks x velocities) = 8 q + r (XCD remap)
};

template <typename T, int P, int CPT, int PD, int BS, int WPE>
__global__ void __launch_bounds__(BS, WPE) k_stream_col3d(const DevTensorPlan pl, const StepArgs sa, const ColGrid cg,
                                                          const T *__restrict__ pin, T *__restrict__ pout) {
  // CPT output columns per thread, TY / CPT rows apart
  constexpr int TX = ColShape<P>::CX * P, TY = CPT * ColShape<P>::CY * P, TYC = TY / CPT;
  constexpr int RX = TX + P + 1, RY = TY + P + 1;
  constexpr int SST = RX + COL_PADS;         // LDS row strides of the staged and x-pass planes
  constexpr int XST = TX + COL_PADX;
  constexpr int SS = SST * RY;               // staged elements per plane and population (LDS)
  constexpr int NSE = RX * RY;               // staged elements per plane and population
  constexpr int NST = (NSE + BS - 1) / BS;
  constexpr int XS = RY * XST;              // x-pass outputs per plane and population (LDS)
  constexpr int NXO = RY * TX;               // x-pass outputs per plane and population
  constexpr int NXI = (NXO + BS - 1) / BS;
  constexpr int L = kColWin<P>;             // z window (planes held per column)
  constexpr int ZM = kColZMax;
  static_assert(BS >= TX * TYC, "CPT output columns per thread");
  static_assert(BS >= TX + TY + ZM, "the set-up threads");
  static_assert(PD % 2 == 0, "even prefetch distance: the buffers of step r + d are d % 2");
  __shared__ T S[2 * 2 * SS];                // the staged plane of f and g (two buffers)
  __shared__ T X[2 * 2 * XS];                // its x-pass output (two buffers)
  __shared__ T WX[TX * (P + 1)], WY[TY * (P + 1)];
  __shared__ int OX[TX], OY[TY];
  __shared__ T WZ[ZM * L];
  __shared__ int EMZ[ZM];

  const int tid = threadIdx.x;
  const int Q = pl.Q;
  const int64_t N = pl.N;
  const int Nx = pl.ax[0].N, Ny = pl.ax[1].N, Nz = pl.ax[2].N;
  // XCD-aware work item: each XCD takes a contiguous range, whose consecutive items are
  // the neighbouring x-y tiles of one (velocity, z chunk): their departure regions overlap
  // and meet in that XCD's L2
  const int bid = blockIdx.x;
  const int xcd = bid & 7, jj = bid >> 3;
  const int item = xcd * cg.q + min(xcd, cg.r) + jj;
  const int ntl = cg.nt0 * cg.nt1;
  const int tl = item % ntl;
  const int rest = item / ntl;
  const int zch = rest % cg.nzc;
  const int i = rest / cg.nzc;
  const int x0 = cg.ox + (tl % cg.nt0) * TX, y0 = cg.oy + (tl / cg.nt0) * TY, z0 = zch * cg.zc;
  const int vx = min(TX, cg.ex - x0), vy = min(TY, cg.ey - y0), vz = min(cg.zc, Nz - z0);
  const AxGeo gx = axis_geo<P>(pl.ax[0], pl.tab_reg[i], x0, vx, TX);
  const AxGeo gy = axis_geo<P>(pl.ax[1], pl.tab_reg[Q + i], y0, vy, TY);
  const AxGeo gz = axis_geo<P>(pl.ax[2], pl.tab_reg[2 * Q + i], z0, vz, cg.zc);

  // weight rows: x (threads 0..TX-1), y (next TY), z (next ZM); positions past a partial
  // tile take the last row (their outputs are never stored)
  int zsr = 0, zlen = 1;
  T wzr[P + 1];
#pragma unroll
  for (int j = 0; j <= P; j++) wzr[j] = T(0);
  if (tid < TX) {
    int off, len;
    T w[P + 1];
    axis_weights<T, P>(pl.ax[0], gx, x0, min(tid, vx - 1), TX, off, len, w);
    OX[tid] = gx.ident ? tid : off;
#pragma unroll
    for (int j = 0; j <= P; j++) WX[tid * (P + 1) + j] = w[j];
  } else if (tid < TX + TY) {
    const int t = tid - TX;
    int off, len;
    T w[P + 1];
    axis_weights<T, P>(pl.ax[1], gy, y0, min(t, vy - 1), TY, off, len, w);
    OY[t] = gy.ident ? t : off;
#pragma unroll
    for (int j = 0; j <= P; j++) WY[t * (P + 1) + j] = w[j];
  } else if (tid < TX + TY + ZM) {
    const int oz = tid - TX - TY;
    int off;
    axis_weights<T, P>(pl.ax[2], gz, z0, min(oz, vz - 1), cg.zc, off, zlen, wzr);
    zsr = gz.ident ? oz : off;
    EMZ[oz] = oz < vz ? zsr + zlen - 1 - oz : 0;
  }
  __syncthreads();
  // D: the largest lag between an output plane and the last plane of its stencil
  int Dz = 0;
  for (int oz = 0; oz < vz; oz++) Dz = max(Dz, EMZ[oz]);
  Dz = __builtin_amdgcn_readfirstlane(Dz);
  if (tid >= TX + TY && tid < TX + TY + ZM) {
    // at the emission of plane oz (after source plane oz + Dz), window slot s holds source
    // plane oz + Dz - (L - 1 - s): stencil plane zsr + j sits in slot L - 1 - lag + j
    const int oz = tid - TX - TY;
    const int lag = oz + Dz - zsr;
#pragma unroll
    for (int s = 0; s < L; s++) {
      const int j = s - (L - 1 - lag);
      T w = T(0);
#pragma unroll
      for (int jj2 = 0; jj2 <= P; jj2++)
        if (jj2 == j && jj2 < zlen) w = wzr[jj2];
      WZ[oz * L + s] = w;
    }
  }
  __syncthreads();

  const double scale = sa.scale ? *sa.scale : 1.0;
  const __amdgpu_buffer_rsrc_t rf = buf_rsrc(pin + (size_t)i * N, N);
  const __amdgpu_buffer_rsrc_t rg = buf_rsrc(pin + ((size_t)Q + i) * N, N);
  const __amdgpu_buffer_rsrc_t wf = buf_rsrc(pout + (size_t)i * N, N);
  const __amdgpu_buffer_rsrc_t wg = buf_rsrc(pout + ((size_t)Q + i) * N, N);
  const int plane = Nx * Ny * (int)sizeof(T);   // bytes per z plane (a population holds < 2^31 bytes)
  // this thread's staged elements: their x-y byte offset within a plane (or none) and
  // their place in the LDS plane (-1: none)
  int xyo[NST], sidx[NST];
#pragma unroll
  for (int s = 0; s < NST; s++) {
    const int e = tid + BS * s;
    const int rx = e % RX, ry = e / RX;
    const bool in = e < NSE && rx < gx.R && ry < gy.R;
    const int gxx = wrap_idx(x0 + gx.rs + rx, Nx), gyy = wrap_idx(y0 + gy.rs + ry, Ny);
    xyo[s] = in ? (gxx + Nx * gyy) * (int)sizeof(T) : -1;
    sidx[s] = e < NSE ? ry * SST + rx : -1;
  }
  // this thread's output columns and their y weights
  const int cx = tid % TX, cyb = tid / TX;
  bool colv[CPT];
  int oyc[CPT], colb[CPT];
  T wy[CPT][P + 1];
#pragma unroll
  for (int c = 0; c < CPT; c++) {
    const int cy = cyb + c * TYC;
    colv[c] = tid < TX * TYC && cx < vx && cy < vy;
    // columns in the boundary layers of a bounded face (x or y) belong to the gather kernel
    for (int fc = 0; fc < pl.nfaces; fc++) {
      const DevFace &F = pl.face[fc];
      const int n3 = F.axis == 0 ? x0 + cx : y0 + cy;
      const int l = F.side == 0 ? n3 : (F.axis == 0 ? Nx : Ny) - 1 - n3;
      if (l < F.depth) colv[c] = false;
    }
    const int ccy = min(cy, TY - 1);
    oyc[c] = OY[ccy];
#pragma unroll
    for (int j = 0; j <= P; j++) wy[c][j] = WY[ccy * (P + 1) + j];
    colb[c] = colv[c] ? (x0 + cx + Nx * (y0 + cy)) * (int)sizeof(T) : 0;
  }
  const int lenx = gx.ident ? 1 : P + 1, leny = gy.ident ? 1 : P + 1;
  // this thread's x-pass position is the same in every sweep (BS is a multiple of TX): its
  // stencil start and weights stay in registers, off the LDS path between the barriers
  static_assert(BS % TX == 0, "one x-pass position per thread");
  const int xt = tid % TX;
  const int oxt = OX[xt];
  T wxt[P + 1];
#pragma unroll
  for (int j = 0; j <= P; j++) wxt[j] = WX[xt * (P + 1) + j];

  // source plane r of the region into registers (r past the region: every offset out of
  // range, the loads return 0)
  auto load_plane = [&](int r, T (&af)[NST], T (&ag)[NST]) __attribute__((always_inline)) {
    const bool real = r < gz.R;
    const int zo = wrap_idx(z0 + gz.rs + min(r, gz.R - 1), Nz) * plane;
#pragma unroll
    for (int s = 0; s < NST; s++) {
      const int off = opaque_off(real && xyo[s] >= 0 ? xyo[s] + zo : kBufOutOfRange);
      af[s] = BufLoad<T>::get(rf, off);
      ag[s] = BufLoad<T>::get(rg, off);
    }
  };
  T zf[CPT][L], zg[CPT][L];
#pragma unroll
  for (int c = 0; c < CPT; c++)
#pragma unroll
    for (int s = 0; s < L; s++) zf[c][s] = zg[c][s] = T(0);
  // one source plane r, one barrier: its staged values (loaded PD planes earlier) into S
  // buffer b, the loads of plane r + PD into the same registers; after the barrier the x-pass
  // of plane r (S_b -> X_b) beside the y-pass of plane r - 1 (X_{1-b}), the window shift and
  // the emission of output plane r - 1 - D (out of range when there is none).  A buffer is
  // written again two planes later, after a barrier that every reader of it has passed.
  // (Against two barriers per plane over single buffers: TGV 96^3 FP64 0.351 -> 0.343 ms per
  // launch on D3Q45, 0.848 -> 0.828 on D3V125; FP32 0.220 -> 0.217 / 0.501 -> 0.489 ms.)
  auto step = [&](int r, int b, T (&af)[NST], T (&ag)[NST]) __attribute__((always_inline)) {
    T *const Sb = S + 2 * SS * b;
    T *const Xw = X + 2 * XS * b;               // this plane's x-pass output
    const T *const Xr = X + 2 * XS * (1 - b);   // the previous plane's, read by the y-pass
#pragma unroll
    for (int s = 0; s < NST; s++) {
      if (sidx[s] >= 0) {
        Sb[sidx[s]] = af[s];
        Sb[SS + sidx[s]] = ag[s];
      }
    }
    load_plane(r + PD, af, ag);
    __syncthreads();
    const int Ry = gy.R;
#pragma unroll
    for (int n = 0; n < NXI; n++) {
      const int it = tid + BS * n;
      const int ry = it / TX;
      if (it < NXO && ry < Ry && xt < vx) {
        const T *sf = Sb + ry * SST + oxt;
        T a = 0, c2 = 0;
#pragma unroll
        for (int j = 0; j <= P; j++) {
          if (j >= lenx) break;
          a += wxt[j] * sf[j];
          c2 += wxt[j] * sf[SS + j];
        }
        Xw[ry * XST + xt] = a;
        Xw[XS + ry * XST + xt] = c2;
      }
    }
    // (every column reads rows of X inside the plane, valid or not, and a column without a
    // node discards its result: no divergent branch around these reads)
#pragma unroll
    for (int c = 0; c < CPT; c++) {
      T a = 0, c2 = 0;
      const T *xf = Xr + oyc[c] * XST + cx;
#pragma unroll
      for (int j = 0; j <= P; j++) {
        if (j >= leny) break;
        a += wy[c][j] * xf[j * XST];
        c2 += wy[c][j] * xf[XS + j * XST];
      }
#pragma unroll
      for (int s = 0; s + 1 < L; s++) {
        zf[c][s] = zf[c][s + 1];
        zg[c][s] = zg[c][s + 1];
      }
      zf[c][L - 1] = a;
      zg[c][L - 1] = c2;
    }
    const int k = r - 1 - Dz;            // the y-pass was of plane r - 1 (k < 0: placeholders)
    const bool kv = k >= 0 && k < vz;
    const T *wz = WZ + min(max(k, 0), ZM - 1) * L;
    T of[CPT], og[CPT];
#pragma unroll
    for (int c = 0; c < CPT; c++) of[c] = og[c] = T(0);
#pragma unroll
    for (int s = 0; s < L; s++) {
      const T w = wz[s];
#pragma unroll
      for (int c = 0; c < CPT; c++) {
        of[c] += w * zf[c][s];
        og[c] += w * zg[c][s];
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; c++) {
      const int off = opaque_off(colv[c] && kv ? colb[c] + (z0 + k) * plane : kBufOutOfRange);
      BufStore<T>::put(wf, off, (T)(scale * (double)of[c]));
      BufStore<T>::put(wg, off, (T)(scale * (double)og[c]));
    }
  };

  // planes -PD .. -1 are placeholders that only issue the loads of planes 0 .. PD-1 (their
  // values are zeros, like the window's planes before 0, and they emit nothing), so that
  // every load is issued inside the loop in the same order: the compiler then waits for a
  // plane's loads only, not for those of the planes after it
  T pf[PD][NST], pg[PD][NST];
#pragma unroll
  for (int d = 0; d < PD; d++)
#pragma unroll
    for (int s = 0; s < NST; s++) pf[d][s] = pg[d][s] = T(0);
  // the previous plane's x-pass output of the first step: zeros, like the window's planes
  // before 0 (the first barrier orders these writes before the reads)
  for (int e = tid; e < 2 * 2 * XS; e += BS) X[e] = T(0);
  // source planes to walk, plus one for the y-pass of the last (the last ones placeholders)
  const int nr = max(gz.R, Dz + vz) + 1;
  for (int r = -PD; r < nr; r += PD) {
#pragma unroll
    for (int d = 0; d < PD; d++) step(r + d, d % 2, pf[d], pg[d]);
  }
}

// The moments and the relaxation of the velocity-split step, in place: a workgroup of NPART
// waves on 64 nodes, wave p holding the streamed values of velocities p QP .. p QP + QP - 1 of
// them in registers (so that the velocity index stays uniform in a wave: the constants
// through the scalar cache, the loads coalesced over the 64 nodes); the moment sums and the
// heat flux of the parts are exchanged through LDS and added in part order, then each wave
// relaxes its velocities (BGK, the Prandtl term and Kupershtokh forcing as in k_relax_nodes).
// The sums are the tiled kernel's terms, added in another order (equal to rounding).  Nodes
// in the boundary layers of a bounded face are left as the gather kernel stored them.
// STATE = 1: no relaxation; the node state (rho, u, T, 1/tau_bar as [6][N] doubles) of the
// nodes outside the boundary layers is stored instead, for a relaxation that the learned
// correction does in its own pass.
template <typename T, int QQ, int NPART, int PR, int STATE>
__global__ void __launch_bounds__(64 * NPART, 2) k_relax_moments(const DevTensorPlan pl, const StepArgs sa,
                                                                        T *__restrict__ pop, double *__restrict__ nstate) {
  constexpr int QP = (QQ + NPART - 1) / NPART;   // velocities per wave
  __shared__ double MS[NPART][6][64];             // each part's sums (5 moments; 6 heat-flux terms)
  if (!STATE && sa.relax_mode == 2) return;   // pure streaming: the stored values are final
  const int64_t N = pl.N;
  const int lane = threadIdx.x & 63;
  const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  const int64_t kc = k < N ? k : N - 1;
  const int i0 = part * QP;
  T fs[QP], gs[QP];
#pragma unroll
  for (int j = 0; j < QP; j++) {
    const int ic = min(i0 + j, QQ - 1);
    fs[j] = pop[(size_t)ic * N + kc];
    gs[j] = pop[((size_t)QQ + ic) * N + kc];
  }
  double rho = 0, j0 = 0, j1 = 0, j2 = 0, E = 0;
#pragma unroll
  for (int j = 0; j < QP; j++) {
    if (i0 + j >= QQ) break;   // (uniform: the last part holds fewer velocities)
    double vi[8];
    vel_consts(pl.vel, i0 + j, vi);
    asm volatile("" : "+s"(vi[0]), "+s"(vi[1]), "+s"(vi[2]) : "v"(fs[j]), "v"(gs[j]));
    const double z2 = vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2];
    const double fv = (double)fs[j], gv = (double)gs[j];
    rho += fv;
    j0 += vi[0] * fv;
    j1 += vi[1] * fv;
    j2 += vi[2] * fv;
    E += z2 * fv + gv;
  }
#pragma unroll
  for (int i = 0; i < QP; i++) asm volatile("" : "+v"(fs[i]), "+v"(gs[i]));
  MS[part][0][lane] = rho;
  MS[part][1][lane] = j0;
  MS[part][2][lane] = j1;
  MS[part][3][lane] = j2;
  MS[part][4][lane] = E;
  __syncthreads();
  rho = j0 = j1 = j2 = E = 0;
#pragma unroll
  for (int q = 0; q < NPART; q++) {
    rho += MS[q][0][lane];
    j0 += MS[q][1][lane];
    j1 += MS[q][2][lane];
    j2 += MS[q][3][lane];
    E += MS[q][4][lane];
  }
  const double r = rho;
  const double u0 = j0 / r, u1 = j1 / r, u2 = j2 / r;
  const double Tn = (E - r * (u0 * u0 + u1 * u1 + u2 * u2)) / (2.0 * r * sa.cv);
  double it = 0.0;
  if (sa.relax_mode == 0) it = 1.0 / sa.tau_bar;
  if (sa.relax_mode == 1) {
    const double mu = sa.mu_ref * pow(Tn / sa.T_ref, sa.mu_exp);
    it = 1.0 / (mu / (r * Tn * sa.dt) + 0.5);
  }
  // nodes in the boundary layers of a bounded face (x or y) were relaxed by the gather kernel
  bool act = k < N;
  if (pl.nfaces > 0) {
    const int Nx = pl.ax[0].N, Ny = pl.ax[1].N, k32 = (int)kc;
    for (int fc = 0; fc < pl.nfaces; fc++) {
      const DevFace &F = pl.face[fc];
      const int n3 = F.axis == 0 ? k32 % Nx : (k32 / Nx) % Ny;
      const int l = F.side == 0 ? n3 : (F.axis == 0 ? Nx : Ny) - 1 - n3;
      if (l < F.depth) act = false;
    }
  }
  if constexpr (STATE) {
    if (part == 0 && act) {
      nstate[k] = r;
      nstate[N + k] = u0;
      nstate[2 * N + k] = u1;
      nstate[3 * N + k] = u2;
      nstate[4 * N + k] = Tn;
      nstate[5 * N + k] = it;
    }
    return;
  }
  const EqNode e = eq_prepare(r, u0, u1, u2, Tn, sa, 3);
  EqNode ef = e;
  if (sa.has_force) ef = eq_forced(r, u0, u1, u2, Tn, sa, 3);
  const double gT = Tn * sa.gbase;
  PrTerm pt;
  if constexpr (PR) {   // Pr != 1
    HeatFlux hq = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < QP; j++) {
      if (i0 + j >= QQ) break;
      double vi[8];
      vel_consts(pl.vel, i0 + j, vi);
      heat_flux_add(hq, vi, u0, u1, u2, (double)fs[j], (double)gs[j]);
    }
    __syncthreads();   // every part has read the moment sums
    MS[part][0][lane] = hq.f0;
    MS[part][1][lane] = hq.f1;
    MS[part][2][lane] = hq.f2;
    MS[part][3][lane] = hq.g0;
    MS[part][4][lane] = hq.g1;
    MS[part][5][lane] = hq.g2;
    __syncthreads();
    hq = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < NPART; q++) {
      hq.f0 += MS[q][0][lane];
      hq.f1 += MS[q][1][lane];
      hq.f2 += MS[q][2][lane];
      hq.g0 += MS[q][3][lane];
      hq.g1 += MS[q][4][lane];
      hq.g2 += MS[q][5][lane];
    }
    pt = pr_term(hq, it, sa, 3);
  }
  const int off = opaque_off(act ? (int)k * (int)sizeof(T) : kBufOutOfRange);
#pragma unroll
  for (int j = 0; j < QP; j++) {
    const int i = i0 + j;
    if (i >= QQ) break;
    double vi[8];
    vel_consts(pl.vel, i, vi);
    const double f = (double)fs[j], g = (double)gs[j];
    const double fe = eq_f(e, vi);
    double fo = f - (f - fe) * it;
    double go = g - (g - gT * fe) * it;
    if constexpr (PR) pr_add(pt, vi, fo, go);
    if (sa.has_force) {
      const double df = eq_f(ef, vi) - fe;
      fo += df;
      go += gT * df;
    }
    BufStore<T>::put(buf_rsrc(pop + (size_t)i * N, N), off, (T)fo);
    BufStore<T>::put(buf_rsrc(pop + ((size_t)QQ + i) * N, N), off, (T)go);
  }
}

// ------------------------------------------------------------------ launcher

namespace {
// single pass: the 2Q streamed values of a node stay in registers (3 waves per SIMD);
// PR = 1 instantiates the Prandtl-number term
template <typename T, int P, int CX, int CY, int BS, int QR, int NTAB>
void launch_tile2d_single(const DevTensorPlan &tp, const StepArgs &a, const TileGrid &tg, int ntiles, const void *pin,
                          void *pout, double *nstate, hipStream_t s) {
  constexpr int WPES = 3;
  if (a.pr_on)
    hipLaunchKernelGGL((k_step_tile2d<T, 2, P, CX, CY, 1, BS, WPES, QR, 1, NTAB>), dim3(ntiles), dim3(BS), 0, s, tp, a,
                       tg, (const T *)pin, (T *)pout, nstate);
  else
    hipLaunchKernelGGL((k_step_tile2d<T, 2, P, CX, CY, 1, BS, WPES, QR, 0, NTAB>), dim3(ntiles), dim3(BS), 0, s, tp, a,
                       tg, (const T *)pin, (T *)pout, nstate);
}

// velocity-split 3D step: the streaming launch (one velocity per workgroup, 576 threads: one
// output column each, two in FP32), then the moments and the relaxation
template <typename T, int P, int CPT>
int launch_col_t(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s, bool relax) {
  // a column per thread (FP64, and FP32 on meshes too short in y for two), 5 waves per SIMD:
  // two workgroups per compute unit (at p = 4 that bound spills: 4 waves, one workgroup)
  constexpr int TX = ColShape<P>::CX * P, TY = CPT * ColShape<P>::CY * P;
  constexpr int BS = (TX * TY / CPT + 63) / 64 * 64;
  constexpr int WPE = P == 4 ? 4 : (sizeof(T) == 8 ? COL_WPE64 : COL_WPE32);
  constexpr int PD = sizeof(T) == 8 ? COL_PD64 : COL_PD32;   // planes loaded ahead
  const DevTensorPlan &tp = Pl->tp;
  ColGrid cg;
  cg.ox = Pl->col_org[0];
  cg.oy = Pl->col_org[1];
  cg.ex = Pl->col_end[0];
  cg.ey = Pl->col_end[1];
  cg.nt0 = (cg.ex - cg.ox + TX - 1) / TX;
  cg.nt1 = (cg.ey - cg.oy + TY - 1) / TY;
  cg.zc = Pl->col_zc * P;
  cg.nzc = (tp.ax[2].N + cg.zc - 1) / cg.zc;
  const int64_t items = (int64_t)cg.nt0 * cg.nt1 * cg.nzc * tp.Q;
  if (items <= 0 || items > 0x7fffffff || cg.zc > kColZMax)
    return fail(SLLBM_EUNSUPPORTED, "velocity-split step: %lld work items, chunk %d", (long long)items, cg.zc);
  cg.q = (int)(items / 8);
  cg.r = (int)(items % 8);
  {
    ProfScope ps(Pl, "k_stream_col", s);
    hipLaunchKernelGGL((k_stream_col3d<T, P, CPT, PD, BS, WPE>), dim3((unsigned)items), dim3(BS), 0, s, tp, a, cg,
                       (const T *)pin, (T *)pout);
  }
  {
    // relax = false: the node state instead of the relaxation (the learned step's
    // correction then relaxes and corrects in one pass)
    ProfScope ps(Pl, relax ? "k_relax_moments" : "k_node_state", s);
    // 64 nodes per workgroup, their velocities over the waves (FP64: 4, FP32: 2 at Q = 45;
    // 4 at Q = 125).  Measured on the 96^3 Taylor-Green mesh against a node per lane: FP64
    // D3Q45 0.268 -> 0.250 ms, FP32 0.152 -> 0.119 ms; the channel's D3Q45 set-up at Pr 0.7,
    // where a node per lane spilled, 1.51 -> 1.17 ms
    const dim3 grid((unsigned)((tp.N + 63) / 64));
    double *ns = Pl->nstate;
#define RM_LAUNCH(QV, NP)                                                                                   \
  {                                                                                                         \
    if (!relax)                                                                                             \
      hipLaunchKernelGGL((k_relax_moments<T, QV, NP, 0, 1>), grid, dim3(64 * NP), 0, s, tp, a, (T *)pout, ns); \
    else if (a.pr_on)                                                                                       \
      hipLaunchKernelGGL((k_relax_moments<T, QV, NP, 1, 0>), grid, dim3(64 * NP), 0, s, tp, a, (T *)pout, ns); \
    else                                                                                                    \
      hipLaunchKernelGGL((k_relax_moments<T, QV, NP, 0, 0>), grid, dim3(64 * NP), 0, s, tp, a, (T *)pout, ns); \
  }
    if (tp.Q == 45) {
      RM_LAUNCH(45, (sizeof(T) == 8 ? 4 : 2))
    } else if (tp.Q == 125) {
      RM_LAUNCH(125, 4)
#undef RM_LAUNCH
    } else {
      return fail(SLLBM_EUNSUPPORTED, "velocity-split step: no relaxation launch for Q = %d", tp.Q);
    }
  }
  return SLLBM_OK;
}

template <typename T, int D, int P, int CX, int CY, int CZ>
int launch_tile_t(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s, bool relax) {
  if constexpr (D == 3) {
    if (Pl->use_col()) {
      if constexpr (sizeof(T) == 4)
        if (Pl->col_cpt == 2) return launch_col_t<T, P, 2>(Pl, a, pin, pout, s, relax);
      return launch_col_t<T, P, 1>(Pl, a, pin, pout, s, relax);
    }
  }
  constexpr int BS = D == 3 ? 512 : 256;   // threads per workgroup
  // 3D schedule: the skewed two-barrier one except at p = 3 in FP64, where its separate
  // y buffer takes the 12 x 12 x 6 tile to 95 KB of LDS and one workgroup per CU.  Tile
  // kernel on the 96^3-node TGV, skewed against four barriers: p = 2 2.16 / 2.28 ms (FP64),
  // 1.32 / 1.59 ms (FP32); p = 3 FP32 1.23 / 1.37 ms; p = 4 2.50 / 2.79 ms (FP64), 1.99 /
  // 2.32 ms (FP32); p = 3 FP64 2.23-2.41 ms skewed (tile shapes and workgroup sizes
  // tried) against 2.01 ms.
  constexpr int SK = (D == 3 && (P != 3 || sizeof(T) == 4)) ? 1 : 0;
  // minimum waves per SIMD the register budget must allow, per launch
  // (the p = 2 and 4 FP32 kernels are held to 6 waves per SIMD, 3 workgroups per CU:
  // unbounded, p = 2 takes 87 VGPRs and 2 workgroups, 11.7 against 7.9 ms on the
  // 128 x 96 x 64 channel, and p = 4 2.00 against 1.73 ms on the 96^3 TGV; at p = 3 the bound
  // spills 112 B per lane and slows the FP32 TGV from 1.23 to 2.17 ms)
  constexpr int WPE = (D == 3 && P != 3 && sizeof(T) == 4) ? 6 : TILE_WPE;
  constexpr int TX = CX * P, TY = CY * P, TZ = (D == 3) ? CZ * P : 1;
  const DevTensorPlan &tp = Pl->tp;
  TileGrid tg;
  tg.nt[0] = (tp.ax[0].N + TX - 1) / TX;
  tg.nt[1] = (tp.ax[1].N + TY - 1) / TY;
  tg.nt[2] = D == 3 ? (tp.ax[2].N + TZ - 1) / TZ : 1;
  int ntiles = tg.nt[0] * tg.nt[1] * tg.nt[2];
  tg.q = ntiles / 8;
  tg.r = ntiles % 8;
  // 2D: the tables of the regular departure points fit the narrow table count (D2V25) or
  // the wide one (D2Q19); plans with a stash-sized Q run single-pass
  const bool wide = Pl->tile_tabs > kTileTabs;
  if constexpr (D == 2) {
    if (tp.Q == kStashQ && !wide) {
      ProfScope ps(Pl, "k_step_tile", s);
      launch_tile2d_single<T, P, CX, CY, BS, kStashQ, kTileTabs>(tp, a, tg, ntiles, pin, pout, Pl->nstate, s);
      return SLLBM_OK;
    }
    if (tp.Q == kStashQ19 && wide) {
      ProfScope ps(Pl, "k_step_tile", s);
      launch_tile2d_single<T, P, CX, CY, BS, kStashQ19, kTileTabsMax>(tp, a, tg, ntiles, pin, pout, Pl->nstate, s);
      return SLLBM_OK;
    }
  }
  {
    ProfScope ps(Pl, "k_step_tile", s);
    if constexpr (D == 3)
      hipLaunchKernelGGL((k_step_tile3d<T, D, P, CX, CY, CZ, BS, WPE, SK>), dim3(ntiles), dim3(BS), 0, s, tp, a, tg,
                         (const T *)pin, (T *)pout, Pl->nstate);
    else if (wide)
      hipLaunchKernelGGL((k_step_tile2d<T, D, P, CX, CY, CZ, BS, WPE, 0, 0, kTileTabsMax>), dim3(ntiles), dim3(BS), 0, s,
                         tp, a, tg, (const T *)pin, (T *)pout, Pl->nstate);
    else
      hipLaunchKernelGGL((k_step_tile2d<T, D, P, CX, CY, CZ, BS, WPE, 0, 0, kTileTabs>), dim3(ntiles), dim3(BS), 0, s,
                         tp, a, tg, (const T *)pin, (T *)pout, Pl->nstate);
  }
  if (!relax) return SLLBM_OK;   // the caller relaxes the stored streamed values itself
  {
    ProfScope ps(Pl, "k_relax_nodes", s);
    // FP64 with even N (rows keep 2-node groups aligned): 16-byte vector accesses, 4 % faster;
    // in FP32 the 8-byte pairs gain nothing
    // (Pr != 1: the instantiation with the quasi-equilibrium term, which reads the populations
    // twice)
    if (sizeof(T) == 8 && tp.N % 2 == 0) {
      const dim3 grid((unsigned)((tp.N / 2 + kBlock - 1) / kBlock));
      if (a.pr_on)
        hipLaunchKernelGGL((k_relax_nodes<T, D, 2, 1>), grid, dim3(kBlock), 0, s, tp, a, (T *)pout,
                           (const double *)Pl->nstate);
      else
        hipLaunchKernelGGL((k_relax_nodes<T, D, 2, 0>), grid, dim3(kBlock), 0, s, tp, a, (T *)pout,
                           (const double *)Pl->nstate);
    } else {
      const dim3 grid((unsigned)((tp.N + kBlock - 1) / kBlock));
      if (a.pr_on)
        hipLaunchKernelGGL((k_relax_nodes<T, D, 1, 1>), grid, dim3(kBlock), 0, s, tp, a, (T *)pout,
                           (const double *)Pl->nstate);
      else
        hipLaunchKernelGGL((k_relax_nodes<T, D, 1, 0>), grid, dim3(kBlock), 0, s, tp, a, (T *)pout,
                           (const double *)Pl->nstate);
    }
  }
  return SLLBM_OK;
}
}  // namespace

int launch_step_tile(sllbm_plan_s *Pl, const StepArgs &a, const void *pin, void *pout, hipStream_t s, bool relax) {
  int D = Pl->mesh.dim, p = Pl->mesh.p;
  bool f32 = Pl->prec == SLLBM_F32;
#define TCASE(DD, PP)                                                                                  \
  if (D == DD && p == PP) {                                                                            \
    constexpr int CX = TileShape<DD, PP>::CX, CY = TileShape<DD, PP>::CY, CZ = TileShape<DD, PP>::CZ; \
    return f32 ? launch_tile_t<float, DD, PP, CX, CY, CZ>(Pl, a, pin, pout, s, relax)                   \
               : launch_tile_t<double, DD, PP, CX, CY, CZ>(Pl, a, pin, pout, s, relax);                 \
  }
  TCASE(2, 2) TCASE(2, 3) TCASE(2, 4) TCASE(3, 2) TCASE(3, 3) TCASE(3, 4)
#undef TCASE
  return fail(SLLBM_EUNSUPPORTED, "no tiled kernel for dim %d order %d", D, p);
}

}  // namespace sllbm
