// Internal structures of libsllbm shared by the host plan builder and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "sllbm.h"

namespace sllbm {

constexpr int kMaxP = 8;      // host geometry supports p <= 8
constexpr int kMaxQ = 128;    // device tables sized for Q <= 128
constexpr int kMaxBC = 16;

// Record an error for sllbm_last_error() and return the code.
int fail(int code, const char *fmt, ...);

// ---------------------------------------------------------------- velocity set
struct VelSet {
  int dim = 0, Q = 0;
  double T0 = 1.0;
  std::vector<double> zeta;   // [Q][dim]
  std::vector<double> w;      // [Q]
  std::vector<int32_t> opp;   // [Q]
};

// ---------------------------------------------------------------- mesh
struct Mesh {
  int dim = 0, p = 0, nodes = 0, kind = 0;
  std::vector<double> xref;   // support points on [-1,1]
  // tensor
  int ncell[3] = {1, 1, 1};
  std::vector<double> edges[3];
  int face_bc[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
  int N[3] = {1, 1, 1};       // nodes per axis
  // curvilinear
  std::vector<double> node_xyz;
  std::vector<int64_t> cell_nodes;
  std::vector<int32_t> cell_face_bc;
  int64_t n_cells = 0;
  // common
  int64_t n_nodes = 0;
  std::vector<sllbm_bc> bcs;
  bool periodic(int a) const { return face_bc[a][0] < 0; }
};

// Support points of one cell on [-1,1] (GLL: ends plus roots of P_p'; GLC: -cos(pi j/p)).
std::vector<double> support_points(int p, int family);
// Barycentric Lagrange weights of the nodes xref at xi (exact 0/1 on a node).
void lagrange_weights(const std::vector<double> &xref, double xi, double *w);
// Integral over [-1,1] of each Lagrange basis function of xref.
std::vector<double> lagrange_integrals(const std::vector<double> &xref);
double tensor_node_coord(const Mesh &m, int a, int n);
// Round one set of n interpolation weights to float so that their exact sum stays 1
// (partition of unity) as closely as float allows: the residual of plain rounding is
// moved into the weight that absorbs it with the smallest leftover.
void round_weights_f32(const double *w, int n, float *out);

// ---------------------------------------------------------------- plan
enum ExcKind : int32_t { EXC_NONE = 0, EXC_WALL = 1, EXC_INLET = 2, EXC_OUTLET = 3 };

// A (boundary layer, velocity) pair on a tensor mesh whose backward path leaves through
// one face.  tab[a] selects the per-axis interpolation table for the axes parallel to
// the face; along the face normal the stencil start and weights are explicit.
struct ExcEntry {
  int32_t kind;
  int32_t src;        // source velocity (bounce-back: opposite), or bc index (inlet)
  int32_t tab[3];     // per-axis table id (ignored along the face axis)
  int32_t start;      // first stencil node along the face axis
  double w[kMaxP + 1];
  float w32[kMaxP + 1];  // the same weights rounded for FP32 plans (see round_weights_f32)
};

// Device view of a tensor-mesh plan; passed to kernels by value.
struct DevAxis {
  int N;
  int periodic;
  int ntab;               // interpolation tables (distinct displacements along the axis)
  const int32_t *start;   // [ntab][N]
  const double *w64;      // [ntab][N][p+1]
  const float *w32;       // same, single precision
  const int32_t *ident;   // [ntab] 1 = zero displacement (identity along this axis)
};

struct DevFace {
  int axis, side;        // axis index and 0 = low, 1 = high
  int depth;             // layers with entries (0 = face not bounded)
  const ExcEntry *e;     // [depth][Q]
  const double *Tw;      // [depth] wall temperature of a thermal layer, NaN otherwise
};

struct DevTensorPlan {
  int dim, p, Q;
  int64_t N;
  DevAxis ax[3];
  const int32_t *tab_reg;   // [3][Q] table id of the regular departure point
  int nfaces;
  DevFace face[2];
  const double *vel;        // [Q][8]: zeta x,y,z, xi x,y,z (= zeta/sqrt(T0)), |xi|^2, w
  const double *vol;        // [N] nodal volumes
};

// Device view of a CSR (curvilinear) plan.
struct DevCsrPlan {
  int dim, p, Q;
  int64_t N;
  int npc;                  // support points per cell, (p+1)^dim
  const int32_t *cell_nodes;// [n_cells][npc]
  const int32_t *row_code;  // [Q][N] the cell of the departure point, | kCsrOpp when the source
                            // is the opposite population (bounce-back); an inlet row: -1 - bc
  const int32_t *opp;       // [Q] opposite velocity
  const double *row_xi;     // FP64 plans: [Q][2][N] reference coordinates (xi, eta) of the departure point in its cell
  const float *row_xf;      // FP32 plans: [Q][N][2] the same coordinates rounded to FP32
  double xref[kMaxP + 1];   // support points on [-1, 1]
  double lam[kMaxP + 1];    // 1 / prod_{b != a} (xref_a - xref_b)
  const double *node_Tw;    // [N] thermal-wall temperature, NaN = none
  const double *vel;
  const double *vol;
};

struct PlanHost;   // host-side tables (defined in sllbm_host.cpp)

}  // namespace sllbm

struct sllbm_mesh_s {
  sllbm::Mesh m;
};

namespace sllbm {
// Per-kernel timing of one plan: HIP events recorded around each launch on the caller's
// stream while enabled; read out (after synchronising on the events) as total time and
// launch count per kernel name.
struct Profiler {
  bool on = false;
  std::vector<std::string> names;
  std::vector<double> total_ms;
  std::vector<int64_t> launches;
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
};
}  // namespace sllbm

namespace sllbm {
// Device memory of library-owned objects: hipMalloc/hipFree, or the caller's functions set
// by sllbm_set_allocator.  Each object keeps the allocator it was created with.
struct DevAllocator {
  void *(*alloc)(size_t bytes, void *ctx) = nullptr;
  void (*release)(void *ptr, void *ctx) = nullptr;
  void *ctx = nullptr;
  hipError_t get(void **p, size_t bytes) const {
    if (!alloc) return hipMalloc(p, bytes);
    *p = alloc(bytes, ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  void put(void *p) const {
    if (!p) return;
    if (release) release(p, ctx);
    else (void)hipFree(p);
  }
};
DevAllocator current_allocator();
}  // namespace sllbm

struct sllbm_plan_s {
  sllbm::DevAllocator dalloc;   // allocator of this plan's device memory
  sllbm::Mesh mesh;
  sllbm::VelSet vel;
  double dt = 0;
  int prec = 0;
  int kernel = 0;               // 0 tensor, 1 csr
  int64_t n_exceptions = 0, n_thermal = 0, table_bytes = 0;
  int has_device = 0;
  int device = -1;
  int tile_ok = 0;              // the LDS-tiled kernel applies to this plan
  int tile_tabs = 0;            // 1 + the largest table id of a regular departure point
  int kernel_choice = 0;        // 0 auto, 1 baseline gather, 2 tiled, 3 tiled with velocity-split 3D steps
  int tile_auto = 0;            // the automatic choice takes the tile: eligible, and at least
                                // kTileMinTiles tiles (fewer leave most compute units idle)
  int col_ok = 0;               // the velocity-split 3D step applies (choice 3; automatic with the tile)
  int col_zc = 0;               // its z chunk, in cells
  int col_cpt = 1;              // its output columns per thread (the tile is that many times as long in y)
  int col_org[2] = {0, 0};      // its x-y tiles start here (a cell boundary past a bounded face's layers)
  int col_end[2] = {0, 0};      // and cover the nodes below this (the last interior cell boundary)
  bool use_tile() const {
    return tile_ok && (kernel_choice == 2 || kernel_choice == 3 || (kernel_choice == 0 && tile_auto));
  }
  // steps of the plan run the velocity-split 3D step (a learned step: its streaming launch and
  // a launch that stores the node state the correction reads)
  bool use_col() const { return col_ok && (kernel_choice == 3 || (kernel_choice == 0 && tile_auto)); }
  sllbm::DevTensorPlan tp{};
  sllbm::DevCsrPlan cp{};
  std::vector<void *> dev_allocs;
  const double *inlet_dev = nullptr;  // [n_bc][5] inlet states (rho, u, T) on the device
  double *scratch = nullptr;    // device scratch: reduction partials + scalars
  double *nstate = nullptr;     // tiled kernel: node state between its two launches, [6][N]
  int64_t scratch_len = 0;      // doubles
  bool force_ready = false;     // the controller's device force has been set (sllbm_force_reset)
  // host copies kept for the GPU-free info path
  std::vector<double> vol;
  sllbm::Profiler prof;
  // learned correction (built on first use): node fields [D+2][N], features [N][n_feat],
  // per-axis derivative stencils [N_a][2][p+1] (node index along the axis, weight)
  double *lfield = nullptr;
  uint16_t *lfeat = nullptr;
  int32_t *ldidx[3] = {nullptr, nullptr, nullptr};
  double *ldw[3] = {nullptr, nullptr, nullptr};
};

namespace sllbm {
// Host plan builders (fill the host vectors, then upload through the allocator callback).
struct HostTables {
  // tensor
  std::vector<int32_t> start[3];
  std::vector<double> w[3];
  std::vector<int32_t> ident[3];
  int ntab[3] = {0, 0, 0};
  std::vector<int32_t> tab_reg;     // [3][Q]
  int nfaces = 0;
  int face_axis[2] = {0, 0}, face_side[2] = {0, 0}, face_depth[2] = {0, 0};
  std::vector<ExcEntry> face_e[2];
  std::vector<double> face_Tw[2];
  // csr
  std::vector<int32_t> row_cell, row_src;
  std::vector<double> row_xi;       // [Q][2][N]
  std::vector<double> node_Tw;
  // common
  std::vector<double> vel;          // [Q][8]
};
int build_tensor_tables(const Mesh &m, const VelSet &v, double dt, HostTables &t, int64_t *n_exc, int64_t *n_th);
int build_csr_tables(const Mesh &m, const VelSet &v, double dt, HostTables &t, int64_t *n_exc, int64_t *n_th);
std::vector<double> node_volumes(const Mesh &m);
// Tile shape (cells per axis) of the LDS-tiled kernel for (dim, p), or false.
bool tile_cells(int D, int P, int c[3]);
// below this many tiles (one per compute unit) the per-node gather kernel, with a node's
// velocities over up to four lanes, steps faster than the tile kernel's sequence of
// per-velocity stages (measured: 80 tiles, 0.24 against 0.65 ms; 4352 tiles, 9.3 against 4.6 ms)
constexpr int64_t kTileMinTiles = 256;
// True if every regular departure stencil of a cell-aligned tile of c[] cells stays in
// the one-cell halo that the tiled kernel stages.
// org / end (optional): the tiles of axis a start at org[a] and cover the nodes below end[a]
// (default: 0 and the axis length)
bool tile_eligible(const Mesh &m, const HostTables &t, const int c[3], const int *org = nullptr,
                   const int *end = nullptr);
// True if the velocity-split 3D step applies with x-y tiles of cx x cy cells and z chunks of
// zc cells: a 3D plan periodic along z (bounded faces on x or y only), every regular stencil
// in the one-cell halo of such a tile, and along z every output plane's stencil inside the
// window of L planes that the kernel holds when it emits that plane.
bool col_eligible(const Mesh &m, const HostTables &t, int cx, int cy, int zc, int L, const int org[2], const int end[2]);
}  // namespace sllbm
