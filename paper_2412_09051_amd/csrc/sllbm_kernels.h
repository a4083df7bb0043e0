// Launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sllbm_internal.h"

namespace sllbm {

constexpr int kBlock = 256;        // threads per block of the node-parallel kernels
constexpr int kRedWidth = 8;       // doubles per block partial: mass, momentum[3], energy, -, -, bad
constexpr int kScratchHead = 64;   // scratch doubles before the block partials
constexpr int kSlotTotals = 0;     // [kRedWidth] final totals
constexpr int kSlotScale = 16;     // mass-rescale factor mass_ref / M
constexpr int kSlotMass = 24;      // final [mass, momentum[3], volume] of the f-only reduction
constexpr int kSlotForce = 32;     // controlled body force [3] (sllbm_force_reset / _update)
constexpr int kSlotForce0 = 36;    // force at the last reset [3]
constexpr int kSlotCtl = 40;       // controller: integral, error, mean momentum, updates

// Step parameters as the kernels see them (all derived on the host per call).
struct StepArgs {
  double gamma, cv, gbase;         // gbase = 2 c_v - D  (g^eq = T gbase f^eq)
  double dt, T0, inv_sqrtT0;
  int relax_mode;
  double tau_bar, mu_ref, T_ref, mu_exp;
  double force[3];
  int has_force;
  double Pr;                       // Prandtl number
  int pr_on;                       // 1: Pr != 1 and a collision: add the quasi-equilibrium term
  const double *force_dev;         // device force [3] of the plan's controller, or nullptr
  const double *scale;             // device mass-rescale factor, or nullptr
  const double *inlet;             // device [n_bc][5] inlet states
};

// The 2D tiled kernel keeps the weight rows of the interpolation tables of the regular
// departure points in LDS: their table ids (one per distinct velocity component along
// an axis) must be below the kernel's table count, kTileTabs (the product rule D2V25: five
// components per axis) or kTileTabsMax (the reduced set D2Q19 needs eleven along x).
constexpr int kTileTabs = 5;
constexpr int kTileTabsMax = 16;

// The 3D tiled kernel reads and writes each population plane through a buffer resource with
// 32-bit byte offsets: its plans hold at most this many bytes per plane.
constexpr int64_t kBufMaxBytes = 0x7ffffff0;

// A curvilinear plan row holds its cell and its source in one word (4 B per row): the cell
// (below 2^30), with this bit set when the source is the opposite population; an inlet row
// holds -1 - bc.
constexpr int32_t kCsrOpp = 1 << 30;

// Cell-aligned tile (cells per axis) of the LDS-tiled step kernel for (dim, order).
template <int D, int P> struct TileShape;
// 2D tiles hold at most 256 nodes: one node per lane of a 256-thread workgroup, so that the
// single-pass kernel keeps a node's streamed values in that lane's registers
template <> struct TileShape<2, 2> { static constexpr int CX = 8, CY = 8, CZ = 1; };
template <> struct TileShape<2, 3> { static constexpr int CX = 8, CY = 3, CZ = 1; };
template <> struct TileShape<2, 4> { static constexpr int CX = 8, CY = 2, CZ = 1; };
#ifndef TILE_3_2
#define TILE_3_2 4, 4, 4
#endif
template <> struct TileShape<3, 2> {
  static constexpr int c[3] = {TILE_3_2};
  static constexpr int CX = c[0], CY = c[1], CZ = c[2];
};
#ifndef TILE_3_3
#define TILE_3_3 4, 4, 2
#endif
template <> struct TileShape<3, 3> {
  static constexpr int c[3] = {TILE_3_3};
  static constexpr int CX = c[0], CY = c[1], CZ = c[2];
};
template <> struct TileShape<3, 4> { static constexpr int CX = 2, CY = 2, CZ = 2; };

// The velocity-split 3D step (one velocity per workgroup on a column of output nodes, then a
// moments-and-relaxation launch with a node's streamed values in registers): x-y tiles of
// 48 x 12 nodes, z chunks of whole cells up to kColZMax planes, a window of kColWin<P>
// y-contracted planes per column; the relaxation launch (a node's velocities over the waves
// of a workgroup) is compiled for these Q.
// (48 x 12 against 24 x 24 on the 96^3 Taylor-Green mesh: the same within 2 % on D3Q45 and
// D3V125; on the 256 x 193 x 128-node channel's D3Q45 set-up 1.60 -> 1.25 ms per streaming
// launch, its longer rows meeting in L2; 36 x 12: no better)
#ifndef COL_TX
#define COL_TX 48
#endif
#ifndef COL_TY
#define COL_TY 12
#endif
template <int P> struct ColShape {
  static constexpr int CX = COL_TX / P, CY = COL_TY / P;   // cells per tile along x and y
};
template <int P> constexpr int kColWin = 3 * P - 1;
// most output columns per thread of the streaming launch (the tile is that many times as long
// in y): two in FP32, one in FP64 (where a second column's window would halve the occupancy).
// FP32 D3Q45 at p = 3 also takes one (96^3 Taylor-Green: 0.267 -> 0.244 ms per streaming
// launch), while D3V125 and the p = 2 channel lose 4-6 % per step with it.
constexpr int col_cpt(int elem_bytes, int p, int Q) { return elem_bytes == 4 && !(p == 3 && Q == 45) ? 2 : 1; }
constexpr int kColZMax = 96;
constexpr bool col_q_supported(int Q) { return Q == 45 || Q == 125; }

int launch_step_csr(sllbm_plan_s *P, const StepArgs &a, const void *pin, void *pout, hipStream_t s);
// relax = false: 3D plans on the two-launch tile path stop after the streaming launch (the
// owned nodes' streamed values and node state stored, the relaxation left to the caller); the
// boundary layers' gather launch still relaxes its nodes.
int launch_step_tile(sllbm_plan_s *P, const StepArgs &a, const void *pin, void *pout, hipStream_t s,
                     bool relax = true);
int launch_init(sllbm_plan_s *P, const StepArgs &a, const double *rho, const double *u, const double *T, void *pop,
                hipStream_t s);
int launch_step(sllbm_plan_s *P, const StepArgs &a, const void *pin, void *pout, hipStream_t s, bool relax = true);
// True if a step of this plan runs the 3D two-launch tile path (streaming launch, node state,
// relaxation launch), whose relaxation launch_step(..., relax = false) leaves out.
bool step_has_relax_launch(const sllbm_plan_s *P);
int launch_moments(sllbm_plan_s *P, const StepArgs &a, const void *pop, double *rho, double *u, double *T,
                   bool totals, hipStream_t s);
// The same with the block partials of the totals in part[kRedWidth * nblocks(N)] and the final
// totals in totals[kRedWidth] (both device memory; totals == nullptr: no reduction).
int launch_moments_to(sllbm_plan_s *P, const StepArgs &a, const void *pop, double *rho, double *u, double *T,
                      double *part, double *totals, hipStream_t s);
int launch_mass_scale(sllbm_plan_s *P, const void *pop, double mass_ref, hipStream_t s);
// Learned correction (sllbm_mlp.hip).  learned_check: the network fits the plan (inputs,
// outputs, device) and the plan's learned-mode buffers exist (allocated on first use).
// launch_mlp_correct: features of pop, network, projected correction added in place.
// launch_relax_correct: after launch_step(..., relax = false) on a plan with a relaxation
// launch, the node fields from the node state, the features, then the relaxation and the
// correction in one pass over pop.
int learned_check(sllbm_plan_s *P, sllbm_mlp m);
int launch_mlp_correct(sllbm_plan_s *P, const sllbm_params *prm, sllbm_mlp m, void *pop, hipStream_t s);
int launch_relax_correct(sllbm_plan_s *P, const StepArgs &a, sllbm_mlp m, void *pop, hipStream_t s);
int launch_force_reset(sllbm_plan_s *P, const double *force0, hipStream_t s);
int launch_force_update(sllbm_plan_s *P, int axis, double target, double kp, double ki, double dt, const void *pop,
                        hipStream_t s);

// Per-kernel timing: while the plan's profiler is on, a ProfScope around a launch
// records HIP events before and after it on the launch stream.
void prof_begin(sllbm_plan_s *P, const char *name, hipStream_t s, int *id, hipEvent_t *a);
void prof_end(sllbm_plan_s *P, int id, hipEvent_t a, hipStream_t s);
struct ProfScope {
  sllbm_plan_s *P;
  hipStream_t s;
  int id = -1;
  hipEvent_t a = nullptr;
  ProfScope(sllbm_plan_s *P_, const char *name, hipStream_t s_) : P(P_), s(s_) { prof_begin(P, name, s, &id, &a); }
  ~ProfScope() { prof_end(P, id, a, s); }
};

}  // namespace sllbm
