/*
 * sllbm.h - C ABI of the MI355X semi-Lagrangian lattice Boltzmann (SLLBM) library.
 *
 * The library advances the compressible SLLBM of Spelten, Wilde, Bedrunka, Reith and
 * Foysi (arXiv 2412.09051) by one time step per call:
 *   - streaming: every node x_k and velocity zeta_i takes the value of the order-p
 *     Lagrange interpolant at the departure point x_k - dt zeta_i
 *     (Sec. 3.1, SLLBM update display, eq:intf and the display after it);
 *   - collision: BGK relaxation of the two population sets f and g towards the
 *     4th-order Hermite equilibrium (Sec. 3.1, f^eq and g^eq displays);
 *   - boundaries: equilibrium inlet (Sec. 3.3.1), bounce-back and isothermal wall
 *     (Sec. 3.3.2, eq:thermalBC), zero-gradient outlet (Sec. 3.3.3), periodic.
 *
 * Conventions shared by every entry point
 *   - Every call returns 0 (SLLBM_OK) or a negative code; sllbm_last_error() returns a
 *     thread-local message for the last failing call of the calling thread.
 *   - Arguments are validated before anything is enqueued: on an error no work was
 *     launched and no caller buffer was touched.
 *   - Handles (sllbm_mesh, sllbm_plan) are owned by the library and must be released
 *     with the matching *_destroy call.  A handle is not thread-safe: calls that use
 *     one plan must be serialised (one host thread, one stream at a time), because the
 *     plan owns a small device scratch area (reductions, mass-rescale factor).
 *   - Population buffers are caller-owned device memory (e.g. torch tensors) holding
 *     2*Q*N elements of the plan precision, laid out as pop[(s*Q + i)*N + k] with
 *     s = 0 for f, s = 1 for g, i the velocity index, k the node index in library
 *     order.  They must be 16-byte aligned.  pop_in and pop_out of a step must not
 *     overlap.
 *   - Library node order on tensor meshes: k = n_x + N_x (n_y + N_y n_z), x fastest,
 *     where along a periodic axis N_a = ncell_a * p and along a bounded axis
 *     N_a = ncell_a * p + 1 (the last node sits on the high face).
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.  All
 *     device work is asynchronous on that stream unless stated otherwise.
 *   - Units: gas constant R = 1, c_v = 1/(gamma - 1); velocities are zeta = sqrt(T0) x
 *     with x the Gauss-Hermite abscissae.
 */
#ifndef SLLBM_H
#define SLLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SLLBM_OK = 0,
  SLLBM_EINVAL = -1,       /* invalid argument, size or enum */
  SLLBM_ENOMEM = -2,       /* host or device allocation failed */
  SLLBM_EGEOM = -3,        /* a departure point cannot be placed (left the mesh untagged,
                              reflected path leaves again, Newton inverse map failed) */
  SLLBM_EHIP = -4,         /* a HIP runtime call failed, or no GPU is present */
  SLLBM_EUNSUPPORTED = -5, /* valid input outside what the GPU path implements (e.g. Pr != 1) */
  SLLBM_EUNSTABLE = -6     /* non-finite value, rho <= 0 or T <= 0 seen by sllbm_moments */
};

typedef struct sllbm_mesh_s *sllbm_mesh;
typedef struct sllbm_plan_s *sllbm_plan;

typedef enum { SLLBM_NODES_GLL = 0, SLLBM_NODES_GLC = 1, SLLBM_NODES_EQUI = 2 } sllbm_nodes;
typedef enum { SLLBM_MESH_TENSOR = 0, SLLBM_MESH_CURVILINEAR = 1 } sllbm_mesh_kind;
typedef enum { SLLBM_BC_PERIODIC = 0, SLLBM_BC_WALL = 1, SLLBM_BC_INLET = 2, SLLBM_BC_OUTLET = 3 } sllbm_bc_kind;
typedef enum { SLLBM_F64 = 0, SLLBM_F32 = 1 } sllbm_prec;

/* One boundary condition (Sec. 3.3).
 *   WALL  : bounce-back (Sec. 3.3.2); T_wall finite adds the isothermal correction
 *           of eq:thermalBC at every node where a trajectory hit this wall; NaN = none.
 *   INLET : equilibrium inlet with state (rho, u, T) (Sec. 3.3.1).
 *   OUTLET: zero-gradient outlet, mirrored departure point (Sec. 3.3.3). */
typedef struct {
  int kind;          /* sllbm_bc_kind */
  double rho;
  double u[3];
  double T;
  double T_wall;
} sllbm_bc;

/* Mesh description (eq:intf: cells with (p+1)^dim support points).  All pointers are
 * host memory and are copied by sllbm_mesh_build.
 *   TENSOR      : tensor product of 1D meshes; edges[a] holds ncell[a]+1 strictly
 *                 increasing coordinates (uniform or stretched).  face_bc[a][0/1] is -1
 *                 on both faces of a periodic axis, otherwise an index into bcs.  At
 *                 most one axis may be bounded.
 *   CURVILINEAR : dim = 2 isoparametric quads of order p: n_nodes unique nodes with
 *                 node_xyz[k*2 + a]; cell_nodes[c*(p+1)^2 + j_x + (p+1) j_y] lists each
 *                 cell's support points in reference order (xi fastest);
 *                 cell_face_bc[c*4 + f] tags the faces xi=-1, xi=+1, eta=-1, eta=+1
 *                 with -1 (interior) or an index into bcs.  Library node order is
 *                 the caller's node order. */
typedef struct {
  int dim;        /* 2 or 3 */
  int order_p;    /* 1..8 (GPU kernels: 2..4) */
  int nodes;      /* sllbm_nodes: support-point family inside each cell */
  int kind;       /* sllbm_mesh_kind */
  int ncell[3];
  const double *edges[3];
  int face_bc[3][2];
  int64_t n_nodes;
  const double *node_xyz;
  int64_t n_cells;
  const int64_t *cell_nodes;
  const int32_t *cell_face_bc;
  int n_bc;
  const sllbm_bc *bcs;
} sllbm_mesh_desc;

/* Build a mesh (host only, no GPU needed).  Returns EINVAL for malformed input. */
int sllbm_mesh_build(const sllbm_mesh_desc *d, sllbm_mesh *out);
/* Number of unique nodes; if xyz != NULL writes n_nodes*dim host doubles, library order. */
int sllbm_mesh_nodes(sllbm_mesh m, int64_t *n_nodes, double *xyz);
/* Integral of every nodal Lagrange function (the nodal quadrature weight V_k used for
 * the totals and the mass rescaling); host output of n_nodes doubles. */
int sllbm_mesh_volumes(sllbm_mesh m, double *vol);
void sllbm_mesh_destroy(sllbm_mesh m);

/* Discrete velocity set (Sec. 3.2). */
typedef struct {
  int dim, Q;
  const double *zeta;        /* [Q][dim] */
  const double *w;           /* [Q] */
  const int32_t *opposite;   /* [Q] index of -zeta_i (bounce-back, Sec. 3.3.2) */
  double T0;                 /* reference temperature of the Hermite expansion */
} sllbm_velset;

/* Product-rule Gauss-Hermite set D{dim}V{n^dim} (Sec. 3.2: n points give quadrature
 * degree 2n-1; n = 5 gives degree 9).  Index i = a_x + n a_y + n^2 a_z over ascending
 * abscissae.  Host outputs: zeta [Q*dim], w [Q], opp [Q] with Q = n^dim. */
int sllbm_velset_gauss_hermite(int dim, int n_per_dim, double T0, double *zeta, double *w, int32_t *opp);
/* Reduced cubature sets of quadrature degree 9 (Sec. 3.2: the smallest known such rules
 * for the Gaussian weight have 19 points in 2D and 45 in 3D, named D2Q19 and D3Q45 there;
 * the paper prints no abscissae).  The rules returned are fixed by the degree-9 moment
 * conditions under a symmetry group that contains -1:
 *   dim 2 (Q = 19): the origin, two regular hexagons with a vertex on +x (|x|^2 =
 *     (48 -+ 8 sqrt 15)/7) and one turned by 30 degrees (|x|^2 = 8, total weight 3/64);
 *   dim 3 (Q = 45): the origin (weight 28/135), icosahedra with the vertices (0, +-1, +-phi)
 *     and their cyclic shifts at |x|^2 = 3 (25/432 each) and 15 (1/2160 each), and the dual
 *     dodecahedron at |x|^2 = 9 (1/216 each).
 * zeta = sqrt(T0) x.  Index 0 is the origin, then the inner and outer hexagon (icosahedron)
 * orbit, then the turned hexagon (dodecahedron).  *Q receives 19 or 45; with zeta, w and
 * opp all NULL nothing else is written (size query), otherwise all three are host outputs
 * of Q*dim, Q and Q elements.  EINVAL for another dim, T0 <= 0 or a partial set of outputs. */
int sllbm_velset_cubature(int dim, double T0, int *Q, double *zeta, double *w, int32_t *opp);

/* Interpolation plan for (mesh, velocity set, dt, precision): for every node and
 * velocity the departure point x_k - dt zeta_i, the boundary case that the backward
 * path meets first, the source population and the interpolation weights
 * (Sec. 3.1 interpolation display, Sec. 3.3).  Built on the host and uploaded to the
 * GPU once; SLLBM_EGEOM names the offending node and velocity in the error message.
 * Without a GPU the host part is still built (sllbm_plan_info works) and every launch
 * returns SLLBM_EHIP.  GPU kernels exist for dim 2 and 3, p = 2..4, Q <= 128.  A curvilinear
 * plan holds each row's cell and source in one 32-bit word: meshes of 2^30 cells or more
 * return SLLBM_EUNSUPPORTED. */
int sllbm_interp_plan(sllbm_mesh m, const sllbm_velset *v, double dt, int prec, sllbm_plan *out);

typedef struct {
  int64_t n_nodes;
  int Q;
  int dim, order_p, prec;
  int64_t n_exceptions;      /* (node, velocity) pairs decided by a boundary */
  int64_t n_thermal_nodes;   /* nodes that receive the isothermal correction */
  int64_t table_bytes;       /* device bytes of the interpolation tables */
  int has_device;            /* 1 if the tables are on a GPU */
  int kernel;                /* step kernel in use: 0 tensor-product per-node gather,
                                1 CSR (curvilinear), 2 tensor-product LDS-tiled, 3 the same
                                with velocity-split 3D steps (see sllbm_plan_select_kernel) */
} sllbm_plan_info_t;
int sllbm_plan_info(sllbm_plan p, sllbm_plan_info_t *info);
/* Choose the step kernel of a tensor-product plan: 0 automatic (tiled when it applies and the
 * mesh has at least 256 tiles, one per compute unit, with velocity-split steps where those
 * apply; smaller meshes step faster on the gather kernel),
 * 1 the per-node gather kernel, 2 the LDS-tiled kernel (SLLBM_EUNSUPPORTED when a
 * departure stencil leaves the one-cell halo the tile stages, e.g. CFL > 1), 3 the tiled
 * kernel with velocity-split 3D steps: the step of Sec. 3.1 as a streaming launch with one
 * velocity per workgroup, walking each departure plane once along z, and a launch that forms
 * the moments from a node's streamed values held in registers and relaxes them
 * (SLLBM_EUNSUPPORTED unless the plan is 3D, periodic along z (bounded faces on x or y, whose
 * boundary layers stay on the gather kernel), on a 45- or 125-velocity set and tiled-eligible
 * with its x-y tiles of 48 x 12 nodes and a halo).  All compute the same step; the
 * choice exists for testing and measurement. */
int sllbm_plan_select_kernel(sllbm_plan p, int kernel);
/* Per-kernel timing of a plan's launches (for measurement, not part of the method).
 * enable = 1 clears the counters and starts recording a HIP event pair around every
 * launch this plan makes, on the stream the launch uses; enable = 0 stops.  Recording
 * adds two event records per launch and no synchronisation (events are waited for only
 * when read, or every 8192 launches).  Returns SLLBM_EHIP for a plan without a device. */
int sllbm_plan_profile(sllbm_plan p, int enable);
/* Times since the last enable: waits for the recorded events, then writes up to `max`
 * entries (kernel name, NUL-terminated in 32 chars; total milliseconds; launch count)
 * into caller-owned host arrays.  Returns the number of distinct kernels (which may
 * exceed max), or a negative error code. */
int sllbm_plan_profile_read(sllbm_plan p, int max, char (*names)[32], double *total_ms, int64_t *launches);
void sllbm_plan_destroy(sllbm_plan p);

/* Device memory of the library's own objects (plans, their learned-mode buffers, networks).
 * By default hipMalloc / hipFree.  A caller that manages device memory itself (a caching
 * allocator, a memory pool) passes alloc(bytes, ctx) -> device pointer (NULL on failure;
 * the memory must be on the device current at the call and stay valid until release) and
 * release(ptr, ctx); both NULL restores the default.  Giving only one is EINVAL.  Each
 * object keeps the functions current when it was created and releases its memory through
 * them on destroy (after the caller's work on it has finished).  Set it before creating
 * handles; the setting itself is guarded by a lock. */
int sllbm_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*release)(void *ptr, void *ctx), void *ctx);

/* Physical parameters of a step. */
typedef struct {
  double gamma;        /* c_v = 1/(gamma-1), R = 1 */
  int relax_mode;      /* 0: constant tau_bar; 1: tau_bar = mu(T)/(rho T dt) + 1/2 with
                          mu = mu_ref (T/T_ref)^mu_exp (tau = mu/p, Sec. 3.1; power law of
                          Sec. 4.3); 2: streaming and boundary schemes only, no collision */
  double tau_bar, mu_ref, T_ref, mu_exp;
  double Pr;           /* Prandtl number, > 0 (EINVAL otherwise).  Pr != 1 adds the collision's
                          quasi-equilibrium term (Sec. 3.1 update display): (1/tau_bar - 1/tau_Pr) h*,
                          tau_Pr = (tau_bar - 1/2)/Pr + 1/2, with h* the lowest-order Hermite part that
                          carries the node's heat flux q (c = zeta - u; q_f = 1/2 sum c|c|^2 f,
                          q_g = 1/2 sum c g): f*_i = w_i (q_f.zeta_i)(|zeta_i|^2 - (D+2)T0)/((D+2)T0^3),
                          g*_i = 2 w_i (q_g.zeta_i)/T0.  The paper defers h* to its references; this
                          form relaxes the heat flux with tau_Pr and leaves rho, j, E and the stress
                          to the BGK term.  On the two-launch tensor path the relaxation then reads
                          the populations twice. */
  double force[3];     /* body force per unit volume, Kupershtokh exact difference (Sec. 4.3) */
  int mass_fix;        /* 1: scale all populations by mass_ref/M before streaming (Sec. 4.3) */
  double mass_ref;
  int force_device;    /* 1: the force is the plan's controlled device value (sllbm_force_reset,
                          sllbm_force_update) and force[] is ignored; EINVAL before a reset */
} sllbm_params;

/* Populations in equilibrium with nodal fields: f = f^eq(rho,u,T), g = g^eq.
 * rho, T: device double [N]; u: device double [dim][N] (component-major). */
int sllbm_init_equilibrium(sllbm_plan p, const sllbm_params *prm, const double *rho, const double *u,
                           const double *T, void *pop, void *stream);

/* One time step: pop_out <- collide(stream(pop_in)).  Both hold post-collision states. */
int sllbm_step(sllbm_plan p, const sllbm_params *prm, const void *pop_in, void *pop_out, void *stream);

/* Force controller of the driven channel (Sec. 4.3: the streamwise force starts from an
 * estimate and is then adjusted by a PI controller that holds the mean momentum).  The
 * force lives in plan-owned device memory, so a controlled run never waits for the host:
 *   e = target - M_axis / V,   I <- I + e dt,   F_axis = F0_axis + kp e + ki I,
 * with M_axis = sum_k V_k sum_i zeta_i,axis f_i(k) and V = sum_k V_k (nodal quadrature
 * volumes) of the populations passed to the update. */
typedef struct {
  int axis;            /* force component controlled, 0 .. dim-1 */
  double target;       /* target mean momentum density (the bulk rho u of the axis) */
  double kp, ki;       /* proportional and integral gains (finite; 0 disables a term) */
  double dt;           /* time since the previous update, >= 0: the integral adds e dt */
} sllbm_force_ctl;
/* Sets the plan's device force and F0 to force0 (host [3]; components beyond dim are
 * taken as 0) and clears the integral.  Enqueued on `stream`; no synchronisation. */
int sllbm_force_reset(sllbm_plan p, const double *force0, void *stream);
/* Measures the mean momentum of pop (device, plan precision, step layout) and applies
 * the controller law on the device.  Steps enqueued after it on the same stream with
 * force_device = 1 use the new force.  EINVAL before sllbm_force_reset. */
int sllbm_force_update(sllbm_plan p, const sllbm_force_ctl *c, const void *pop, void *stream);
/* Synchronises the stream and writes the controller state to host [7]: force[3],
 * integral I, last error e, last mean momentum, number of updates since the reset. */
int sllbm_force_read(sllbm_plan p, double *state_host, void *stream);

/* Nodal rho, u ([dim][N]), T of a population set (eq:density, eq:momentum, energy display
 * read as total energy), each output optional (NULL), device doubles.  If totals_host
 * != NULL the call also reduces the nodal-quadrature totals [mass, momentum[dim], energy]
 * (deterministic order), synchronises the stream and writes them to host memory; it
 * returns SLLBM_EUNSTABLE if any node has a non-finite value, rho <= 0 or T <= 0. */
int sllbm_moments(sllbm_plan p, const sllbm_params *prm, const void *pop, double *rho, double *u, double *T,
                  double *totals_host, void *stream);

/* sllbm_moments for callers that cannot allocate device memory (code under stream capture,
 * serving loops, hosts that forbid allocation): same arguments, outputs and errors, but the
 * block partials and totals of the reduction live in a fixed scratch array that the library
 * holds on each GPU for the life of the process (8 MiB), so the call allocates nothing.
 * Limit: plans of at most 2^25 = 33,554,432 nodes; larger plans get SLLBM_EINVAL before any
 * launch.  All calls on one GPU share that scratch: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller. */
int sllbm_moments_noalloc(sllbm_plan p, const sllbm_params *prm, const void *pop, double *rho, double *u, double *T,
                          double *totals_host, void *stream);

/* ------------------------------------------------------------------------------------
 * Learned post-collision correction (tensor-product plans)
 *
 * A small network maps the moments of a node and their gradients to a correction of the
 * node's post-collision populations on a coarse mesh; it is trained on restricted runs
 * of a finer mesh.  The plain step stays the method; the correction is a separate call
 * after it, so leaving it out falls back to the plain method.
 *
 * Features of node k (n_feat = (D+2)(D+1): 12 in 2D, 20 in 3D), in this order:
 *   rho - 1, u_a / sqrt(T0) (a < D), T / T0 - 1, then for each of those D+2 fields q and
 *   each axis a: h_a dq/dx_a, the derivative of the cell interpolant (eq:intf) along a at
 *   the node averaged over the cells that share the node on that axis, h_a the mean
 *   length of those cells.  Stored as BF16 (round to nearest even), row-major [N][n_feat].
 * Network: three tanh layers of width 64 and a linear output y of n_out = 2Q values;
 *   matrix-product inputs in BF16 (MFMA), sums and master weights in FP32.  Parameters,
 *   flat FP32 in the order W1 [n_in][64], b1, W2 [64][64], b2, W3, b3, W4 [64][n_out], b4.
 * Correction: pop_k += P (w rho_k * y_k), the output scaled by w_i rho_k (w repeated for
 *   f and g), projected off the collision invariants (mass, momentum, total energy) in the
 *   inner product weighted by 1/w_i, so that no moment of the node changes.
 * Training targets: t_k = P (pop_true - pop_plain)_k / (w rho_k), rho_k of pop_plain;
 *   loss = mean over rows and outputs of (y - t)^2; Adam (0.9, 0.999, 1e-8).
 * ------------------------------------------------------------------------------------ */
typedef struct sllbm_mlp_s *sllbm_mlp;

/* A network with n_in <= 32 inputs and n_out <= 256 outputs (width 64 and depth 3 only,
 * else SLLBM_EUNSUPPORTED), on the current device.  Weights uniform in
 * +-1/sqrt(fan_in) from a splitmix64 counter stream of `seed`, biases 0, Adam state 0. */
int sllbm_mlp_create(int n_in, int width, int depth, int n_out, uint64_t seed, sllbm_mlp *out);
void sllbm_mlp_destroy(sllbm_mlp m);
int sllbm_mlp_num_params(sllbm_mlp m, int64_t *n);
/* Copy the FP32 master parameters to / from host memory (set also resets Adam). */
int sllbm_mlp_get_params(sllbm_mlp m, float *host);
int sllbm_mlp_set_params(sllbm_mlp m, const float *host);

/* Node features of a population field (see above) into feat_bf16 (device, [N][n_feat],
 * 8-byte aligned: SLLBM_EINVAL otherwise). */
int sllbm_features(sllbm_plan p, const sllbm_params *prm, const void *pop, uint16_t *feat_bf16, void *stream);
/* y = network(x) for `rows` rows of BF16 inputs [rows][n_in] (device); y device FP32
 * [rows][n_out]. */
int sllbm_mlp_forward(sllbm_mlp m, const uint16_t *x_bf16, int64_t rows, float *y, void *stream);
/* In place on a post-collision population field of plan p: features, network, scaled and
 * projected correction added.  The network's n_in / n_out must match the plan. */
int sllbm_mlp_correct(sllbm_plan p, const sllbm_params *prm, sllbm_mlp m, void *pop, void *stream);
/* One step of the learned method: sllbm_step followed by sllbm_mlp_correct on its result,
 * with the same arguments, layouts and errors as those two calls (the network's n_in / n_out
 * must match the plan).  On 3D plans stepped by the LDS-tiled kernel the relaxation and the
 * correction share one pass over the populations: the streaming launch stores the streamed
 * values and each node's state, the node fields (rho, u, T of the post-collision state: the
 * collision keeps rho and T, Kupershtokh forcing adds F dt / rho to u) and their gradients
 * come from that state, and one launch relaxes the stored values and adds the projected
 * correction.  Elsewhere it runs the two calls. */
int sllbm_step_learned(sllbm_plan p, const sllbm_params *prm, sllbm_mlp m, const void *pop_in, void *pop_out,
                       void *stream);
/* Training targets of every node of plan p into t (device FP32 [N][2Q]). */
int sllbm_learned_targets(sllbm_plan p, const void *pop_plain, const void *pop_true, float *t, void *stream);
/* Injection of a fine population field onto a nested coarse mesh: coarse node (jx,jy,jz)
 * takes fine node (r jx, r jy, r jz).  The meshes must be nested at that ratio (checked
 * on the node coordinates: SLLBM_EINVAL otherwise), with the same velocity set and
 * precision. */
int sllbm_restrict(sllbm_plan fine, sllbm_plan coarse, int ratio, const void *pop_fine, void *pop_coarse,
                   void *stream);
/* Loss and parameter gradient over `rows` rows (inputs BF16 [rows][n_in], targets FP32
 * [rows][n_out], device), without updating: grad_host (nparams floats) and loss_host
 * optional; synchronises the stream when either is given. */
int sllbm_mlp_gradient(sllbm_mlp m, const uint16_t *x_bf16, const float *t, int64_t rows, float *grad_host,
                       float *loss_host, void *stream);
/* One training step: loss and gradient over the rows, then one Adam update of the FP32
 * master weights with learning rate lr.  loss_host optional (synchronises when given). */
int sllbm_mlp_train_step(sllbm_mlp m, const uint16_t *x_bf16, const float *t, int64_t rows, float lr,
                         float *loss_host, void *stream);

const char *sllbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SLLBM_H */
