/*
 * Oracle: plain, slow FP64 CPU reference of one time step of the compressible
 * semi-Lagrangian lattice Boltzmann method (SLLBM) of Spelten et al.,
 * arXiv 2412.09051.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
 * this file; only tests, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code with the HIP library: velocity sets, support points and
 * quadrature weights arrive from the oracle's own numpy setup (oracle/__init__.py),
 * and every formula below is written out again from the paper.
 *
 * What one step computes, for every node x_k and velocity zeta_i
 * (Sec. 3.1, SLLBM update display and the interpolation display after eq:intf):
 *   1. departure point x_DP = x_k - dt*zeta_i; walk the backward segment; the first
 *      non-periodic boundary crossed decides bounce-back / inlet / outlet
 *      (Sec. 3.3.1-3.3.3);
 *   2. evaluate the order-p Lagrange interpolant of the cell containing the departure
 *      point with the full tensor-product formula (eq:intf);
 *   3. conserved moments (eq:density, eq:momentum, energy display; total-energy
 *      reading), isothermal-wall correction (eq:thermalBC);
 *   4. BGK relaxation against the 4th-order Hermite equilibrium (f^eq and g^eq
 *      displays), optional Kupershtokh forcing (Sec. 4.3 forcing displays).
 * The state stored between steps is the post-collision population set.
 * Collision happens at the nodes and the post-collision field is interpolated; by
 * linearity this is the update display read with nodal equilibria interpolated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EGEOM -3
#define OR_EINVAL -1

#define OR_BC_PERIODIC 0
#define OR_BC_WALL 1
#define OR_BC_INLET 2
#define OR_BC_OUTLET 3

#define OR_MAXP 8
#define OR_MAXQ 128

typedef struct {
  int dim, p, Q;
  const double *zeta; /* [Q][dim] physical abscissae */
  const double *w;    /* [Q] weights */
  const int *opp;     /* [Q] index of -zeta_i */
  double T0;          /* reference temperature of the Hermite expansion */
  const double *xref; /* [p+1] support points on [-1,1], ascending */
  int ncell[3];
  const double *edges[3]; /* [ncell+1] cell boundaries per axis */
  int periodic[3];
  int face_bc[3][2];  /* boundary index per (axis, low/high face); -1 if periodic */
  int n_bc;
  const int *bc_kind;    /* [n_bc] */
  const double *bc_val;  /* [n_bc][6] rho, u0, u1, u2, T, T_wall (NaN: no thermal wall) */
  double gamma, dt;
  int relax_mode;        /* 0 constant tau_bar, 1 power-law viscosity, 2 streaming only */
  double tau_bar, mu_ref, T_ref, mu_exp;
  double force[3];
  int mass_fix;          /* 1: rescale populations to mass_ref before streaming */
  double mass_ref;
  const double *node_vol;/* [N] integral of each nodal Lagrange function */
} or_tensor;

/* ------------------------------------------------------------------------- */
/* Hermite tensors and the equilibrium (Sec. 3.1, f^eq display, N = 4)         */
/* ------------------------------------------------------------------------- */

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* Probabilists' Hermite tensors H^(n)(xi) for n = 0..4, components flattened
 * with the first index slowest.  Offsets: n=0 at 0, n=1 at 1, n=2 at 1+D, ... */
static void hermite_tensors(int D, const double *xi, double *H) {
  int o1 = 1, o2 = o1 + D, o3 = o2 + D * D, o4 = o3 + D * D * D;
  H[0] = 1.0;
  for (int a = 0; a < D; a++) H[o1 + a] = xi[a];
  for (int a = 0; a < D; a++)
    for (int b = 0; b < D; b++)
      H[o2 + a * D + b] = xi[a] * xi[b] - kd(a, b);
  for (int a = 0; a < D; a++)
    for (int b = 0; b < D; b++)
      for (int c = 0; c < D; c++)
        H[o3 + (a * D + b) * D + c] = xi[a] * xi[b] * xi[c]
            - (xi[a] * kd(b, c) + xi[b] * kd(a, c) + xi[c] * kd(a, b));
  for (int a = 0; a < D; a++)
    for (int b = 0; b < D; b++)
      for (int c = 0; c < D; c++)
        for (int d = 0; d < D; d++)
          H[o4 + ((a * D + b) * D + c) * D + d] =
              xi[a] * xi[b] * xi[c] * xi[d]
              - (xi[a] * xi[b] * kd(c, d) + xi[a] * xi[c] * kd(b, d) + xi[a] * xi[d] * kd(b, c)
                 + xi[b] * xi[c] * kd(a, d) + xi[b] * xi[d] * kd(a, c) + xi[c] * xi[d] * kd(a, b))
              + (kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c));
}

/* Hermite coefficients of the Maxwellian with density rho, velocity u and
 * temperature T, in units scaled by sqrt(T0): ut = u/sqrt(T0), th = T/T0. */
static void maxwell_coeffs(int D, double rho, const double *u, double T, double T0, double *A) {
  int o1 = 1, o2 = o1 + D, o3 = o2 + D * D, o4 = o3 + D * D * D;
  double ut[3] = {0, 0, 0};
  for (int a = 0; a < D; a++) ut[a] = u[a] / sqrt(T0);
  double t = T / T0 - 1.0;
  A[0] = rho;
  for (int a = 0; a < D; a++) A[o1 + a] = rho * ut[a];
  for (int a = 0; a < D; a++)
    for (int b = 0; b < D; b++)
      A[o2 + a * D + b] = rho * (ut[a] * ut[b] + t * kd(a, b));
  for (int a = 0; a < D; a++)
    for (int b = 0; b < D; b++)
      for (int c = 0; c < D; c++)
        A[o3 + (a * D + b) * D + c] = rho * (ut[a] * ut[b] * ut[c]
            + t * (kd(a, b) * ut[c] + kd(a, c) * ut[b] + kd(b, c) * ut[a]));
  for (int a = 0; a < D; a++)
    for (int b = 0; b < D; b++)
      for (int c = 0; c < D; c++)
        for (int d = 0; d < D; d++)
          A[o4 + ((a * D + b) * D + c) * D + d] = rho * (
              ut[a] * ut[b] * ut[c] * ut[d]
              + t * (kd(a, b) * ut[c] * ut[d] + kd(a, c) * ut[b] * ut[d] + kd(a, d) * ut[b] * ut[c]
                     + kd(b, c) * ut[a] * ut[d] + kd(b, d) * ut[a] * ut[c] + kd(c, d) * ut[a] * ut[b])
              + t * t * (kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c)));
}

static int herm_len(int D) { return 1 + D + D * D + D * D * D + D * D * D * D; }

/* f^eq_i = w_i sum_{n<=4} (1/n!) a^(n) : H^(n)_i  for all i.  Htab holds the
 * Hermite tensors of every velocity (Q * herm_len(D)). */
static void feq_all(int D, int Q, const double *w, const double *Htab, double T0,
                    double rho, const double *u, double T, double *feq) {
  double A[1 + 3 + 9 + 27 + 81];
  int L = herm_len(D);
  maxwell_coeffs(D, rho, u, T, T0, A);
  int len[5] = {1, D, D * D, D * D * D, D * D * D * D};
  double fact[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
  for (int i = 0; i < Q; i++) {
    const double *H = Htab + (size_t)i * L;
    double s = 0.0;
    int off = 0;
    for (int n = 0; n <= 4; n++) {
      double c = 0.0;
      for (int m = 0; m < len[n]; m++) c += A[off + m] * H[off + m];
      s += c / fact[n];
      off += len[n];
    }
    feq[i] = w[i] * s;
  }
}

static double *make_htab(int D, int Q, const double *zeta, double T0) {
  int L = herm_len(D);
  double *H = (double *)malloc(sizeof(double) * (size_t)Q * L);
  for (int i = 0; i < Q; i++) {
    double xi[3] = {0, 0, 0};
    for (int a = 0; a < D; a++) xi[a] = zeta[i * D + a] / sqrt(T0);
    hermite_tensors(D, xi, H + (size_t)i * L);
  }
  return H;
}

/* Public: equilibrium of one state for every velocity; g^eq = T (2 c_v - D) f^eq
 * with c_v = 1/(gamma-1) (g^eq display). */
int or_equilibrium(int D, int Q, const double *zeta, const double *w, double T0, double gamma,
                   double rho, const double *u, double T, double *feq, double *geq) {
  double *H = make_htab(D, Q, zeta, T0);
  feq_all(D, Q, w, H, T0, rho, u, T, feq);
  double cv = 1.0 / (gamma - 1.0);
  if (geq)
    for (int i = 0; i < Q; i++) geq[i] = T * (2.0 * cv - D) * feq[i];
  free(H);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Tensor-product mesh geometry                                                */
/* ------------------------------------------------------------------------- */

static int axis_nodes(const or_tensor *m, int a) {
  return m->ncell[a] * m->p + (m->periodic[a] ? 0 : 1);
}

static double node_coord(const or_tensor *m, int a, int n) {
  int p = m->p;
  int c = n / p, b = n % p;
  if (c == m->ncell[a]) return m->edges[a][m->ncell[a]];
  double lo = m->edges[a][c], hi = m->edges[a][c + 1];
  return lo + 0.5 * (1.0 + m->xref[b]) * (hi - lo);
}

/* Lagrange basis l_j(xi) = prod_{m != j} (xi - x_m)/(x_j - x_m)  (eq:intf). */
static void lagrange(int p, const double *xref, double xi, double *l) {
  for (int j = 0; j <= p; j++) {
    double v = 1.0;
    for (int q = 0; q <= p; q++)
      if (q != j) v *= (xi - xref[q]) / (xref[j] - xref[q]);
    l[j] = v;
  }
}

/* Locate coordinate x (already inside [lo,hi]) on axis a: cell index and
 * reference coordinate.  A point on an interior face takes the larger cell.
 * A point that equals a support point gets that point's exact reference
 * coordinate, so the interpolant returns the nodal value. */
static void locate_axis(const or_tensor *m, int a, double x, int *cell, double *xi) {
  int n = m->ncell[a];
  const double *e = m->edges[a];
  int lo = 0, hi = n; /* invariant: e[lo] <= x, answer in [lo, hi) */
  if (x < e[0]) x = e[0];
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (e[mid] <= x) lo = mid; else hi = mid;
  }
  int c = lo;
  double h = e[c + 1] - e[c];
  double r = 2.0 * (x - e[c]) / h - 1.0;
  for (int j = 0; j <= m->p; j++) {
    double xn = e[c] + 0.5 * (1.0 + m->xref[j]) * h;
    if (j == m->p) xn = e[c + 1];
    if (x == xn) { r = m->xref[j]; break; }
  }
  *cell = c;
  *xi = r;
}

typedef struct {
  int kind;     /* 0: interpolate; 1: inlet equilibrium */
  int src;      /* source velocity */
  double dp[3]; /* departure point to interpolate at */
  int bc;       /* boundary index that decided the case, -1 none */
  int thermal;  /* 1 if a thermal wall was hit */
} or_trace;

static double wrap(double x, double lo, double hi) {
  double L = hi - lo;
  while (x < lo) x += L;
  while (x >= hi) x -= L;
  return x;
}

static int inside_nonperiodic(const or_tensor *m, const double *x) {
  for (int a = 0; a < m->dim; a++) {
    if (m->periodic[a]) continue;
    if (x[a] < m->edges[a][0] || x[a] > m->edges[a][m->ncell[a]]) return 0;
  }
  return 1;
}

/* Walk the backward segment x_k -> x_k - dt zeta_i; the first non-periodic face
 * crossed decides the boundary case (Sec. 3.3).  A departure point exactly on a
 * face counts as inside. */
static int trace(const or_tensor *m, const double *xk, int i, or_trace *t) {
  int D = m->dim;
  double d[3] = {0, 0, 0};
  for (int a = 0; a < D; a++) d[a] = m->dt * m->zeta[i * D + a];
  double best = 2.0;
  int ba = -1, bs = 0;
  for (int a = 0; a < D; a++) {
    if (m->periodic[a] || d[a] == 0.0) continue;
    double lo = m->edges[a][0], hi = m->edges[a][m->ncell[a]];
    double end = xk[a] - d[a];
    double s = 2.0;
    int side = 0;
    if (end < lo) { s = (xk[a] - lo) / d[a]; side = 0; }
    else if (end > hi) { s = (xk[a] - hi) / d[a]; side = 1; }
    if (s < best) { best = s; ba = a; bs = side; }
  }
  t->thermal = 0;
  t->bc = -1;
  if (ba < 0) {
    t->kind = 0;
    t->src = i;
    for (int a = 0; a < D; a++) t->dp[a] = xk[a] - d[a];
  } else {
    int bc = m->face_bc[ba][bs];
    int kind = m->bc_kind[bc];
    t->bc = bc;
    if (kind == OR_BC_WALL) {
      /* Sec. 3.3.2: wall point x_W = x_k - s dt zeta_i, remaining path iota =
       * dt zeta_i - (x_k - x_W) travelled back from the wall, opposite population. */
      double s = best;
      t->kind = 0;
      t->src = m->opp[i];
      for (int a = 0; a < D; a++) {
        double xw = xk[a] - s * d[a];
        double iota = d[a] - (xk[a] - xw);
        t->dp[a] = xw + iota;
      }
      /* the wall-normal coordinate is mathematically inside; absorb rounding */
      for (int a = 0; a < D; a++) {
        if (m->periodic[a]) continue;
        double lo = m->edges[a][0], hi = m->edges[a][m->ncell[a]], tol = 1e-12 * (hi - lo);
        if (t->dp[a] < lo && t->dp[a] > lo - tol) t->dp[a] = lo;
        if (t->dp[a] > hi && t->dp[a] < hi + tol) t->dp[a] = hi;
      }
      if (!inside_nonperiodic(m, t->dp)) return OR_EGEOM;
      if (!isnan(m->bc_val[bc * 6 + 5])) t->thermal = 1;
    } else if (kind == OR_BC_INLET) {
      t->kind = 1;
      t->src = i;
    } else if (kind == OR_BC_OUTLET) {
      /* Sec. 3.3.3: restart from the arrival point in the opposite direction. */
      t->kind = 0;
      t->src = i;
      double sf = 1.0;
      for (int a = 0; a < D; a++) {
        if (m->periodic[a] || d[a] == 0.0) continue;
        double lo = m->edges[a][0], hi = m->edges[a][m->ncell[a]];
        double end = xk[a] + d[a];
        if (end > hi) { double f = (hi - xk[a]) / d[a]; if (f < sf) sf = f; }
        if (end < lo) { double f = (lo - xk[a]) / d[a]; if (f < sf) sf = f; }
      }
      for (int a = 0; a < D; a++) t->dp[a] = xk[a] + sf * d[a];
    } else {
      return OR_EINVAL;
    }
  }
  for (int a = 0; a < D; a++)
    if (m->periodic[a]) t->dp[a] = wrap(t->dp[a], m->edges[a][0], m->edges[a][m->ncell[a]]);
  return OR_OK;
}

/* Full tensor-product Lagrange interpolation of one population field at x (eq:intf). */
static double interp(const or_tensor *m, const double *field, const double *x, const int *Nax) {
  int D = m->dim, p = m->p;
  int cell[3] = {0, 0, 0};
  double l[3][OR_MAXP + 1];
  for (int a = 0; a < 3; a++)
    for (int j = 0; j <= p; j++) l[a][j] = (j == 0) ? 1.0 : 0.0;
  for (int a = 0; a < D; a++) {
    double xi;
    locate_axis(m, a, x[a], &cell[a], &xi);
    lagrange(p, m->xref, xi, l[a]);
  }
  int nz = (D == 3) ? p + 1 : 1;
  double v = 0.0;
  for (int jz = 0; jz < nz; jz++)
    for (int jy = 0; jy <= p; jy++)
      for (int jx = 0; jx <= p; jx++) {
        int n[3] = {cell[0] * p + jx, cell[1] * p + jy, (D == 3) ? cell[2] * p + jz : 0};
        for (int a = 0; a < D; a++)
          if (m->periodic[a]) n[a] %= Nax[a];
        size_t k = (size_t)n[0] + (size_t)Nax[0] * ((size_t)n[1] + (size_t)Nax[1] * (size_t)n[2]);
        double wgt = l[0][jx] * l[1][jy] * (D == 3 ? l[2][jz] : 1.0);
        v += wgt * field[k];
      }
  return v;
}

static void node_xyz(const or_tensor *m, const int *Nax, size_t k, double *x) {
  size_t r = k;
  int n[3] = {0, 0, 0};
  for (int a = 0; a < m->dim; a++) { n[a] = (int)(r % (size_t)Nax[a]); r /= (size_t)Nax[a]; }
  for (int a = 0; a < 3; a++) x[a] = (a < m->dim) ? node_coord(m, a, n[a]) : 0.0;
}

size_t or_tensor_num_nodes(const or_tensor *m) {
  size_t N = 1;
  for (int a = 0; a < m->dim; a++) N *= (size_t)axis_nodes(m, a);
  return N;
}

int or_tensor_coords(const or_tensor *m, double *xyz) {
  int Nax[3] = {1, 1, 1};
  for (int a = 0; a < m->dim; a++) Nax[a] = axis_nodes(m, a);
  size_t N = or_tensor_num_nodes(m);
  for (size_t k = 0; k < N; k++) {
    double x[3];
    node_xyz(m, Nax, k, x);
    for (int a = 0; a < m->dim; a++) xyz[k * m->dim + a] = x[a];
  }
  return OR_OK;
}

/* Conserved moments of one node (eq:density, eq:momentum, energy display read as
 * total energy: sum(|zeta|^2 f + g) = rho|u|^2 + 2 rho c_v T). */
static void node_moments(int D, int Q, const double *zeta, double cv, const double *f, const double *g,
                         double *rho, double *u, double *T) {
  double r = 0, j[3] = {0, 0, 0}, E = 0;
  for (int i = 0; i < Q; i++) {
    double z2 = 0;
    r += f[i];
    for (int a = 0; a < D; a++) { j[a] += zeta[i * D + a] * f[i]; z2 += zeta[i * D + a] * zeta[i * D + a]; }
    E += z2 * f[i] + g[i];
  }
  double uu = 0;
  for (int a = 0; a < 3; a++) { u[a] = (a < D) ? j[a] / r : 0.0; uu += u[a] * u[a]; }
  *rho = r;
  *T = (E - r * uu) / (2.0 * r * cv);
}

/* Post-collision populations of one node k (f into fo[Q], g into go[Q]) from the
 * (already rescaled) input set src. */
static int node_update(const or_tensor *m, const double *H, const int *Nax, const double *src,
                       const double *inlet, size_t k, double *fo, double *go, int64_t *bad_i) {
  int D = m->dim, Q = m->Q;
  size_t N = or_tensor_num_nodes(m);
  double cv = 1.0 / (m->gamma - 1.0);
  double xk[3];
  node_xyz(m, Nax, k, xk);
  double fs[OR_MAXQ], gs[OR_MAXQ], fe[OR_MAXQ], fe2[OR_MAXQ];
  int thermal = 0;
  double Tw = 0.0;
  for (int i = 0; i < Q; i++) {
    or_trace t;
    int rc = trace(m, xk, i, &t);
    if (rc != OR_OK) { *bad_i = i; return rc; }
    if (t.kind == 1) {
      fs[i] = inlet[(size_t)t.bc * 2 * Q + i];
      gs[i] = inlet[(size_t)t.bc * 2 * Q + Q + i];
    } else {
      fs[i] = interp(m, src + (size_t)t.src * N, t.dp, Nax);
      gs[i] = interp(m, src + ((size_t)Q + t.src) * N, t.dp, Nax);
    }
    if (t.thermal) { thermal = 1; Tw = m->bc_val[t.bc * 6 + 5]; }
  }
  double rho, u[3], T;
  node_moments(D, Q, m->zeta, cv, fs, gs, &rho, u, &T);
  if (thermal) {
    /* eq:thermalBC: f_i += f^eq_i(rho,u,T_w) - f^eq_i(rho,u,T), same for g with
     * g^eq; afterwards the node temperature is T_w. */
    feq_all(D, Q, m->w, H, m->T0, rho, u, Tw, fe);
    feq_all(D, Q, m->w, H, m->T0, rho, u, T, fe2);
    for (int i = 0; i < Q; i++) {
      fs[i] += fe[i] - fe2[i];
      gs[i] += Tw * (2.0 * cv - D) * fe[i] - T * (2.0 * cv - D) * fe2[i];
    }
    T = Tw;
  }
  if (m->relax_mode == 2) {
    for (int i = 0; i < Q; i++) { fo[i] = fs[i]; go[i] = gs[i]; }
    return OR_OK;
  }
  /* Relaxation time: tau = mu/p with p = rho R T, R = 1, as a dimensionless
   * tau_bar = tau/dt + 1/2 (Sec. 3.1; reading of the units). */
  double tb = m->tau_bar;
  if (m->relax_mode == 1) {
    double mu = m->mu_ref * pow(T / m->T_ref, m->mu_exp);
    tb = mu / (rho * T * m->dt) + 0.5;
  }
  feq_all(D, Q, m->w, H, m->T0, rho, u, T, fe);
  double gfac = T * (2.0 * cv - D);
  for (int i = 0; i < Q; i++) {
    fo[i] = fs[i] - (fs[i] - fe[i]) / tb;
    go[i] = gs[i] - (gs[i] - gfac * fe[i]) / tb;
  }
  int has_force = 0;
  for (int a = 0; a < D; a++) if (m->force[a] != 0.0) has_force = 1;
  if (has_force) {
    /* Kupershtokh exact difference: delta h_i = h^eq(rho,u+du,T) - h^eq(rho,u,T),
     * du = F dt / rho, added after the collision. */
    double u2[3] = {u[0], u[1], u[2]};
    for (int a = 0; a < D; a++) u2[a] += m->force[a] * m->dt / rho;
    feq_all(D, Q, m->w, H, m->T0, rho, u2, T, fe2);
    for (int i = 0; i < Q; i++) {
      fo[i] += fe2[i] - fe[i];
      go[i] += gfac * (fe2[i] - fe[i]);
    }
  }
  return OR_OK;
}

/* Input set for streaming: pin itself, or a copy rescaled by mass_ref / M (Sec. 4.3,
 * mass-loss remedy) with M = sum_k V_k rho_k, V_k the integral of the nodal basis. */
static double *prepare_source(const or_tensor *m, const double *pin) {
  if (!m->mass_fix) return NULL;
  size_t N = or_tensor_num_nodes(m);
  int Q = m->Q;
  double M = 0.0;
  for (size_t k = 0; k < N; k++) {
    double r = 0;
    for (int i = 0; i < Q; i++) r += pin[(size_t)i * N + k];
    M += m->node_vol[k] * r;
  }
  double c = m->mass_ref / M;
  double *scaled = (double *)malloc(sizeof(double) * 2 * (size_t)Q * N);
  for (size_t q = 0; q < 2 * (size_t)Q * N; q++) scaled[q] = c * pin[q];
  return scaled;
}

/* Equilibria of the inlet states (Sec. 3.3.1). */
static double *inlet_table(const or_tensor *m, const double *H) {
  int D = m->dim, Q = m->Q;
  double cv = 1.0 / (m->gamma - 1.0);
  double *inlet = (double *)calloc((size_t)(m->n_bc > 0 ? m->n_bc : 1) * 2 * Q, sizeof(double));
  for (int b = 0; b < m->n_bc; b++) {
    if (m->bc_kind[b] != OR_BC_INLET) continue;
    const double *v = m->bc_val + b * 6;
    feq_all(D, Q, m->w, H, m->T0, v[0], v + 1, v[4], inlet + (size_t)b * 2 * Q);
    for (int i = 0; i < Q; i++)
      inlet[(size_t)b * 2 * Q + Q + i] = v[4] * (2.0 * cv - D) * inlet[(size_t)b * 2 * Q + i];
  }
  return inlet;
}

/* One SLLBM time step on a tensor-product mesh.  pop layout: [(s*Q + i)*N + k],
 * s = 0 for f, 1 for g.  On a geometry error the offending node and velocity are
 * written to err[0], err[1]. */
int or_tensor_step(const or_tensor *m, const double *pin, double *pout, int64_t *err) {
  int D = m->dim, Q = m->Q;
  int Nax[3] = {1, 1, 1};
  for (int a = 0; a < D; a++) Nax[a] = axis_nodes(m, a);
  size_t N = or_tensor_num_nodes(m);
  double *H = make_htab(D, Q, m->zeta, m->T0);
  double *scaled = prepare_source(m, pin);
  const double *src = scaled ? scaled : pin;
  double *inlet = inlet_table(m, H);
  int status = OR_OK;
  int64_t ek = -1, ei = -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (size_t k = 0; k < N; k++) {
    if (status != OR_OK) continue;
    double fo[OR_MAXQ], go[OR_MAXQ];
    int64_t bi = -1;
    int rc = node_update(m, H, Nax, src, inlet, k, fo, go, &bi);
    if (rc != OR_OK) {
#pragma omp critical
      { status = rc; ek = (int64_t)k; ei = bi; }
      continue;
    }
    for (int i = 0; i < Q; i++) {
      pout[(size_t)i * N + k] = fo[i];
      pout[((size_t)Q + i) * N + k] = go[i];
    }
  }
  if (err) { err[0] = ek; err[1] = ei; }
  free(inlet);
  free(scaled);
  free(H);
  return status;
}

/* The same step evaluated at a list of nodes only: out[j][2Q] (f then g) for node
 * nodes[j].  Used to check large runs at sampled nodes. */
int or_tensor_step_nodes(const or_tensor *m, const double *pin, const int64_t *nodes, int64_t n, double *out,
                         int64_t *err) {
  int D = m->dim, Q = m->Q;
  int Nax[3] = {1, 1, 1};
  for (int a = 0; a < D; a++) Nax[a] = axis_nodes(m, a);
  double *H = make_htab(D, Q, m->zeta, m->T0);
  double *scaled = prepare_source(m, pin);
  const double *src = scaled ? scaled : pin;
  double *inlet = inlet_table(m, H);
  int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < n; j++) {
    if (status != OR_OK) continue;
    int64_t bi = -1;
    int rc = node_update(m, H, Nax, src, inlet, (size_t)nodes[j], out + (size_t)j * 2 * Q,
                         out + (size_t)j * 2 * Q + Q, &bi);
    if (rc != OR_OK) {
#pragma omp critical
      { status = rc; if (err) { err[0] = nodes[j]; err[1] = bi; } }
    }
  }
  free(inlet);
  free(scaled);
  free(H);
  return status;
}

/* Populations from nodal (rho, u, T): f = f^eq, g = g^eq. */
int or_tensor_init(const or_tensor *m, const double *rho, const double *u, const double *T, double *pop) {
  int D = m->dim, Q = m->Q;
  size_t N = or_tensor_num_nodes(m);
  double cv = 1.0 / (m->gamma - 1.0);
  double *H = make_htab(D, Q, m->zeta, m->T0);
#pragma omp parallel for
  for (size_t k = 0; k < N; k++) {
    double fe[OR_MAXQ], uk[3] = {0, 0, 0};
    for (int a = 0; a < D; a++) uk[a] = u[k * D + a];
    feq_all(D, Q, m->w, H, m->T0, rho[k], uk, T[k], fe);
    for (int i = 0; i < Q; i++) {
      pop[(size_t)i * N + k] = fe[i];
      pop[((size_t)Q + i) * N + k] = T[k] * (2.0 * cv - D) * fe[i];
    }
  }
  free(H);
  return OR_OK;
}

/* Nodal rho, u, T of a population set (generic: N nodes, any mesh). */
int or_moments(int D, int Q, const double *zeta, double gamma, size_t N, const double *pop,
               double *rho, double *u, double *T) {
  double cv = 1.0 / (gamma - 1.0);
#pragma omp parallel for
  for (size_t k = 0; k < N; k++) {
    double f[OR_MAXQ], g[OR_MAXQ], uk[3];
    for (int i = 0; i < Q; i++) { f[i] = pop[(size_t)i * N + k]; g[i] = pop[((size_t)Q + i) * N + k]; }
    node_moments(D, Q, zeta, cv, f, g, &rho[k], uk, &T[k]);
    for (int a = 0; a < D; a++) u[k * D + a] = uk[a];
  }
  return OR_OK;
}
