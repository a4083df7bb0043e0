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
 *      displays), the quasi-equilibrium term for Pr != 1 (add_quasi_eq), optional
 *      Kupershtokh forcing (Sec. 4.3 forcing displays).
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
  double Pr;             /* Prandtl number (1: no quasi-equilibrium term) */
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
      /* a reflected point outside the box (rounding, a channel thinner than the path,
       * a corner) is replaced by its nearest point of the box */
      for (int a = 0; a < D; a++) {
        if (m->periodic[a]) continue;
        double lo = m->edges[a][0], hi = m->edges[a][m->ncell[a]];
        if (t->dp[a] < lo) t->dp[a] = lo;
        if (t->dp[a] > hi) t->dp[a] = hi;
      }
      if (!isnan(m->bc_val[bc * 6 + 5])) t->thermal = 1;
    } else if (kind == OR_BC_INLET) {
      t->kind = 1;
      t->src = i;
    } else if (kind == OR_BC_OUTLET) {
      /* Sec. 3.3.3: restart from the arrival point in the opposite direction, i.e.
       * population i at x_k + dt zeta_i; should that point lie outside the box too,
       * its nearest point of the box (each bounded coordinate clamped). */
      t->kind = 0;
      t->src = i;
      for (int a = 0; a < D; a++) {
        t->dp[a] = xk[a] + d[a];
        if (m->periodic[a]) continue;
        double lo = m->edges[a][0], hi = m->edges[a][m->ncell[a]];
        if (t->dp[a] < lo) t->dp[a] = lo;
        if (t->dp[a] > hi) t->dp[a] = hi;
      }
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

/* Quasi-equilibrium term of the collision (Sec. 3.1 update display: h gains
 * (1/tau - 1/tau_Pr) h*, tau_Pr = (tau - 1/2)/Pr + 1/2).  The paper defers h* to its
 * references; reading: the lowest-order Hermite terms that carry the node's heat flux and
 * no moment of order <= 2, so that the heat flux relaxes with tau_Pr and the stress with
 * tau.  With c = zeta - u, q_f = 1/2 sum_i c |c|^2 f_i and q_g = 1/2 sum_i c g_i (the
 * equilibria carry none):
 *   f*_i = w_i (q_f . zeta_i)(|zeta_i|^2 - (D+2) T0) / ((D+2) T0^3),
 *   g*_i = 2 w_i (q_g . zeta_i) / T0.
 * Adds coef * f*_i to fo[i] and coef * g*_i to go[i]. */
static void add_quasi_eq(int D, int Q, const double *zeta, const double *w, double T0, const double *u,
                         const double *fs, const double *gs, double coef, double *fo, double *go) {
  double qf[3] = {0.0, 0.0, 0.0}, qg[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; i++) {
    double c[3] = {0.0, 0.0, 0.0}, c2 = 0.0;
    for (int a = 0; a < D; a++) {
      c[a] = zeta[i * D + a] - u[a];
      c2 += c[a] * c[a];
    }
    for (int a = 0; a < D; a++) {
      qf[a] += 0.5 * c[a] * c2 * fs[i];
      qg[a] += 0.5 * c[a] * gs[i];
    }
  }
  for (int i = 0; i < Q; i++) {
    double z2 = 0.0, qfz = 0.0, qgz = 0.0;
    for (int a = 0; a < D; a++) {
      double z = zeta[i * D + a];
      z2 += z * z;
      qfz += qf[a] * z;
      qgz += qg[a] * z;
    }
    fo[i] += coef * w[i] * qfz * (z2 - (D + 2) * T0) / ((D + 2) * T0 * T0 * T0);
    go[i] += coef * 2.0 * w[i] * qgz / T0;
  }
}

/* 1/tau_bar - 1/tau_bar_Pr with tau_bar_Pr = (tau_bar - 1/2)/Pr + 1/2 (Sec. 3.1). */
static double pr_coef(double tb, double Pr) {
  return 1.0 / tb - 1.0 / ((tb - 0.5) / Pr + 0.5);
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
  if (m->Pr != 1.0) add_quasi_eq(D, Q, m->zeta, m->w, m->T0, u, fs, gs, pr_coef(tb, m->Pr), fo, go);
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

/* ========================================================================= */
/* Curvilinear (isoparametric quadrilateral) meshes, dim = 2                   */
/* ========================================================================= */

typedef struct {
  int p, Q;
  const double *zeta, *w;
  const int *opp;
  double T0;
  const double *xref;
  int64_t n_nodes;
  const double *xyz;        /* [n_nodes][2] */
  int64_t n_cells;
  const int64_t *cell_nodes;/* [n_cells][(p+1)^2], xi fastest */
  const int *face_bc;       /* [n_cells][4]: xi-, xi+, eta-, eta+ ; -1 interior */
  int n_bc;
  const int *bc_kind;
  const double *bc_val;     /* [n_bc][6] */
  double gamma, dt;
  int relax_mode;
  double tau_bar, mu_ref, T_ref, mu_exp;
  double force[2];
  int mass_fix;
  double mass_ref;
  const double *node_vol;
  double Pr;
  /* bucket grid over cell bounding boxes (built by or_curv_prepare) */
  double bx0, by0, bh;
  int bnx, bny;
  int64_t *bstart, *bcells;
} or_curv;

/* derivative of the Lagrange basis, product rule */
static void lagrange_d(int p, const double *xref, double xi, double *dl) {
  for (int j = 0; j <= p; j++) {
    double s = 0.0;
    for (int k = 0; k <= p; k++) {
      if (k == j) continue;
      double t = 1.0 / (xref[j] - xref[k]);
      for (int q = 0; q <= p; q++)
        if (q != j && q != k) t *= (xi - xref[q]) / (xref[j] - xref[q]);
      s += t;
    }
    dl[j] = s;
  }
}

/* isoparametric map x(xi, eta) = sum_j X_j l_jx(xi) l_jy(eta) and its Jacobian */
static void cell_map(const or_curv *m, int64_t c, double xi, double eta, double *x, double J[2][2]) {
  int p = m->p, n1 = p + 1;
  double lx[OR_MAXP + 1], ly[OR_MAXP + 1], dx[OR_MAXP + 1], dy[OR_MAXP + 1];
  lagrange(p, m->xref, xi, lx);
  lagrange(p, m->xref, eta, ly);
  lagrange_d(p, m->xref, xi, dx);
  lagrange_d(p, m->xref, eta, dy);
  x[0] = x[1] = 0;
  J[0][0] = J[0][1] = J[1][0] = J[1][1] = 0;
  const int64_t *cn = m->cell_nodes + c * n1 * n1;
  for (int jy = 0; jy <= p; jy++)
    for (int jx = 0; jx <= p; jx++) {
      const double *X = m->xyz + 2 * cn[jx + n1 * jy];
      for (int a = 0; a < 2; a++) {
        x[a] += X[a] * lx[jx] * ly[jy];
        J[a][0] += X[a] * dx[jx] * ly[jy];
        J[a][1] += X[a] * lx[jx] * dy[jy];
      }
    }
}

#define OR_CURV_TOL 1e-10

/* Newton iteration for x(xi) = x in cell c from reference point r0 (steps damped to
 * 0.5); returns 1 and the converged point if it converged. */
static int cell_newton(const or_curv *m, int64_t c, const double *x, const double *r0, double *r) {
  r[0] = r0[0];
  r[1] = r0[1];
  for (int it = 0; it < 60; it++) {
    double X[2], J[2][2];
    cell_map(m, c, r[0], r[1], X, J);
    double e0 = x[0] - X[0], e1 = x[1] - X[1];
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (det == 0.0) return 0;
    double d0 = (J[1][1] * e0 - J[0][1] * e1) / det;
    double d1 = (-J[1][0] * e0 + J[0][0] * e1) / det;
    double sz = fabs(d0) > fabs(d1) ? fabs(d0) : fabs(d1);
    if (sz > 0.5) { d0 *= 0.5 / sz; d1 *= 0.5 / sz; }
    r[0] += d0;
    r[1] += d1;
    if (fabs(r[0]) > 4.0 || fabs(r[1]) > 4.0) return 0;
    if (fabs(d0) + fabs(d1) < 1e-11) {
      /* quadratic convergence: two more corrections reach the rounding level, which
       * in a thin cell can itself be ~1e-13 in reference units */
      for (int extra = 0; extra < 2; extra++) {
        cell_map(m, c, r[0], r[1], X, J);
        e0 = x[0] - X[0];
        e1 = x[1] - X[1];
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (det == 0.0) return 0;
        r[0] += (J[1][1] * e0 - J[0][1] * e1) / det;
        r[1] += (-J[1][0] * e0 + J[0][0] * e1) / det;
      }
      return 1;
    }
  }
  return 0; /* no convergence from this start */
}

static int in_ref_square(const double *r) {
  return fabs(r[0]) <= 1.0 + OR_CURV_TOL && fabs(r[1]) <= 1.0 + OR_CURV_TOL;
}

/* Inverse of the isoparametric map of cell c; 1 if x lies in the cell (reference
 * coordinates within 1e-10 of [-1,1]^2).  Starts from the support point nearest to x,
 * then from a 3x3 grid of reference points. */
static int cell_inverse(const or_curv *m, int64_t c, const double *x, double *xi) {
  int n1 = m->p + 1;
  const int64_t *cn = m->cell_nodes + c * n1 * n1;
  double best = 1e300, r0[2] = {0, 0}, r[2];
  for (int jy = 0; jy <= m->p; jy++)
    for (int jx = 0; jx <= m->p; jx++) {
      const double *X = m->xyz + 2 * cn[jx + n1 * jy];
      double d = (X[0] - x[0]) * (X[0] - x[0]) + (X[1] - x[1]) * (X[1] - x[1]);
      if (d < best) { best = d; r0[0] = m->xref[jx]; r0[1] = m->xref[jy]; }
      if (d == 0.0) {  /* a support point: its exact reference coordinates */
        xi[0] = m->xref[jx];
        xi[1] = m->xref[jy];
        return 1;
      }
    }
  /* a start may converge to a root of the polynomial map outside the cell (or not
   * at all, near a degenerate corner): then the next start is tried */
  int ok = cell_newton(m, c, x, r0, r) && in_ref_square(r);
  for (int t = 0; !ok && t < 9; t++) {
    double s0[2] = {-0.6 + 0.6 * (t % 3), -0.6 + 0.6 * (t / 3)};
    ok = cell_newton(m, c, x, s0, r) && in_ref_square(r);
  }
  if (!ok) return 0;
  xi[0] = r[0] < -1.0 ? -1.0 : (r[0] > 1.0 ? 1.0 : r[0]);
  xi[1] = r[1] < -1.0 ? -1.0 : (r[1] > 1.0 ? 1.0 : r[1]);
  return 1;
}

int or_curv_prepare(or_curv *m, double cell_size) {
  /* uniform bucket grid of width cell_size over all cell bounding boxes */
  int n1 = m->p + 1;
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int64_t k = 0; k < m->n_nodes; k++) {
    double X = m->xyz[2 * k], Y = m->xyz[2 * k + 1];
    if (X < x0) x0 = X;
    if (X > x1) x1 = X;
    if (Y < y0) y0 = Y;
    if (Y > y1) y1 = Y;
  }
  m->bh = cell_size;
  m->bx0 = x0 - cell_size;
  m->by0 = y0 - cell_size;
  m->bnx = (int)((x1 - m->bx0) / cell_size) + 2;
  m->bny = (int)((y1 - m->by0) / cell_size) + 2;
  int64_t nb = (int64_t)m->bnx * m->bny;
  int64_t *cnt = (int64_t *)calloc(nb + 1, sizeof(int64_t));
  /* a cell's box: its support points' box, widened by 5% for curved edges */
  for (int pass = 0; pass < 2; pass++) {
    for (int64_t c = 0; c < m->n_cells; c++) {
      double cx0 = 1e300, cx1 = -1e300, cy0 = 1e300, cy1 = -1e300;
      for (int j = 0; j < n1 * n1; j++) {
        const double *X = m->xyz + 2 * m->cell_nodes[c * n1 * n1 + j];
        if (X[0] < cx0) cx0 = X[0];
        if (X[0] > cx1) cx1 = X[0];
        if (X[1] < cy0) cy0 = X[1];
        if (X[1] > cy1) cy1 = X[1];
      }
      double gx = 0.05 * (cx1 - cx0) + 1e-12, gy = 0.05 * (cy1 - cy0) + 1e-12;
      int i0 = (int)((cx0 - gx - m->bx0) / cell_size), i1 = (int)((cx1 + gx - m->bx0) / cell_size);
      int j0 = (int)((cy0 - gy - m->by0) / cell_size), j1 = (int)((cy1 + gy - m->by0) / cell_size);
      for (int bj = j0; bj <= j1; bj++)
        for (int bi = i0; bi <= i1; bi++) {
          if (bi < 0 || bj < 0 || bi >= m->bnx || bj >= m->bny) continue;
          int64_t b = (int64_t)bj * m->bnx + bi;
          if (pass == 0) cnt[b + 1]++;
          else m->bcells[m->bstart[b] + cnt[b]++] = c;
        }
    }
    if (pass == 0) {
      m->bstart = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
      m->bstart[0] = 0;
      for (int64_t b = 0; b < nb; b++) m->bstart[b + 1] = m->bstart[b] + cnt[b + 1];
      m->bcells = (int64_t *)malloc(sizeof(int64_t) * (m->bstart[nb] + 1));
      memset(cnt, 0, sizeof(int64_t) * (nb + 1));
    }
  }
  free(cnt);
  return OR_OK;
}

void or_curv_release(or_curv *m) {
  free(m->bstart);
  free(m->bcells);
  m->bstart = m->bcells = NULL;
}

/* cell containing x (the largest cell index on shared faces), -1 if outside */
static int64_t curv_locate(const or_curv *m, const double *x, double *xi) {
  int bi = (int)((x[0] - m->bx0) / m->bh), bj = (int)((x[1] - m->by0) / m->bh);
  if (bi < 0 || bj < 0 || bi >= m->bnx || bj >= m->bny) return -1;
  int64_t b = (int64_t)bj * m->bnx + bi, best = -1;
  double r[2];
  int n1 = m->p + 1;
  for (int64_t q = m->bstart[b]; q < m->bstart[b + 1]; q++) {
    int64_t c = m->bcells[q];
    if (c <= best) continue;
    /* bounding box of the support points, widened by 5% for curved edges */
    double cx0 = 1e300, cx1 = -1e300, cy0 = 1e300, cy1 = -1e300;
    for (int j = 0; j < n1 * n1; j++) {
      const double *X = m->xyz + 2 * m->cell_nodes[c * n1 * n1 + j];
      if (X[0] < cx0) cx0 = X[0];
      if (X[0] > cx1) cx1 = X[0];
      if (X[1] < cy0) cy0 = X[1];
      if (X[1] > cy1) cy1 = X[1];
    }
    double gx = 0.05 * (cx1 - cx0) + 1e-12, gy = 0.05 * (cy1 - cy0) + 1e-12;
    if (x[0] < cx0 - gx || x[0] > cx1 + gx || x[1] < cy0 - gy || x[1] > cy1 + gy) continue;
    if (cell_inverse(m, c, x, r)) { best = c; xi[0] = r[0]; xi[1] = r[1]; }
  }
  return best;
}

/* Point and tangent of face f of cell c at face parameter t. */
static void face_curve(const or_curv *m, int64_t c, int f, double t, double *x, double *dx) {
  int p = m->p, n1 = p + 1;
  double l[OR_MAXP + 1], dl[OR_MAXP + 1];
  lagrange(p, m->xref, t, l);
  lagrange_d(p, m->xref, t, dl);
  x[0] = x[1] = dx[0] = dx[1] = 0.0;
  for (int j = 0; j <= p; j++) {
    int jx = f == 0 ? 0 : (f == 1 ? p : j), jy = f == 2 ? 0 : (f == 3 ? p : j);
    const double *X = m->xyz + 2 * m->cell_nodes[c * n1 * n1 + jx + n1 * jy];
    for (int a = 0; a < 2; a++) {
      x[a] += X[a] * l[j];
      dx[a] += X[a] * dl[j];
    }
  }
}

/* Nearest point of the mesh boundary to y, over every tagged face: each face sampled at
 * 65 parameters, then the sign change of d|face(t) - y|^2/dt next to the best sample
 * bisected.  Returns the cell, with y's projection in its reference coordinates. */
static int64_t curv_project(const or_curv *m, const double *y, double *xi) {
  double best = 1e300;
  int64_t cb = -1;
  for (int64_t c = 0; c < m->n_cells; c++)
    for (int f = 0; f < 4; f++) {
      if (m->face_bc[c * 4 + f] < 0) continue;
      int jb = 0;
      double db = 1e300, x[2], dx[2];
      for (int j = 0; j <= 64; j++) {
        face_curve(m, c, f, -1.0 + j / 32.0, x, dx);
        double dd = (x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]);
        if (dd < db) { db = dd; jb = j; }
      }
      double t = -1.0 + jb / 32.0;
      if (db < best * 4.0 + 1e-30) {
        /* derivative of the squared distance, h(t) = (face(t) - y) . face'(t) */
        double lo = t - 1.0 / 32.0, hi = t + 1.0 / 32.0, hl, hh;
        if (lo < -1.0) lo = -1.0;
        if (hi > 1.0) hi = 1.0;
        face_curve(m, c, f, lo, x, dx);
        hl = (x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1];
        face_curve(m, c, f, hi, x, dx);
        hh = (x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1];
        if (hl < 0.0 && hh > 0.0) {
          for (int it = 0; it < 100; it++) {
            double mid = 0.5 * (lo + hi);
            face_curve(m, c, f, mid, x, dx);
            if ((x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1] < 0.0) lo = mid; else hi = mid;
          }
          t = 0.5 * (lo + hi);
        } else {
          t = hl >= 0.0 ? lo : hi;   /* the minimum sits at an end of the bracket */
        }
        face_curve(m, c, f, t, x, dx);
        double dd = (x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]);
        if (dd < best) {
          best = dd;
          cb = c;
          xi[0] = f == 0 ? -1.0 : (f == 1 ? 1.0 : t);
          xi[1] = f == 2 ? -1.0 : (f == 3 ? 1.0 : t);
        }
      }
    }
  return cb;
}

/* Outward unit normal of face f of cell c at face parameter t: perpendicular to the face
 * curve, on the other side from the cell's point half a reference unit inward from the
 * face (the normal component of that offset is positive in any unfolded cell, at a
 * degenerate corner too). */
static void face_normal(const or_curv *m, int64_t c, int f, double t, double *n) {
  double x[2], dx[2], y[2], J[2][2];
  face_curve(m, c, f, t, x, dx);
  double xi = f == 0 ? -0.5 : (f == 1 ? 0.5 : t), eta = f == 2 ? -0.5 : (f == 3 ? 0.5 : t);
  cell_map(m, c, xi, eta, y, J);
  double len = sqrt(dx[0] * dx[0] + dx[1] * dx[1]);
  n[0] = dx[1] / len;
  n[1] = -dx[0] / len;
  if (n[0] * (y[0] - x[0]) + n[1] * (y[1] - x[1]) > 0.0) {
    n[0] = -n[0];
    n[1] = -n[1];
  }
}

/* For a path x0 + s v tangent to face f of cell c at x0 = face(t0): whether its end x0 + v
 * lies beyond the face curve (a convex boundary, which the path then leaves) rather than
 * on it (a straight face, along which it stays).  The end is projected onto the face's
 * polynomial curve (extended past its ends if need be) by bisection on the derivative
 * of the squared distance, near t0; beyond = on the outward side by more than rounding. */
static int beyond_face(const or_curv *m, int64_t c, int f, double t0, const double *x0, const double *v,
                       double scale) {
  double y[2] = {x0[0] + v[0], x0[1] + v[1]}, x[2], dx[2];
  double lo = t0 - 0.5, hi = t0 + 0.5;
  face_curve(m, c, f, lo, x, dx);
  double hlo = (x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1];
  for (int it = 0; it < 100; it++) {
    double mid = 0.5 * (lo + hi);
    face_curve(m, c, f, mid, x, dx);
    double h = (x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1];
    if ((h > 0.0) == (hlo > 0.0)) { lo = mid; hlo = h; } else hi = mid;
  }
  double t = 0.5 * (lo + hi), n[2];
  face_curve(m, c, f, t, x, dx);
  face_normal(m, c, f, t, n);
  return n[0] * (y[0] - x[0]) + n[1] * (y[1] - x[1]) > 1e-12 * scale;
}

/* Where x0 + s v (x0 inside the mesh or on its boundary, s in [0,1]) first meets the
 * boundary, and that boundary's tag; *bc = -1 if it never does.  Every tagged face is
 * intersected with the line: h(t) = (face(t) - x0) x v is sampled at 65 even parameters
 * and at the face's support points, every sign change is bisected in t, and a root gives
 * s = (face(t) - x0).v / |v|^2.  A root at x0 itself (x0 a boundary node) counts only if
 * the path leaves the mesh there: v . n_out > 0, or a tangent path whose end lies beyond
 * the face curve (beyond_face).  Crossing points closer than 1e-9 max(1, |x0|) are one point (a
 * junction of boundary segments): the smaller tag wins. */
static double curv_exit(const or_curv *m, const double *x0, const double *v, int *bc) {
  int p = m->p, n1 = p + 1;
  double vv = v[0] * v[0] + v[1] * v[1], vlen = sqrt(vv);
  double scale = fmax(1.0, fmax(fabs(x0[0]), fabs(x0[1])));
  double tie = 1e-9 * scale / fmax(fabs(v[0]), fabs(v[1]));
  double sx0 = fmin(x0[0], x0[0] + v[0]), sx1 = fmax(x0[0], x0[0] + v[0]);
  double sy0 = fmin(x0[1], x0[1] + v[1]), sy1 = fmax(x0[1], x0[1] + v[1]);
  double sbest = 1e300;
  *bc = -1;
  double ts[65 + OR_MAXP + 1];
  int nt = 0;
  for (int j = 0; j <= 64; j++) ts[nt++] = -1.0 + j / 32.0;
  for (int j = 1; j < p; j++) ts[nt++] = m->xref[j];
  for (int a = 1; a < nt; a++)             /* insertion sort: the samples in order */
    for (int b = a; b > 0 && ts[b] < ts[b - 1]; b--) {
      double tmp = ts[b];
      ts[b] = ts[b - 1];
      ts[b - 1] = tmp;
    }
  for (int64_t c = 0; c < m->n_cells; c++)
    for (int f = 0; f < 4; f++) {
      int tag = m->face_bc[c * 4 + f];
      if (tag < 0) continue;
      /* the face's box (its support points, widened by 10% for the curve) against the
       * segment's */
      double fx0 = 1e300, fx1 = -1e300, fy0 = 1e300, fy1 = -1e300;
      for (int j = 0; j <= p; j++) {
        int jx = f == 0 ? 0 : (f == 1 ? p : j), jy = f == 2 ? 0 : (f == 3 ? p : j);
        const double *X = m->xyz + 2 * m->cell_nodes[c * n1 * n1 + jx + n1 * jy];
        fx0 = fmin(fx0, X[0]);
        fx1 = fmax(fx1, X[0]);
        fy0 = fmin(fy0, X[1]);
        fy1 = fmax(fy1, X[1]);
      }
      double w = 0.1 * fmax(fx1 - fx0, fy1 - fy0) + 1e-12;
      if (sx1 < fx0 - w || sx0 > fx1 + w || sy1 < fy0 - w || sy0 > fy1 + w) continue;
      double hprev = 0.0, tprev = -1.0;
      for (int j = 0; j < nt; j++) {
        double x[2], dx[2];
        face_curve(m, c, f, ts[j], x, dx);
        double h = (x[0] - x0[0]) * v[1] - (x[1] - x0[1]) * v[0];
        double troot;
        int have = 0;
        if (h == 0.0) {
          troot = ts[j];
          have = 1;
        } else if (j > 0 && hprev != 0.0 && (h > 0.0) != (hprev > 0.0)) {
          double lo = tprev, hi = ts[j], hlo = hprev;
          for (int it = 0; it < 100; it++) {
            double mid = 0.5 * (lo + hi), xm[2], dm[2];
            face_curve(m, c, f, mid, xm, dm);
            double hm = (xm[0] - x0[0]) * v[1] - (xm[1] - x0[1]) * v[0];
            if (hm == 0.0) { lo = hi = mid; break; }
            if ((hm > 0.0) == (hlo > 0.0)) { lo = mid; hlo = hm; } else hi = mid;
          }
          troot = 0.5 * (lo + hi);
          have = 1;
        }
        hprev = h;
        tprev = ts[j];
        if (!have) continue;
        double xr[2], dr[2];
        face_curve(m, c, f, troot, xr, dr);
        double sr = ((xr[0] - x0[0]) * v[0] + (xr[1] - x0[1]) * v[1]) / vv;
        if (sr < -1e-9 || sr > 1.0 + 1e-9) continue;
        double dist = fabs(xr[0] - x0[0]) + fabs(xr[1] - x0[1]);
        if (dist <= 1e-12 * scale) {
          /* the root is x0: only a path that leaves the mesh here counts */
          double n[2];
          face_normal(m, c, f, troot, n);
          double nv = n[0] * v[0] + n[1] * v[1];
          if (nv < -1e-12 * vlen) continue;
          if (nv <= 1e-12 * vlen && !beyond_face(m, c, f, troot, x0, v, scale)) continue;
          sr = 0.0;
        }
        if (sr < 0.0) sr = 0.0;
        if (sr < sbest - tie) {
          sbest = sr;
          *bc = tag;
        } else if (sr <= sbest + tie) {
          if (sr < sbest) sbest = sr;
          if (tag < *bc) *bc = tag;
        }
      }
    }
  return *bc < 0 ? 0.0 : sbest;
}

/* Departure-point geometry of the Q (velocity, node k) pairs, row i stored at index
 * i * stride: kind 0 interpolates population src in cell at xi; kind 1 takes the inlet
 * state of boundary src.  *thermal = a thermal wall met by some path of node k, else -1.
 * Returns OR_OK, or OR_EGEOM with the failing velocity in *bad_i. */
static int curv_node_geometry(const or_curv *m, int64_t k, int64_t stride, int64_t *cell, double *xi, int *src,
                              int *kind, int *thermal, int *bad_i) {
  *thermal = -1;
  const double *xk = m->xyz + 2 * k;
  for (int i = 0; i < m->Q; i++) {
    int64_t q = (int64_t)i * stride;
    double d[2] = {m->dt * m->zeta[2 * i], m->dt * m->zeta[2 * i + 1]};
    double dp[2] = {xk[0] - d[0], xk[1] - d[1]}, r[2];
    int64_t c = curv_locate(m, dp, r);
    src[q] = i;
    kind[q] = 0;
    if (c < 0) {
      /* the backward path leaves the mesh: the first boundary crossed decides */
      double v[2] = {-d[0], -d[1]};
      int bc;
      double s = curv_exit(m, xk, v, &bc);
      if (bc < 0) { *bad_i = i; return OR_EGEOM; }
      int bk = m->bc_kind[bc];
      if (bk == OR_BC_WALL) {
        /* Sec. 3.3.2: remaining path travelled back from the wall point x_k - s d */
        double xw[2] = {xk[0] - s * d[0], xk[1] - s * d[1]};
        for (int a = 0; a < 2; a++) dp[a] = xw[a] + (d[a] - (xk[a] - xw[a]));
        c = curv_locate(m, dp, r);
        /* reflected out of the mesh again (a corner, a thin gap): nearest boundary point */
        if (c < 0) c = curv_project(m, dp, r);
        if (c < 0) { *bad_i = i; return OR_EGEOM; }
        src[q] = m->opp[i];
        if (!isnan(m->bc_val[6 * bc + 5])) *thermal = bc;
      } else if (bk == OR_BC_INLET) {
        kind[q] = 1;
        src[q] = bc;
      } else if (bk == OR_BC_OUTLET) {
        /* Sec. 3.3.3: population i at x_k + d; outside the mesh, at the nearest
         * boundary point (orthogonal projection) */
        dp[0] = xk[0] + d[0];
        dp[1] = xk[1] + d[1];
        c = curv_locate(m, dp, r);
        if (c < 0) c = curv_project(m, dp, r);
        if (c < 0) { *bad_i = i; return OR_EGEOM; }
      } else {
        *bad_i = i;
        return OR_EGEOM;
      }
    }
    cell[q] = c;
    xi[2 * q] = r[0];
    xi[2 * q + 1] = r[1];
  }
  return OR_OK;
}

/* Departure-point geometry of every (velocity, node) pair, rows [Q][N]. */
int or_curv_geometry(const or_curv *m, int64_t *cell, double *xi, int *src, int *kind, int *thermal_bc,
                     int64_t *err) {
  int64_t N = m->n_nodes;
  int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < N; k++) {
    if (status != OR_OK) continue;
    int bad = -1;
    int rc = curv_node_geometry(m, k, N, cell + k, xi + 2 * k, src + k, kind + k, thermal_bc + k, &bad);
    if (rc != OR_OK) {
#pragma omp critical
      { status = rc; err[0] = k; err[1] = bad; }
    }
  }
  return status;
}

/* One node's new populations (Sec. 3.2-3.4): interpolate every row of its geometry
 * (rows at index i * stride), the thermal-wall correction, then BGK relaxation and the
 * force term.  out[i] = f_i, out[Q + i] = g_i, at index i * ostride. */
static void curv_node_update(const or_curv *m, const double *H, const double *inlet, const double *in,
                             const int64_t *cell, const double *xi, const int *src, const int *kind, int64_t stride,
                             int thermal, double *out, int64_t ostride) {
  int Q = m->Q, D = 2, p = m->p, n1 = p + 1;
  int64_t N = m->n_nodes;
  double cv = 1.0 / (m->gamma - 1.0);
  double fs[OR_MAXQ], gs[OR_MAXQ], fe[OR_MAXQ], fe2[OR_MAXQ];
  for (int i = 0; i < Q; i++) {
    int64_t q = (int64_t)i * stride;
    if (kind[q] == 1) {
      fs[i] = inlet[(size_t)src[q] * 2 * Q + i];
      gs[i] = inlet[(size_t)src[q] * 2 * Q + Q + i];
      continue;
    }
    double lx[OR_MAXP + 1], ly[OR_MAXP + 1];
    lagrange(p, m->xref, xi[2 * q], lx);
    lagrange(p, m->xref, xi[2 * q + 1], ly);
    const int64_t *cn = m->cell_nodes + cell[q] * n1 * n1;
    const double *F = in + (size_t)src[q] * N, *G = in + ((size_t)Q + src[q]) * N;
    double a = 0, b = 0;
    for (int jy = 0; jy <= p; jy++)
      for (int jx = 0; jx <= p; jx++) {
        double wgt = lx[jx] * ly[jy];
        a += wgt * F[cn[jx + n1 * jy]];
        b += wgt * G[cn[jx + n1 * jy]];
      }
    fs[i] = a;
    gs[i] = b;
  }
  double rho, u[3], T;
  node_moments(D, Q, m->zeta, cv, fs, gs, &rho, u, &T);
  if (thermal >= 0) {
    double Tw = m->bc_val[6 * thermal + 5];
    feq_all(D, Q, m->w, H, m->T0, rho, u, Tw, fe);
    feq_all(D, Q, m->w, H, m->T0, rho, u, T, fe2);
    for (int i = 0; i < Q; i++) {
      fs[i] += fe[i] - fe2[i];
      gs[i] += Tw * (2.0 * cv - D) * fe[i] - T * (2.0 * cv - D) * fe2[i];
    }
    T = Tw;
  }
  if (m->relax_mode == 2) {
    for (int i = 0; i < Q; i++) {
      out[(size_t)i * ostride] = fs[i];
      out[((size_t)Q + i) * ostride] = gs[i];
    }
    return;
  }
  double tb = m->tau_bar;
  if (m->relax_mode == 1) tb = m->mu_ref * pow(T / m->T_ref, m->mu_exp) / (rho * T * m->dt) + 0.5;
  feq_all(D, Q, m->w, H, m->T0, rho, u, T, fe);
  double gfac = T * (2.0 * cv - D);
  int has_force = m->force[0] != 0.0 || m->force[1] != 0.0;
  if (has_force) {
    double u2[3] = {u[0] + m->force[0] * m->dt / rho, u[1] + m->force[1] * m->dt / rho, 0.0};
    feq_all(D, Q, m->w, H, m->T0, rho, u2, T, fe2);
  }
  double fo[OR_MAXQ], go[OR_MAXQ];
  for (int i = 0; i < Q; i++) {
    fo[i] = fs[i] - (fs[i] - fe[i]) / tb;
    go[i] = gs[i] - (gs[i] - gfac * fe[i]) / tb;
  }
  if (m->Pr != 1.0) add_quasi_eq(D, Q, m->zeta, m->w, m->T0, u, fs, gs, pr_coef(tb, m->Pr), fo, go);
  for (int i = 0; i < Q; i++) {
    if (has_force) {
      fo[i] += fe2[i] - fe[i];
      go[i] += gfac * (fe2[i] - fe[i]);
    }
    out[(size_t)i * ostride] = fo[i];
    out[((size_t)Q + i) * ostride] = go[i];
  }
}

/* The step's inputs shared by all nodes: the populations to stream (scaled by
 * mass_ref / M first when the mass fix is on, M = sum_k V_k rho_k) and the inlet
 * equilibria [n_bc][2Q].  *scaled is the buffer to free (or NULL). */
static const double *curv_prepare(const or_curv *m, const double *pin, double **scaled, double **inlet) {
  int Q = m->Q, D = 2;
  int64_t N = m->n_nodes;
  double cv = 1.0 / (m->gamma - 1.0);
  double *H = make_htab(D, Q, m->zeta, m->T0);
  const double *in = pin;
  *scaled = NULL;
  if (m->mass_fix) {
    double M = 0.0;
    for (int64_t k = 0; k < N; k++) {
      double r = 0;
      for (int i = 0; i < Q; i++) r += pin[(size_t)i * N + k];
      M += m->node_vol[k] * r;
    }
    *scaled = (double *)malloc(sizeof(double) * 2 * (size_t)Q * N);
    for (size_t q = 0; q < 2 * (size_t)Q * N; q++) (*scaled)[q] = (m->mass_ref / M) * pin[q];
    in = *scaled;
  }
  *inlet = (double *)calloc((size_t)(m->n_bc > 0 ? m->n_bc : 1) * 2 * Q, sizeof(double));
  for (int b = 0; b < m->n_bc; b++) {
    if (m->bc_kind[b] != OR_BC_INLET) continue;
    const double *v = m->bc_val + b * 6;
    feq_all(D, Q, m->w, H, m->T0, v[0], v + 1, v[4], *inlet + (size_t)b * 2 * Q);
    for (int i = 0; i < Q; i++)
      (*inlet)[(size_t)b * 2 * Q + Q + i] = v[4] * (2.0 * cv - D) * (*inlet)[(size_t)b * 2 * Q + i];
  }
  free(H);
  return in;
}

int or_curv_step(const or_curv *m, const int64_t *cell, const double *xi, const int *src, const int *kind,
                 const int *thermal_bc, const double *pin, double *pout) {
  int64_t N = m->n_nodes;
  double *scaled, *inlet;
  const double *in = curv_prepare(m, pin, &scaled, &inlet);
  double *H = make_htab(2, m->Q, m->zeta, m->T0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < N; k++)
    curv_node_update(m, H, inlet, in, cell + k, xi + 2 * k, src + k, kind + k, N, thermal_bc[k], pout + k, N);
  free(inlet);
  free(scaled);
  free(H);
  return OR_OK;
}

/* The step at a sample of nodes only (geometry computed for those nodes alone):
 * out[n][2Q] = (f_0..f_Q-1, g_0..g_Q-1) of node nodes[n].  err = (node, velocity) of
 * a geometry failure. */
int or_curv_step_nodes(const or_curv *m, const double *pin, const int64_t *nodes, int64_t n, double *out,
                       int64_t *err) {
  int Q = m->Q;
  double *scaled, *inlet;
  const double *in = curv_prepare(m, pin, &scaled, &inlet);
  double *H = make_htab(2, Q, m->zeta, m->T0);
  int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t s = 0; s < n; s++) {
    if (status != OR_OK) continue;
    int64_t cell[OR_MAXQ];
    double xi[2 * OR_MAXQ];
    int src[OR_MAXQ], kind[OR_MAXQ], th, bad = -1;
    int rc = curv_node_geometry(m, nodes[s], 1, cell, xi, src, kind, &th, &bad);
    if (rc != OR_OK) {
#pragma omp critical
      { status = rc; err[0] = nodes[s]; err[1] = bad; }
      continue;
    }
    curv_node_update(m, H, inlet, in, cell, xi, src, kind, 1, th, out + s * 2 * Q, 1);
  }
  free(inlet);
  free(scaled);
  free(H);
  return status;
}

/* populations in equilibrium with nodal fields, any mesh (u is [N][D]) */
int or_init_generic(int D, int Q, const double *zeta, const double *w, double T0, double gamma, int64_t N,
                    const double *rho, const double *u, const double *T, double *pop) {
  double cv = 1.0 / (gamma - 1.0);
  double *H = make_htab(D, Q, zeta, T0);
#pragma omp parallel for
  for (int64_t k = 0; k < N; k++) {
    double fe[OR_MAXQ], uk[3] = {0, 0, 0};
    for (int a = 0; a < D; a++) uk[a] = u[k * D + a];
    feq_all(D, Q, w, H, T0, rho[k], uk, T[k], fe);
    for (int i = 0; i < Q; i++) {
      pop[(size_t)i * N + k] = fe[i];
      pop[((size_t)Q + i) * N + k] = T[k] * (2.0 * cv - D) * fe[i];
    }
  }
  free(H);
  return OR_OK;
}

/* point location of one point (test hook) */
int64_t or_curv_locate(const or_curv *m, const double *x, double *xi) { return curv_locate(m, x, xi); }
double or_curv_exit(const or_curv *m, const double *x0, const double *v, int *bc) { return curv_exit(m, x0, v, bc); }
