// Host half of libsllbm: errors, velocity sets, support points, meshes and the
// interpolation-plan builder (departure points, boundary cases, weights).
// Nothing here touches the GPU; sllbm_device.hip uploads what is built here.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>

#include "sllbm_internal.h"
#include "sllbm_kernels.h"

namespace sllbm {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// ------------------------------------------------------------------ support points

// Legendre P_n and its first two derivatives by the three-term recurrence.
static void legendre(int n, double x, double *P, double *dP, double *d2P) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *P = 1; *dP = 0; *d2P = 0; return; }
  for (int k = 2; k <= n; k++) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  double den = 1.0 - x * x;
  *dP = n * (p0 - x * p1) / den;
  *d2P = (2.0 * x * (*dP) - n * (n + 1.0) * p1) / den;
}

std::vector<double> support_points(int p, int family) {
  std::vector<double> x(p + 1);
  if (family == SLLBM_NODES_EQUI) {
    for (int j = 0; j <= p; j++) x[j] = -1.0 + 2.0 * j / p;
  } else if (family == SLLBM_NODES_GLC) {
    for (int j = 0; j <= p; j++) x[j] = -std::cos(M_PI * j / p);
  } else {
    // Gauss-Lobatto-Legendre: +-1 and the roots of P_p', by Newton from the
    // Chebyshev-Lobatto points.
    x[0] = -1.0;
    x[p] = 1.0;
    for (int j = 1; j < p; j++) {
      double r = -std::cos(M_PI * j / p);
      for (int it = 0; it < 100; it++) {
        double P, dP, d2P;
        legendre(p, r, &P, &dP, &d2P);
        double dr = dP / d2P;
        r -= dr;
        if (std::fabs(dr) < 1e-16) break;
      }
      x[j] = r;
    }
    for (int j = 1; j < p; j++)  // symmetrise
      if (j < p - j) { double s = 0.5 * (x[p - j] - x[j]); x[j] = -s; x[p - j] = s; }
    if (p % 2 == 0) x[p / 2] = 0.0;
  }
  return x;
}

void lagrange_weights(const std::vector<double> &xr, double xi, double *w) {
  int n = (int)xr.size();
  for (int j = 0; j < n; j++)
    if (xi == xr[j]) {
      for (int m = 0; m < n; m++) w[m] = (m == j) ? 1.0 : 0.0;
      return;
    }
  // second (true) barycentric form
  double den = 0.0;
  double lam[kMaxP + 1];
  for (int j = 0; j < n; j++) {
    double l = 1.0;
    for (int m = 0; m < n; m++)
      if (m != j) l *= (xr[j] - xr[m]);
    lam[j] = 1.0 / l;
  }
  for (int j = 0; j < n; j++) {
    w[j] = lam[j] / (xi - xr[j]);
    den += w[j];
  }
  for (int j = 0; j < n; j++) w[j] /= den;
}

std::vector<double> lagrange_integrals(const std::vector<double> &xr) {
  // Solve sum_j V_j x_j^m = int_{-1}^1 x^m dx, m = 0..p (Vandermonde moment system).
  int n = (int)xr.size();
  std::vector<double> A(n * n), b(n);
  for (int m = 0; m < n; m++) {
    for (int j = 0; j < n; j++) A[m * n + j] = std::pow(xr[j], m);
    b[m] = (m % 2 == 0) ? 2.0 / (m + 1.0) : 0.0;
  }
  for (int c = 0; c < n; c++) {  // Gaussian elimination with partial pivoting
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    for (int k = 0; k < n; k++) std::swap(A[c * n + k], A[piv * n + k]);
    std::swap(b[c], b[piv]);
    for (int r = c + 1; r < n; r++) {
      double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; k++) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  std::vector<double> V(n);
  for (int r = n - 1; r >= 0; r--) {
    double s = b[r];
    for (int k = r + 1; k < n; k++) s -= A[r * n + k] * V[k];
    V[r] = s / A[r * n + r];
  }
  return V;
}

void round_weights_f32(const double *w, int n, float *out) {
  double s = 0.0;
  for (int j = 0; j < n; j++) {
    out[j] = (float)w[j];
    s += (double)out[j];
  }
  double best = std::fabs(1.0 - s);
  int bj = -1;
  float bv = 0.0f;
  for (int j = 0; j < n; j++) {
    if (out[j] == 0.0f) continue;
    float cand = (float)((double)out[j] + (1.0 - s));
    double res = std::fabs(1.0 - (s - (double)out[j] + (double)cand));
    if (res < best) { best = res; bj = j; bv = cand; }
  }
  if (bj >= 0) out[bj] = bv;
}

double tensor_node_coord(const Mesh &m, int a, int n) {
  int c = n / m.p, b = n % m.p;
  if (c == m.ncell[a]) return m.edges[a][m.ncell[a]];
  double lo = m.edges[a][c], hi = m.edges[a][c + 1];
  return lo + 0.5 * (1.0 + m.xref[b]) * (hi - lo);
}

std::vector<double> node_volumes(const Mesh &m) {
  std::vector<double> li = lagrange_integrals(m.xref);
  std::vector<double> V;
  if (m.kind == SLLBM_MESH_TENSOR) {
    std::vector<double> va[3];
    for (int a = 0; a < 3; a++) {
      va[a].assign(m.N[a], a < m.dim ? 0.0 : 1.0);
      if (a >= m.dim) continue;
      for (int c = 0; c < m.ncell[a]; c++) {
        double h = m.edges[a][c + 1] - m.edges[a][c];
        for (int j = 0; j <= m.p; j++) {
          int n = c * m.p + j;
          if (m.periodic(a)) n %= m.N[a];
          va[a][n] += 0.5 * h * li[j];
        }
      }
    }
    V.resize(m.n_nodes);
    for (int z = 0; z < m.N[2]; z++)
      for (int y = 0; y < m.N[1]; y++)
        for (int x = 0; x < m.N[0]; x++)
          V[(size_t)x + (size_t)m.N[0] * ((size_t)y + (size_t)m.N[1] * z)] = va[0][x] * va[1][y] * va[2][z];
  } else {
    // isoparametric quads: V_k = sum over cells of int l_k |J| d xi, by a tensor
    // Gauss rule of the oracle-independent kind: the same Vandermonde integrals
    // applied to |J| l_k sampled at the support points would be inexact, so use
    // a (p+2)-point Legendre-Gauss rule built from Newton on P_{p+2}.
    int q = m.p + 2;
    std::vector<double> xg(q), wg(q);
    for (int j = 0; j < q; j++) {
      double r = -std::cos(M_PI * (j + 0.75) / (q + 0.5));
      for (int it = 0; it < 100; it++) {
        double P, dP, d2P;
        legendre(q, r, &P, &dP, &d2P);
        double dr = P / dP;
        r -= dr;
        if (std::fabs(dr) < 1e-16) break;
      }
      double P, dP, d2P;
      legendre(q, r, &P, &dP, &d2P);
      xg[j] = r;
      wg[j] = 2.0 / ((1.0 - r * r) * dP * dP);
    }
    int np1 = m.p + 1;
    V.assign(m.n_nodes, 0.0);
    std::vector<double> lx(np1), ly(np1), dlx(np1), dly(np1);
    for (int64_t c = 0; c < m.n_cells; c++) {
      const int64_t *cn = &m.cell_nodes[c * np1 * np1];
      for (int gy = 0; gy < q; gy++)
        for (int gx = 0; gx < q; gx++) {
          lagrange_weights(m.xref, xg[gx], lx.data());
          lagrange_weights(m.xref, xg[gy], ly.data());
          // derivatives of the basis by the product rule
          for (int j = 0; j < np1; j++) {
            double s = 0.0;
            for (int k = 0; k < np1; k++) {
              if (k == j) continue;
              double t = 1.0 / (m.xref[j] - m.xref[k]);
              for (int l = 0; l < np1; l++)
                if (l != j && l != k) t *= (xg[gx] - m.xref[l]) / (m.xref[j] - m.xref[l]);
              s += t;
            }
            dlx[j] = s;
            s = 0.0;
            for (int k = 0; k < np1; k++) {
              if (k == j) continue;
              double t = 1.0 / (m.xref[j] - m.xref[k]);
              for (int l = 0; l < np1; l++)
                if (l != j && l != k) t *= (xg[gy] - m.xref[l]) / (m.xref[j] - m.xref[l]);
              s += t;
            }
            dly[j] = s;
          }
          double J[2][2] = {{0, 0}, {0, 0}};
          for (int jy = 0; jy < np1; jy++)
            for (int jx = 0; jx < np1; jx++) {
              const double *X = &m.node_xyz[2 * cn[jx + np1 * jy]];
              for (int a = 0; a < 2; a++) {
                J[a][0] += X[a] * dlx[jx] * ly[jy];
                J[a][1] += X[a] * lx[jx] * dly[jy];
              }
            }
          double det = std::fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
          for (int jy = 0; jy < np1; jy++)
            for (int jx = 0; jx < np1; jx++) V[cn[jx + np1 * jy]] += wg[gx] * wg[gy] * det * lx[jx] * ly[jy];
        }
    }
  }
  return V;
}

// ------------------------------------------------------------------ tensor plan

namespace {

struct AxisBuilder {
  const Mesh &m;
  int a;
  std::map<uint64_t, int> ids;
  HostTables &t;
  AxisBuilder(const Mesh &mm, int aa, HostTables &tt) : m(mm), a(aa), t(tt) {}

  double lo() const { return m.edges[a][0]; }
  double hi() const { return m.edges[a][m.ncell[a]]; }

  // Cell and reference coordinate of a coordinate inside [lo, hi]; a point on an
  // interior face takes the cell above it.
  void locate(double x, int *cell, double *xi) const {
    const std::vector<double> &e = m.edges[a];
    int c = (int)(std::upper_bound(e.begin(), e.end(), x) - e.begin()) - 1;
    c = std::max(0, std::min(c, m.ncell[a] - 1));
    *cell = c;
    *xi = 2.0 * (x - e[c]) / (e[c + 1] - e[c]) - 1.0;
  }

  // 1D table for departure points x_n - d (identity when d == 0).  On a bounded axis a
  // departure point outside the domain gets a harmless in-range stencil with zero
  // weights: the boundary entries of the face decide those pairs.
  int table(double d) {
    uint64_t key;
    std::memcpy(&key, &d, 8);
    auto it = ids.find(key);
    if (it != ids.end()) return it->second;
    int id = t.ntab[a]++;
    ids[key] = id;
    int N = m.N[a], p = m.p;
    t.ident[a].push_back(d == 0.0 ? 1 : 0);
    for (int n = 0; n < N; n++) {
      double w[kMaxP + 1];
      int start;
      if (d == 0.0) {
        int c = std::min(n / p, m.ncell[a] - 1);
        int b = n - c * p;
        start = c * p;
        for (int j = 0; j <= p; j++) w[j] = (j == b) ? 1.0 : 0.0;
      } else {
        double x = tensor_node_coord(m, a, n) - d;
        bool out = false;
        if (m.periodic(a)) {
          double L = hi() - lo();
          while (x < lo()) x += L;
          while (x >= hi()) x -= L;
        } else if (x < lo() || x > hi()) {
          out = true;
        }
        if (out) {
          // nearest in-range cell, so that stencil starts stay non-decreasing along the
          // axis and a tile's departure region stays local
          start = (x < lo()) ? 0 : (m.ncell[a] - 1) * p;
          for (int j = 0; j <= p; j++) w[j] = 0.0;
        } else {
          int c;
          double xi;
          locate(x, &c, &xi);
          start = c * p;
          lagrange_weights(m.xref, xi, w);
        }
      }
      t.start[a].push_back(start);
      for (int j = 0; j <= p; j++) t.w[a].push_back(w[j]);
    }
    return id;
  }
};

}  // namespace

int build_tensor_tables(const Mesh &m, const VelSet &v, double dt, HostTables &t, int64_t *n_exc, int64_t *n_th) {
  int D = m.dim, Q = v.Q, p = m.p;
  int bounded = -1, nb = 0;
  for (int a = 0; a < D; a++)
    if (!m.periodic(a)) { bounded = a; nb++; }
  if (nb > 1)
    return fail(SLLBM_EUNSUPPORTED, "tensor meshes support at most one bounded axis (found %d); "
                                    "describe the mesh as curvilinear instead", nb);
  std::vector<AxisBuilder> ab;
  for (int a = 0; a < 3; a++) ab.emplace_back(m, a, t);
  t.tab_reg.assign(3 * Q, 0);
  for (int a = 0; a < 3; a++) {
    if (a >= D) {
      // unused axis: one identity table over a single node
      t.ntab[a] = 1;
      t.ident[a] = {1};
      t.start[a] = {0};
      t.w[a].assign(p + 1, 0.0);
      t.w[a][0] = 1.0;
      continue;
    }
    for (int i = 0; i < Q; i++) t.tab_reg[a * Q + i] = ab[a].table(dt * v.zeta[i * D + a]);
  }
  *n_exc = 0;
  *n_th = 0;
  t.nfaces = 0;
  if (bounded < 0) return SLLBM_OK;
  int a = bounded;
  double lo = m.edges[a][0], hi = m.edges[a][m.ncell[a]];
  double dmax = 0.0;
  for (int i = 0; i < Q; i++) dmax = std::max(dmax, std::fabs(dt * v.zeta[i * D + a]));
  for (int side = 0; side < 2; side++) {
    int f = t.nfaces++;
    t.face_axis[f] = a;
    t.face_side[f] = side;
    int bc = m.face_bc[a][side];
    const sllbm_bc &B = m.bcs[bc];
    std::vector<ExcEntry> rows;
    std::vector<double> Tw;
    int depth = 0;
    for (int l = 0; l < m.N[a]; l++) {
      int n = side == 0 ? l : m.N[a] - 1 - l;
      double x = tensor_node_coord(m, a, n);
      double dist = side == 0 ? x - lo : hi - x;
      if (dist > dmax) break;
      bool any = false, thermal = false;
      for (int i = 0; i < Q; i++) {
        ExcEntry e;
        std::memset(&e, 0, sizeof(e));
        double d = dt * v.zeta[i * D + a];
        double end = x - d;
        bool crosses = side == 0 ? (end < lo) : (end > hi);
        if (crosses) {
          any = true;
          (*n_exc) += 1;  // per layer; scaled by the layer's node count below
          if (B.kind == SLLBM_BC_INLET) {
            e.kind = EXC_INLET;
            e.src = bc;
          } else if (B.kind == SLLBM_BC_WALL) {
            // Sec. 3.3.2: wall at fraction s of the backward path; remaining path back
            // from the wall; opposite population at x_k + (1 - 2 s) dt zeta_i.
            double s = (x - (side == 0 ? lo : hi)) / d;
            // a reflected point outside the domain (a channel thinner than the path,
            // or rounding) is replaced by its nearest boundary point
            double y = std::max(lo, std::min(hi, x + (1.0 - 2.0 * s) * d));
            e.kind = EXC_WALL;
            e.src = v.opp[i];
            int c;
            double xi;
            ab[a].locate(y, &c, &xi);
            e.start = c * p;
            lagrange_weights(m.xref, xi, e.w);
            round_weights_f32(e.w, p + 1, e.w32);
            for (int b = 0; b < D; b++)
              if (b != a) e.tab[b] = ab[b].table(-(1.0 - 2.0 * s) * dt * v.zeta[i * D + b]);
            if (std::isfinite(B.T_wall)) thermal = true;
          } else if (B.kind == SLLBM_BC_OUTLET) {
            // Sec. 3.3.3: population i at x_k + dt zeta_i; outside the domain, its
            // nearest boundary point (the bounded coordinate clamped)
            double y = std::max(lo, std::min(hi, x + d));
            e.kind = EXC_OUTLET;
            e.src = i;
            int c;
            double xi;
            ab[a].locate(y, &c, &xi);
            e.start = c * p;
            lagrange_weights(m.xref, xi, e.w);
            round_weights_f32(e.w, p + 1, e.w32);
            for (int b = 0; b < D; b++)
              if (b != a) e.tab[b] = ab[b].table(-dt * v.zeta[i * D + b]);
          } else {
            return fail(SLLBM_EINVAL, "bounded face with boundary kind %d", B.kind);
          }
        }
        rows.push_back(e);
      }
      Tw.push_back(thermal ? B.T_wall : std::numeric_limits<double>::quiet_NaN());
      if (any) depth = l + 1;
    }
    rows.resize((size_t)depth * Q);
    Tw.resize(depth);
    t.face_depth[f] = depth;
    t.face_e[f] = rows;
    t.face_Tw[f] = Tw;
  }
  // scale counters by the number of nodes in one layer
  int64_t layer = 1;
  for (int b = 0; b < D; b++)
    if (b != a) layer *= m.N[b];
  *n_exc *= layer;
  int64_t nth = 0;
  for (int f = 0; f < t.nfaces; f++)
    for (double T : t.face_Tw[f])
      if (std::isfinite(T)) nth++;
  *n_th = nth * layer;
  return SLLBM_OK;
}

}  // namespace sllbm

using namespace sllbm;

// ------------------------------------------------------------------ C ABI (host only)

extern "C" const char *sllbm_last_error(void) { return g_err.c_str(); }

extern "C" int sllbm_velset_gauss_hermite(int dim, int n, double T0, double *zeta, double *w, int32_t *opp) {
  if (dim < 1 || dim > 3 || n < 1 || n > 12 || !(T0 > 0) || !zeta || !w || !opp)
    return fail(SLLBM_EINVAL, "velset: need dim in 1..3, n in 1..12, T0 > 0 and non-NULL outputs");
  // 1D rule for the weight exp(-x^2/2)/sqrt(2 pi): roots of the Hermite polynomial He_n
  // (He_{k+1} = x He_k - k He_{k-1}) by bisection on a fine grid then Newton; weights
  // n! / (n He_{n-1}(x))^2.
  auto he = [n](double x, double *Hn, double *Hn1) {
    double h0 = 1.0, h1 = x;
    if (n == 1) { *Hn = x; *Hn1 = 1.0; return; }
    for (int k = 1; k < n; k++) {
      double h2 = x * h1 - k * h0;
      h0 = h1;
      h1 = h2;
    }
    *Hn = h1;
    *Hn1 = h0;
  };
  std::vector<double> x;
  double R = 2.0 * std::sqrt((double)n) + 1.0;
  int steps = 20000;
  double dummy;
  // grid offset by half a step, so that no grid point is a root (x = 0 for odd n)
  auto grid = [&](int s) { return -R + 2.0 * R * (s + 0.5) / steps; };
  double prev;
  he(grid(0), &prev, &dummy);
  for (int s = 1; s < steps && (int)x.size() < n; s++) {
    double cur;
    he(grid(s), &cur, &dummy);
    if ((prev < 0) != (cur < 0)) {
      double a = grid(s - 1), b = grid(s), fa = prev;
      for (int it = 0; it < 200 && b - a > 0; it++) {  // bisection to the last bit
        double mid = 0.5 * (a + b), fm;
        if (mid == a || mid == b) break;
        he(mid, &fm, &dummy);
        if ((fm < 0) == (fa < 0)) { a = mid; fa = fm; } else { b = mid; }
      }
      x.push_back(0.5 * (a + b));
    }
    prev = cur;
  }
  if ((int)x.size() != n) return fail(SLLBM_EINVAL, "velset: Hermite root search failed");
  std::sort(x.begin(), x.end());
  for (int j = 0; j < n / 2; j++) {  // symmetrise
    double s = 0.5 * (x[n - 1 - j] - x[j]);
    x[j] = -s;
    x[n - 1 - j] = s;
  }
  if (n % 2) x[n / 2] = 0.0;
  std::vector<double> w1(n);
  double nf = 1.0;
  for (int k = 2; k <= n; k++) nf *= k;
  for (int j = 0; j < n; j++) {
    double Hn, Hn1;
    he(x[j], &Hn, &Hn1);
    w1[j] = nf / ((double)n * n * Hn1 * Hn1);
  }
  int Q = 1;
  for (int d = 0; d < dim; d++) Q *= n;
  for (int i = 0; i < Q; i++) {
    int r = i, a[3] = {0, 0, 0};
    for (int d = 0; d < dim; d++) { a[d] = r % n; r /= n; }
    double wi = 1.0;
    int o = 0, mul = 1;
    for (int d = 0; d < dim; d++) {
      zeta[i * dim + d] = std::sqrt(T0) * x[a[d]];
      wi *= w1[a[d]];
      o += (n - 1 - a[d]) * mul;
      mul *= n;
    }
    w[i] = wi;
    opp[i] = o;
  }
  return SLLBM_OK;
}

extern "C" int sllbm_velset_cubature(int dim, double T0, int *Q, double *zeta, double *w, int32_t *opp) {
  const bool none = !zeta && !w && !opp, all = zeta && w && opp;
  if ((dim != 2 && dim != 3) || !(T0 > 0) || !Q || !(none || all))
    return fail(SLLBM_EINVAL, "velset_cubature: need dim 2 or 3, T0 > 0, non-NULL Q and either all or none "
                              "of zeta, w, opp");
  // Degree-9 rules for the weight exp(-|x|^2/2)/(2 pi)^(D/2) with 19 / 45 points, each an
  // origin plus three orbits of a finite rotation group (hexagonal / icosahedral), in
  // closed form.  Radii^2 s and total orbit weights W:
  //   2D: hexagon at 0 deg (a vertex on +x) with s = (48 - 8 sqrt15)/7 and (48 + 8 sqrt15)/7,
  //       hexagon at 30 deg with s = 8, W = 3/64; the two inner weights solve
  //       W1 s1 + W2 s2 = 13/8, W1 s1^2 + W2 s2^2 = 5.
  //   3D: icosahedra with s = 3 (W = 25/36) and s = 15 (W = 1/180), the dual dodecahedron
  //       with s = 9 (W = 5/54), origin 28/135.
  // Index order: origin; inner, outer hexagon-0 (icosahedron); hexagon-30 (dodecahedron).
  const int q = dim == 2 ? 19 : 45;
  *Q = q;
  if (none) return SLLBM_OK;
  std::vector<double> v;  // q * dim unit-scale abscissae (T0 = 1)
  std::vector<double> wt;
  auto orbit = [&](const std::vector<double> &dirs, double s, double Wtot) {
    const int n = (int)dirs.size() / dim;
    const double r = std::sqrt(s);
    for (int k = 0; k < n; k++) {
      double nrm = 0.0;
      for (int d = 0; d < dim; d++) nrm += dirs[k * dim + d] * dirs[k * dim + d];
      nrm = std::sqrt(nrm);
      for (int d = 0; d < dim; d++) v.push_back(r * dirs[k * dim + d] / nrm);
      wt.push_back(Wtot / n);
    }
  };
  for (int d = 0; d < dim; d++) v.push_back(0.0);
  if (dim == 2) {
    const double h = std::sqrt(3.0) / 2.0;
    // vertex k at angle k pi/3 (hex0) and pi/6 + k pi/3 (hex30), k = 0..5
    const std::vector<double> hex0 = {1, 0, 0.5, h, -0.5, h, -1, 0, -0.5, -h, 0.5, -h};
    const std::vector<double> hex30 = {h, 0.5, 0, 1, -h, 0.5, -h, -0.5, 0, -1, h, -0.5};
    const double r15 = std::sqrt(15.0);
    const double s1 = (48.0 - 8.0 * r15) / 7.0, s2 = (48.0 + 8.0 * r15) / 7.0;
    const double W1 = (5.0 - 1.625 * s2) / (s1 * (s1 - s2)), W2 = (5.0 - 1.625 * s1) / (s2 * (s2 - s1));
    const double W3 = 3.0 / 64.0;
    wt.push_back(1.0 - W1 - W2 - W3);
    orbit(hex0, s1, W1);
    orbit(hex0, s2, W2);
    orbit(hex30, 8.0, W3);
  } else {
    const double ph = 0.5 * (1.0 + std::sqrt(5.0));
    // cyclic shifts c = 0, 1, 2 of (0, a, b): 0 on axis c, +-a on axis c+1, +-b on axis c+2,
    // sign of a outer, + before -
    auto shifts = [](double a, double b, std::vector<double> &o) {
      for (int c = 0; c < 3; c++)
        for (int sa = 0; sa < 2; sa++)
          for (int sb = 0; sb < 2; sb++) {
            double e[3] = {0, 0, 0};
            e[(c + 1) % 3] = sa ? -a : a;
            e[(c + 2) % 3] = sb ? -b : b;
            o.insert(o.end(), e, e + 3);
          }
    };
    std::vector<double> ico, dod;
    shifts(1.0, ph, ico);
    for (int j = 0; j < 8; j++)  // cube vertices, x's sign fastest
      for (int b = 0; b < 3; b++) dod.push_back((j >> b) & 1 ? -1.0 : 1.0);
    shifts(ph, 1.0 / ph, dod);
    wt.push_back(28.0 / 135.0);
    orbit(ico, 3.0, 25.0 / 36.0);
    orbit(ico, 15.0, 1.0 / 180.0);
    orbit(dod, 9.0, 5.0 / 54.0);
  }
  const double st = std::sqrt(T0);
  for (int i = 0; i < q; i++) {
    w[i] = wt[i];
    for (int d = 0; d < dim; d++) zeta[i * dim + d] = st * v[i * dim + d];
  }
  for (int i = 0; i < q; i++) {
    opp[i] = -1;
    for (int j = 0; j < q && opp[i] < 0; j++) {
      bool neg = true;
      for (int d = 0; d < dim; d++) neg = neg && zeta[j * dim + d] == -zeta[i * dim + d];
      if (neg) opp[i] = j;
    }
    if (opp[i] < 0) return fail(SLLBM_EINVAL, "velset_cubature: no opposite for velocity %d", i);
  }
  return SLLBM_OK;
}

extern "C" int sllbm_mesh_build(const sllbm_mesh_desc *d, sllbm_mesh *out) {
  if (!d || !out) return fail(SLLBM_EINVAL, "mesh_build: NULL argument");
  *out = nullptr;
  if (d->dim < 2 || d->dim > 3) return fail(SLLBM_EINVAL, "mesh_build: dim must be 2 or 3 (got %d)", d->dim);
  if (d->order_p < 1 || d->order_p > kMaxP) return fail(SLLBM_EINVAL, "mesh_build: order_p must be in 1..%d", kMaxP);
  if (d->nodes < 0 || d->nodes > 2) return fail(SLLBM_EINVAL, "mesh_build: unknown node family %d", d->nodes);
  if (d->n_bc < 0 || d->n_bc > kMaxBC || (d->n_bc > 0 && !d->bcs))
    return fail(SLLBM_EINVAL, "mesh_build: n_bc must be in 0..%d with bcs != NULL", kMaxBC);
  sllbm_mesh_s *ms = new (std::nothrow) sllbm_mesh_s();
  if (!ms) return fail(SLLBM_ENOMEM, "mesh_build: out of host memory");
  Mesh &m = ms->m;
  m.dim = d->dim;
  m.p = d->order_p;
  m.nodes = d->nodes;
  m.kind = d->kind;
  m.xref = support_points(m.p, m.nodes);
  m.bcs.assign(d->bcs, d->bcs + d->n_bc);
  for (const sllbm_bc &b : m.bcs) {
    if (b.kind < SLLBM_BC_WALL || b.kind > SLLBM_BC_OUTLET) {
      delete ms;
      return fail(SLLBM_EINVAL, "mesh_build: boundary kind %d is not wall/inlet/outlet", b.kind);
    }
    if (b.kind == SLLBM_BC_INLET && !(b.rho > 0 && b.T > 0)) {
      delete ms;
      return fail(SLLBM_EINVAL, "mesh_build: inlet state needs rho > 0 and T > 0");
    }
  }
  if (m.kind == SLLBM_MESH_TENSOR) {
    m.n_nodes = 1;
    for (int a = 0; a < 3; a++) {
      if (a >= m.dim) {
        m.ncell[a] = 1;
        m.N[a] = 1;
        m.edges[a] = {0.0, 1.0};
        continue;
      }
      if (d->ncell[a] < 1 || !d->edges[a]) {
        delete ms;
        return fail(SLLBM_EINVAL, "mesh_build: axis %d needs ncell >= 1 and edges", a);
      }
      m.ncell[a] = d->ncell[a];
      m.edges[a].assign(d->edges[a], d->edges[a] + d->ncell[a] + 1);
      for (int c = 0; c < m.ncell[a]; c++)
        if (!(m.edges[a][c + 1] > m.edges[a][c])) {
          delete ms;
          return fail(SLLBM_EINVAL, "mesh_build: edges of axis %d are not strictly increasing at %d", a, c);
        }
      int lo = d->face_bc[a][0], hi = d->face_bc[a][1];
      if ((lo < 0) != (hi < 0) || lo >= d->n_bc || hi >= d->n_bc) {
        delete ms;
        return fail(SLLBM_EINVAL, "mesh_build: axis %d faces must be both periodic (-1) or both valid bc indices", a);
      }
      m.face_bc[a][0] = lo;
      m.face_bc[a][1] = hi;
      m.N[a] = m.ncell[a] * m.p + (lo < 0 ? 0 : 1);
      if (lo < 0 && m.N[a] < m.p + 1) {
        delete ms;
        return fail(SLLBM_EINVAL, "mesh_build: periodic axis %d needs at least 2 cells", a);
      }
      m.n_nodes *= m.N[a];
    }
  } else if (m.kind == SLLBM_MESH_CURVILINEAR) {
    if (m.dim != 2) { delete ms; return fail(SLLBM_EUNSUPPORTED, "mesh_build: curvilinear meshes are 2D"); }
    if (d->n_nodes < 1 || !d->node_xyz || d->n_cells < 1 || !d->cell_nodes || !d->cell_face_bc) {
      delete ms;
      return fail(SLLBM_EINVAL, "mesh_build: curvilinear mesh needs nodes, cells and face tags");
    }
    int npc = (m.p + 1) * (m.p + 1);
    m.n_nodes = d->n_nodes;
    m.n_cells = d->n_cells;
    m.node_xyz.assign(d->node_xyz, d->node_xyz + 2 * d->n_nodes);
    m.cell_nodes.assign(d->cell_nodes, d->cell_nodes + npc * d->n_cells);
    m.cell_face_bc.assign(d->cell_face_bc, d->cell_face_bc + 4 * d->n_cells);
    for (int64_t v : m.cell_nodes)
      if (v < 0 || v >= m.n_nodes) { delete ms; return fail(SLLBM_EINVAL, "mesh_build: cell node index out of range"); }
    for (int32_t b : m.cell_face_bc)
      if (b < -1 || b >= d->n_bc) { delete ms; return fail(SLLBM_EINVAL, "mesh_build: face bc index out of range"); }
  } else {
    delete ms;
    return fail(SLLBM_EINVAL, "mesh_build: unknown mesh kind %d", m.kind);
  }
  *out = ms;
  return SLLBM_OK;
}

extern "C" int sllbm_mesh_nodes(sllbm_mesh ms, int64_t *n_nodes, double *xyz) {
  if (!ms || !n_nodes) return fail(SLLBM_EINVAL, "mesh_nodes: NULL argument");
  const Mesh &m = ms->m;
  *n_nodes = m.n_nodes;
  if (!xyz) return SLLBM_OK;
  if (m.kind == SLLBM_MESH_CURVILINEAR) {
    std::memcpy(xyz, m.node_xyz.data(), sizeof(double) * 2 * m.n_nodes);
    return SLLBM_OK;
  }
  std::vector<double> c[3];
  for (int a = 0; a < m.dim; a++) {
    c[a].resize(m.N[a]);
    for (int n = 0; n < m.N[a]; n++) c[a][n] = tensor_node_coord(m, a, n);
  }
  for (int z = 0; z < m.N[2]; z++)
    for (int y = 0; y < m.N[1]; y++)
      for (int x = 0; x < m.N[0]; x++) {
        size_t k = (size_t)x + (size_t)m.N[0] * ((size_t)y + (size_t)m.N[1] * z);
        xyz[k * m.dim + 0] = c[0][x];
        xyz[k * m.dim + 1] = c[1][y];
        if (m.dim == 3) xyz[k * m.dim + 2] = c[2][z];
      }
  return SLLBM_OK;
}

extern "C" int sllbm_mesh_volumes(sllbm_mesh ms, double *vol) {
  if (!ms || !vol) return fail(SLLBM_EINVAL, "mesh_volumes: NULL argument");
  std::vector<double> V = node_volumes(ms->m);
  std::memcpy(vol, V.data(), sizeof(double) * V.size());
  return SLLBM_OK;
}

extern "C" void sllbm_mesh_destroy(sllbm_mesh m) { delete m; }

namespace sllbm {

bool tile_cells(int D, int P, int c[3]) {
#define TSHAPE(DD, PP) {TileShape<DD, PP>::CX, TileShape<DD, PP>::CY, TileShape<DD, PP>::CZ}
  static const int shape[2][3][3] = {{TSHAPE(2, 2), TSHAPE(2, 3), TSHAPE(2, 4)},
                                     {TSHAPE(3, 2), TSHAPE(3, 3), TSHAPE(3, 4)}};
#undef TSHAPE
  if (D < 2 || D > 3 || P < 2 || P > 4) return false;
  for (int a = 0; a < 3; a++) c[a] = shape[D - 2][P - 2][a];
  return true;
}

bool tile_eligible(const Mesh &m, const HostTables &t, const int c[3], const int *org, const int *end) {
  int P = m.p;
  // the kernel holds byte offsets within a staged region's span of a population in 32 bits
  const int64_t span = m.dim == 3 ? (int64_t)m.N[0] * m.N[1] * (c[2] * P + P + 1)
                                  : (int64_t)m.N[0] * (c[1] * P + P + 1);
  if (span * (int64_t)sizeof(double) >= ((int64_t)1 << 31)) return false;
  // the 2D tile keeps the tables of the regular departure points in LDS (boundary entries
  // may add more tables; the gather kernel reads those); the 3D tile reads each velocity's
  // weight rows from the tables in device memory, so any number of tables will do
  if (m.dim == 2)
    for (size_t q = 0; q < t.tab_reg.size(); q++)
      if (t.tab_reg[q] >= kTileTabsMax) return false;
  for (int a = 0; a < m.dim; a++) {
    int T = c[a] * P, N = m.N[a];
    if (m.periodic(a) && N <= T + P) return false;
    std::vector<char> used(t.ntab[a], 0);
    for (size_t q = 0; q < t.tab_reg.size() / 3; q++) used[t.tab_reg[a * (t.tab_reg.size() / 3) + q]] = 1;
    const int o = org ? org[a] : 0, e = end ? end[a] : N;
    for (int tb = 0; tb < t.ntab[a]; tb++) {
      if (!used[tb] || t.ident[a][tb]) continue;
      for (int n0 = o; n0 < e; n0 += T) {
        int v = std::min(T, e - n0);
        int lo = 1 << 30, hi = -(1 << 30), first = 0, last = 0;
        for (int k = 0; k < v; k++) {
          int r = t.start[a][(size_t)tb * N + n0 + k] - n0;
          if (r > T) r -= N;
          else if (r < -P) r += N;
          if (r < -P || r > T) return false;
          lo = std::min(lo, r);
          hi = std::max(hi, r);
          if (k == 0) first = r;
          last = r;
        }
        if (first != lo || last != hi || hi - lo > T) return false;
      }
    }
  }
  return true;
}

bool col_eligible(const Mesh &m, const HostTables &t, int cx, int cy, int zc, int L, const int org[2], const int end[2]) {
  const int P = m.p;
  if (m.dim != 3 || !m.periodic(2)) return false;
  // bounded axes: x or y (their boundary layers' nodes are left to the gather kernel, as in
  // the tiled kernel); z is walked in chunks and must be periodic
  for (int f = 0; f < t.nfaces; f++)
    if (t.face_axis[f] == 2) return false;
  const int c[3] = {cx, cy, zc};
  const int o3[3] = {org[0], org[1], 0}, e3[3] = {end[0], end[1], m.N[2]};
  if (!tile_eligible(m, t, c, o3, e3)) return false;
  // along z: the kernel emits output plane k of a chunk after source plane k + D of the
  // chunk's departure region, D the largest lag of a stencil's last plane behind its output
  // plane; stencil plane j of k then sits lag = k + D - (its first plane) planes back
  const int Q = (int)(t.tab_reg.size() / 3), N = m.N[2], T = zc * P;
  for (int q = 0; q < Q; q++) {
    const int tb = t.tab_reg[2 * Q + q];
    if (t.ident[2][tb]) continue;
    for (int n0 = 0; n0 < N; n0 += T) {
      const int v = std::min(T, N - n0);
      std::vector<int> rel(v);
      for (int k = 0; k < v; k++) {
        int r = t.start[2][(size_t)tb * N + n0 + k] - n0;
        if (r > T) r -= N;
        else if (r < -P) r += N;
        rel[k] = r;
      }
      int D = 0;
      for (int k = 0; k < v; k++) D = std::max(D, rel[k] - rel[0] + P - k);
      for (int k = 0; k < v; k++) {
        const int lag = k + D - (rel[k] - rel[0]);
        if (lag < P || lag > L - 1) return false;
      }
    }
  }
  return true;
}

}  // namespace sllbm
