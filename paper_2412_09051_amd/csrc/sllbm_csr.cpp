// Curvilinear (isoparametric quadrilateral) plan builder: for every (velocity, node)
// pair the departure point x_k - dt zeta_i, the boundary case met first along the
// backward path (Sec. 3.3), the cell that contains the final departure point and its
// (p+1)^2 interpolation weights (eq:intf).  The rows are stored CSR-by-cell for the
// GPU: cell id, source velocity (or inlet index) and weights, SoA over nodes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

#include "sllbm_internal.h"

namespace sllbm {
namespace {

constexpr double kInsideTol = 1e-10;   // reference-coordinate tolerance of "inside a cell"

// Lagrange basis values and derivatives at xi (barycentric weights for the values,
// derivative by differentiating the barycentric form).
void basis_and_deriv(const std::vector<double> &xr, double xi, double *l, double *dl) {
  int n = (int)xr.size();
  lagrange_weights(xr, xi, l);
  for (int j = 0; j < n; j++) {
    double s = 0.0;
    for (int k = 0; k < n; k++) {
      if (k == j) continue;
      double t = 1.0 / (xr[j] - xr[k]);
      for (int q = 0; q < n; q++)
        if (q != j && q != k) t *= (xi - xr[q]) / (xr[j] - xr[q]);
      s += t;
    }
    dl[j] = s;
  }
}

struct Geo {
  const Mesh &m;
  int p, n1, npc;
  std::vector<double> box;            // [c][4] x0 x1 y0 y1 (widened)
  double bx0 = 0, by0 = 0, bh = 1;
  int bnx = 1, bny = 1;
  std::vector<int64_t> bstart, bcells; // bucket -> cells
  // boundary faces: (cell, face) with bbox; bucketed the same way
  std::vector<int64_t> fcell;
  std::vector<int> fside;
  std::vector<double> fbox;
  std::vector<int64_t> fbstart, fbfaces;

  explicit Geo(const Mesh &mm) : m(mm), p(mm.p), n1(mm.p + 1), npc((mm.p + 1) * (mm.p + 1)) {}

  const double *X(int64_t node) const { return &m.node_xyz[2 * node]; }
  int64_t cn(int64_t c, int j) const { return m.cell_nodes[c * npc + j]; }

  void cell_map(int64_t c, double xi, double eta, double *x, double J[2][2]) const {
    double lx[kMaxP + 1], ly[kMaxP + 1], dx[kMaxP + 1], dy[kMaxP + 1];
    basis_and_deriv(m.xref, xi, lx, dx);
    basis_and_deriv(m.xref, eta, ly, dy);
    x[0] = x[1] = 0;
    J[0][0] = J[0][1] = J[1][0] = J[1][1] = 0;
    for (int jy = 0; jy <= p; jy++)
      for (int jx = 0; jx <= p; jx++) {
        const double *P = X(cn(c, jx + n1 * jy));
        for (int a = 0; a < 2; a++) {
          x[a] += P[a] * lx[jx] * ly[jy];
          J[a][0] += P[a] * dx[jx] * ly[jy];
          J[a][1] += P[a] * lx[jx] * dy[jy];
        }
      }
  }

  bool newton(int64_t c, const double *x, double r0, double s0, double *r) const {
    r[0] = r0;
    r[1] = s0;
    for (int it = 0; it < 60; it++) {
      double y[2], J[2][2];
      cell_map(c, r[0], r[1], y, J);
      double e0 = x[0] - y[0], e1 = x[1] - y[1];
      double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      if (!(std::fabs(det) > 0.0)) return false;
      double d0 = (J[1][1] * e0 - J[0][1] * e1) / det, d1 = (J[0][0] * e1 - J[1][0] * e0) / det;
      double sz = std::max(std::fabs(d0), std::fabs(d1));
      if (sz > 0.5) { d0 *= 0.5 / sz; d1 *= 0.5 / sz; }
      r[0] += d0;
      r[1] += d1;
      if (std::fabs(r[0]) > 4.0 || std::fabs(r[1]) > 4.0) return false;
      if (std::fabs(d0) + std::fabs(d1) < 1e-11) {
        // converging quadratically: two plain corrections reach the rounding level
        // (about 1e-13 reference units in a thin cell, so no tighter test is reliable)
        for (int extra = 0; extra < 2; extra++) {
          cell_map(c, r[0], r[1], y, J);
          e0 = x[0] - y[0];
          e1 = x[1] - y[1];
          det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          if (!(std::fabs(det) > 0.0)) return false;
          r[0] += (J[1][1] * e0 - J[0][1] * e1) / det;
          r[1] += (J[0][0] * e1 - J[1][0] * e0) / det;
        }
        return true;
      }
    }
    return false;   // not converged: the caller tries another start
  }

  // reference coordinates of x in cell c, if inside (within kInsideTol)
  bool inverse(int64_t c, const double *x, double *r) const {
    double best = std::numeric_limits<double>::infinity();
    int bj = 0;
    for (int j = 0; j < npc; j++) {
      const double *P = X(cn(c, j));
      double d = (P[0] - x[0]) * (P[0] - x[0]) + (P[1] - x[1]) * (P[1] - x[1]);
      if (d == 0.0) {
        r[0] = m.xref[j % n1];
        r[1] = m.xref[j / n1];
        return true;
      }
      if (d < best) { best = d; bj = j; }
    }
    auto inside = [&](bool ok) {
      return ok && std::fabs(r[0]) <= 1.0 + kInsideTol && std::fabs(r[1]) <= 1.0 + kInsideTol;
    };
    // from the nearest support point Newton finds the cell's own root when x is inside;
    // a root found outside settles it.  Only a start that does not converge (next to a
    // degenerate corner) falls back to a 3x3 grid of starts.
    bool conv = newton(c, x, m.xref[bj % n1], m.xref[bj / n1], r);
    bool ok = inside(conv);
    if (!conv)
      for (int t = 0; !ok && t < 9; t++) ok = inside(newton(c, x, -0.6 + 0.6 * (t % 3), -0.6 + 0.6 * (t / 3), r));
    if (!ok) return false;
    r[0] = std::max(-1.0, std::min(1.0, r[0]));
    r[1] = std::max(-1.0, std::min(1.0, r[1]));
    return true;
  }

  int bucket_of(double x, double y, int *bi, int *bj) const {
    *bi = (int)std::floor((x - bx0) / bh);
    *bj = (int)std::floor((y - by0) / bh);
    return *bi >= 0 && *bj >= 0 && *bi < bnx && *bj < bny;
  }

  // node -> cells containing it (CSR)
  std::vector<int64_t> ncell_start, ncell_list;

  void build_node_cells() {
    ncell_start.assign(m.n_nodes + 1, 0);
    for (int64_t q = 0; q < m.n_cells * npc; q++) ncell_start[m.cell_nodes[q] + 1]++;
    for (int64_t k = 0; k < m.n_nodes; k++) ncell_start[k + 1] += ncell_start[k];
    ncell_list.resize(ncell_start[m.n_nodes]);
    std::vector<int64_t> fill(ncell_start.begin(), ncell_start.end() - 1);
    for (int64_t c = 0; c < m.n_cells; c++)
      for (int j = 0; j < npc; j++) ncell_list[fill[cn(c, j)]++] = c;
  }

  // the cell containing x, trying first the cells around node k (a departure point
  // lies within one short step of its node); -1 outside the mesh.  On a face shared by
  // two cells either one serves: the interpolant is continuous across it.
  int64_t locate_near(int64_t k, const double *x, double *r) const {
    for (int64_t q = ncell_start[k]; q < ncell_start[k + 1]; q++) {
      int64_t c = ncell_list[q];
      const double *B = &box[4 * c];
      if (x[0] < B[0] || x[0] > B[1] || x[1] < B[2] || x[1] > B[3]) continue;
      if (inverse(c, x, r)) return c;
    }
    return locate(x, r);
  }

  // the cell containing x (largest index on shared faces), -1 outside the mesh
  int64_t locate(const double *x, double *r) const {
    int bi, bj;
    if (!bucket_of(x[0], x[1], &bi, &bj)) return -1;
    int64_t b = (int64_t)bj * bnx + bi, best = -1;
    double t[2];
    for (int64_t q = bstart[b]; q < bstart[b + 1]; q++) {
      int64_t c = bcells[q];
      if (c <= best) continue;
      const double *B = &box[4 * c];
      if (x[0] < B[0] || x[0] > B[1] || x[1] < B[2] || x[1] > B[3]) continue;
      if (inverse(c, x, t)) { best = c; r[0] = t[0]; r[1] = t[1]; }
    }
    return best;
  }

  // boundary face curve: support points along face f of cell c, parameter t in [-1,1]
  void face_point(int64_t c, int f, double t, double *x, double *dx) const {
    double l[kMaxP + 1], dl[kMaxP + 1];
    basis_and_deriv(m.xref, t, l, dl);
    x[0] = x[1] = dx[0] = dx[1] = 0;
    for (int j = 0; j <= p; j++) {
      int jx = f == 0 ? 0 : (f == 1 ? p : j);
      int jy = f == 2 ? 0 : (f == 3 ? p : j);
      const double *P = X(cn(c, jx + n1 * jy));
      for (int a = 0; a < 2; a++) {
        x[a] += P[a] * l[j];
        dx[a] += P[a] * dl[j];
      }
    }
  }

  // unit normal of face f of cell c at face parameter t (point x, tangent tc), pointing
  // out of the cell: away from the point half a reference unit inward of the face
  void outward_normal(int64_t c, int f, double t, const double *tc, const double *x, double *n) const {
    double y[2], J[2][2];
    cell_map(c, f == 0 ? -0.5 : (f == 1 ? 0.5 : t), f == 2 ? -0.5 : (f == 3 ? 0.5 : t), y, J);
    double len = std::hypot(tc[0], tc[1]);
    n[0] = tc[1] / len;
    n[1] = -tc[0] / len;
    if (n[0] * (y[0] - x[0]) + n[1] * (y[1] - x[1]) > 0.0) {
      n[0] = -n[0];
      n[1] = -n[1];
    }
  }

  // a path x0 + s v tangent to face f of cell c at x0 = face(t0) leaves the mesh there
  // only if the face curves away from it (a convex boundary): its end x0 + v, projected
  // onto the face curve by Newton (extended past the face's ends if need be), lies on the
  // outward side by more than rounding.  Along a straight face the path stays on it.
  bool tangent_end_beyond(int64_t c, int f, double t0, const double *x0, const double *v, double xscale) const {
    double y[2] = {x0[0] + v[0], x0[1] + v[1]}, x[2], dx[2];
    double t = t0;
    for (int it = 0; it < 8; it++) {
      face_point(c, f, t, x, dx);
      double g = (x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1];
      t -= g / (dx[0] * dx[0] + dx[1] * dx[1]);   // Gauss-Newton on |face(t) - y|^2
    }
    face_point(c, f, t, x, dx);
    double n[2];
    outward_normal(c, f, t, dx, x, n);
    return n[0] * (y[0] - x[0]) + n[1] * (y[1] - x[1]) > 1e-12 * xscale;
  }

  // first boundary face crossed by x0 + s v, s in [0, 1]: returns s and the bc index
  bool first_crossing(const double *x0, const double *v, double *s_out, int *bc_out) const {
    double xs0 = std::min(x0[0], x0[0] + v[0]), xs1 = std::max(x0[0], x0[0] + v[0]);
    double ys0 = std::min(x0[1], x0[1] + v[1]), ys1 = std::max(x0[1], x0[1] + v[1]);
    int i0, j0, i1, j1;
    bucket_of(xs0, ys0, &i0, &j0);
    bucket_of(xs1, ys1, &i1, &j1);
    i0 = std::max(0, i0 - 1);
    j0 = std::max(0, j0 - 1);
    i1 = std::min(bnx - 1, i1 + 1);
    j1 = std::min(bny - 1, j1 + 1);
    double best = std::numeric_limits<double>::infinity();
    double scale = std::fabs(x0[0]) + std::fabs(x0[1]) + std::fabs(v[0]) + std::fabs(v[1]);
    double xscale = std::max(1.0, std::max(std::fabs(x0[0]), std::fabs(x0[1])));
    double tie = 1e-9 * xscale / std::max(std::fabs(v[0]), std::fabs(v[1]));
    int bbc = -1;
    for (int bj = j0; bj <= j1; bj++)
      for (int bi = i0; bi <= i1; bi++) {
        int64_t b = (int64_t)bj * bnx + bi;
        for (int64_t q = fbstart[b]; q < fbstart[b + 1]; q++) {
          int64_t fi = fbfaces[q];
          const double *B = &fbox[4 * fi];
          if (xs1 < B[0] || xs0 > B[1] || ys1 < B[2] || ys0 > B[3]) continue;
          int64_t c = fcell[fi];
          int f = fside[fi];
          // solve face(t) = x0 + s v for (t, s), Newton from several t
          for (int st = 0; st < 5; st++) {
            double t = -1.0 + 0.5 * st, s = 0.0;
            bool ok = false;
            for (int it = 0; it < 50; it++) {
              double x[2], dx[2];
              face_point(c, f, t, x, dx);
              double e0 = x[0] - x0[0] - s * v[0], e1 = x[1] - x0[1] - s * v[1];
              // at grazing incidence the steps stall at the rounding floor of s while
              // the residual is already at the rounding level of the coordinates
              if (it > 0 && std::fabs(e0) + std::fabs(e1) <= 4e-16 * scale) { ok = true; break; }
              // Jacobian of (t, s) -> face(t) - x0 - s v
              double a = dx[0], bb = -v[0], cc = dx[1], dd = -v[1];
              double det = a * dd - bb * cc;
              if (!(std::fabs(det) > 0.0)) break;
              double dt_ = (dd * e0 - bb * e1) / det, ds = (a * e1 - cc * e0) / det;
              t -= dt_;
              s -= ds;
              if (std::fabs(t) > 3.0) break;
              // t and s are O(1): a step below 1e-12 is converged to rounding level
              if (std::fabs(dt_) + std::fabs(ds) < 1e-12) { ok = true; break; }
            }
            if (!ok) continue;
            if (std::fabs(t) <= 1.0 + 1e-9 && s >= -1e-9 && s <= 1.0 + 1e-9) {
              int tag = m.cell_face_bc[c * 4 + f];
              double xc[2], tc[2];
              face_point(c, f, t, xc, tc);
              if (std::fabs(xc[0] - x0[0]) + std::fabs(xc[1] - x0[1]) <= 1e-12 * xscale) {
                // the crossing is x0 itself (a boundary node): it counts only if the
                // path leaves the mesh there, tangent paths included
                double n[2];
                outward_normal(c, f, t, tc, xc, n);
                double nv = n[0] * v[0] + n[1] * v[1], vl = std::hypot(v[0], v[1]);
                if (nv < -1e-12 * vl) continue;
                if (nv <= 1e-12 * vl && !tangent_end_beyond(c, f, t, x0, v, xscale)) continue;
                s = 0.0;
              }
              s = std::max(0.0, s);
              // where two boundary segments meet, the path crosses both at once
              // (crossing points closer than 1e-9 max(1, |x0|)): the segment with the
              // smaller tag decides
              if (s < best - tie) {
                best = s;
                bbc = tag;
              } else if (s <= best + tie) {
                best = std::min(best, s);
                bbc = std::min(bbc, tag);
              }
            }
          }
        }
      }
    if (bbc < 0) {
      // no transversal crossing: the path touches the boundary tangentially (a double
      // root, typically at s = 0 from a boundary node on a convex boundary).  Bracket the
      // exit by bisection on point location and take the nearest boundary face's tag.
      double lo = 0.0, hi = 1.0, r[2];
      for (int it = 0; it < 60; it++) {
        double mid = 0.5 * (lo + hi), y[2] = {x0[0] + mid * v[0], x0[1] + mid * v[1]};
        if (locate(y, r) >= 0) lo = mid; else hi = mid;
      }
      double y[2] = {x0[0] + lo * v[0], x0[1] + lo * v[1]};
      int64_t c;
      int tag = std::numeric_limits<int>::max();
      if (!project_to_boundary(y, std::fabs(v[0]) + std::fabs(v[1]), &c, r, &tag) ||
          tag == std::numeric_limits<int>::max())
        return false;
      *s_out = lo;
      *bc_out = tag;
      return true;
    }
    *s_out = best;
    *bc_out = bbc;
    return true;
  }

  // nearest point of the mesh boundary to y (orthogonal projection onto the tagged
  // faces near y): its cell and reference coordinates
  bool project_to_boundary(const double *y, double reach, int64_t *c_out, double *r_out, int *tag_out = nullptr) const {
    int i0, j0, i1, j1;
    bucket_of(y[0] - reach, y[1] - reach, &i0, &j0);
    bucket_of(y[0] + reach, y[1] + reach, &i1, &j1);
    i0 = std::max(0, i0 - 1);
    j0 = std::max(0, j0 - 1);
    i1 = std::min(bnx - 1, i1 + 1);
    j1 = std::min(bny - 1, j1 + 1);
    double best = std::numeric_limits<double>::infinity();
    for (int bj = j0; bj <= j1; bj++)
      for (int bi = i0; bi <= i1; bi++) {
        int64_t b = (int64_t)bj * bnx + bi;
        for (int64_t q = fbstart[b]; q < fbstart[b + 1]; q++) {
          int64_t fi = fbfaces[q];
          int64_t c = fcell[fi];
          int f = fside[fi];
          for (int st = 0; st < 5; st++) {
            // Gauss-Newton on |face(t) - y|^2 with t kept in [-1, 1]
            double t = -1.0 + 0.5 * st, x[2], dx[2];
            for (int it = 0; it < 60; it++) {
              face_point(c, f, t, x, dx);
              double g = (x[0] - y[0]) * dx[0] + (x[1] - y[1]) * dx[1];
              double h = dx[0] * dx[0] + dx[1] * dx[1];
              double tn = std::max(-1.0, std::min(1.0, t - g / h));
              bool done = std::fabs(tn - t) < 1e-15;
              t = tn;
              if (done) break;
            }
            face_point(c, f, t, x, dx);
            double dd = (x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]);
            int tag = m.cell_face_bc[c * 4 + f];
            // equally near faces (a junction of boundary segments): the smaller tag
            bool tie = std::isfinite(best) && std::fabs(dd - best) <= 1e-24 + 1e-12 * best;
            if ((dd < best && !tie) || (tie && tag_out && tag < *tag_out)) {
              best = std::min(dd, best);
              *c_out = c;
              if (tag_out) *tag_out = tag;
              r_out[0] = f == 0 ? -1.0 : (f == 1 ? 1.0 : t);
              r_out[1] = f == 2 ? -1.0 : (f == 3 ? 1.0 : t);
            }
          }
        }
      }
    return std::isfinite(best);
  }

  void build_buckets() {
    int64_t nc = m.n_cells;
    box.resize(4 * nc);
    std::vector<double> ext(nc);
    double gx0 = 1e300, gx1 = -1e300, gy0 = 1e300, gy1 = -1e300;
    for (int64_t c = 0; c < nc; c++) {
      double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
      for (int j = 0; j < npc; j++) {
        const double *P = X(cn(c, j));
        x0 = std::min(x0, P[0]);
        x1 = std::max(x1, P[0]);
        y0 = std::min(y0, P[1]);
        y1 = std::max(y1, P[1]);
      }
      double wx = 0.05 * (x1 - x0) + 1e-12, wy = 0.05 * (y1 - y0) + 1e-12;
      box[4 * c] = x0 - wx;
      box[4 * c + 1] = x1 + wx;
      box[4 * c + 2] = y0 - wy;
      box[4 * c + 3] = y1 + wy;
      ext[c] = std::max(x1 - x0, y1 - y0);
      gx0 = std::min(gx0, box[4 * c]);
      gx1 = std::max(gx1, box[4 * c + 1]);
      gy0 = std::min(gy0, box[4 * c + 2]);
      gy1 = std::max(gy1, box[4 * c + 3]);
    }
    std::vector<double> e2 = ext;
    std::nth_element(e2.begin(), e2.begin() + e2.size() / 2, e2.end());
    bh = std::max(e2[e2.size() / 2], std::max(gx1 - gx0, gy1 - gy0) / 2000.0);
    bx0 = gx0 - bh;
    by0 = gy0 - bh;
    bnx = (int)((gx1 - bx0) / bh) + 2;
    bny = (int)((gy1 - by0) / bh) + 2;
    auto fill = [&](const std::vector<double> &bx, int64_t n, std::vector<int64_t> &start, std::vector<int64_t> &items) {
      int64_t nb = (int64_t)bnx * bny;
      std::vector<int64_t> cnt(nb + 1, 0);
      for (int pass = 0; pass < 2; pass++) {
        for (int64_t c = 0; c < n; c++) {
          int i0, j0, i1, j1;
          bucket_of(bx[4 * c], bx[4 * c + 2], &i0, &j0);
          bucket_of(bx[4 * c + 1], bx[4 * c + 3], &i1, &j1);
          for (int bj = std::max(0, j0); bj <= std::min(bny - 1, j1); bj++)
            for (int bi = std::max(0, i0); bi <= std::min(bnx - 1, i1); bi++) {
              int64_t b = (int64_t)bj * bnx + bi;
              if (pass == 0) cnt[b + 1]++;
              else items[start[b] + cnt[b]++] = c;
            }
        }
        if (pass == 0) {
          start.assign(nb + 1, 0);
          for (int64_t b = 0; b < nb; b++) start[b + 1] = start[b] + cnt[b + 1];
          items.assign(start[nb], 0);
          std::fill(cnt.begin(), cnt.end(), 0);
        }
      }
    };
    fill(box, nc, bstart, bcells);
    for (int64_t c = 0; c < nc; c++)
      for (int f = 0; f < 4; f++) {
        if (m.cell_face_bc[c * 4 + f] < 0) continue;
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int j = 0; j <= p; j++) {
          int jx = f == 0 ? 0 : (f == 1 ? p : j);
          int jy = f == 2 ? 0 : (f == 3 ? p : j);
          const double *P = X(cn(c, jx + n1 * jy));
          x0 = std::min(x0, P[0]);
          x1 = std::max(x1, P[0]);
          y0 = std::min(y0, P[1]);
          y1 = std::max(y1, P[1]);
        }
        double w = 0.1 * std::max(x1 - x0, y1 - y0) + 1e-12;
        fcell.push_back(c);
        fside.push_back(f);
        fbox.insert(fbox.end(), {x0 - w, x1 + w, y0 - w, y1 + w});
      }
    fill(fbox, (int64_t)fcell.size(), fbstart, fbfaces);
  }
};

}  // namespace

int build_csr_tables(const Mesh &m, const VelSet &v, double dt, HostTables &t, int64_t *n_exc, int64_t *n_th) {
  if (m.dim != 2) return fail(SLLBM_EUNSUPPORTED, "curvilinear plans are 2D");
  Geo g(m);
  g.build_buckets();
  g.build_node_cells();
  const int Q = v.Q;
  const int64_t N = m.n_nodes;
  t.row_cell.assign((size_t)Q * N, -1);
  t.row_src.assign((size_t)Q * N, 0);
  t.row_xi.assign((size_t)Q * 2 * N, 0.0);
  t.node_Tw.assign(N, std::numeric_limits<double>::quiet_NaN());
  std::atomic<int> status{SLLBM_OK};
  std::atomic<int64_t> bad_k{-1}, bad_i{-1}, exc{0};
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int64_t k0, int64_t k1) {
    int64_t local_exc = 0;
    for (int64_t k = k0; k < k1 && status.load() == SLLBM_OK; k++) {
      const double *xk = g.X(k);
      for (int i = 0; i < Q; i++) {
        double d[2] = {dt * v.zeta[2 * i], dt * v.zeta[2 * i + 1]};
        double dp[2] = {xk[0] - d[0], xk[1] - d[1]}, r[2];
        int src = i;
        int64_t c = g.locate_near(k, dp, r);
        if (c < 0) {
          local_exc++;
          double mv[2] = {-d[0], -d[1]}, s;
          int bc;
          if (!g.first_crossing(xk, mv, &s, &bc)) {
            status = SLLBM_EGEOM; bad_k = k; bad_i = i;
            return;
          }
          const sllbm_bc &B = m.bcs[bc];
          if (B.kind == SLLBM_BC_WALL) {
            // Sec. 3.3.2: opposite population at x_k + (1 - 2 s) dt zeta_i
            dp[0] = xk[0] + (1.0 - 2.0 * s) * d[0];
            dp[1] = xk[1] + (1.0 - 2.0 * s) * d[1];
            c = g.locate_near(k, dp, r);
            // reflected out of the mesh again (a corner, a thin gap): the nearest
            // boundary point
            if (c < 0 && !g.project_to_boundary(dp, std::fabs(d[0]) + std::fabs(d[1]), &c, r)) c = -1;
            if (c < 0) { status = SLLBM_EGEOM; bad_k = k; bad_i = i; return; }
            src = v.opp[i];
            if (std::isfinite(B.T_wall)) t.node_Tw[k] = B.T_wall;
          } else if (B.kind == SLLBM_BC_INLET) {
            t.row_cell[(size_t)i * N + k] = -1;
            t.row_src[(size_t)i * N + k] = bc;
            continue;
          } else if (B.kind == SLLBM_BC_OUTLET) {
            // Sec. 3.3.3: population i at x_k + dt zeta_i; outside the mesh, at the
            // nearest boundary point (the per-axis clamp of a tensor mesh)
            dp[0] = xk[0] + d[0];
            dp[1] = xk[1] + d[1];
            c = g.locate_near(k, dp, r);
            if (c < 0 && !g.project_to_boundary(dp, std::fabs(d[0]) + std::fabs(d[1]), &c, r)) c = -1;
            if (c < 0) { status = SLLBM_EGEOM; bad_k = k; bad_i = i; return; }
          } else {
            status = SLLBM_EGEOM; bad_k = k; bad_i = i;
            return;
          }
        }
        t.row_cell[(size_t)i * N + k] = (int32_t)c;
        t.row_src[(size_t)i * N + k] = src;
        t.row_xi[((size_t)i * 2) * N + k] = r[0];
        t.row_xi[((size_t)i * 2 + 1) * N + k] = r[1];
      }
    }
    exc += local_exc;
  };
  std::vector<std::thread> pool;
  int64_t chunk = (N + nth - 1) / nth;
  for (unsigned w = 0; w < nth; w++) {
    int64_t k0 = w * chunk, k1 = std::min<int64_t>(N, k0 + chunk);
    if (k0 < k1) pool.emplace_back(work, k0, k1);
  }
  for (auto &th : pool) th.join();
  if (status != SLLBM_OK)
    return fail(SLLBM_EGEOM, "departure point of node %lld velocity %lld cannot be placed in the mesh",
                (long long)bad_k.load(), (long long)bad_i.load());
  *n_exc = exc.load();
  int64_t nthm = 0;
  for (double T : t.node_Tw)
    if (std::isfinite(T)) nthm++;
  *n_th = nthm;
  return SLLBM_OK;
}

}  // namespace sllbm
