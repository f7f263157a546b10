/*
 * fco_sphere.c -- cubed-sphere geometry and shallow-water solver of the CPU
 * oracle (test infrastructure only).
 *
 * Sec. 2 / Sec. 4: six mapped trees cover the sphere; the wave-propagation
 * update runs in computational coordinates with a capacity (cell area over
 * computational area) and edge metrics.  The paper names the geometry and
 * the method it follows for mapped grids (Calhoun, Helzel and LeVeque,
 * SIAM Review 2008); the formulas below are that method written out.
 *
 * Mapping (gnomonic, equiangular).  Tree t is cube face t with centre c,
 * axes u, v (u x v = c); the reference point (xi, eta) goes to the cube
 * point c + T(xi) u + T(eta) v, T(s) = tan((s - 1/2) pi/2), then to the
 * unit sphere.  T(0) = -1, T(1) = 1 and T(1 - s) = -T(s) exactly, so a
 * point on a cube edge gets the same coordinates from either face.
 *
 * Pillow sphere (two trees; the paper's Sec. 5 sphere example maps one
 * quadtree to each hemisphere, after Calhoun, Helzel and LeVeque).  The map
 * here is this oracle's own choice of such a map: with x = 2 xi - 1, y =
 * 2 eta - 1 and d = max(|x|, |y|), the square of half-width d goes to the
 * circle of polar angle theta = d pi / 2 about the tree's pole, each point
 * along its own direction (x, y) / |(x, y)|:
 *   tree 0: (sin theta x / rho, sin theta y / rho, cos theta), rho = |(x, y)|;
 *   tree 1: the same with the second and third components negated (so that
 *     both trees are right-handed seen from outside).
 * The square's boundary (d = 1) goes to the equator, exactly (sin = 1,
 * cos = 0 there); tree 0's face eta = 0 meets tree 1's face eta = 1 and
 * its face eta = 1 meets tree 1's eta = 0 (tangential coordinates the same
 * way), and the faces xi = 0 and xi = 1 meet their namesakes with the
 * tangential coordinate reversed.  Each square corner is a point where only
 * the two trees' corner cells meet (each with a straight angle); the region
 * beyond it, reached across either face, is the own tree's corner mirrored
 * through that point.
 *
 * Geometry of a patch, for its cells and its two ghost layers: a corner
 * point outside the patch's tree is carried into the tree that contains it
 * and mapped there, so ghost cells have the geometry of the cells whose
 * values they hold.  At a cube vertex no tree holds the corner region of
 * the ghost layers (three faces leave no room for a fourth quadrant): the
 * cells of that region, and edges between two of them, take the patch's own
 * face mapping extended; an edge between such a cell and any other cell
 * keeps the canonical points, which the neighbouring patch sees as well.
 *   capacity kappa = (area of the spherical quadrilateral) / dxi^2, area as
 *     two spherical triangles (a, b, c) + (a, c, d) with the solid-angle
 *     formula of Van Oosterom and Strackee;
 *   edge from corner a to corner b: gamma = (great-circle length) / dxi,
 *     unit normal n along (b x a) for xi-edges and (a x b) for eta-edges
 *     (both point towards increasing index), unit tangent t = r_m x n with
 *     r_m the normalised midpoint a + b;
 *   cell centre: the image of the centre of the computational cell.
 *
 * Equations: shallow water with 3D Cartesian momentum, q = (h, hu, hv, hw).
 * At an edge the momenta are rotated into (n, t), the 1D Roe problem gives
 * three waves, which are rotated back; speeds are scaled by gamma.  The
 * mass component is advanced in flux form, F = gamma (m_l + m_r).n / 2 -
 * (A+dq - A-dq)_h / 2, so that mass is conserved on curved cells.
 * Transverse splitting uses the frame and gamma of the receiving cell's
 * transverse edge and the Roe averages of the normal edge's states.  After
 * a step the momentum is projected onto the tangent plane at the cell
 * centre.
 */
#include "fco_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double FACE[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {0, 1, 0}, {-1, 0, 0}},
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

static double tline(int64_t X) {
  const int64_t d = 2 * X - FCO_SIDE;
  if (d == 0) return 0.0;
  const int64_t ad = d < 0 ? -d : d;
  const double t = ad == FCO_SIDE ? 1.0
                                  : tan(ldexp((double)ad, -FCO_S) * 0.78539816339744830962);
  return d < 0 ? -t : t;
}

int fco_pillow_trees(int32_t ntrees, const fco_tree *trees) {
  static const int32_t NF[4] = {0, 1, 3, 2}, OR[4] = {1, 1, 0, 0};
  if (ntrees != 2) return 0;
  for (int t = 0; t < 2; ++t)
    for (int f = 0; f < 4; ++f)
      if (trees[t].bc[f] != 0 || trees[t].nbr_tree[f] != 1 - t ||
          trees[t].nbr_face[f] != NF[f] || trees[t].orient[f] != OR[f])
        return 0;
  return 1;
}

static void pillow_point(int32_t t, int64_t X, int64_t Y, double r[3]) {
  const double x = ldexp((double)(2 * X - FCO_SIDE), -FCO_S);
  const double y = ldexp((double)(2 * Y - FCO_SIDE), -FCO_S);
  const double d = fmax(fabs(x), fabs(y));
  double s = 0.0, c = 1.0, ux = 0.0, uy = 0.0;
  if (d > 0.0) {
    const double rho = sqrt(x * x + y * y);
    ux = x / rho;
    uy = y / rho;
    if (d == 1.0) {
      s = 1.0;
      c = 0.0;
    } else {
      s = sin(d * 1.57079632679489661923);
      c = cos(d * 1.57079632679489661923);
    }
  }
  r[0] = s * ux;
  r[1] = t == 1 ? 0.0 - s * uy : s * uy;
  r[2] = t == 1 ? 0.0 - c : c;
}

static void cube_point(int32_t t, int64_t X, int64_t Y, double r[3]) {
  const double a = tline(X), b = tline(Y);
  double p[3];
  for (int c = 0; c < 3; ++c) p[c] = FACE[t][0][c] + a * FACE[t][1][c] + b * FACE[t][2][c];
  const double s = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  for (int c = 0; c < 3; ++c) r[c] = p[c] / s;
}

static void face_point(const fco_mesh *mesh, int32_t t, int64_t X, int64_t Y, double r[3]) {
  if (mesh->pillow)
    pillow_point(t, X, Y, r);
  else
    cube_point(t, X, Y, r);
}

/* sphere point of tree coordinates (X, Y) of tree t, carried into the tree
 * that contains it (closed trees; own face extended at a cube vertex) */
static void map_point(const fco_mesh *mesh, int32_t t, int64_t X, int64_t Y,
                      double r[3]) {
  const int ox = X < 0 || X > FCO_SIDE, oy = Y < 0 || Y > FCO_SIDE;
  int32_t t2 = t;
  int64_t x = X, y = Y;
  if (ox && !oy) {
    fco_cross_face(mesh->trees, t, X < 0 ? 0 : 1, &x, &y, &t2);
  } else if (oy && !ox) {
    fco_cross_face(mesh->trees, t, Y < 0 ? 2 : 3, &x, &y, &t2);
  } else if (ox && oy) {
    if (fco_locate(mesh->trees, t, X, Y, &t2, &x, &y) != 0) {
      t2 = t;   /* cube vertex: no tree holds the point */
      x = X;
      y = Y;
    }
  }
  face_point(mesh, t2, x, y, r);
}

static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* solid angle of the spherical triangle (a, b, c), counter-clockwise (Van
 * Oosterom and Strackee).  The triple product a.(b x c) of three nearly
 * parallel unit vectors is formed as a.((b - a) x (c - a)), equal in exact
 * arithmetic: the differences of close points are exact and the cross
 * product of the short vectors keeps full relative accuracy, where b x c
 * itself would lose it to cancellation (a relative error of order eps / h^2
 * for a cell of angular size h). */
static double tri(const double a[3], const double b[3], const double c[3]) {
  double u[3], v[3], w[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = b[k] - a[k];
    v[k] = c[k] - a[k];
  }
  cross3(u, v, w);
  return 2.0 * atan2(dot3(a, w), 1.0 + dot3(a, b) + dot3(b, c) + dot3(c, a));
}

/* a x b of two nearly parallel unit vectors, formed as ((a + b) / 2) x
 * (b - a): equal in exact arithmetic, accurate for close points, and
 * exactly negated when a and b are swapped (so that a cell edge is the same
 * whichever side computes it). */
static void cross_close(const double a[3], const double b[3], double o[3]) {
  double mid[3], d[3];
  for (int k = 0; k < 3; ++k) {
    mid[k] = 0.5 * (a[k] + b[k]);
    d[k] = b[k] - a[k];
  }
  cross3(mid, d, o);
}

/* table offsets, in frames: capacity, centre, edges (gamma, n, t per
 * direction), and the chord b - a of each low-side edge (per direction) */
enum { GK = 0, GC = 1, GE = 4, GD = 18, GN = 24 };

/* corner points of patch p: canonical (carried into the tree that holds
 * them) and the patch's own face mapping extended (used for the corner
 * region at a cube vertex, which no tree covers) */
static void patch_corners(const fco_mesh *mesh, int64_t p, double *cor, double *ext) {
  const int32_t m = mesh->m;
  const fco_leaf *a = &mesh->leaves[p];
  const int64_t size = FCO_SIDE >> a->level, cs = size / m;
  const int64_t x0 = (int64_t)a->ix * size, y0 = (int64_t)a->iy * size;
  const int NC = m + 5;
  for (int J = -2; J <= m + 2; ++J)
    for (int I = -2; I <= m + 2; ++I) {
      const int64_t X = x0 + I * cs, Y = y0 + J * cs;
      map_point(mesh, a->tree, X, Y, &cor[3 * ((J + 2) * NC + (I + 2))]);
      face_point(mesh, a->tree, X, Y, &ext[3 * ((J + 2) * NC + (I + 2))]);
    }
}

/* 1 if frame cell (i, j) of patch p lies in a corner region at a cube
 * vertex (no tree holds it) */
static int vertex_cell(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j) {
  const int32_t m = mesh->m;
  if ((i >= 1 && i <= m) || (j >= 1 && j <= m)) return 0;
  const fco_leaf *a = &mesh->leaves[p];
  const int64_t size = FCO_SIDE >> a->level, cs = size / m;
  const int64_t X = (int64_t)a->ix * size + (2 * i - 1) * cs / 2;
  const int64_t Y = (int64_t)a->iy * size + (2 * j - 1) * cs / 2;
  int32_t t2;
  int64_t x2, y2;
  return fco_locate(mesh->trees, a->tree, X, Y, &t2, &x2, &y2) == 2;
}

int fco_sphere_build(fco_mesh *mesh) {
  const int32_t m = mesh->m;
  const int64_t FR = fco_frame(m), n = mesh->n;
  mesh->geo = (double *)malloc(sizeof(double) * GN * FR * n);
  if (!mesh->geo) return -1;
  const int NC = m + 5;   /* corner indices -2 .. m+2 */
  double *cor = (double *)malloc(sizeof(double) * 6 * NC * NC);
  if (!cor) return -1;
  double *ext = cor + 3 * NC * NC;
  for (int64_t p = 0; p < n; ++p) {
    const fco_leaf *a = &mesh->leaves[p];
    const int64_t size = FCO_SIDE >> a->level, cs = size / m;
    const int64_t x0 = (int64_t)a->ix * size, y0 = (int64_t)a->iy * size;
    const double dx = ldexp(1.0, -a->level) / m;
    patch_corners(mesh, p, cor, ext);
#define PT(arr, I, J) (&(arr)[3 * (((J) + 2) * NC + ((I) + 2))])
    double *g = mesh->geo + p * GN * FR;
    for (int32_t j = -1; j <= m + 2; ++j)
      for (int32_t i = -1; i <= m + 2; ++i) {
        const int64_t f = fco_fidx(m, i, j);
        const int vc = vertex_cell(mesh, p, i, j);
        const double *src = vc ? ext : cor;
        const double *A = PT(src, i - 1, j - 1), *B = PT(src, i, j - 1),
                     *Cc = PT(src, i, j), *D = PT(src, i - 1, j);
        g[GK * FR + f] = (tri(A, B, Cc) + tri(A, Cc, D)) / (dx * dx);
        map_point(mesh, a->tree, x0 + (2 * i - 1) * cs / 2, y0 + (2 * j - 1) * cs / 2,
                  &g[GC * FR + 3 * f]);
        for (int dir = 0; dir < 2; ++dir) {
          /* the low-side edge is shared with cell (i-1, j) or (i, j-1) */
          const int vn = dir == 0 ? vertex_cell(mesh, p, i - 1, j)
                                  : vertex_cell(mesh, p, i, j - 1);
          const double *es = (vc && vn) ? ext : cor;
          const double *ea = PT(es, i - 1, j - 1);
          const double *eb = dir == 0 ? PT(es, i - 1, j) : PT(es, i, j - 1);
          double cr[3], nn[3], rm[3], tt[3];
          cross_close(ea, eb, cr);
          const double len = sqrt(dot3(cr, cr));
          const double sg = dir == 0 ? -1.0 : 1.0;     /* xi-edge: b x a */
          for (int c = 0; c < 3; ++c) nn[c] = sg * cr[c] / len;
          for (int c = 0; c < 3; ++c) rm[c] = ea[c] + eb[c];
          const double rl = sqrt(dot3(rm, rm));
          for (int c = 0; c < 3; ++c) rm[c] /= rl;
          cross3(rm, nn, tt);
          double *ch = &g[GD * FR + (dir * FR + f) * 3];
          for (int c = 0; c < 3; ++c) ch[c] = eb[c] - ea[c];
          double *e = &g[GE * FR + (dir * FR + f) * 7];
          e[0] = atan2(len, dot3(ea, eb)) / dx;
          for (int c = 0; c < 3; ++c) e[1 + c] = nn[c];
          for (int c = 0; c < 3; ++c) e[4 + c] = tt[c];
        }
      }
#undef PT
  }
  free(cor);
  return 0;
}

double fco_sphere_kappa(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j) {
  const int64_t FR = fco_frame(mesh->m);
  return mesh->geo[p * GN * FR + GK * FR + fco_fidx(mesh->m, i, j)];
}

void fco_sphere_edge(const fco_mesh *mesh, int64_t p, int32_t dir, int32_t i,
                     int32_t j, double *gamma, double n[3], double t[3]) {
  const int64_t FR = fco_frame(mesh->m);
  const double *e = &mesh->geo[p * GN * FR + GE * FR +
                               (dir * FR + fco_fidx(mesh->m, i, j)) * 7];
  *gamma = e[0];
  for (int c = 0; c < 3; ++c) {
    n[c] = e[1 + c];
    t[c] = e[4 + c];
  }
}

void fco_sphere_centre(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j,
                       double r[3]) {
  const int64_t FR = fco_frame(mesh->m);
  const double *c = &mesh->geo[p * GN * FR + GC * FR + 3 * fco_fidx(mesh->m, i, j)];
  for (int k = 0; k < 3; ++k) r[k] = c[k];
}

double fco_rotation_edge(const fco_mesh *mesh, const fco_params *par, int64_t p,
                         int32_t dir, int32_t i, int32_t j) {
  const int64_t FR = fco_frame(mesh->m);
  const double *ch = &mesh->geo[p * GN * FR + GD * FR + (dir * FR + fco_fidx(mesh->m, i, j)) * 3];
  const double *w = par->axis;
  const double wl = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double omega = 2.0 * 3.14159265358979323846 / par->period;
  const double dx = ldexp(1.0, -mesh->leaves[p].level) / mesh->m;
  /* the xi-edge runs from corner (i-1, j-1) to (i-1, j) and higher i lies
   * to its right; the eta-edge runs from (i-1, j-1) to (i, j-1) with higher
   * j to its left: the flux towards higher index is +dpsi and -dpsi */
  const double dpsi = omega * (w[0] * ch[0] + w[1] * ch[1] + w[2] * ch[2]) / wl;
  return (dir == 0 ? dpsi : -dpsi) / dx;
}

/* ---- solver ------------------------------------------------------------ */
typedef fco_edge_geom edge_geom;

/* Normal Riemann problem at an edge: waves W[w*4+k] (3D momentum), speeds
 * s[w] (times gamma), fluctuations; *fl = mass flux through the edge. */
int fco_rp_sphere(const fco_params *par, const edge_geom *e, const double *ql,
                  const double *qr, double *W, double *s, double *am,
                  double *ap, double *fl) {
  const double hl = ql[0], hr = qr[0];
  if (!(hl > 0.0) || !(hr > 0.0)) return -1;
  const double nl = ql[1] * e->n[0] + ql[2] * e->n[1] + ql[3] * e->n[2];
  const double nr = qr[1] * e->n[0] + qr[2] * e->n[1] + qr[3] * e->n[2];
  const double tl = ql[1] * e->t[0] + ql[2] * e->t[1] + ql[3] * e->t[2];
  const double tr = qr[1] * e->t[0] + qr[2] * e->t[1] + qr[3] * e->t[2];
  const double sl = sqrt(hl), sr = sqrt(hr);
  const double u = (nl / sl + nr / sr) / (sl + sr);
  const double v = (tl / sl + tr / sr) / (sl + sr);
  const double c = sqrt(par->g * 0.5 * (hl + hr));
  const double d0 = hr - hl, d1 = nr - nl, d2 = tr - tl;
  const double a1 = ((u + c) * d0 - d1) / (2.0 * c);
  const double a2 = d2 - v * d0;
  const double a3 = (d1 - (u - c) * d0) / (2.0 * c);
  /* waves in (h, normal, tangential), then rotated to 3D */
  const double w1[3] = {a1, a1 * (u - c), a1 * v};
  const double w2[3] = {0.0, 0.0, a2};
  const double w3[3] = {a3, a3 * (u + c), a3 * v};
  const double *wl[3] = {w1, w2, w3};
  const double sp[3] = {u - c, u, u + c};
  for (int w = 0; w < 3; ++w) {
    W[w * 4 + 0] = wl[w][0];
    for (int k = 0; k < 3; ++k) W[w * 4 + 1 + k] = wl[w][1] * e->n[k] + wl[w][2] * e->t[k];
    s[w] = e->gamma * sp[w];
  }
  for (int k = 0; k < 4; ++k) {
    am[k] = 0.0;
    ap[k] = 0.0;
    for (int w = 0; w < 3; ++w) {
      am[k] += fmin(s[w], 0.0) * W[w * 4 + k];
      ap[k] += fmax(s[w], 0.0) * W[w * 4 + k];
    }
  }
  if (fl) *fl = 0.5 * e->gamma * (nl + nr) - 0.5 * (ap[0] - am[0]);
  return 3;
}

/* Part of the fluctuation psi that crosses the transverse edge tedge of
 * the receiving cell: down-going (up = 0, its lower edge) or up-going
 * (up = 1, its upper edge); Roe averages from the normal edge's states. */
int fco_tsplit_sphere(const fco_params *par, const double *ql, const double *qr,
                      const edge_geom *tedge, const double *psi, double *out,
                      int up) {
  const double hl = ql[0], hr = qr[0];
  if (!(hl > 0.0) || !(hr > 0.0)) return -1;
  const double sl = sqrt(hl), sr = sqrt(hr);
  double ub[3];
  for (int k = 0; k < 3; ++k) ub[k] = (ql[1 + k] / sl + qr[1 + k] / sr) / (sl + sr);
  const double c = sqrt(par->g * 0.5 * (hl + hr));
  const double *n = tedge->n, *t = tedge->t;
  const double un = ub[0] * n[0] + ub[1] * n[1] + ub[2] * n[2];
  const double ut = ub[0] * t[0] + ub[1] * t[1] + ub[2] * t[2];
  const double pn = psi[1] * n[0] + psi[2] * n[1] + psi[3] * n[2];
  const double pt = psi[1] * t[0] + psi[2] * t[1] + psi[3] * t[2];
  const double b1 = ((un + c) * psi[0] - pn) / (2.0 * c);
  const double b2 = pt - ut * psi[0];
  const double b3 = (pn - (un - c) * psi[0]) / (2.0 * c);
  const double lam[3] = {tedge->gamma * (un - c), tedge->gamma * un,
                         tedge->gamma * (un + c)};
  /* eigenvectors (1, (un - c) n + ut t), (0, t), (1, (un + c) n + ut t) */
  double R[3][4];
  R[0][0] = 1.0; R[1][0] = 0.0; R[2][0] = 1.0;
  for (int k = 0; k < 3; ++k) {
    R[0][1 + k] = (un - c) * n[k] + ut * t[k];
    R[1][1 + k] = t[k];
    R[2][1 + k] = (un + c) * n[k] + ut * t[k];
  }
  const double beta[3] = {b1, b2, b3};
  for (int k = 0; k < 4; ++k) {
    out[k] = 0.0;
    for (int w = 0; w < 3; ++w) {
      const double l = up ? fmax(lam[w], 0.0) : fmin(lam[w], 0.0);
      out[k] += l * beta[w] * R[w][k];
    }
  }
  return 0;
}

/* momentum of interior cells onto the tangent plane at the cell centre */
void fco_sphere_project(const fco_mesh *mesh, const fco_params *par, double *qn) {
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t FR = fco_frame(m);
  for (int64_t p = 0; p < mesh->n; ++p)
    for (int32_t j = 1; j <= m; ++j)
      for (int32_t i = 1; i <= m; ++i) {
        double r[3];
        fco_sphere_centre(mesh, p, i, j, r);
        double *q = &qn[p * meqn * FR + fco_fidx(m, i, j)];
        const double mr = q[1 * FR] * r[0] + q[2 * FR] * r[1] + q[3 * FR] * r[2];
        for (int k = 0; k < 3; ++k) q[(1 + k) * FR] -= mr * r[k];
      }
}
