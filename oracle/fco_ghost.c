/*
 * fco_ghost.c -- ghost-cell fill of the CPU oracle (test infrastructure
 * only).
 *
 * Sec. 3 of the paper: every patch is surrounded by two ghost layers; a
 * same-level neighbour copies its edge cells into them, finer neighbours
 * average their edge cells into them, and a coarser neighbour fills them by
 * interpolation that is conservative and limited.
 *
 * The oracle states this as one definition, applied cell by cell:
 *
 *   the ghost cell takes its value from the leaf L that contains its
 *   centre (carried through the tree connectivity when the centre lies in
 *   another tree):  level(L) = l      -> copy the coincident cell,
 *                   level(L) = l + 1  -> kappa-weighted mean of the 2x2
 *                                        L-cells inside the ghost cell,
 *                   level(L) = l - 1  -> Q_c + sx*dx + sy*dy from the L-cell
 *                                        c containing the centre, with
 *                                        minmod slopes of L's ghost-extended
 *                                        data and offsets dx, dy = +-1/4 of
 *                                        a coarse cell.
 *
 * Readings where the paper is silent: minmod as the limiter of the
 * interpolation; walls are handled first (xi-walls, then eta-walls):
 * a reflecting wall mirrors the frame with the normal momentum negated, an
 * extrapolation wall repeats the first interior cell; a corner region at
 * which no leaf exists (valence-3 vertex of the cubed sphere) takes the
 * mean of the two face ghosts obtained by mirroring one index.
 *
 * Values of L's ghost-extended array that the interpolation slopes need are
 * evaluated by the same definition, recursively.  With full (face and
 * corner) 2:1 balance and m >= 4 that recursion never interpolates twice;
 * the depth is returned so that tests can confirm it.
 */
#include "fco_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  const fco_mesh *mesh;
  const fco_params *par;
  const double *q;
  int32_t depth_max;
  int32_t error;
  /* sub-cycling (NULL qold: the state q alone): a leaf coarser than
   * fill_level contributes (1 - alpha[l]) qold + alpha[l] q, its state
   * interpolated linearly in time between the start and the end of its
   * current step */
  const double *qold;
  const double *alpha;
  int32_t fill_level;
} gctx;

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) <= fabs(b) ? a : b;
}

static double kappa_of(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j) {
  return mesh->sphere ? fco_sphere_kappa(mesh, p, i, j) : 1.0;
}

static void interior(const gctx *g, int64_t p, int32_t i, int32_t j,
                     double *out) {
  const int32_t m = g->mesh->m, meqn = g->par->meqn;
  const int64_t F = fco_frame(m);
  const int32_t lev = g->mesh->leaves[p].level;
  if (g->qold && lev < g->fill_level) {
    const double a = g->alpha[lev];
    for (int k = 0; k < meqn; ++k) {
      const int64_t o = (p * meqn + k) * F + fco_fidx(m, i, j);
      out[k] = (1.0 - a) * g->qold[o] + a * g->q[o];
    }
    return;
  }
  for (int k = 0; k < meqn; ++k)
    out[k] = g->q[(p * meqn + k) * F + fco_fidx(m, i, j)];
}

void fco_frame_value(gctx *g, int64_t p, int32_t i, int32_t j, double *out,
                     int32_t depth);

/* Value at a ghost-cell centre, located in leaf L (tree coords x, y). */
static void from_leaf(gctx *g, int64_t L, int32_t lev, int64_t x, int64_t y,
                      double *out, int32_t depth) {
  const fco_mesh *mesh = g->mesh;
  const int32_t m = mesh->m, meqn = g->par->meqn;
  const fco_leaf *a = &mesh->leaves[L];
  const int64_t size = FCO_SIDE >> a->level, cs = size / m;
  const int64_t u = x - (int64_t)a->ix * size, v = y - (int64_t)a->iy * size;
  if (a->level == lev) {
    interior(g, L, (int32_t)(u / cs) + 1, (int32_t)(v / cs) + 1, out);
  } else if (a->level == lev + 1) {
    /* the centre is the common corner of four L cells */
    int32_t i0 = (int32_t)(u / cs), j0 = (int32_t)(v / cs);
    double acc[FCO_MAXEQ] = {0}, w = 0.0, c[FCO_MAXEQ];
    for (int b = 0; b < 4; ++b) {
      int32_t ii = i0 + (b & 1), jj = j0 + (b >> 1);
      double kap = kappa_of(mesh, L, ii, jj);
      interior(g, L, ii, jj, c);
      for (int k = 0; k < meqn; ++k) acc[k] += kap * c[k];
      w += kap;
    }
    for (int k = 0; k < meqn; ++k) out[k] = acc[k] / w;
  } else if (a->level == lev - 1) {
    int32_t ic = (int32_t)(u / cs) + 1, jc = (int32_t)(v / cs) + 1;
    /* offset of the fine centre from the coarse centre, in coarse cells */
    double dx = (2 * u > (2 * ic - 1) * cs) ? 0.25 : -0.25;
    double dy = (2 * v > (2 * jc - 1) * cs) ? 0.25 : -0.25;
    double qc[FCO_MAXEQ], qe[FCO_MAXEQ], qw[FCO_MAXEQ], qn[FCO_MAXEQ],
        qs[FCO_MAXEQ];
    if (depth + 1 > g->depth_max) g->depth_max = depth + 1;
    interior(g, L, ic, jc, qc);
    fco_frame_value(g, L, ic + 1, jc, qe, depth + 1);
    fco_frame_value(g, L, ic - 1, jc, qw, depth + 1);
    fco_frame_value(g, L, ic, jc + 1, qn, depth + 1);
    fco_frame_value(g, L, ic, jc - 1, qs, depth + 1);
    for (int k = 0; k < meqn; ++k) {
      double sx = minmod(qe[k] - qc[k], qc[k] - qw[k]);
      double sy = minmod(qn[k] - qc[k], qc[k] - qs[k]);
      out[k] = qc[k] + dx * sx + dy * sy;
    }
  } else {
    g->error = 1;   /* not 2:1 balanced */
    for (int k = 0; k < meqn; ++k) out[k] = NAN;
  }
}

/* normal momentum component negated by a reflecting wall of axis `axis` */
static int normal_component(const fco_params *par, int axis) {
  if (par->physics == FCO_SHALLOW) return 1 + axis;
  return -1;
}

void fco_frame_value(gctx *g, int64_t p, int32_t i, int32_t j, double *out,
                     int32_t depth) {
  const fco_mesh *mesh = g->mesh;
  const int32_t m = mesh->m, meqn = g->par->meqn;
  if (i >= 1 && i <= m && j >= 1 && j <= m) {
    interior(g, p, i, j, out);
    return;
  }
  /* physical walls: xi first, then eta */
  for (int axis = 0; axis < 2; ++axis) {
    int32_t idx = axis == 0 ? i : j;
    int f = -1;
    if (idx < 1) f = 2 * axis;
    else if (idx > m) f = 2 * axis + 1;
    if (f < 0 || !fco_wall_face(mesh, p, f)) continue;
    int bc = mesh->trees[mesh->leaves[p].tree].bc[f];
    int32_t mir;
    if (bc == 1) mir = (f % 2 == 0) ? 1 - idx : 2 * m + 1 - idx;
    else mir = (f % 2 == 0) ? 1 : m;
    if (axis == 0) fco_frame_value(g, p, mir, j, out, depth);
    else fco_frame_value(g, p, i, mir, out, depth);
    int nc = normal_component(g->par, axis);
    if (bc == 1 && nc >= 0) out[nc] = -out[nc];
    return;
  }
  /* location rule */
  const fco_leaf *a = &mesh->leaves[p];
  const int64_t size = FCO_SIDE >> a->level, half = size / (2 * m);
  int64_t x = (int64_t)a->ix * size + (2 * i - 1) * half;
  int64_t y = (int64_t)a->iy * size + (2 * j - 1) * half;
  int32_t t2;
  int64_t x2, y2;
  int r = fco_locate(mesh->trees, a->tree, x, y, &t2, &x2, &y2);
  if (r == 2) {
    /* valence-3 corner: mean of the two mirrored face ghosts */
    int32_t mi = (i < 1) ? 1 - i : 2 * m + 1 - i;
    int32_t mj = (j < 1) ? 1 - j : 2 * m + 1 - j;
    double va[FCO_MAXEQ], vb[FCO_MAXEQ];
    fco_frame_value(g, p, i, mj, va, depth);
    fco_frame_value(g, p, mi, j, vb, depth);
    for (int k = 0; k < meqn; ++k) out[k] = 0.5 * (va[k] + vb[k]);
    return;
  }
  int64_t L = (r == 0) ? fco_leaf_at(mesh, t2, x2, y2) : -1;
  if (L < 0) {
    g->error = 2;
    for (int k = 0; k < meqn; ++k) out[k] = NAN;
    return;
  }
  from_leaf(g, L, a->level, x2, y2, out, depth);
}

int fco_ghost_fill(const fco_mesh *mesh, const fco_params *par, double *q,
                   int32_t *max_depth) {
  if (!mesh || !par || !q || par->meqn < 1 || par->meqn > FCO_MAXEQ ||
      par->m != mesh->m)
    return -1;
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t F = fco_frame(m);
  int32_t depth = 0, error = 0;
  /* every ghost value is evaluated from interior values only, so patches
   * can be filled in any order (fco_set_threads: whole patches per thread) */
#pragma omp parallel num_threads(fco_threads()) reduction(max : depth) reduction(| : error)
  {
    gctx g = {mesh, par, q, 0, 0, NULL, NULL, 0};
    double v[FCO_MAXEQ];
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < mesh->n; ++p)
      for (int32_t j = -1; j <= m + 2; ++j)
        for (int32_t i = -1; i <= m + 2; ++i) {
          int gi = (i < 1 || i > m), gj = (j < 1 || j > m);
          if (!gi && !gj) continue;
          /* the four outermost corner cells are never read by the step */
          if ((i == -1 || i == m + 2) && (j == -1 || j == m + 2)) continue;
          fco_frame_value(&g, p, i, j, v, 0);
          for (int k = 0; k < meqn; ++k)
            q[(p * meqn + k) * F + fco_fidx(m, i, j)] = v[k];
        }
    depth = g.depth_max > depth ? g.depth_max : depth;
    error |= g.error;
  }
  if (max_depth) *max_depth = depth;
  return error ? -2 : 0;
}

int fco_ghost_fill_level(const fco_mesh *mesh, const fco_params *par, double *q,
                         const double *qold, const double *alpha, int32_t level) {
  if (!mesh || !par || !q || !qold || !alpha || par->meqn < 1 ||
      par->meqn > FCO_MAXEQ || par->m != mesh->m)
    return -1;
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t F = fco_frame(m);
  int32_t error = 0;
#pragma omp parallel num_threads(fco_threads()) reduction(| : error)
  {
    gctx g = {mesh, par, q, 0, 0, qold, alpha, level};
    double v[FCO_MAXEQ];
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < mesh->n; ++p) {
      if (mesh->leaves[p].level != level) continue;
      for (int32_t j = -1; j <= m + 2; ++j)
        for (int32_t i = -1; i <= m + 2; ++i) {
          int gi = (i < 1 || i > m), gj = (j < 1 || j > m);
          if (!gi && !gj) continue;
          if ((i == -1 || i == m + 2) && (j == -1 || j == m + 2)) continue;
          fco_frame_value(&g, p, i, j, v, 0);
          for (int k = 0; k < meqn; ++k)
            q[(p * meqn + k) * F + fco_fidx(m, i, j)] = v[k];
        }
    }
    error |= g.error;
  }
  return error ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* Regrid transfer (Sec. 3: interpolate coarse data to newly created   */
/* fine patches, average fine data to a newly created coarse patch).   */
/* Every new cell is filled by the same three-way rule as a ghost cell, */
/* applied to the old mesh; the old data carry filled ghost frames.    */
int fco_transfer(const fco_mesh *old_mesh, const fco_mesh *new_mesh,
                 const fco_params *par, const double *q_old, double *q_new) {
  if (!old_mesh || !new_mesh || old_mesh->m != new_mesh->m) return -1;
  const int32_t m = new_mesh->m, meqn = par->meqn;
  const int64_t F = fco_frame(m);
  gctx g = {old_mesh, par, q_old, 0, 0, NULL, NULL, 0};
  double v[FCO_MAXEQ];
  for (int64_t p = 0; p < new_mesh->n; ++p) {
    const fco_leaf *a = &new_mesh->leaves[p];
    const int64_t size = FCO_SIDE >> a->level, half = size / (2 * m);
    /* old leaf covering this new leaf (or lying inside it) */
    int64_t o = fco_leaf_at(old_mesh, a->tree, (int64_t)a->ix * size + half,
                            (int64_t)a->iy * size + half);
    if (o < 0) return -2;
    const fco_leaf *b = &old_mesh->leaves[o];
    int coarser = b->level < a->level;
    double fix[FCO_MAXEQ] = {0};
    for (int32_t j = 1; j <= m; ++j)
      for (int32_t i = 1; i <= m; ++i) {
        int64_t x = (int64_t)a->ix * size + (2 * i - 1) * half;
        int64_t y = (int64_t)a->iy * size + (2 * j - 1) * half;
        int64_t L = fco_leaf_at(old_mesh, a->tree, x, y);
        if (L < 0) return -2;
        const fco_leaf *c = &old_mesh->leaves[L];
        if (c->level < a->level - 1) {
          /* two or more levels: general offsets from the coarse centre */
          const int64_t cs_old = (FCO_SIDE >> c->level) / m;
          const int64_t u = x - (int64_t)c->ix * (FCO_SIDE >> c->level);
          const int64_t w = y - (int64_t)c->iy * (FCO_SIDE >> c->level);
          int32_t ic = (int32_t)(u / cs_old) + 1, jc = (int32_t)(w / cs_old) + 1;
          double dx = ((double)u - (ic - 0.5) * (double)cs_old) / (double)cs_old;
          double dy = ((double)w - (jc - 0.5) * (double)cs_old) / (double)cs_old;
          double qc[FCO_MAXEQ], qe[FCO_MAXEQ], qw[FCO_MAXEQ], qn[FCO_MAXEQ],
              qs[FCO_MAXEQ];
          fco_frame_value(&g, L, ic, jc, qc, 0);
          fco_frame_value(&g, L, ic + 1, jc, qe, 0);
          fco_frame_value(&g, L, ic - 1, jc, qw, 0);
          fco_frame_value(&g, L, ic, jc + 1, qn, 0);
          fco_frame_value(&g, L, ic, jc - 1, qs, 0);
          for (int k = 0; k < meqn; ++k)
            v[k] = qc[k] + dx * minmod(qe[k] - qc[k], qc[k] - qw[k]) +
                   dy * minmod(qn[k] - qc[k], qc[k] - qs[k]);
        } else {
          from_leaf(&g, L, a->level, x, y, v, 0);
        }
        for (int k = 0; k < meqn; ++k)
          q_new[(p * meqn + k) * F + fco_fidx(m, i, j)] = v[k];
      }
    (void)fix;
    if (coarser && new_mesh->sphere) {
      /* mapped cells: shift the interpolated children of every old cell so
       * that their capacity-weighted sum equals the old cell's content */
      const int64_t size_o = FCO_SIDE >> b->level;
      for (int32_t j = 1; j <= m; ++j)
        for (int32_t i = 1; i <= m; ++i) {
          /* handle each old coarse cell once: at its lower-left child */
          if (((i - 1) & 1) || ((j - 1) & 1)) continue;
          int64_t x = (int64_t)a->ix * size + (2 * i - 1) * half;
          int64_t y = (int64_t)a->iy * size + (2 * j - 1) * half;
          int64_t L = fco_leaf_at(old_mesh, a->tree, x, y);
          const fco_leaf *c = &old_mesh->leaves[L];
          if (c->level != a->level - 1) continue;
          int64_t cs_o = size_o / m;
          int32_t ic = (int32_t)((x - (int64_t)c->ix * size_o) / cs_o) + 1;
          int32_t jc = (int32_t)((y - (int64_t)c->iy * size_o) / cs_o) + 1;
          double qc[FCO_MAXEQ];
          interior(&g, L, ic, jc, qc);
          double kc = fco_sphere_kappa(old_mesh, L, ic, jc);
          double ksum = 0.0, qsum[FCO_MAXEQ] = {0};
          for (int b2 = 0; b2 < 4; ++b2) {
            int32_t ii = i + (b2 & 1), jj = j + (b2 >> 1);
            double kf = fco_sphere_kappa(new_mesh, p, ii, jj);
            ksum += kf;
            for (int k = 0; k < meqn; ++k)
              qsum[k] += kf * q_new[(p * meqn + k) * F + fco_fidx(m, ii, jj)];
          }
          /* kappa is relative to the cell's own computational area; a
           * coarse cell has four times the computational area of a child */
          for (int k = 0; k < meqn; ++k) {
            double shift = (4.0 * kc * qc[k] - qsum[k]) / ksum;
            for (int b2 = 0; b2 < 4; ++b2) {
              int32_t ii = i + (b2 & 1), jj = j + (b2 >> 1);
              q_new[(p * meqn + k) * F + fco_fidx(m, ii, jj)] += shift;
            }
          }
        }
    }
  }
  return g.error ? -3 : 0;
}
