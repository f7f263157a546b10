/*
 * fco_regrid.c -- refinement tags and mesh modification of the CPU oracle
 * (test infrastructure only).
 *
 * Sec. 2: the only information passed to the mesher is a set of per-patch
 * refine / coarsen flags computed from the numerical state; the mesher then
 * refines, coarsens and restores 2:1 balance.  Sec. 5: a patch is tagged for
 * refinement when its criterion exceeds a threshold, and a family of 2^d
 * patches is coarsened when the parent patch would not be tagged.
 *
 * Criteria:
 *   0: max - min of the first component over the patch interior (Sec. 5);
 *   1: max over interior cells of |grad h| by central differences over the
 *      ghost-extended data, in physical spacing.
 * The parent test uses the 2x2 (capacity-weighted) averages of the four
 * children, central differences inside and one-sided differences on the
 * outer ring (reading: no parent ghost cells are formed).
 * Comparisons are made on squared quantities with no fused operations so
 * that an independent implementation can reproduce every decision exactly.
 *
 * Tags: +1 refine (criterion true, level < lmax); -1 on all four members
 * of a family of leaf siblings above lmin none of which is tagged +1 and
 * whose parent fails the criterion; 0 otherwise.
 * Apply: refine +1 leaves, merge families tagged -1, then restore balance
 * by refinement only (a merge that would break balance is undone).
 */
#include "fco_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double qv(const double *q, int32_t m, int32_t meqn, int64_t p, int k,
                 int32_t i, int32_t j) {
  return q[(p * meqn + k) * fco_frame(m) + fco_fidx(m, i, j)];
}

/* physical spacing between the centres of cells a and b of patch p */
static double spacing(const fco_mesh *mesh, int64_t p, int32_t ia, int32_t ja,
                      int32_t ib, int32_t jb) {
  if (!mesh->sphere) {
    int32_t n = abs(ib - ia) + abs(jb - ja);
    return n * (ldexp(1.0, -mesh->leaves[p].level) / mesh->m);
  }
  double ra[3], rb[3];
  fco_sphere_centre(mesh, p, ia, ja, ra);
  fco_sphere_centre(mesh, p, ib, jb, rb);
  double cx = ra[1] * rb[2] - ra[2] * rb[1];
  double cy = ra[2] * rb[0] - ra[0] * rb[2];
  double cz = ra[0] * rb[1] - ra[1] * rb[0];
  double dot = ra[0] * rb[0] + ra[1] * rb[1] + ra[2] * rb[2];
  return atan2(sqrt(cx * cx + cy * cy + cz * cz), dot);
}

/* criterion value of patch p: max - min of h (criterion 0) or the largest
 * squared gradient of h (criterion 1); the patch passes when the value
 * exceeds thr (criterion 0) or thr^2 (criterion 1) */
static double refine_value(const fco_mesh *mesh, const fco_params *par,
                           const double *q, int64_t p, int criterion) {
  const int32_t m = mesh->m, meqn = par->meqn;
  if (criterion == 0) {
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t j = 1; j <= m; ++j)
      for (int32_t i = 1; i <= m; ++i) {
        double v = qv(q, m, meqn, p, 0, i, j);
        lo = fmin(lo, v);
        hi = fmax(hi, v);
      }
    return hi - lo;
  }
  double best = 0.0;
  for (int32_t j = 1; j <= m; ++j)
    for (int32_t i = 1; i <= m; ++i) {
      double gx = (qv(q, m, meqn, p, 0, i + 1, j) - qv(q, m, meqn, p, 0, i - 1, j)) /
                  spacing(mesh, p, i - 1, j, i + 1, j);
      double gy = (qv(q, m, meqn, p, 0, i, j + 1) - qv(q, m, meqn, p, 0, i, j - 1)) /
                  spacing(mesh, p, i, j - 1, i, j + 1);
      double s = gx * gx;
      s = s + gy * gy;
      best = fmax(best, s);
    }
  return best;
}

static int passes(int criterion, double value, double thr) {
  return criterion == 0 ? value > thr : value > thr * thr;
}

/* criterion value of the averaged parent of the family kids[0..3] */
static double parent_value(const fco_mesh *mesh, const fco_params *par,
                           const double *q, const int64_t kids[4], int criterion) {
  const int32_t m = mesh->m, meqn = par->meqn, h = m / 2;
  double *P = (double *)malloc(sizeof(double) * m * m);
  double *cx = (double *)malloc(sizeof(double) * m * m * 3);
  for (int32_t J = 1; J <= m; ++J)
    for (int32_t I = 1; I <= m; ++I) {
      int c = ((I - 1) >= h) + 2 * ((J - 1) >= h);
      int64_t kp = kids[c];
      int32_t ii = 2 * ((I - 1) % h) + 1, jj = 2 * ((J - 1) % h) + 1;
      double acc = 0.0, w = 0.0;
      double r[3] = {0, 0, 0};
      for (int b = 0; b < 4; ++b) {
        int32_t i2 = ii + (b & 1), j2 = jj + (b >> 1);
        double kap = mesh->sphere ? fco_sphere_kappa(mesh, kp, i2, j2) : 1.0;
        acc += kap * qv(q, m, meqn, kp, 0, i2, j2);
        w += kap;
        if (mesh->sphere) {
          double rc[3];
          fco_sphere_centre(mesh, kp, i2, j2, rc);
          for (int d = 0; d < 3; ++d) r[d] += rc[d];
        }
      }
      P[(J - 1) * m + (I - 1)] = acc / w;
      if (mesh->sphere) {
        double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int d = 0; d < 3; ++d) cx[((J - 1) * m + (I - 1)) * 3 + d] = r[d] / nr;
      }
    }
  double res = 0.0;
  if (criterion == 0) {
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t k = 0; k < m * m; ++k) {
      lo = fmin(lo, P[k]);
      hi = fmax(hi, P[k]);
    }
    res = hi - lo;
  } else {
    const double dxp = ldexp(1.0, -(mesh->leaves[kids[0]].level - 1)) / m;
    for (int32_t J = 1; J <= m; ++J)
      for (int32_t I = 1; I <= m; ++I) {
        int32_t ia = I > 1 ? I - 1 : I, ib = I < m ? I + 1 : I;
        int32_t ja = J > 1 ? J - 1 : J, jb = J < m ? J + 1 : J;
        double sx, sy;
        if (mesh->sphere) {
          const double *a = &cx[((J - 1) * m + (ia - 1)) * 3];
          const double *b = &cx[((J - 1) * m + (ib - 1)) * 3];
          double c0 = a[1] * b[2] - a[2] * b[1], c1 = a[2] * b[0] - a[0] * b[2],
                 c2 = a[0] * b[1] - a[1] * b[0];
          sx = atan2(sqrt(c0 * c0 + c1 * c1 + c2 * c2),
                     a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
          a = &cx[((ja - 1) * m + (I - 1)) * 3];
          b = &cx[((jb - 1) * m + (I - 1)) * 3];
          c0 = a[1] * b[2] - a[2] * b[1]; c1 = a[2] * b[0] - a[0] * b[2];
          c2 = a[0] * b[1] - a[1] * b[0];
          sy = atan2(sqrt(c0 * c0 + c1 * c1 + c2 * c2),
                     a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
        } else {
          sx = (ib - ia) * dxp;
          sy = (jb - ja) * dxp;
        }
        double gx = (P[(J - 1) * m + (ib - 1)] - P[(J - 1) * m + (ia - 1)]) / sx;
        double gy = (P[(jb - 1) * m + (I - 1)] - P[(ja - 1) * m + (I - 1)]) / sy;
        double s = gx * gx;
        s = s + gy * gy;
        res = fmax(res, s);
      }
  }
  free(P);
  free(cx);
  return res;
}

/* the four members of the complete family whose first child is p, or 0 */
static int family_of(const fco_mesh *mesh, int64_t p, int64_t kids[4]) {
  const fco_leaf *a = &mesh->leaves[p];
  if (a->level == 0 || (a->ix & 1) || (a->iy & 1)) return 0;
  for (int c = 0; c < 4; ++c) {
    kids[c] = fco_find(mesh, a->tree, a->level, a->ix + (c & 1), a->iy + (c >> 1));
    if (kids[c] < 0) return 0;
  }
  return 1;
}

int fco_tag_values(const fco_mesh *mesh, const fco_params *par, const double *q,
                   int32_t criterion, double *refine, double *parent) {
  if (!mesh || !par || !q || !refine || !parent || (criterion != 0 && criterion != 1))
    return -1;
  for (int64_t p = 0; p < mesh->n; ++p) {
    int64_t kids[4];
    refine[p] = refine_value(mesh, par, q, p, criterion);
    parent[p] = family_of(mesh, p, kids) ? parent_value(mesh, par, q, kids, criterion)
                                         : NAN;
  }
  return 0;
}

int fco_tags(const fco_mesh *mesh, const fco_params *par, const double *q,
             int32_t criterion, double threshold, int32_t lmin, int32_t lmax,
             int8_t *tags) {
  if (!mesh || !par || !q || !tags || (criterion != 0 && criterion != 1))
    return -1;
  const int64_t n = mesh->n;
  char *crit = (char *)malloc((size_t)n);
  for (int64_t p = 0; p < n; ++p) {
    crit[p] = (char)passes(criterion, refine_value(mesh, par, q, p, criterion), threshold);
    tags[p] = (crit[p] && mesh->leaves[p].level < lmax) ? 1 : 0;
  }
  for (int64_t p = 0; p < n; ++p) {
    const fco_leaf *a = &mesh->leaves[p];
    int64_t kids[4];
    if (a->level <= lmin || !family_of(mesh, p, kids)) continue;
    int ok = 1;
    for (int c = 0; c < 4; ++c)
      if (tags[kids[c]] == 1) ok = 0;
    if (!ok) continue;
    if (!passes(criterion, parent_value(mesh, par, q, kids, criterion), threshold))
      for (int c = 0; c < 4; ++c) tags[kids[c]] = -1;
  }
  free(crit);
  return 0;
}

int fco_regrid(const fco_mesh *mesh, const int8_t *tags, int32_t lmin,
               int32_t lmax, int64_t cap, fco_leaf *out, int64_t *nout) {
  const int64_t n = mesh->n;
  fco_leaf *tmp = (fco_leaf *)malloc(sizeof(fco_leaf) * (size_t)(4 * n));
  int64_t k = 0;
  for (int64_t p = 0; p < n; ++p) {
    const fco_leaf *a = &mesh->leaves[p];
    if (tags[p] > 0 && a->level < lmax) {
      for (int c = 0; c < 4; ++c) {
        fco_leaf ch = {a->tree, a->level + 1, 2 * a->ix + (c & 1),
                       2 * a->iy + (c >> 1)};
        tmp[k++] = ch;
      }
      continue;
    }
    if (tags[p] < 0 && a->level > lmin) {
      /* the family merges only when all four siblings are leaves tagged -1 */
      int all = 1;
      int32_t bx = a->ix & ~1, by = a->iy & ~1;
      for (int c = 0; c < 4 && all; ++c) {
        int64_t s = fco_find(mesh, a->tree, a->level, bx + (c & 1), by + (c >> 1));
        if (s < 0 || tags[s] >= 0) all = 0;
      }
      if (all) {
        if (a->ix == bx && a->iy == by) {
          fco_leaf par = {a->tree, a->level - 1, a->ix / 2, a->iy / 2};
          tmp[k++] = par;
        }
        continue;
      }
    }
    tmp[k++] = *a;
  }
  int rc = fco_balance(mesh->ntrees, mesh->trees, k, tmp, cap, out, nout);
  free(tmp);
  return rc;
}

/* Per-patch statistics for learned tagging (an extension; the paper tags by
 * a threshold on one criterion, Sec. 5).  For each of the first three
 * components (zero where meqn is smaller): min, max and plain mean over the
 * interior cells, and log(1 + the largest |grad q_k|) by the same central
 * differences as criterion 1 (needs filled ghosts); then the level; then
 * three zeros.  feats[p * 16 + f].  The logarithm keeps gradients near the
 * criterion threshold apart after standardisation and bfloat16 rounding:
 * across a forest the largest gradients span about four decades. */
int fco_features(const fco_mesh *mesh, const fco_params *par, const double *q,
                 double *feats) {
  const int32_t m = mesh->m, meqn = par->meqn;
  for (int64_t p = 0; p < mesh->n; ++p) {
    double *f = feats + p * 16;
    for (int f0 = 0; f0 < 16; ++f0) f[f0] = 0.0;
    for (int k = 0; k < 3 && k < meqn; ++k) {
      double lo = INFINITY, hi = -INFINITY, sum = 0.0, gmax = 0.0;
      for (int32_t j = 1; j <= m; ++j)
        for (int32_t i = 1; i <= m; ++i) {
          double v = qv(q, m, meqn, p, k, i, j);
          lo = fmin(lo, v);
          hi = fmax(hi, v);
          sum += v;
          double gx = (qv(q, m, meqn, p, k, i + 1, j) - qv(q, m, meqn, p, k, i - 1, j)) /
                      spacing(mesh, p, i - 1, j, i + 1, j);
          double gy = (qv(q, m, meqn, p, k, i, j + 1) - qv(q, m, meqn, p, k, i, j - 1)) /
                      spacing(mesh, p, i, j - 1, i, j + 1);
          gmax = fmax(gmax, sqrt(gx * gx + gy * gy));
        }
      f[4 * k + 0] = lo;
      f[4 * k + 1] = hi;
      f[4 * k + 2] = sum / ((double)m * m);
      f[4 * k + 3] = log1p(gmax);
    }
    f[12] = mesh->leaves[p].level;
  }
  return 0;
}

/* Refinement buffer for tags applied several steps after they are computed
 * (an extension, used with learned tagging): a leaf below lmax that touches
 * (over a face or a corner) a leaf tagged +1 is tagged +1 as well; other
 * tags are unchanged.  The touching leaves are found by locating the
 * centres of the first ghost ring of the patch at its own resolution. */
int fco_dilate_tags(const fco_mesh *mesh, const int8_t *in, int32_t lmax,
                    int8_t *out) {
  const int32_t m = mesh->m;
  for (int64_t p = 0; p < mesh->n; ++p) {
    const fco_leaf *a = &mesh->leaves[p];
    out[p] = in[p];
    if (in[p] == 1 || a->level >= lmax) continue;
    const int64_t side = (int64_t)1 << (FCO_S - a->level), half = side / (2 * m);
    for (int32_t j = 0; j <= m + 1 && out[p] != 1; ++j)
      for (int32_t i = 0; i <= m + 1; ++i) {
        if (i != 0 && i != m + 1 && j != 0 && j != m + 1) continue;
        const int64_t x = a->ix * side + (2 * i - 1) * half;
        const int64_t y = a->iy * side + (2 * j - 1) * half;
        int32_t t;
        int64_t xx, yy;
        if (fco_locate(mesh->trees, a->tree, x, y, &t, &xx, &yy) != 0) continue;
        const int64_t q = fco_leaf_at(mesh, t, xx, yy);
        if (q >= 0 && in[q] == 1) {
          out[p] = 1;
          break;
        }
      }
  }
  return 0;
}
