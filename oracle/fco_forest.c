/*
 * fco_forest.c -- forest of quadtrees for the CPU oracle (test
 * infrastructure only).
 *
 * Leaves are kept in space-filling-curve order: tree-major, then Morton
 * order of the leaf's lower-left corner (Sec. 4: the leaf ordering follows
 * a space filling curve).  Neighbour relations are not tabulated: every
 * question "which leaf contains this point" is answered by walking the
 * tree connectivity (Sec. 2: blocks carry their own coordinates and are
 * glued by a connectivity; Sec. 4: neighbour access across blocks applies
 * a coordinate transformation) and probing a hash of the leaves.
 *
 * 2:1 balance (Sec. 2: neighbouring patches differ in size by at most a
 * factor of two) is taken over faces and corners.  fco_balance returns the
 * coarsest balanced forest that refines its input, found by the plain
 * fixed-point iteration "refine every leaf that touches a leaf more than one
 * level finer, until none is left".
 */
#include "fco_internal.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Morton key of a leaf: interleave x (even bits) and y (odd bits) of  */
/* the lower-left corner expressed at the finest resolution 2^-S.      */
static uint64_t morton(int64_t x, int64_t y) {
  uint64_t k = 0;
  for (int b = 0; b < FCO_S; ++b) {
    k |= (uint64_t)((x >> b) & 1) << (2 * b);
    k |= (uint64_t)((y >> b) & 1) << (2 * b + 1);
  }
  return k;
}

static uint64_t leaf_key(const fco_leaf *a) {
  int sh = FCO_S - a->level;
  return morton((int64_t)a->ix << sh, (int64_t)a->iy << sh);
}

static int cmp_leaf(const void *pa, const void *pb) {
  const fco_leaf *a = (const fco_leaf *)pa, *b = (const fco_leaf *)pb;
  if (a->tree != b->tree) return a->tree < b->tree ? -1 : 1;
  uint64_t ka = leaf_key(a), kb = leaf_key(b);
  if (ka != kb) return ka < kb ? -1 : 1;
  if (a->level != b->level) return a->level < b->level ? -1 : 1;
  return 0;
}

int fco_sfc_sort(int64_t n, fco_leaf *leaves) {
  if (n < 0 || (n > 0 && !leaves)) return -1;
  qsort(leaves, (size_t)n, sizeof(fco_leaf), cmp_leaf);
  return 0;
}

/* ------------------------------------------------------------------ */
static uint64_t hmix(int32_t tree, int32_t level, int64_t ix, int64_t iy) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
  uint64_t v[4] = {(uint64_t)tree, (uint64_t)level, (uint64_t)ix,
                   (uint64_t)iy};
  for (int k = 0; k < 4; ++k) {
    h ^= v[k] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
  }
  return h;
}

int64_t fco_find(const fco_mesh *mesh, int32_t tree, int32_t level,
                 int64_t ix, int64_t iy) {
  if (level < 0 || level > mesh->maxlevel) return -1;
  uint64_t mask = (uint64_t)mesh->hcap - 1;
  uint64_t h = hmix(tree, level, ix, iy) & mask;
  for (;;) {
    int64_t s = mesh->hslot[h];
    if (s < 0) return -1;
    const fco_leaf *a = &mesh->leaves[s];
    if (a->tree == tree && a->level == level && a->ix == ix && a->iy == iy)
      return s;
    h = (h + 1) & mask;
  }
}

int64_t fco_leaf_at(const fco_mesh *mesh, int32_t tree, int64_t x,
                    int64_t y) {
  if (x < 0 || y < 0 || x >= FCO_SIDE || y >= FCO_SIDE) return -1;
  for (int32_t l = 0; l <= mesh->maxlevel; ++l) {
    int64_t s = fco_find(mesh, tree, l, x >> (FCO_S - l), y >> (FCO_S - l));
    if (s >= 0) return s;
  }
  return -1;
}

/* ------------------------------------------------------------------ */
/* Carry a point that lies beyond face f of tree t into the neighbour  */
/* tree.  The distance d beyond the face becomes the distance inside   */
/* the neighbour's face; the tangential coordinate is kept or mirrored */
/* according to the orientation.                                       */
int fco_cross_face(const fco_tree *trees, int32_t t, int32_t f, int64_t *x,
                   int64_t *y, int32_t *tout) {
  const fco_tree *T = &trees[t];
  if (T->bc[f] != 0) return -1;
  int32_t t2 = T->nbr_tree[f], f2 = T->nbr_face[f], o = T->orient[f];
  int32_t a = f / 2, s = f % 2, a2 = f2 / 2, s2 = f2 % 2;
  int64_t nrm = (a == 0) ? *x : *y;
  int64_t tan = (a == 0) ? *y : *x;
  int64_t d = (s == 0) ? -nrm : nrm - FCO_SIDE;
  int64_t n2 = (s2 == 0) ? d : FCO_SIDE - d;
  int64_t t2c = o ? FCO_SIDE - tan : tan;
  if (a2 == 0) { *x = n2; *y = t2c; } else { *x = t2c; *y = n2; }
  *tout = t2;
  return 0;
}

static int outside_face(int64_t v, int axis) {
  if (v < 0) return 2 * axis;
  if (v >= FCO_SIDE) return 2 * axis + 1;
  return -1;
}

/* Follow faces until the point is inside a tree; at most two crossings. */
static int walk(const fco_tree *trees, int32_t t, int64_t x, int64_t y,
                int first_axis, int32_t *to, int64_t *xo, int64_t *yo) {
  int axis = first_axis;
  for (int hop = 0; hop < 3; ++hop) {
    int fx = outside_face(x, 0), fy = outside_face(y, 1);
    if (fx < 0 && fy < 0) { *to = t; *xo = x; *yo = y; return 0; }
    int f;
    if (fx >= 0 && fy >= 0) f = (axis == 0) ? fx : fy;
    else f = (fx >= 0) ? fx : fy;
    if (fco_cross_face(trees, t, f, &x, &y, &t) != 0) return 1;
    axis = 1 - axis;
  }
  return 3;
}

int fco_locate(const fco_tree *trees, int32_t tree, int64_t x, int64_t y,
               int32_t *tout, int64_t *xout, int64_t *yout) {
  int fx = outside_face(x, 0), fy = outside_face(y, 1);
  if (fx < 0 || fy < 0) {
    int r = walk(trees, tree, x, y, 0, tout, xout, yout);
    return r == 0 ? 0 : (r == 1 ? 1 : 3);
  }
  /* corner region: both crossing orders must agree on a tree */
  int32_t ta, tb;
  int64_t xa, ya, xb, yb;
  int ra = walk(trees, tree, x, y, 0, &ta, &xa, &ya);
  int rb = walk(trees, tree, x, y, 1, &tb, &xb, &yb);
  if (ra == 0 && rb == 0) {
    if (ta == tb && xa == xb && ya == yb) {
      *tout = ta; *xout = xa; *yout = ya;
      return 0;
    }
    return 2;
  }
  if (ra == 1 && rb == 1) return 1;
  return 3;
}

int fco_wall_face(const fco_mesh *mesh, int64_t p, int32_t f) {
  const fco_leaf *a = &mesh->leaves[p];
  int64_t last = ((int64_t)1 << a->level) - 1;
  int on = 0;
  switch (f) {
    case 0: on = (a->ix == 0); break;
    case 1: on = (a->ix == last); break;
    case 2: on = (a->iy == 0); break;
    default: on = (a->iy == last); break;
  }
  return on && mesh->trees[a->tree].bc[f] != 0;
}

/* ------------------------------------------------------------------ */
static int check_trees(int32_t ntrees, const fco_tree *trees) {
  for (int32_t t = 0; t < ntrees; ++t)
    for (int f = 0; f < 4; ++f) {
      const fco_tree *T = &trees[t];
      if (T->bc[f] < 0 || T->bc[f] > 2) return -1;
      if (T->bc[f] != 0) continue;
      int32_t t2 = T->nbr_tree[f], f2 = T->nbr_face[f];
      if (t2 < 0 || t2 >= ntrees || f2 < 0 || f2 > 3) return -1;
      if (T->orient[f] < 0 || T->orient[f] > 1) return -1;
      const fco_tree *U = &trees[t2];
      if (U->bc[f2] != 0 || U->nbr_tree[f2] != t || U->nbr_face[f2] != f ||
          U->orient[f2] != T->orient[f])
        return -1;
    }
  return 0;
}

fco_mesh *fco_mesh_new(int32_t ntrees, const fco_tree *trees, int64_t n,
                       const fco_leaf *leaves, int32_t m, int32_t sphere) {
  if (ntrees <= 0 || n <= 0 || !trees || !leaves) return NULL;
  if (m < 4 || (m & (m - 1))) return NULL;   /* power of two, >= 4 */
  if (check_trees(ntrees, trees) != 0) return NULL;
  /* leaves must be SFC-sorted and tile every tree exactly */
  int32_t maxlevel = 0;
  int64_t k = 0;
  for (int32_t t = 0; t < ntrees; ++t) {
    uint64_t next = 0;
    const uint64_t end = (uint64_t)1 << (2 * FCO_S);
    while (k < n && leaves[k].tree == t) {
      const fco_leaf *a = &leaves[k];
      if (a->level < 0 || a->level > 20) return NULL;
      int64_t side = (int64_t)1 << a->level;
      if (a->ix < 0 || a->iy < 0 || a->ix >= side || a->iy >= side)
        return NULL;
      if (leaf_key(a) != next) return NULL;
      next += (uint64_t)1 << (2 * (FCO_S - a->level));
      if (a->level > maxlevel) maxlevel = a->level;
      ++k;
    }
    if (next != end) return NULL;
  }
  if (k != n) return NULL;

  fco_mesh *mesh = (fco_mesh *)calloc(1, sizeof(fco_mesh));
  mesh->ntrees = ntrees;
  mesh->trees = (fco_tree *)malloc(sizeof(fco_tree) * ntrees);
  memcpy(mesh->trees, trees, sizeof(fco_tree) * ntrees);
  mesh->n = n;
  mesh->leaves = (fco_leaf *)malloc(sizeof(fco_leaf) * n);
  memcpy(mesh->leaves, leaves, sizeof(fco_leaf) * n);
  mesh->m = m;
  mesh->sphere = sphere;
  mesh->maxlevel = maxlevel;
  int64_t cap = 16;
  while (cap < 2 * n) cap <<= 1;
  mesh->hcap = cap;
  mesh->hslot = (int64_t *)malloc(sizeof(int64_t) * cap);
  for (int64_t s = 0; s < cap; ++s) mesh->hslot[s] = -1;
  for (int64_t s = 0; s < n; ++s) {
    const fco_leaf *a = &leaves[s];
    uint64_t h = hmix(a->tree, a->level, a->ix, a->iy) & (uint64_t)(cap - 1);
    while (mesh->hslot[h] >= 0) h = (h + 1) & (uint64_t)(cap - 1);
    mesh->hslot[h] = s;
  }
  mesh->pillow = sphere && ntrees == 2;
  if (sphere && ((ntrees != 6 && !fco_pillow_trees(ntrees, trees)) ||
                 fco_sphere_build(mesh) != 0)) {
    fco_mesh_free(mesh);
    return NULL;
  }
  return mesh;
}

void fco_mesh_free(fco_mesh *mesh) {
  if (!mesh) return;
  free(mesh->trees);
  free(mesh->leaves);
  free(mesh->hslot);
  free(mesh->geo);
  free(mesh);
}

int64_t fco_mesh_size(const fco_mesh *mesh) { return mesh ? mesh->n : -1; }

int fco_locate_leaf(const fco_mesh *mesh, int32_t tree, int64_t x, int64_t y,
                    int64_t *leaf) {
  int32_t t2;
  int64_t x2, y2;
  int r = fco_locate(mesh->trees, tree, x, y, &t2, &x2, &y2);
  *leaf = -1;
  if (r != 0) return r;
  *leaf = fco_leaf_at(mesh, t2, x2, y2);
  return *leaf >= 0 ? 0 : 3;
}

/* ------------------------------------------------------------------ */
/* Balance.  A leaf A at level l must be refined when any leaf touching */
/* it (across a face or a corner, through the connectivity) has a      */
/* level above l + 1.  Touching leaves are found with probe points just */
/* outside A, spaced by the finest leaf size present, so that every    */
/* leaf touching A contains at least one probe.                        */
static int needs_refine(const fco_mesh *mesh, int64_t p) {
  const fco_leaf *a = &mesh->leaves[p];
  int32_t lf = mesh->maxlevel;
  if (a->level >= lf - 1) return 0;
  int64_t size = FCO_SIDE >> a->level;
  int64_t step = FCO_SIDE >> lf, half = step / 2;
  int64_t x0 = (int64_t)a->ix * size, y0 = (int64_t)a->iy * size;
  int64_t nprobe = size / step;
  for (int f = 0; f < 4; ++f) {
    for (int64_t k = 0; k < nprobe; ++k) {
      int64_t t = k * step + half, x, y;
      switch (f) {
        case 0: x = x0 - half; y = y0 + t; break;
        case 1: x = x0 + size + half; y = y0 + t; break;
        case 2: x = x0 + t; y = y0 - half; break;
        default: x = x0 + t; y = y0 + size + half; break;
      }
      int64_t b;
      if (fco_locate_leaf(mesh, a->tree, x, y, &b) == 0 &&
          mesh->leaves[b].level > a->level + 1)
        return 1;
    }
  }
  for (int c = 0; c < 4; ++c) {
    int64_t x = (c & 1) ? x0 + size + half : x0 - half;
    int64_t y = (c & 2) ? y0 + size + half : y0 - half;
    int64_t b;
    if (fco_locate_leaf(mesh, a->tree, x, y, &b) == 0 &&
        mesh->leaves[b].level > a->level + 1)
      return 1;
  }
  return 0;
}

int fco_is_balanced(const fco_mesh *mesh) {
  for (int64_t p = 0; p < mesh->n; ++p)
    if (needs_refine(mesh, p)) return 0;
  return 1;
}

int fco_balance(int32_t ntrees, const fco_tree *trees, int64_t n,
                const fco_leaf *in, int64_t cap, fco_leaf *out,
                int64_t *nout) {
  fco_leaf *cur = (fco_leaf *)malloc(sizeof(fco_leaf) * (size_t)n);
  memcpy(cur, in, sizeof(fco_leaf) * (size_t)n);
  int64_t ncur = n;
  fco_sfc_sort(ncur, cur);
  for (;;) {
    fco_mesh *mesh = fco_mesh_new(ntrees, trees, ncur, cur, 4, 0);
    if (!mesh) { free(cur); return -1; }
    char *mark = (char *)calloc((size_t)ncur, 1);
    int64_t nmark = 0;
    for (int64_t p = 0; p < ncur; ++p)
      if (needs_refine(mesh, p)) { mark[p] = 1; ++nmark; }
    fco_mesh_free(mesh);
    if (nmark == 0) { free(mark); break; }
    fco_leaf *nxt = (fco_leaf *)malloc(sizeof(fco_leaf) * (size_t)(ncur + 3 * nmark));
    int64_t k = 0;
    for (int64_t p = 0; p < ncur; ++p) {
      if (!mark[p]) { nxt[k++] = cur[p]; continue; }
      for (int c = 0; c < 4; ++c) {
        fco_leaf ch = {cur[p].tree, cur[p].level + 1, 2 * cur[p].ix + (c & 1),
                       2 * cur[p].iy + (c >> 1)};
        nxt[k++] = ch;
      }
    }
    free(mark);
    free(cur);
    cur = nxt;
    ncur = k;
    fco_sfc_sort(ncur, cur);
  }
  *nout = ncur;
  if (ncur > cap) { free(cur); return -2; }
  memcpy(out, cur, sizeof(fco_leaf) * (size_t)ncur);
  free(cur);
  return 0;
}

/* ---- threads of the per-patch loops ---------------------------------- */
static int32_t g_threads = 1;

void fco_set_threads(int32_t n) { g_threads = n < 1 ? 1 : n; }

int32_t fco_threads(void) { return g_threads; }
