/* fco_internal.h -- private declarations of the CPU oracle (test
 * infrastructure only; see fco.h). */
#ifndef FCO_INTERNAL_H
#define FCO_INTERNAL_H

#include "fco.h"

struct fco_mesh {
  int32_t ntrees;
  fco_tree *trees;
  int64_t n;
  fco_leaf *leaves;
  int32_t m;
  int32_t sphere;     /* 1: trees are the six gnomonic cubed-sphere faces,
                         or the two hemispheres of the pillow sphere   */
  int32_t pillow;     /* sphere of two trees (fco_sphere.c)             */
  int32_t maxlevel;
  int64_t hcap;
  int64_t *hslot;     /* open-addressing table of leaf indices, -1 = free */
  double *geo;        /* sphere: per-patch cell and edge geometry (fco_sphere.c) */
};

/* frame index of cell (i, j), i, j in -1..m+2 */
static inline int64_t fco_fidx(int32_t m, int32_t i, int32_t j) {
  return (int64_t)(j + 1) * (m + 4) + (i + 1);
}
static inline int64_t fco_frame(int32_t m) { return (int64_t)(m + 4) * (m + 4); }

int64_t fco_find(const fco_mesh *mesh, int32_t tree, int32_t level,
                 int64_t ix, int64_t iy);
/* Map a point given in tree coordinates (units of 2^-FCO_S) into the tree
 * that contains it.  Returns 0 if found, 1 if it lies beyond a physical
 * boundary, 2 at a valence-3 corner (no tree contains it), 3 otherwise. */
int fco_locate(const fco_tree *trees, int32_t tree, int64_t x, int64_t y,
               int32_t *tout, int64_t *xout, int64_t *yout);
/* Carry a point beyond face f of tree t into the neighbour tree (in place);
 * -1 if the face is a physical boundary. */
int fco_cross_face(const fco_tree *trees, int32_t t, int32_t f, int64_t *x,
                   int64_t *y, int32_t *tout);
/* geometry tables of a sphere mesh (called by fco_mesh_new) */
int fco_sphere_build(fco_mesh *mesh);
/* 1 if the two trees are glued as the pillow sphere (fco_sphere.c) */
int fco_pillow_trees(int32_t ntrees, const fco_tree *trees);
/* leaf (index) containing an in-tree point, -1 if none */
int64_t fco_leaf_at(const fco_mesh *mesh, int32_t tree, int64_t x, int64_t y);
/* 1 if face f of leaf p lies on a physical boundary of its tree */
int fco_wall_face(const fco_mesh *mesh, int64_t p, int32_t f);

/* geometry of one edge: gamma = arc length / computational length, unit
 * normal n and unit tangent t (3D) */
typedef struct {
  double gamma;
  double n[3], t[3];
  double vel;          /* FCO_SWIRL: the edge's normal velocity */
} fco_edge_geom;

/* sphere solver pieces (fco_sphere.c) */
int fco_rp_sphere(const fco_params *par, const fco_edge_geom *e, const double *ql,
                  const double *qr, double *W, double *s, double *am,
                  double *ap, double *fl);
int fco_tsplit_sphere(const fco_params *par, const double *ql, const double *qr,
                      const fco_edge_geom *tedge, const double *psi, double *out,
                      int up);
void fco_sphere_project(const fco_mesh *mesh, const fco_params *par, double *qn);

/* Cell geometry of mapped (sphere) trees: capacity kappa of cell (i, j)
 * of patch p, computed from the mapping (fco_sphere.c). */
double fco_sphere_kappa(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j);
/* Edge data of the edge on the low side of cell (i, j) in direction dir
 * (0: xi-edge between (i-1, j) and (i, j); 1: eta-edge between (i, j-1)
 * and (i, j)): gamma = arc length / computational length, unit normal n
 * (pointing towards increasing index) and unit tangent t, both 3D. */
void fco_sphere_edge(const fco_mesh *mesh, int64_t p, int32_t dir,
                     int32_t i, int32_t j, double *gamma, double n[3],
                     double t[3]);
/* unit vector of the cell centre (i, j) of patch p */
void fco_sphere_centre(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j,
                       double r[3]);

#endif
