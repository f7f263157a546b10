/*
 * fco.h -- CPU FP64 oracle for leaf-patch AMR wave propagation.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is a plain, slow, independent
 * restatement of what one time step of the forest-of-quadtrees leaf-patch
 * method computes (ForestClaw, Burstedde, Calhoun, Mandli, Terrel, arXiv
 * 1308.1472).  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header, table or
 * constant with the HIP library it checks.
 *
 * Conventions (2D, quadtrees):
 *   - every tree is the unit square [0,1]^2 with a mapping of its own
 *     (Sec. 2);
 *   - a leaf at level l with integer coordinates (ix, iy) in [0, 2^l)^2
 *     covers [ix, ix+1] 2^-l x [iy, iy+1] 2^-l and houses one m x m patch
 *     (Sec. 2, the 1:1 leaf <-> patch correspondence);
 *   - patch cells (i, j), i, j = 1..m, and two ghost layers (Sec. 3) with
 *     i or j in {-1, 0, m+1, m+2};
 *   - face ids 0 = xi-low, 1 = xi-high, 2 = eta-low, 3 = eta-high;
 *   - per-patch state is stored "framed": q[p][k][(j+1)*(m+4) + (i+1)],
 *     i.e. a (m+4)^2 array per component with i fastest.
 */
#ifndef FCO_H
#define FCO_H

#include <stdint.h>

#define FCO_S 30                      /* tree side = 2^30 integer units  */
#define FCO_SIDE ((int64_t)1 << FCO_S)
#define FCO_MAXEQ 4

typedef struct { int32_t tree, level, ix, iy; } fco_leaf;

/* Per tree face: bc == 0 means connected to (nbr_tree, nbr_face) with
 * orient 0 (tangential coordinate runs the same way) or 1 (reversed);
 * bc == 1 reflecting wall; bc == 2 zero-order extrapolation. */
typedef struct {
  int32_t nbr_tree[4], nbr_face[4], orient[4], bc[4];
} fco_tree;

/* FCO_SWIRL: a scalar carried by a prescribed divergence-free flow (the
 * paper's Sec. 5 advection example, whose field the paper does not give;
 * the stand-in here is the classic swirl stream function
 *   psi(x, y, t) = sin^2(pi x) sin^2(pi y) cos(pi t / T) / pi
 * on each tree's unit square, period T = par->period).  The equation is
 * the colour equation q_t + u q_x + v q_y = 0 with (u, v) = (psi_y, -psi_x);
 * every cell edge carries the normal velocity of psi's difference between
 * the edge's two corners over its length (so the discrete field is exactly
 * divergence free), taken at the middle of the step (par->time + dt / 2). */
/* FCO_ROTATION: the colour equation on the cubed sphere carried by a rigid
 * rotation (the paper's Sec. 5 sphere example), velocity u = Omega w x r with
 * unit axis w = par->axis normalised and Omega = 2 pi / par->period.  u is
 * the surface curl of the stream function psi = Omega w.r, so the flux of u
 * through a great-circle edge from corner a to corner b is psi's difference
 * between them, Omega w.(b - a), up to the orientation of the edge: every
 * edge carries that flux over its computational length, signed towards
 * higher index (exactly divergence free).  The update is the capacity form
 * of the colour equation; no reflux (not a conservation law). */
enum { FCO_ADVECTION = 0, FCO_SHALLOW = 1, FCO_SPHERE = 2, FCO_SWIRL = 3,
       FCO_ROTATION = 4 };

typedef struct {
  int32_t m;           /* cells per patch side (even, >= 4)            */
  int32_t meqn;        /* 1 advection, 3 planar shallow water, 4 sphere */
  int32_t physics;     /* FCO_ADVECTION / FCO_SHALLOW / FCO_SPHERE      */
  int32_t limiter;     /* 0 none, 1 minmod, 2 superbee, 3 van Leer, 4 MC */
  int32_t transverse;  /* 0 none, 1 fluctuations, 2 fluctuations + corrections */
  int32_t pad;
  double g;            /* gravity (shallow water)                      */
  double ax, ay;       /* advection velocity (computational coords)    */
  double period;       /* FCO_SWIRL: period T of the flow              */
  double time;         /* FCO_SWIRL: time of the state a step starts from */
  double axis[3];      /* FCO_ROTATION: rotation axis (any length > 0)   */
} fco_params;

typedef struct fco_mesh fco_mesh;

#ifdef __cplusplus
extern "C" {
#endif

/* ---- forest ------------------------------------------------------- */
int  fco_sfc_sort(int64_t n, fco_leaf *leaves);
fco_mesh *fco_mesh_new(int32_t ntrees, const fco_tree *trees, int64_t n,
                       const fco_leaf *leaves, int32_t m, int32_t sphere);
void fco_mesh_free(fco_mesh *mesh);
int64_t fco_mesh_size(const fco_mesh *mesh);
int  fco_is_balanced(const fco_mesh *mesh);
int  fco_balance(int32_t ntrees, const fco_tree *trees, int64_t n,
                 const fco_leaf *in, int64_t cap, fco_leaf *out,
                 int64_t *nout);
int  fco_locate_leaf(const fco_mesh *mesh, int32_t tree, int64_t x,
                     int64_t y, int64_t *leaf);

/* ---- threads -------------------------------------------------------- */
/* Number of threads the ghost fill and the per-patch loop of the step
 * split whole patches over (default 1; only timing changes: each patch is
 * computed exactly as with one thread).  The reflux, sums and everything
 * else stay serial. */
void fco_set_threads(int32_t n);
int32_t fco_threads(void);

/* ---- ghost fill, step, sums ---------------------------------------- */
int  fco_ghost_fill(const fco_mesh *mesh, const fco_params *par, double *q,
                    int32_t *max_depth);
int  fco_step(const fco_mesh *mesh, const fco_params *par, const double *q,
              double *qn, double dt, int32_t reflux, double *numax);
/* Ghost fill of the level-`level` patches only, at a time inside the
 * current steps of the coarser levels: a coarser leaf's interior value is
 * (1 - alpha[l]) qold + alpha[l] q (alpha indexed by that leaf's level). */
int  fco_ghost_fill_level(const fco_mesh *mesh, const fco_params *par, double *q,
                          const double *qold, const double *alpha, int32_t level);
/* One sub-cycled step of the coarsest level present (planar forests):
 * level l steps with dt 2^-l (dt: the step of a level-0 patch), 2^(l - lmin)
 * times, coarse to fine with the finer levels' corrections carried back; q
 * framed in (ghosts ignored), qn framed out (interiors); *numax the largest
 * Courant number of all the steps. */
int  fco_step_subcycled(const fco_mesh *mesh, const fco_params *par, const double *q,
                        double *qn, double dt, double *numax);
int  fco_sums(const fco_mesh *mesh, const fco_params *par, const double *q,
              double *sums);

/* ---- regrid --------------------------------------------------------- */
int  fco_tags(const fco_mesh *mesh, const fco_params *par, const double *q,
              int32_t criterion, double threshold, int32_t lmin,
              int32_t lmax, int8_t *tags);
/* per patch: its criterion value (refine[p]) and, when p is the first
 * child of a complete family, the value of the averaged parent (parent[p],
 * NaN otherwise); a value passes when it exceeds thr (criterion 0) or thr^2
 * (criterion 1) */
int  fco_tag_values(const fco_mesh *mesh, const fco_params *par, const double *q,
                    int32_t criterion, double *refine, double *parent);
int  fco_regrid(const fco_mesh *mesh, const int8_t *tags, int32_t lmin,
                int32_t lmax, int64_t cap, fco_leaf *out, int64_t *nout);
int  fco_transfer(const fco_mesh *old_mesh, const fco_mesh *new_mesh,
                  const fco_params *par, const double *q_old, double *q_new);

/* ---- learned tagging (extension; see fco_mlp.c) ------------------- */
int  fco_features(const fco_mesh *mesh, const fco_params *par, const double *q,
                  double *feats);
double fco_bf16(double x);
double fco_mlp(const double *P, const double *norm, int64_t M, const double *x,
               const int32_t *y, const double *cw, double scale, int32_t round,
               double *logits, double *grad);
void fco_adam(int64_t n, double *P, const double *g, double *m1, double *m2,
              int32_t t, double lr, double beta1, double beta2, double eps);
void fco_learned_tags(int64_t M, const double *logits, const int8_t *plain,
                      double confidence, int8_t *tags);
int  fco_dilate_tags(const fco_mesh *mesh, const int8_t *in, int32_t lmax,
                     int8_t *out);

/* ---- pieces exposed for pinning ------------------------------------ */
double fco_phi(int32_t limiter, double theta);
int  fco_riemann(const fco_params *par, int32_t dir, const double *ql,
                 const double *qr, double *waves, double *speeds,
                 double *amdq, double *apdq);
/* FCO_SWIRL: the stream function, and the normal velocity of the
 * dir-edge at coordinate a (x for dir 0, y for dir 1) spanning [b0, b1] in
 * the other coordinate, at time t (tree coordinates) */
double fco_swirl_psi(const fco_params *par, double x, double y, double t);
double fco_swirl_edge(const fco_params *par, int32_t dir, double a, double b0,
                      double b1, double t);
/* FCO_ROTATION: the flux of the rigid rotation through the low-side
 * dir-edge of frame cell (i, j) of patch p over the computational cell
 * size, signed towards higher index (mesh built with sphere = 1) */
double fco_rotation_edge(const fco_mesh *mesh, const fco_params *par, int64_t p,
                         int32_t dir, int32_t i, int32_t j);
/* transverse split of a fluctuation psi from the dir-edge with states ql,
 * qr into the parts moving down (bm) and up (bp) the other direction
 * (planar physics) */
int  fco_tsplit(const fco_params *par, int32_t dir, const double *ql,
                const double *qr, const double *psi, double *bm, double *bp);

#ifdef __cplusplus
}
#endif
#endif
