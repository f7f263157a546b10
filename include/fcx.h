/*
 * fcx.h -- C ABI of the MI355X leaf-patch AMR library (libfcx.so).
 *
 * One time step of the forest-of-quadtrees leaf-patch method of
 * Burstedde, Calhoun, Mandli and Terrel (ForestClaw, arXiv 1308.1472):
 * every leaf of a 2:1-balanced forest houses one m x m finite-volume patch
 * with two ghost layers (Sec. 2, Sec. 3); a step fills the ghost cells from
 * neighbouring patches (copy, average, limited interpolation; Sec. 3) and
 * advances every patch by the wave-propagation algorithm the paper adopts
 * from Clawpack (Sec. 3).
 *
 * Conventions
 *   - A tree is the reference square [0,1]^2 (Sec. 2).  A leaf
 *     (tree, level, ix, iy) covers [ix, ix+1] 2^-level x [iy, iy+1] 2^-level.
 *   - Patch ids are positions in the uploaded leaf array, which must be in
 *     space-filling-curve order: tree-major, then Morton order of the
 *     lower-left corner (x in the even bits).  fcx_sfc_sort produces it.
 *   - State "q" (device memory, owned by the caller) is compact:
 *     q[((p*meqn + k)*m + (j-1))*m + (i-1)] for patch p, component k,
 *     cell (i, j), i, j = 1..m.  Element type float (precision 32) or
 *     double (precision 64).
 *   - Ghost buffer "ghost" (device, caller-owned) holds the two-layer frame
 *     of every patch: ghost[(p*meqn + k)*G + g], G = 8m + 16, with g
 *     = (j+1)(m+4) + (i+1) for rows j = -1, 0; 2(m+4) + (j-m-1)(m+4) + (i+1)
 *     for rows j = m+1, m+2 (i = -1..m+2); 4(m+4) + 4(j-1) + s for rows
 *     j = 1..m with s = 0, 1, 2, 3 for i = -1, 0, m+1, m+2.  The four
 *     outermost corner cells are never read or written.
 *   - dt, nu_max and sums are device doubles.
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream).
 *     Every call that takes a stream only enqueues work on it.
 *
 * Errors: every entry point returns FCX_OK (0) or a negative code; none
 * throws or aborts.  fcx_last_error() returns a message for the calling
 * thread, owned by the library and valid until the next call.
 */
#ifndef FCX_H
#define FCX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCX_OK 0
#define FCX_EINVAL (-1)    /* bad argument, size or unsorted leaves        */
#define FCX_EBALANCE (-2)  /* forest not 2:1 balanced over faces, corners  */
#define FCX_ENOMEM (-3)    /* device or host allocation failed             */
#define FCX_EHIP (-4)      /* HIP runtime error (text in fcx_last_error)   */
#define FCX_ECFL (-5)      /* reported through fcx_next_dt's status word   */
#define FCX_ENEG (-6)      /* non-positive depth met by a Riemann solve    */
#define FCX_ESTATE (-7)    /* call out of order (e.g. no forest uploaded)  */

/* FCX_SWIRL: a scalar carried by a prescribed divergence-free flow, the
 * colour equation q_t + u q_x + v q_y = 0 with (u, v) = (psi_y, -psi_x) and
 * the stream function psi(x, y, t) = sin^2(pi x) sin^2(pi y) cos(pi t / T)
 * / pi on each tree's unit square (T = period): a stand-in for the
 * unpublished field of the paper's Sec. 5 advection example.  Each cell
 * edge carries the normal velocity of psi's difference between its two
 * corners over its length (the discrete field is exactly divergence free),
 * at the middle of the step: t is the context's simulated time
 * (fcx_sim_time) plus dt / 2.  The equation is not in conservation form,
 * so fcx_reflux leaves the state as it is.  Planar forests, global time
 * step only (fcx_advance_subcycled and batches refuse it). */
/* FCX_ROTATION (Sec. 5, the sphere example: a 0/1 colour field carried by
 * a rigid rotation of the sphere): the colour equation on the cubed sphere
 * (the six trees and geometry of FCX_SPHERE, see fcx_sphere_geometry) or on
 * the two-tree (pillow) sphere of the example, one tree per hemisphere:
 * tree t's faces 0 and 1 glued to the other tree's faces 0 and 1 with
 * orient 1, its face 2 to the other's face 3 and face 3 to face 2 with
 * orient 0 (fcx_create recognises either gluing), with
 * velocity u = Omega w x r, w = axis / |axis|, Omega = 2 pi / period.  u is
 * the surface curl of psi = Omega w.r, so the flux of u through a cell
 * edge is psi's difference between the edge's corners: each edge carries
 * it over the computational cell size, signed towards higher index,
 * formed as Omega (2 / dxi) sin(gamma dxi / 2) (w.t) from the edge's
 * arc-length factor gamma and tangent t (the chord between the corners
 * has length 2 sin(theta / 2) and the direction of t).  The update is the
 * capacity form of the colour equation (divided by kappa); no reflux (not
 * a conservation law).  Plain steps only: fcx_patch_step, fcx_ghost_fill,
 * fcx_next_dt, fcx_conservation_sums (capacity weighted), the regrid
 * calls and fcx_run with fused = 0; fused and sub-cycled steps, features
 * and batches return FCX_EINVAL. */
enum { FCX_ADVECTION = 0, FCX_SHALLOW = 1, FCX_SPHERE = 2, FCX_SWIRL = 3,
       FCX_ROTATION = 4 };

typedef struct fcx_ctx fcx_ctx;
typedef struct fcx_batch fcx_batch;

typedef struct {
  int32_t tree, level, ix, iy;
} fcx_leaf;

/* Tree connectivity (Sec. 2: blocks glued by a connectivity; Sec. 4:
 * neighbour access across blocks applies a coordinate transformation).
 * Face ids 0 = xi-low, 1 = xi-high, 2 = eta-low, 3 = eta-high.  bc[f] = 0:
 * face f is glued to face nbr_face[f] of tree nbr_tree[f]; orient[f] = 0
 * if the tangential coordinates run the same way, 1 if reversed.
 * bc[f] = 1: reflecting wall; bc[f] = 2: zero-order extrapolation. */
typedef struct {
  int32_t nbr_tree[4], nbr_face[4], orient[4], bc[4];
} fcx_tree;

typedef struct {
  int32_t m;           /* cells per patch side: 8, 16 or 32               */
  int32_t precision;   /* 32 or 64: element type of q and ghost           */
  int32_t physics;     /* FCX_ADVECTION (meqn 1), FCX_SHALLOW (meqn 3),
                          FCX_SPHERE (meqn 4: h and 3D momentum on the
                          cubed sphere; see fcx_sphere_geometry) or
                          FCX_SWIRL or FCX_ROTATION (meqn 1)              */
  int32_t limiter;     /* wave limiter: 0 none, 1 minmod, 2 superbee,
                          3 van Leer, 4 MC (LeVeque 2002, Sec. 6.12)      */
  int32_t transverse;  /* 0 none, 1 fluctuations, 2 fluctuations and
                          second-order corrections                         */
  int32_t tile;        /* cells per LDS tile side: 8 or 16 (0 = default) */
  int32_t threads;     /* threads per tile workgroup: T*T or 2*T*T
                          (0 = left to the library: 2*T*T for FP64
                          16 x 16 tiles and for FP32 16 x 16 tiles of a
                          forest with at most four tiles per compute
                          unit, else T*T); advection tiles ignore it:
                          one wavefront per tile, four per workgroup     */
  int32_t redo;        /* CFL rule (LeVeque 2002, Sec. 4.4; Clawpack's
                          time-step control): 1 = an attempt whose largest
                          Courant number exceeds cfl_max is rejected and
                          redone with the reduced dt, in fcx_advance,
                          fcx_run and batches; 0 = such a step is kept and
                          flagged (status bit 0)                           */
  double g;            /* gravity (shallow water)                         */
  double ax, ay;       /* advection velocity in reference coordinates     */
  double cfl_desired;  /* target Courant number for the next dt           */
  double cfl_max;      /* larger Courant numbers reject or flag the step  */
  double period;       /* FCX_SWIRL: period T of the flow (> 0);
                          FCX_ROTATION: time of one turn (> 0)            */
  double axis[3];      /* FCX_ROTATION: rotation axis (nonzero)           */
} fcx_config;

const char *fcx_last_error(void);
int32_t fcx_version(void);

/* ---- host-only forest utilities (integer work; no device needed) ---- */

/* Sort leaves in place into space-filling-curve order. */
int fcx_sfc_sort(int64_t n, fcx_leaf *leaves);

/* Coarsest forest that refines `in` (a tiling of every tree, any order)
 * and is 2:1 balanced across faces and corners, through the connectivity
 * (Sec. 2: the 2:1 balance condition).  Writes at most `cap` leaves in SFC
 * order to `out` and their number to *n_out (FCX_EINVAL if cap is short,
 * with *n_out set to the size needed). */
int fcx_balance(int32_t n_trees, const fcx_tree *trees, int64_t n,
                const fcx_leaf *in, int64_t cap, fcx_leaf *out,
                int64_t *n_out);

/* Regrid of a balanced forest from per-leaf tags (Sec. 2: per-patch flags
 * are the only mesher input): refine leaves tagged +1 (below lmax), merge
 * complete families of leaf siblings all tagged -1 (above lmin), then
 * restore 2:1 balance by refinement (a merge that would break it is
 * undone).  `leaves` must be SFC-sorted and balanced; writes the new forest
 * in SFC order (FCX_EINVAL with *n_out set if cap is short). */
int fcx_regrid_leaves(int32_t n_trees, const fcx_tree *trees, int64_t n,
                      const fcx_leaf *leaves, const int8_t *tags, int32_t lmin,
                      int32_t lmax, int64_t cap, fcx_leaf *out, int64_t *n_out);

/* ---- context -------------------------------------------------------- */

/* Creates a context for one forest on the current HIP device.  The
 * connectivity is copied. */
int fcx_create(const fcx_config *cfg, int32_t n_trees, const fcx_tree *trees,
               fcx_ctx **out);
int fcx_destroy(fcx_ctx *ctx);

/* Uploads a forest (Sec. 2: the leaf <-> patch correspondence).  Leaves
 * must be SFC-sorted and tile every tree; FCX_EBALANCE if not 2:1 balanced
 * (faces and corners), FCX_EINVAL otherwise.  Builds the neighbour records
 * (Sec. 2: constant-time neighbour lookup with relative orientation) and
 * copies them to the device.  Synchronous. */
int fcx_upload_forest(fcx_ctx *ctx, int64_t n, const fcx_leaf *leaves);

int64_t fcx_num_patches(const fcx_ctx *ctx);
int64_t fcx_state_elems(const fcx_ctx *ctx);   /* P * meqn * m * m        */
int64_t fcx_ghost_elems(const fcx_ctx *ctx);   /* P * meqn * (8m + 16)    */
int fcx_get_leaves(const fcx_ctx *ctx, int64_t cap, fcx_leaf *out);

/* Read-only host copy of the current forest's patch tables (Sec. 2: each
 * leaf's neighbours and their orientation), for tests and tools; waits for
 * the device.  recs: P records of 24 int32 (level, ix, iy, flags, 12
 * neighbour ids: faces 0-3 two slots each, then corners 0-3; 8 orientation
 * codes: faces, then corners); phislot: P face-term slots (-1: none);
 * family: P flags (1 at the first child of a complete family of leaf
 * siblings); counts: {slots, xi items, eta items}.  With items / aux (either
 * may be null), the coarse-fine items in reflux order, 8 int32 each (coarse
 * patch, face, two fine patches, their faces, their reversal flags), and
 * their companions, 6 int32 each (the other direction's items at the low and
 * high end, the coarse and the two fine face-term slots, the coarse level);
 * FCX_EINVAL if there are more than cap_items. */
int fcx_patch_table(fcx_ctx *ctx, int64_t cap_items, void *recs, int32_t *phislot,
                    int32_t *family, int32_t *counts, void *items, void *aux);

/* ---- the time step -------------------------------------------------- */

/* Ghost fill (Sec. 3): each ghost cell takes its value from the leaf that
 * contains its centre: copy from a same-level leaf, mean of the 2x2 cells of
 * a finer leaf, or limited (minmod) conservative linear interpolation from a
 * coarser leaf; reflecting / extrapolation walls; at a corner where no leaf
 * exists (three trees meeting) the mean of the two mirrored face ghosts.
 * Reads q, writes ghost. */
int fcx_ghost_fill(fcx_ctx *ctx, const void *q, void *ghost, void *stream);

/* Wave-propagation update of every patch (Sec. 3; LeVeque 1997): Riemann
 * problems at all edges, limited second-order corrections, transverse
 * propagation, for the given dt.  Reads q and ghost, writes q_new (must not
 * alias q).  Raises *nu_max (device double, atomically) to the largest
 * Courant number seen at interior edges; records the face terms used by
 * fcx_reflux in the context. */
int fcx_patch_step(fcx_ctx *ctx, const void *q, const void *ghost, void *q_new,
                   const double *dt, double *nu_max, void *stream);

/* Same result as fcx_ghost_fill followed by fcx_patch_step, in one launch:
 * ghost values are evaluated from q directly into LDS; no ghost buffer. */
int fcx_fused_step(fcx_ctx *ctx, const void *q, void *q_new, const double *dt,
                   double *nu_max, void *stream);

/* Coarse-fine correction with one global dt (Sec. 4: fine-level corrections
 * are carried back to the coarse level): each coarse cell at a
 * coarse-fine face gets the sum of the two fine face terms instead of its
 * own.  Needs the face terms of the preceding patch step on the same q. */
int fcx_reflux(fcx_ctx *ctx, const void *q, void *q_new, const double *dt,
               void *stream);

/* dt <- dt * cfl_desired / nu_max (unchanged if nu_max == 0); nu_max <- 0;
 * status (device int32): bit 0 set if nu_max > cfl_max (FCX_ECFL), bit 1 if
 * a non-positive depth was met since the last call (FCX_ENEG), bit 2 if a
 * ghost value needed nested interpolation, bit 3 if an attempt was rejected
 * and redone (redo on; then bit 0 is not set for it).  Bits are sticky
 * until the caller clears them.  This call never rejects: the caller
 * decides on a redo (fcx_advance and fcx_run apply the config's rule). */
int fcx_next_dt(fcx_ctx *ctx, double *nu_max, double *dt, int32_t *status,
                void *stream);

/* One whole step of the fused path in one call: fcx_fused_step (q ->
 * q_new), then fcx_reflux and fcx_next_dt in one launch (dt is updated for
 * the next step, nu_max cleared, status flags raised); same result as the
 * three calls.  With cfg.redo = 1 an attempt whose nu_max exceeds cfl_max is
 * rejected: q_new receives q unchanged, dt is reduced to
 * dt * cfl_desired / nu_max and status bit 3 is raised, so the next call
 * on (q_new -> q) redoes the step.  Planar forests only. */
int fcx_advance(fcx_ctx *ctx, const void *q, void *q_new, double *dt,
                double *nu_max, int32_t *status, void *stream);

/* Sub-cycled step (Sec. 4: per-level time steps, coarse to fine, with the
 * finer levels' correction factors carried back; Sec. 3: time-accurate
 * coarse data fill the ghost cells of finer patches).  Level l steps with
 * dt * 2^-l (*dt is the step of a level-0 patch, so all levels run at one
 * Courant number); one call is one step of the coarsest level present, in
 * which level l takes 2^(l - lmin) steps.  For each substep of a level: its
 * ghost cells at the substep's time (a coarser leaf's state interpolated
 * linearly in time within its own step), its step, and its fine-side face
 * terms w [dx_f (f(q_f) - f(q_c)) - phi_f], w = 1/2, accumulated at faces
 * with the next coarser level; after the two substeps of the next finer
 * level, this level's cells at those faces take -dt_l / dx^2 (sum of the
 * fine terms - phi_c) (Berger and Colella's flux correction).  Reads q
 * (never written), writes q_new; `work` (a state of the same size) and
 * `ghost` are scratch of the caller.  nu_max, dt and status as fcx_advance
 * (the CFL rule over all the substeps; with cfg.redo a rejected step leaves
 * q_new = q).  Planar forests; plain launches (no fused gather). */
int fcx_advance_subcycled(fcx_ctx *ctx, const void *q, void *q_new, void *work,
                          void *ghost, double *dt, double *nu_max, int32_t *status,
                          void *stream);

/* Counters of the steps taken on this context since fcx_create, read after
 * the device has finished: out[0] accepted steps, out[1] rejected attempts,
 * out[2] accepted cell updates (interior cells advanced). */
int fcx_step_stats(const fcx_ctx *ctx, int64_t *out);

/* Simulated time covered by the accepted steps of this context since
 * fcx_create (the sum of their dt; a sub-cycled step counts the step of its
 * coarsest level), read after the device has finished. */
int fcx_sim_time(const fcx_ctx *ctx, double *t);

/* A run of `steps` whole steps on two caller buffers of `cap` elements
 * each (enough for the finest forest the run can reach): step n = step0 +
 * k first regrids when regrid_every > 0, n > 0 and n % regrid_every == 0
 * (fcx_regrid with the given criterion, then fcx_regrid_transfer into the
 * other buffer, using `ghost` of ghost_cap elements), then advances into
 * the other buffer: mode (`fused`) 1: fcx_advance; 0: fcx_ghost_fill,
 * fcx_patch_step, fcx_reflux and fcx_next_dt; 2: fcx_advance_subcycled
 * (a step of the coarsest level; *dt is then a level-0 patch's step; the
 * work buffer is the library's).  The state starts in q0; *which
 * receives the buffer (0 or 1) holding the final state, *cell_updates the
 * number of interior cells advanced.  FCX_ENOMEM if a capacity is short
 * (the state is then where the last completed step left it).  On the
 * sphere only with fused = 0. */
int fcx_run(fcx_ctx *ctx, int32_t fused, void *q0, void *q1, int64_t cap,
            void *ghost, int64_t ghost_cap, int32_t steps, int32_t step0,
            int32_t regrid_every, int32_t criterion, double threshold,
            int32_t lmin, int32_t lmax, double *dt, double *nu_max,
            int32_t *status, int32_t *which, int64_t *cell_updates,
            void *stream);

/* sums[k] = sum over interior cells of q_k * cell area, in FP64, reduced in
 * a fixed order (deterministic). */
int fcx_conservation_sums(fcx_ctx *ctx, const void *q, double *sums,
                          void *stream);

/* fcx_conservation_sums for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and the same result bit for bit, but the per-patch
 * partial sums go to a fixed device array of the library (1048576 doubles,
 * 8 MiB, on every device the library runs on, held until the process ends)
 * instead of the context's buffer, and the call allocates nothing.
 * FCX_EINVAL if patches x components exceeds 1048576.  Every call on one
 * device shares that array: calls that overlap on one device (different
 * streams, or host threads) race; order them on one stream.  Nothing in the
 * array needs clearing between calls. */
int fcx_conservation_sums_noalloc(fcx_ctx *ctx, const void *q, double *sums,
                                  void *stream);

/* ---- regrid (Sec. 2: per-patch flags are the only mesher input) ----- */

/* tags (device int8, one per patch): +1 if the criterion exceeds the
 * threshold and level < lmax; -1 on the four members of a family of leaf
 * siblings above lmin, none tagged +1, whose averaged parent stays below
 * the threshold; 0 otherwise.  criterion 0: max - min of component 0 over
 * the interior (Sec. 5); 1: max |grad q_0| by central differences over the
 * ghost-extended data (needs a ghost fill of the same q).  On the sphere the
 * spacing is the great-circle distance of the cell centres and the parent
 * average is capacity weighted. */
int fcx_regrid_tags(fcx_ctx *ctx, const void *q, const void *ghost,
                    int32_t criterion, double threshold, int32_t lmin,
                    int32_t lmax, int8_t *tags, void *stream);

/* Applies host tags: refine +1, merge families tagged -1, restore balance by
 * refinement.  The context switches to the new forest; the old one is kept
 * for fcx_regrid_transfer.  *n_new receives the new patch count.
 * old_to_new (host, caller-allocated, one entry per old patch; NULL: not
 * wanted) maps each old patch, so that the caller can carry per-patch data
 * of its own (Sec. 2: the mesher sees only flags): >= 0 the patch is kept
 * with that new index; -2 - k it was refined, its four children are new
 * patches k .. k+3; -1 it was merged into a new parent. */
int fcx_regrid_apply(fcx_ctx *ctx, const int8_t *tags_host, int32_t lmin,
                     int32_t lmax, int64_t *n_new, int64_t *old_to_new);

/* fcx_ghost_fill of q into ghost, fcx_regrid_tags, the tags to the host
 * and fcx_regrid_apply (old_to_new as there), in one call (the calling thread polls until the
 * stream has reached the tags, so it spins for as long as the work queued
 * before them takes).  The new forest's tables are copied to the device in the order of
 * `stream`: later calls that use them go on the same stream or wait for it.
 * The ghost buffer then holds the fill that fcx_regrid_transfer needs;
 * *n_new receives the new patch count. */
int fcx_regrid(fcx_ctx *ctx, const void *q, void *ghost, int32_t criterion,
               double threshold, int32_t lmin, int32_t lmax, int64_t *n_new,
               int64_t *old_to_new, void *stream);

/* Data transfer after fcx_regrid_apply (Sec. 3: interpolate to new fine
 * patches, average to new coarse patches): kept patches copy, refined ones
 * interpolate with minmod slopes (the old ghost buffer must hold a fill of
 * q_old), merged ones take the mean of the 2x2 children cells.  On the
 * sphere the mean is capacity weighted and the four children of a refined
 * cell are shifted by one common amount so that their capacity-weighted sum
 * equals the coarse cell's content (conservative). */
int fcx_regrid_transfer(fcx_ctx *ctx, const void *q_old, const void *ghost_old,
                        void *q_new, void *stream);

/* ---- batches of independent forests ---------------------------------- */

/* A batch advances every leaf of n independent forests (each created and
 * uploaded as its own context; their m and physics may differ, their
 * precision must agree) in one fused ghost-gather + update launch per tile
 * class (8 x 8 tiles for m = 8, the tuned tile size otherwise): one
 * workgroup per tile, or persistent workgroups that take tiles through
 * per-XCD work counters.
 * The contexts must outlive the batch.  The state of all forests is one
 * caller-owned buffer: forest f starts at fcx_batch_state_offset(f) and uses
 * the compact layout of its own context.  dt, nu_max and status are device
 * arrays of n entries (per forest; status bits as fcx_next_dt's, raised by
 * the forest they concern); cfl_desired, cfl_max and redo are those of the
 * first forest (with redo on, a forest's rejected attempt leaves its state
 * unchanged in q_new and its next attempt uses the reduced dt). */
int fcx_batch_create(int32_t n, fcx_ctx *const *forests, fcx_batch **out);
int fcx_batch_destroy(fcx_batch *batch);
int64_t fcx_batch_state_elems(const fcx_batch *batch);
int64_t fcx_batch_state_offset(const fcx_batch *batch, int32_t f);
int64_t fcx_batch_num_patches(const fcx_batch *batch);

/* Tunables (chosen by the autotuner): tile of forests with m >= 16 (8 or
 * 16), threads per 8 x 8 tile (64 or 128) and per 16 x 16 tile (256 or 512;
 * advection tiles run one wavefront each whatever these say), launch form
 * (0: a workgroup per tile -- for advection, resident wavefronts that each
 * walk a run of the tiles with a simple halo, and a workgroup per four of
 * the others; 1: persistent workgroups).  Drops any captured graph. */
int fcx_batch_set_tuning(fcx_batch *batch, int32_t tile_big, int32_t threads8,
                         int32_t threads16, int32_t persistent);

/* One step of every forest: fused ghost gather + update (per forest: its own
 * dt), reflux, per-forest next dt as fcx_next_dt.  q_new must not alias q.
 * With launch form 0, an advection class whose tiles have both kinds of
 * halo runs its general-halo tiles on a stream of the batch's own, forked
 * from `stream` before the class and joined back into it before the reflux
 * (so the step stays ordered on `stream`, and a capture of `stream` takes
 * both branches); calls that overlap on one batch race. */
int fcx_batch_step(fcx_batch *batch, const void *q, void *q_new, double *dt,
                   double *nu_max, int32_t *status, void *stream);

/* Records `steps` batch steps, alternating q_a -> q_b -> q_a ..., into a HIP
 * graph (captured on a private stream; no memset nodes).  The pointers are
 * baked into the graph and must stay valid until the next capture or
 * fcx_batch_destroy.  After an odd number of steps the state is in q_b. */
int fcx_batch_capture(fcx_batch *batch, int32_t steps, void *q_a, void *q_b,
                      double *dt, double *nu_max, int32_t *status);
int fcx_batch_replay(fcx_batch *batch, void *stream);

/* The work split of the current tuning: items[c] tiles of class c (0:
 * advection 8 x 8, 1: shallow water 8 x 8, 2: advection with the tuned tile
 * of forests with m >= 16, 3: shallow water with it), of which simple[c]
 * have a halo of strip copies only (advection classes; 0 for the others).
 * items and simple are host arrays of 4 entries. */
int fcx_batch_class_items(const fcx_batch *batch, int32_t *items, int32_t *simple);

/* Per-forest counters since fcx_batch_create, read after the device has
 * finished: out[3 f + 0] accepted steps, out[3 f + 1] rejected attempts,
 * out[3 f + 2] accepted cell updates of forest f. */
int fcx_batch_step_stats(const fcx_batch *batch, int64_t *out);

/* sums[4 f + k]: FP64 conservation sums of forest f (k < meqn; others 0),
 * reduced in a fixed order. */
int fcx_batch_sums(fcx_batch *batch, const void *q, double *sums, void *stream);

/* ---- cubed sphere (Sec. 2: six mapped trees; Sec. 4: capacity and edge
 * metrics of mapped blocks) ---------------------------------------------
 *
 * With physics FCX_SPHERE the six trees are the faces of the cube, tree t
 * spanned by centre c_t and axes u_t, v_t (u x v = c):
 *   0: (+x, +y, +z)  1: (+y, -x, +z)  2: (-x, -y, +z)  3: (-y, +x, +z)
 *   4: (+z, +y, -x)  5: (-z, +y, +x)
 * glued edge to edge as the cube dictates (fcx_create checks it).  A point
 * (xi, eta) of tree t maps to c + T(xi) u + T(eta) v normalised to the unit
 * sphere, T(s) = tan((s - 1/2) pi/2) (gnomonic, equiangular).  The state is
 * (h, hu, hv, hw) with Cartesian momentum; each edge solves the Roe problem
 * in its (normal, tangent) frame with speeds scaled by the edge length; mass
 * is advanced in flux form; momentum is projected on the tangent plane
 * after the step.  fcx_patch_step, fcx_ghost_fill, fcx_reflux (which also
 * makes the mass face terms of same-level faces across cube edges agree:
 * call it after every step), fcx_next_dt, fcx_conservation_sums (capacity
 * weighted), the regrid calls (tags, apply, transfer, fcx_regrid), fcx_run
 * with plain steps and fcx_dilate_tags support the sphere; fused steps,
 * features and batches return FCX_EINVAL. */

/* Geometry table of every patch (device doubles, caller-owned, P * 18 *
 * (m+4)^2 values), per patch 18 frames of (m+4)^2 values indexed by frame
 * cell (i, j), i, j = -1 .. m+2, at (j+1)(m+4) + (i+1):
 *   frame 0: capacity kappa = cell area / dxi^2;
 *   frames 1-3 (interleaved, 3 per cell): unit vector of the cell centre;
 *   frames 4-10 (7 per cell): the cell's low-side xi-edge: gamma = arc
 *     length / dxi, unit normal (towards higher i), unit tangent;
 *   frames 11-17: the same for the low-side eta-edge.
 * Ghost cells carry the geometry of the cells they copy (points outside
 * the tree are mapped in the tree that holds them); at a cube vertex, where
 * no tree covers the corner region, that region uses the patch's own face
 * mapping extended.
 * Two-tree sphere (FCX_ROTATION only): with x = 2 xi - 1, y = 2 eta - 1 and
 * d = max(|x|, |y|), tree 0's point is (sin(th) x / rho, sin(th) y / rho,
 * cos(th)), th = d pi / 2, rho = |(x, y)|; tree 1 negates the second and
 * third components.  Beyond a square corner (where only the two trees'
 * corner cells meet) the ghost region is the own tree's corner mirrored
 * through that point. */
int fcx_sphere_geometry(fcx_ctx *ctx, double *geo, void *stream);   /* FCX_SPHERE, FCX_ROTATION */

/* ---- learned tagging (an extension of the Sec. 5 criterion tags) ------
 *
 * A small network predicts, per patch, the tag the criterion will give a
 * few steps later, so that regridding can run less often.  Inputs are 16
 * per-patch statistics (fcx_features); the network is 16 -> 64 -> 64 -> 3
 * with GELU (exact erf form) after both hidden layers; the 3 outputs are
 * logits of refine / keep / coarsen.  Parameters (caller-owned device FP32
 * array of FCX_MLP_PARAMS values, row = input unit, column = output unit):
 *   W1[16][64] b1[64] W2[64][64] b2[64] W3[64][3] b3[3]
 * norm (device FP32[32]): mu[16] then sigma[16]; inputs are used as
 * (x - mu) / sigma.  Products run on the matrix cores with bfloat16
 * operands (round to nearest even: normalised inputs, weights, hidden
 * activations, and in the backward pass the logit and pre-activation
 * gradients) and FP32 accumulation; the rest is FP32.  Row-major arrays:
 * x[rows][16], logits[rows][3]. */
#define FCX_MLP_INPUTS 16
#define FCX_MLP_HIDDEN 64
#define FCX_MLP_CLASSES 3
#define FCX_MLP_PARAMS 5443

/* feats[p * 16 + f] (device FP32): for each of the first three components
 * (zero where meqn is smaller) its min, max and mean over the interior and
 * log(1 + its largest |grad|) by central differences in reference
 * coordinates; then the patch level; then three zeros.  Needs a ghost fill
 * of q. */
int fcx_features(fcx_ctx *ctx, const void *q, const void *ghost, float *feats,
                 void *stream);

/* logits[rows][3] of the network on x[rows][16]. */
int fcx_mlp_forward(const float *params, const float *norm, int64_t rows,
                    const float *x, float *logits, void *stream);

/* Overwrites *loss with scale * sum_r class_weight[y_r] * (-log softmax_r[y_r])
 * and grad[FCX_MLP_PARAMS] with its gradient (labels: device int32, 0
 * refine, 1 keep, 2 coarsen; rows with other labels contribute nothing;
 * class_weight: device FP32[3]).  Accumulation order is not fixed (FP32
 * atomics), so results vary in the last bits between calls. */
int fcx_mlp_backward(const float *params, const float *norm, int64_t rows,
                     const float *x, const int32_t *labels,
                     const float *class_weight, float scale, float *grad,
                     float *loss, void *stream);

/* One Adam update at step t >= 1 (Kingma and Ba 2015, with bias
 * correction) of n parameters; m1 and m2 are the caller's moment arrays
 * (zero before step 1). */
int fcx_adam_step(int64_t n, float *params, const float *grad, float *m1,
                  float *m2, int32_t t, float lr, float beta1, float beta2,
                  float eps, void *stream);

/* tags[r] (device int8) from logits with the criterion as fallback: +1
 * where plain[r] is +1; plain[r] where the largest softmax probability is
 * below `confidence`; otherwise +1 / 0 / -1 for the most likely class
 * refine / keep / coarsen (lowest class on ties). */
int fcx_learned_tags(int64_t rows, const float *logits, const int8_t *plain,
                     float confidence, int8_t *tags, void *stream);

/* Refinement buffer for tags used several steps after they were computed:
 * out[p] = +1 if in[p] = +1, or if the level of p is below lmax and a patch
 * touching p over a face or a corner has in = +1; out[p] = in[p] otherwise.
 * in and out are device int8 arrays of one entry per patch; no aliasing. */
int fcx_dilate_tags(fcx_ctx *ctx, const int8_t *in, int32_t lmax, int8_t *out,
                    void *stream);

#ifdef __cplusplus
}
#endif
#endif
