/*
 * fco_step.c -- one wave-propagation time step on every leaf patch, for the
 * CPU oracle (test infrastructure only).
 *
 * Sec. 3 of the paper: each patch is advanced by the wave-propagation
 * algorithm of LeVeque (JCP 1997; "Finite Volume Methods for Hyperbolic
 * Problems", 2002) -- piecewise-constant states, a Riemann problem at every
 * cell edge giving waves and speeds, wave limiters for the second-order
 * corrections, and (from the cited unsplit method) transverse propagation.
 * For systems a Roe solver is used (Roe 1981, cited in Sec. 3).
 *
 * Per patch, on the ghost-extended array Q (time level n) and a given dt:
 *   xi-sweep over rows j = 0..m+1, edges i-1/2 for i = 0..m+2:
 *     Riemann(Q[i-1], Q[i]) -> waves W^p, speeds s^p,
 *     A-dq = sum min(s,0) W,  A+dq = sum max(s,0) W;
 *   at edges i = 1..m+1: theta^p = W^p_upwind . W^p / W^p . W^p (upwind
 *     edge i-3/2 if s > 0, else i+1/2), limited wave phi(theta) W,
 *     correction flux Ft = 1/2 sum |s| (1 - nu |s|) Wlim with
 *     nu = 1/2 (dt/(kappa_l dx) + dt/(kappa_r dx));
 *   transverse (mode 2): A-dq + C and A+dq - C, C = sum |s|(1-nu|s|) Wlim,
 *     split by the eta-eigenstructure into down/up parts that are
 *     subtracted, times dt/(2 kappa dx) of the receiving cell, from the
 *     eta-correction flux of the cell's lower/upper edge;
 *   eta-sweep symmetric (both sweeps read Q^n: the scheme is unsplit);
 *   update of interior cells with the unmodified fluctuations:
 *     Q' = Q - dt/(kappa dx) [A+dq(i-1/2) + A-dq(i+1/2) + Ft(i+1/2) - Ft(i-1/2)]
 *            - dt/(kappa dy) [B+dq(j-1/2) + B-dq(j+1/2) + Gt(j+1/2) - Gt(j-1/2)].
 * Accumulation order is fixed: xi-rows ascending, then eta-columns
 * ascending, edges ascending inside each.
 *
 * Reflux (reading of Sec. 4, where fine-level corrections are carried back to
 * the coarse level after each step; here with one global dt): at every coarse-fine face
 * the coarse cell's face term is replaced by the sum of the fine face
 * terms.  The Roe property turns the missing f(Q_fine) - f(Q_coarse) into
 * the fluctuation sum of one extra Riemann problem per fine cell.
 *
 * Cubed sphere (reading): the mass component is in flux form, so its fine
 * face terms replace the coarse one as they are; and at same-level faces
 * across cube edges the mass face term of the higher-numbered patch is set
 * to minus its neighbour's, which keeps mass exact also next to the cube
 * vertices, where the two sides' transverse terms read different corner
 * ghost values.
 */
#include "fco_internal.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MW 3   /* at most three waves */

double fco_phi(int32_t limiter, double th) {
  switch (limiter) {
    case 0: return 1.0;                                   /* Lax-Wendroff */
    case 1: return fmax(0.0, fmin(1.0, th));              /* minmod */
    case 2: return fmax(0.0, fmax(fmin(1.0, 2.0 * th), fmin(2.0, th)));
    case 3: return (th + fabs(th)) / (1.0 + fabs(th));    /* van Leer */
    case 4: return fmax(0.0, fmin(fmin(0.5 * (1.0 + th), 2.0), 2.0 * th));
    default: return NAN;
  }
}

/* ---------------- edge geometry (Cartesian or mapped) ---------------- */
typedef fco_edge_geom edge_geom;   /* gamma = 1 on Cartesian grids */

/* ---------------- Riemann solvers ------------------------------------ */
/* Normal solvers fill waves[w*meqn+k], speeds[w], amdq, apdq; return the
 * number of waves, or -1 if a depth is not positive. */
static int rp_advection(const fco_params *par, int dir, const double *ql,
                        const double *qr, double *W, double *s, double *am,
                        double *ap) {
  double a = dir == 0 ? par->ax : par->ay;
  W[0] = qr[0] - ql[0];
  s[0] = a;
  am[0] = fmin(a, 0.0) * W[0];
  ap[0] = fmax(a, 0.0) * W[0];
  return 1;
}

/* colour equation with the edge's own normal velocity (FCO_SWIRL,
 * FCO_ROTATION) */
static int rp_swirl(const edge_geom *e, const double *ql, const double *qr,
                    double *W, double *s, double *am, double *ap) {
  W[0] = qr[0] - ql[0];
  s[0] = e->vel;
  am[0] = fmin(e->vel, 0.0) * W[0];
  ap[0] = fmax(e->vel, 0.0) * W[0];
  return 1;
}

static const double kPi = 3.14159265358979323846;

double fco_swirl_psi(const fco_params *par, double x, double y, double t) {
  const double sx = sin(kPi * x), sy = sin(kPi * y);
  return sx * sx * sy * sy * cos(kPi * t / par->period) / kPi;
}

double fco_swirl_edge(const fco_params *par, int32_t dir, double a, double b0,
                      double b1, double t) {
  if (dir == 0)   /* u = psi_y across an x = a edge */
    return (fco_swirl_psi(par, a, b1, t) - fco_swirl_psi(par, a, b0, t)) / (b1 - b0);
  /* v = -psi_x across a y = a edge */
  return -(fco_swirl_psi(par, b1, a, t) - fco_swirl_psi(par, b0, a, t)) / (b1 - b0);
}

typedef struct { double u, v, c; } roe_avg;

/* Roe averages of the edge pair, velocities in the (normal, tangential)
 * frame given by the momentum indices mu, mv */
static int roe_average(const fco_params *par, const double *ql,
                       const double *qr, int mu, int mv, roe_avg *r) {
  double hl = ql[0], hr = qr[0];
  if (!(hl > 0.0) || !(hr > 0.0)) return -1;
  double sl = sqrt(hl), sr = sqrt(hr);
  r->u = (ql[mu] / sl + qr[mu] / sr) / (sl + sr);
  r->v = (ql[mv] / sl + qr[mv] / sr) / (sl + sr);
  r->c = sqrt(par->g * 0.5 * (hl + hr));
  return 0;
}

static int rp_shallow(const fco_params *par, int dir, const double *ql,
                      const double *qr, double *W, double *s, double *am,
                      double *ap) {
  const int mu = 1 + dir, mv = 2 - dir;
  roe_avg r;
  if (roe_average(par, ql, qr, mu, mv, &r) != 0) return -1;
  double d0 = qr[0] - ql[0], d1 = qr[mu] - ql[mu], d2 = qr[mv] - ql[mv];
  double a1 = ((r.u + r.c) * d0 - d1) / (2.0 * r.c);
  double a2 = d2 - r.v * d0;
  double a3 = (d1 - (r.u - r.c) * d0) / (2.0 * r.c);
  memset(W, 0, sizeof(double) * 3 * 3);
  W[0 * 3 + 0] = a1; W[0 * 3 + mu] = a1 * (r.u - r.c); W[0 * 3 + mv] = a1 * r.v;
  W[1 * 3 + mv] = a2;
  W[2 * 3 + 0] = a3; W[2 * 3 + mu] = a3 * (r.u + r.c); W[2 * 3 + mv] = a3 * r.v;
  s[0] = r.u - r.c; s[1] = r.u; s[2] = r.u + r.c;
  for (int k = 0; k < 3; ++k) {
    am[k] = 0.0;
    ap[k] = 0.0;
    for (int w = 0; w < 3; ++w) {
      am[k] += fmin(s[w], 0.0) * W[w * 3 + k];
      ap[k] += fmax(s[w], 0.0) * W[w * 3 + k];
    }
  }
  return 3;
}

/* Transverse splitting of a normal fluctuation asdq (from the edge with
 * states ql, qr) into parts moving down / up in the other direction. */
static int tsplit_advection(const fco_params *par, int dir, const double *asdq,
                            double *bm, double *bp) {
  double b = dir == 0 ? par->ay : par->ax;
  bm[0] = fmin(b, 0.0) * asdq[0];
  bp[0] = fmax(b, 0.0) * asdq[0];
  return 0;
}

static int tsplit_shallow(const fco_params *par, int dir, const double *ql,
                          const double *qr, const double *psi, double *bm,
                          double *bp) {
  const int mu = 1 + dir, mv = 2 - dir;
  roe_avg r;
  if (roe_average(par, ql, qr, mu, mv, &r) != 0) return -1;
  double b1 = ((r.v + r.c) * psi[0] - psi[mv]) / (2.0 * r.c);
  double b2 = psi[mu] - r.u * psi[0];
  double b3 = (psi[mv] - (r.v - r.c) * psi[0]) / (2.0 * r.c);
  double lam[3] = {r.v - r.c, r.v, r.v + r.c};
  double R[3][3];
  R[0][0] = 1.0; R[0][mu] = r.u; R[0][mv] = r.v - r.c;
  R[1][0] = 0.0; R[1][mu] = 1.0; R[1][mv] = 0.0;
  R[2][0] = 1.0; R[2][mu] = r.u; R[2][mv] = r.v + r.c;
  double beta[3] = {b1, b2, b3};
  for (int k = 0; k < 3; ++k) {
    bm[k] = 0.0;
    bp[k] = 0.0;
    for (int w = 0; w < 3; ++w) {
      bm[k] += fmin(lam[w], 0.0) * beta[w] * R[w][k];
      bp[k] += fmax(lam[w], 0.0) * beta[w] * R[w][k];
    }
  }
  return 0;
}

int fco_tsplit(const fco_params *par, int32_t dir, const double *ql,
               const double *qr, const double *psi, double *bm, double *bp) {
  switch (par->physics) {
    case FCO_ADVECTION: return tsplit_advection(par, dir, psi, bm, bp);
    case FCO_SHALLOW: return tsplit_shallow(par, dir, ql, qr, psi, bm, bp);
    default: return -1;
  }
}

/* sphere solvers live in fco_sphere.c; *fl receives the mass flux there */
static int riemann(const fco_params *par, int dir, const edge_geom *e,
                   const double *ql, const double *qr, double *W, double *s,
                   double *am, double *ap, double *fl) {
  switch (par->physics) {
    case FCO_ADVECTION: return rp_advection(par, dir, ql, qr, W, s, am, ap);
    case FCO_SHALLOW: return rp_shallow(par, dir, ql, qr, W, s, am, ap);
    case FCO_SPHERE: return fco_rp_sphere(par, e, ql, qr, W, s, am, ap, fl);
    case FCO_SWIRL:
    case FCO_ROTATION: return rp_swirl(e, ql, qr, W, s, am, ap);
    default: return -1;
  }
}

int fco_riemann(const fco_params *par, int32_t dir, const double *ql,
                const double *qr, double *waves, double *speeds, double *amdq,
                double *apdq) {
  edge_geom e = {1.0, {0}, {0}};
  return riemann(par, dir, &e, ql, qr, waves, speeds, amdq, apdq, NULL);
}

/* ---------------- one patch ------------------------------------------ */
typedef struct {
  int32_t m, meqn;
  double *F[2], *AM[2], *AP[2];   /* [edge 0..m+2][row 0..m+1][meqn] */
  double *FL[2];                   /* sphere: mass flux [edge][row] */
  double *W, *S;                   /* one row: [edge][MW][meqn], [edge][MW] */
  double *kap;                     /* frame of capacities */
  edge_geom *eg;                   /* one row of edge geometry */
  edge_geom *tg;                   /* transverse edges of one row */
} work;

static int64_t eidx(int32_t m, int32_t e, int32_t r) {
  return (int64_t)e * (m + 2) + r;
}

static void cell_of(int d, int32_t nidx, int32_t r, int32_t *i, int32_t *j) {
  if (d == 0) { *i = nidx; *j = r; } else { *i = r; *j = nidx; }
}

static double qval(const double *Q, int32_t m, int k, int32_t i, int32_t j) {
  return Q[k * fco_frame(m) + fco_fidx(m, i, j)];
}

static int step_patch(const fco_mesh *mesh, const fco_params *par, int64_t p,
                      const double *Q, double *Qn, double dt, work *wk,
                      double *phi, double *numax) {
  const int32_t m = mesh->m, meqn = par->meqn;
  const fco_leaf *a = &mesh->leaves[p];
  const double dx = ldexp(1.0, -a->level) / m;   /* computational spacing */
  const int64_t NE = (int64_t)(m + 3) * (m + 2);
  /* FCO_SWIRL: tree coordinates of the patch's corner and the mid-step time;
   * the edge between cells n-1 and n of direction d at cell c of the other
   * direction lies at (n - 1) dx and spans [(c - 1) dx, c dx] */
  const double x0 = ldexp((double)a->ix, -a->level), y0 = ldexp((double)a->iy, -a->level);
  const double tmid = par->time + 0.5 * dt;
#define SWIRL_VEL(d, n, c)                                                           \
  fco_swirl_edge(par, (d), ((d) == 0 ? x0 : y0) + ((n) - 1) * dx,                    \
                 ((d) == 0 ? y0 : x0) + ((c) - 1) * dx, ((d) == 0 ? y0 : x0) + (c) * dx, tmid)
  for (int d = 0; d < 2; ++d) {
    memset(wk->F[d], 0, sizeof(double) * NE * meqn);
    memset(wk->AM[d], 0, sizeof(double) * NE * meqn);
    memset(wk->AP[d], 0, sizeof(double) * NE * meqn);
  }
  for (int32_t j = -1; j <= m + 2; ++j)
    for (int32_t i = -1; i <= m + 2; ++i)
      wk->kap[fco_fidx(m, i, j)] =
          mesh->sphere ? fco_sphere_kappa(mesh, p, i, j) : 1.0;
#define KAP(i, j) (wk->kap[fco_fidx(m, (i), (j))])
  double nmax = 0.0;
  double ql[FCO_MAXEQ], qr[FCO_MAXEQ], cq[FCO_MAXEQ], amt[FCO_MAXEQ],
      apt[FCO_MAXEQ], bm[FCO_MAXEQ], bp[FCO_MAXEQ];
  int nw = 0;
  for (int d = 0; d < 2; ++d) {
    double *F = wk->F[d], *FO = wk->F[1 - d];
    for (int32_t r = 0; r <= m + 1; ++r) {
      /* Riemann problems at every edge of the row */
      for (int32_t e = 0; e <= m + 2; ++e) {
        int32_t il, jl, ir, jr;
        cell_of(d, e - 1, r, &il, &jl);
        cell_of(d, e, r, &ir, &jr);
        for (int k = 0; k < meqn; ++k) {
          ql[k] = qval(Q, m, k, il, jl);
          qr[k] = qval(Q, m, k, ir, jr);
        }
        edge_geom *eg = &wk->eg[e];
        if (mesh->sphere) {
          fco_sphere_edge(mesh, p, d, ir, jr, &eg->gamma, eg->n, eg->t);
        } else {
          eg->gamma = 1.0;
        }
        if (par->physics == FCO_SWIRL) eg->vel = SWIRL_VEL(d, e, r);
        if (par->physics == FCO_ROTATION) eg->vel = fco_rotation_edge(mesh, par, p, d, ir, jr);
        nw = riemann(par, d, eg, ql, qr, &wk->W[e * MW * meqn], &wk->S[e * MW],
                     &wk->AM[d][eidx(m, e, r) * meqn],
                     &wk->AP[d][eidx(m, e, r) * meqn], &wk->FL[d][eidx(m, e, r)]);
        if (nw < 0) return -4;
      }
      /* limiter, correction and transverse terms at edges 1..m+1 */
      for (int32_t e = 1; e <= m + 1; ++e) {
        int32_t il, jl, ir, jr;
        cell_of(d, e - 1, r, &il, &jl);
        cell_of(d, e, r, &ir, &jr);
        double dtdl = dt / (KAP(il, jl) * dx), dtdr = dt / (KAP(ir, jr) * dx);
        double nu = 0.5 * (dtdl + dtdr);
        for (int k = 0; k < meqn; ++k) cq[k] = 0.0;
        for (int w = 0; w < nw; ++w) {
          const double *Wc = &wk->W[(e * MW + w) * meqn];
          double sw = wk->S[e * MW + w];
          if (r >= 1 && r <= m) {
            nmax = fmax(nmax, dtdr * fmax(sw, 0.0));
            nmax = fmax(nmax, dtdl * fmax(-sw, 0.0));
          }
          double wn2 = 0.0;
          for (int k = 0; k < meqn; ++k) wn2 += Wc[k] * Wc[k];
          if (wn2 == 0.0) continue;
          int32_t up = sw > 0.0 ? e - 1 : e + 1;
          const double *Wu = &wk->W[(up * MW + w) * meqn];
          double dot = 0.0;
          for (int k = 0; k < meqn; ++k) dot += Wu[k] * Wc[k];
          double lim = fco_phi(par->limiter, dot / wn2);
          double as = fabs(sw);
          for (int k = 0; k < meqn; ++k)
            cq[k] += as * (1.0 - nu * as) * lim * Wc[k];
        }
        double *Fe = &F[eidx(m, e, r) * meqn];
        for (int k = 0; k < meqn; ++k) Fe[k] += 0.5 * cq[k];
        if (par->transverse == 0) continue;
        const double *AMe = &wk->AM[d][eidx(m, e, r) * meqn];
        const double *APe = &wk->AP[d][eidx(m, e, r) * meqn];
        for (int k = 0; k < meqn; ++k) {
          ql[k] = qval(Q, m, k, il, jl);
          qr[k] = qval(Q, m, k, ir, jr);
          amt[k] = AMe[k] + (par->transverse == 2 ? cq[k] : 0.0);
          apt[k] = APe[k] - (par->transverse == 2 ? cq[k] : 0.0);
        }
        /* left-going part enters column e-1, right-going part column e;
         * the lower edge of row r has index r, the upper edge r+1 */
        for (int side = 0; side < 2; ++side) {
          const double *psi = side == 0 ? amt : apt;
          int32_t col = side == 0 ? e - 1 : e;
          double dtd = side == 0 ? dtdl : dtdr;
          int rc;
          if (par->physics == FCO_ADVECTION) {
            rc = tsplit_advection(par, d, psi, bm, bp);
          } else if (par->physics == FCO_SWIRL || par->physics == FCO_ROTATION) {
            /* down through the receiving cell's lower transverse edge, up
             * through its upper one, each at that edge's own velocity */
            double vlo, vhi;
            if (par->physics == FCO_SWIRL) {
              vlo = SWIRL_VEL(1 - d, r, col);
              vhi = SWIRL_VEL(1 - d, r + 1, col);
            } else {
              int32_t ci, cj, ui, uj;
              cell_of(d, col, r, &ci, &cj);
              cell_of(d, col, r + 1, &ui, &uj);
              vlo = fco_rotation_edge(mesh, par, p, 1 - d, ci, cj);
              vhi = fco_rotation_edge(mesh, par, p, 1 - d, ui, uj);
            }
            bm[0] = fmin(vlo, 0.0) * psi[0];
            bp[0] = fmax(vhi, 0.0) * psi[0];
            rc = 0;
          } else if (par->physics == FCO_SHALLOW) {
            rc = tsplit_shallow(par, d, ql, qr, psi, bm, bp);
          } else {
            /* transverse edges of the receiving cell, lower and upper */
            int32_t ci, cj, ui, uj;
            cell_of(d, col, r, &ci, &cj);
            cell_of(d, col, r + 1, &ui, &uj);
            edge_geom lo, hi;
            fco_sphere_edge(mesh, p, 1 - d, ci, cj, &lo.gamma, lo.n, lo.t);
            fco_sphere_edge(mesh, p, 1 - d, ui, uj, &hi.gamma, hi.n, hi.t);
            rc = fco_tsplit_sphere(par, ql, qr, &lo, psi, bm, 0);
            if (rc == 0) rc = fco_tsplit_sphere(par, ql, qr, &hi, psi, bp, 1);
          }
          if (rc != 0) return -4;
          double *Flo = &FO[eidx(m, r, col) * meqn];
          double *Fhi = &FO[eidx(m, r + 1, col) * meqn];
          for (int k = 0; k < meqn; ++k) {
            Flo[k] -= 0.5 * dtd * bm[k];
            Fhi[k] -= 0.5 * dtd * bp[k];
          }
        }
      }
    }
  }
  /* update */
  const int64_t FR = fco_frame(m);
  for (int32_t j = 1; j <= m; ++j)
    for (int32_t i = 1; i <= m; ++i) {
      double dtd = dt / (KAP(i, j) * dx);
      for (int k = 0; k < meqn; ++k) {
        double fx, gy;
        if (par->physics == FCO_SPHERE && k == 0) {   /* mass in flux form */
          fx = wk->FL[0][eidx(m, i + 1, j)] - wk->FL[0][eidx(m, i, j)];
          gy = wk->FL[1][eidx(m, j + 1, i)] - wk->FL[1][eidx(m, j, i)];
        } else {
          fx = wk->AP[0][eidx(m, i, j) * meqn + k] + wk->AM[0][eidx(m, i + 1, j) * meqn + k];
          gy = wk->AP[1][eidx(m, j, i) * meqn + k] + wk->AM[1][eidx(m, j + 1, i) * meqn + k];
        }
        fx = fx + (wk->F[0][eidx(m, i + 1, j) * meqn + k] -
                   wk->F[0][eidx(m, i, j) * meqn + k]);
        gy = gy + (wk->F[1][eidx(m, j + 1, i) * meqn + k] -
                   wk->F[1][eidx(m, j, i) * meqn + k]);
        Qn[k * FR + fco_fidx(m, i, j)] =
            Q[k * FR + fco_fidx(m, i, j)] - dtd * fx - dtd * gy;
      }
    }
  /* face terms for the reflux: the cell's own contribution through each
   * patch face, times the computational face length dx */
  if (phi) {
    for (int f = 0; f < 4; ++f)
      for (int32_t t = 1; t <= m; ++t)
        for (int k = 0; k < meqn; ++k) {
          const int fd = f / 2;
          const int64_t ei = eidx(m, (f & 1) ? m + 1 : 1, t);
          double fluct;
          if (par->physics == FCO_SPHERE && k == 0)   /* flux form: -F in, +F out */
            fluct = (f & 1) ? wk->FL[fd][ei] : -wk->FL[fd][ei];
          else
            fluct = (f & 1) ? wk->AM[fd][ei * meqn + k] : wk->AP[fd][ei * meqn + k];
          const double corr = wk->F[fd][ei * meqn + k];
          const double v = (f & 1) ? fluct + corr : fluct - corr;
          phi[((int64_t)f * m + (t - 1)) * meqn + k] = dx * v;
        }
  }
#undef KAP
#undef SWIRL_VEL
  *numax = nmax;
  return 0;
}

/* ---------------- reflux --------------------------------------------- */
/* fine-cell position in the leaf that contains point (x, y) of tree t */
static int fine_cell(const fco_mesh *mesh, int32_t t, int64_t x, int64_t y,
                     int64_t *L, int32_t *i, int32_t *j, int32_t *tt,
                     int64_t *xx, int64_t *yy) {
  if (fco_locate(mesh->trees, t, x, y, tt, xx, yy) != 0) return -1;
  *L = fco_leaf_at(mesh, *tt, *xx, *yy);
  if (*L < 0) return -1;
  const fco_leaf *a = &mesh->leaves[*L];
  int64_t size = FCO_SIDE >> a->level, cs = size / mesh->m;
  *i = (int32_t)((*xx - (int64_t)a->ix * size) / cs) + 1;
  *j = (int32_t)((*yy - (int64_t)a->iy * size) / cs) + 1;
  return 0;
}

static int reflux(const fco_mesh *mesh, const fco_params *par, const double *q,
                  double *qn, double dt, const double *phi) {
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t FR = fco_frame(m);
  double W[MW * FCO_MAXEQ], S[MW], am[FCO_MAXEQ], ap[FCO_MAXEQ];
  double ql[FCO_MAXEQ], qr[FCO_MAXEQ], qc[FCO_MAXEQ], qf[FCO_MAXEQ];
  for (int f = 0; f < 4; ++f) {
    const int d = f / 2, hi = f % 2;
    for (int64_t p = 0; p < mesh->n; ++p) {
      if (fco_wall_face(mesh, p, f)) continue;
      const fco_leaf *a = &mesh->leaves[p];
      const int64_t size = FCO_SIDE >> a->level, cs = size / m;
      const int64_t x0 = (int64_t)a->ix * size, y0 = (int64_t)a->iy * size;
      const double dx = ldexp(1.0, -a->level) / m;
      for (int32_t t = 1; t <= m; ++t) {
        int32_t ic = d == 0 ? (hi ? m : 1) : t;
        int32_t jc = d == 0 ? t : (hi ? m : 1);
        double corr[FCO_MAXEQ] = {0};
        int fine = 1;
        for (int k2 = 0; k2 < 2 && fine; ++k2) {
          /* centre of the k2-th fine cell across the face, and a point a
           * quarter fine cell closer to the face (same fine cell) */
          int64_t nrm_out = hi ? size + cs / 4 : -cs / 4;
          int64_t nrm_in = hi ? size + cs / 8 : -cs / 8;
          int64_t tan = (int64_t)(t - 1) * cs + (k2 == 0 ? cs / 4 : 3 * cs / 4);
          int64_t xa, ya, xb, yb;
          if (d == 0) { xa = x0 + nrm_out; ya = y0 + tan; xb = x0 + nrm_in; yb = ya; }
          else { xa = x0 + tan; ya = y0 + nrm_out; xb = xa; yb = y0 + nrm_in; }
          int64_t L, L2, X, Y, X2, Y2;
          int32_t fi, fj, fi2, fj2, tt, tt2;
          if (fine_cell(mesh, a->tree, xa, ya, &L, &fi, &fj, &tt, &X, &Y) != 0 ||
              fine_cell(mesh, a->tree, xb, yb, &L2, &fi2, &fj2, &tt2, &X2, &Y2) != 0)
            return -5;
          if (mesh->sphere && k2 == 0 && mesh->leaves[L].level == a->level &&
              tt != a->tree && L < p) {
            /* same-level faces across cube edges: the mass face term of the
             * higher-numbered patch becomes minus its neighbour's, so that
             * both sides agree also next to a cube vertex (where their
             * transverse terms read different corner ghosts) */
            int ffs;
            if (X2 != X) ffs = X2 > X ? 1 : 0;
            else ffs = Y2 > Y ? 3 : 2;
            const int32_t fts = (ffs < 2) ? fj : fi;
            const double phin = phi[((L * 4 + ffs) * m + (fts - 1)) * meqn];
            const double phio = phi[((p * 4 + f) * m + (t - 1)) * meqn];
            const double ks = fco_sphere_kappa(mesh, p, ic, jc);
            qn[(p * meqn) * FR + fco_fidx(m, ic, jc)] -=
                dt / (ks * dx * dx) * (-phin - phio);
          }
          if (mesh->leaves[L].level != a->level + 1) { fine = 0; break; }
          /* the direction towards the coarse cell, in the fine leaf's frame,
           * names the fine leaf's face */
          int ff;
          if (X2 != X) ff = X2 > X ? 1 : 0;
          else ff = Y2 > Y ? 3 : 2;
          int32_t ft = (ff < 2) ? fj : fi;
          const double *phif = &phi[((L * 4 + ff) * m + (ft - 1)) * meqn];
          for (int k = 0; k < meqn; ++k) {
            qc[k] = q[(p * meqn + k) * FR + fco_fidx(m, ic, jc)];
            qf[k] = q[(L * meqn + k) * FR + fco_fidx(m, fi, fj)];
          }
          for (int k = 0; k < meqn; ++k) {
            ql[k] = hi ? qc[k] : qf[k];
            qr[k] = hi ? qf[k] : qc[k];
          }
          edge_geom eg = {1.0, {0}, {0}};
          double flen = 0.5 * dx;
          if (mesh->sphere) {
            /* the fine edge, seen from the fine leaf */
            int32_t ei = fi, ej = fj, ed = ff / 2;
            if (ff == 1) ei = fi + 1;
            if (ff == 3) ej = fj + 1;
            fco_sphere_edge(mesh, L, ed, ei, ej, &eg.gamma, eg.n, eg.t);
            /* orient the normal from the left state to the right state */
            double sgn = 1.0;
            if ((ff % 2 == 1) != (hi == 0)) sgn = -1.0;
            for (int c = 0; c < 3; ++c) eg.n[c] *= sgn;
            for (int c = 0; c < 3; ++c) eg.t[c] *= sgn;
          }
          if (riemann(par, d, &eg, ql, qr, W, S, am, ap, NULL) < 0) return -4;
          /* the mass of a sphere is in flux form: its face terms already
           * are fluxes, so the fine terms replace the coarse one as they are */
          for (int k = 0; k < meqn; ++k)
            corr[k] += (mesh->sphere && k == 0 ? 0.0 : flen * (am[k] + ap[k])) - phif[k];
        }
        if (!fine) continue;
        const double *phic = &phi[((p * 4 + f) * m + (t - 1)) * meqn];
        double kc = mesh->sphere ? fco_sphere_kappa(mesh, p, ic, jc) : 1.0;
        for (int k = 0; k < meqn; ++k)
          qn[(p * meqn + k) * FR + fco_fidx(m, ic, jc)] -=
              dt / (kc * dx * dx) * (corr[k] - phic[k]);
      }
    }
  }
  return 0;
}

int fco_step(const fco_mesh *mesh, const fco_params *par, const double *q,
             double *qn, double dt, int32_t do_reflux, double *numax) {
  if (!mesh || !par || !q || !qn || par->m != mesh->m || par->meqn < 1 ||
      par->meqn > FCO_MAXEQ)
    return -1;
  if ((par->physics == FCO_SPHERE || par->physics == FCO_ROTATION) != (mesh->sphere != 0))
    return -1;
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t NE = (int64_t)(m + 3) * (m + 2), FR = fco_frame(m);
  double *phi = do_reflux
                    ? (double *)malloc(sizeof(double) * mesh->n * 4 * m * meqn)
                    : NULL;
  double nmax = 0.0;
  int rc = 0;
  /* patches are independent given the filled frames: with more than one
   * thread (fco_set_threads) each takes whole patches with a work area of
   * its own; every patch's arithmetic is the same as with one */
#pragma omp parallel num_threads(fco_threads()) reduction(max : nmax) reduction(| : rc)
  {
    work wk;
    wk.m = m;
    wk.meqn = meqn;
    for (int d = 0; d < 2; ++d) {
      wk.F[d] = (double *)malloc(sizeof(double) * NE * meqn);
      wk.AM[d] = (double *)malloc(sizeof(double) * NE * meqn);
      wk.AP[d] = (double *)malloc(sizeof(double) * NE * meqn);
      wk.FL[d] = (double *)calloc(NE, sizeof(double));
    }
    wk.W = (double *)malloc(sizeof(double) * (m + 3) * MW * meqn);
    wk.S = (double *)malloc(sizeof(double) * (m + 3) * MW);
    wk.kap = (double *)malloc(sizeof(double) * FR);
    wk.eg = (edge_geom *)malloc(sizeof(edge_geom) * (m + 3));
    wk.tg = NULL;
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < mesh->n; ++p) {
      double nu = 0.0;
      rc |= step_patch(mesh, par, p, &q[p * meqn * FR], &qn[p * meqn * FR], dt,
                       &wk, phi ? &phi[p * 4 * m * meqn] : NULL, &nu) != 0;
      nmax = fmax(nmax, nu);
    }
    for (int d = 0; d < 2; ++d) {
      free(wk.F[d]);
      free(wk.AM[d]);
      free(wk.AP[d]);
      free(wk.FL[d]);
    }
    free(wk.W);
    free(wk.S);
    free(wk.kap);
    free(wk.eg);
  }
  if (rc) rc = -1;
  /* the colour equation is not in conservation form: no reflux */
  if (rc == 0 && do_reflux && par->physics != FCO_SWIRL && par->physics != FCO_ROTATION)
    rc = reflux(mesh, par, q, qn, dt, phi);
  if (rc == 0 && par->physics == FCO_SPHERE) fco_sphere_project(mesh, par, qn);
  free(phi);
  if (numax) *numax = nmax;
  return rc;
}

/* ---------------- sub-cycled step -------------------------------------- */
/* Per-level time steps (Sec. 4: one exchange per level and time step, the
 * levels visited from coarse to fine and correction factors carried back
 * from fine to coarse; Sec. 3: time-accurate coarse data fill the ghost
 * cells of finer patches), in the recursive form of the block-structured
 * AMR codes the paper cites (Berger and Oliger 1984; flux correction of
 * Berger and Colella 1989).  Level l steps with dt_l = dt 2^-l (dt is the
 * step of a level-0 patch, so every level runs at the same Courant number):
 * one step of the coarsest level lmin takes 2^(l - lmin) steps at level l:
 *
 *   advance(l, t):  keep the level-l states at time t (old); fill the
 *     level-l ghost cells at time t (a coarser leaf, which is inside its own
 *     step, gives (1 - a) old + a new with a its fraction of that step);
 *     step the level-l patches by dt_l; add this substep's fine-side terms
 *     to the accumulators psi of their faces that border level l - 1;
 *     then advance(l + 1, t), advance(l + 1, t + dt_l / 2) and correct the
 *     level-l cells at faces with level-(l + 1) patches.
 *
 * Fine-side term of a substep at one fine face cell, w = dt_l / dt_{l-1}
 * = 1/2:   w [ dx_f (f(q_f) - f(q_c)) - phi_f ]   with q_f the fine cell at
 * the substep's start and q_c the coarse cell at the start of the coarse
 * level's step (f(q_f) - f(q_c) as the sum of the pair's fluctuations,
 * Roe's property).  The coarse cell then takes
 *   -dt_{l-1} / dx_c^2 (psi of its two fine cells - phi_c),
 * which with a single substep (w = 1) is the reflux of the global-dt step.
 * Planar forests only. */

/* The fine cell across position t (1..m) of face f of patch p, half k2: its
 * leaf L, cell (fi, fj), face ff towards p and position ft along that face.
 * Returns 1 if the leaf across is one level finer, 0 if not, < 0 on error. */
static int cf_pair(const fco_mesh *mesh, int64_t p, int f, int32_t t, int k2,
                   int64_t *L, int32_t *fi, int32_t *fj, int *ff, int32_t *ft) {
  const int32_t m = mesh->m;
  const int d = f / 2, hi = f % 2;
  const fco_leaf *a = &mesh->leaves[p];
  const int64_t size = FCO_SIDE >> a->level, cs = size / m;
  const int64_t x0 = (int64_t)a->ix * size, y0 = (int64_t)a->iy * size;
  int64_t nrm_out = hi ? size + cs / 4 : -cs / 4;
  int64_t nrm_in = hi ? size + cs / 8 : -cs / 8;
  int64_t tan = (int64_t)(t - 1) * cs + (k2 == 0 ? cs / 4 : 3 * cs / 4);
  int64_t xa, ya, xb, yb;
  if (d == 0) { xa = x0 + nrm_out; ya = y0 + tan; xb = x0 + nrm_in; yb = ya; }
  else { xa = x0 + tan; ya = y0 + nrm_out; xb = xa; yb = y0 + nrm_in; }
  int64_t L2, X, Y, X2, Y2;
  int32_t fi2, fj2, tt, tt2;
  if (fine_cell(mesh, a->tree, xa, ya, L, fi, fj, &tt, &X, &Y) != 0 ||
      fine_cell(mesh, a->tree, xb, yb, &L2, &fi2, &fj2, &tt2, &X2, &Y2) != 0)
    return -5;
  if (mesh->leaves[*L].level != a->level + 1) return 0;
  if (X2 != X) *ff = X2 > X ? 1 : 0;
  else *ff = Y2 > Y ? 3 : 2;
  *ft = (*ff < 2) ? *fj : *fi;
  return 1;
}

typedef struct {
  const fco_mesh *mesh;
  const fco_params *par;
  int32_t lmin, lmax;
  double *cur, *old, *tmp;            /* framed states per patch */
  double *phi, *psi;                  /* [P][4][m][meqn] face terms */
  double t_old[FCO_S + 1], dtl[FCO_S + 1];
  work wk;
  double numax;
} subcycle;

/* psi of level-lf patches += w [dx_f (f(q_f) - f(q_c)) - phi_f] at their
 * faces with level lf - 1 (q_f, q_c: states at the starts of the steps) */
static int accumulate_fine(subcycle *S, int32_t lf, double w) {
  const fco_mesh *mesh = S->mesh;
  const fco_params *par = S->par;
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t FR = fco_frame(m);
  double W[MW * FCO_MAXEQ], Sp[MW], am[FCO_MAXEQ], ap[FCO_MAXEQ];
  double ql[FCO_MAXEQ], qr[FCO_MAXEQ];
  for (int f = 0; f < 4; ++f) {
    const int d = f / 2, hi = f % 2;
    for (int64_t p = 0; p < mesh->n; ++p) {
      if (mesh->leaves[p].level != lf - 1 || fco_wall_face(mesh, p, f)) continue;
      const double dx = ldexp(1.0, -mesh->leaves[p].level) / m;
      for (int32_t t = 1; t <= m; ++t) {
        const int32_t ic = d == 0 ? (hi ? m : 1) : t;
        const int32_t jc = d == 0 ? t : (hi ? m : 1);
        for (int k2 = 0; k2 < 2; ++k2) {
          int64_t L;
          int32_t fi, fj, ft;
          int ff;
          const int r = cf_pair(mesh, p, f, t, k2, &L, &fi, &fj, &ff, &ft);
          if (r < 0) return r;
          if (r == 0) break;
          for (int k = 0; k < meqn; ++k) {
            const double qc = S->old[(p * meqn + k) * FR + fco_fidx(m, ic, jc)];
            const double qf = S->old[(L * meqn + k) * FR + fco_fidx(m, fi, fj)];
            ql[k] = hi ? qc : qf;
            qr[k] = hi ? qf : qc;
          }
          edge_geom eg = {1.0, {0}, {0}};
          if (riemann(par, d, &eg, ql, qr, W, Sp, am, ap, NULL) < 0) return -4;
          double *ps = &S->psi[((L * 4 + ff) * m + (ft - 1)) * meqn];
          const double *pf = &S->phi[((L * 4 + ff) * m + (ft - 1)) * meqn];
          for (int k = 0; k < meqn; ++k)
            ps[k] += w * (0.5 * dx * (am[k] + ap[k]) - pf[k]);
        }
      }
    }
  }
  return 0;
}

/* level-lc cells at faces with level lc + 1: -dt / dx^2 (psi - phi_c),
 * xi faces first, then eta faces */
static int correct_coarse(subcycle *S, int32_t lc) {
  const fco_mesh *mesh = S->mesh;
  const int32_t m = mesh->m, meqn = S->par->meqn;
  const int64_t FR = fco_frame(m);
  const double dt = S->dtl[lc];
  for (int f = 0; f < 4; ++f) {
    const int d = f / 2, hi = f % 2;
    for (int64_t p = 0; p < mesh->n; ++p) {
      if (mesh->leaves[p].level != lc || fco_wall_face(mesh, p, f)) continue;
      const double dx = ldexp(1.0, -lc) / m;
      for (int32_t t = 1; t <= m; ++t) {
        const int32_t ic = d == 0 ? (hi ? m : 1) : t;
        const int32_t jc = d == 0 ? t : (hi ? m : 1);
        double corr[FCO_MAXEQ] = {0};
        int fine = 1;
        for (int k2 = 0; k2 < 2 && fine; ++k2) {
          int64_t L;
          int32_t fi, fj, ft;
          int ff;
          const int r = cf_pair(mesh, p, f, t, k2, &L, &fi, &fj, &ff, &ft);
          if (r < 0) return r;
          if (r == 0) { fine = 0; break; }
          const double *ps = &S->psi[((L * 4 + ff) * m + (ft - 1)) * meqn];
          for (int k = 0; k < meqn; ++k) corr[k] += ps[k];
        }
        if (!fine) continue;
        const double *phic = &S->phi[((p * 4 + f) * m + (t - 1)) * meqn];
        for (int k = 0; k < meqn; ++k)
          S->cur[(p * meqn + k) * FR + fco_fidx(m, ic, jc)] -=
              dt / (dx * dx) * (corr[k] - phic[k]);
      }
    }
  }
  return 0;
}

static int advance_level(subcycle *S, int32_t l, double t) {
  const fco_mesh *mesh = S->mesh;
  const fco_params *par = S->par;
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t FR = fco_frame(m), PS = (int64_t)meqn * FR;
  const double dt = S->dtl[l];
  /* the level-l states at time t */
  for (int64_t p = 0; p < mesh->n; ++p)
    if (mesh->leaves[p].level == l)
      memcpy(&S->old[p * PS], &S->cur[p * PS], sizeof(double) * PS);
  S->t_old[l] = t;
  /* ghost cells of level l at time t */
  double alpha[FCO_S + 1];
  for (int32_t lv = 0; lv <= FCO_S; ++lv)
    alpha[lv] = lv < l && lv >= S->lmin ? (t - S->t_old[lv]) / S->dtl[lv] : 0.0;
  int rc = fco_ghost_fill_level(mesh, par, S->cur, S->old, alpha, l);
  if (rc != 0) return rc;
  /* the level-l patches, then their new interiors */
  for (int64_t p = 0; p < mesh->n; ++p) {
    if (mesh->leaves[p].level != l) continue;
    double nu = 0.0;
    rc = step_patch(mesh, par, p, &S->cur[p * PS], &S->tmp[p * PS], dt, &S->wk,
                    &S->phi[p * 4 * m * meqn], &nu);
    if (rc != 0) return rc;
    S->numax = fmax(S->numax, nu);
  }
  for (int64_t p = 0; p < mesh->n; ++p) {
    if (mesh->leaves[p].level != l) continue;
    for (int k = 0; k < meqn; ++k)
      for (int32_t j = 1; j <= m; ++j)
        for (int32_t i = 1; i <= m; ++i) {
          const int64_t o = p * PS + k * FR + fco_fidx(m, i, j);
          S->cur[o] = S->tmp[o];
        }
  }
  /* this substep's terms at faces with the next coarser level */
  if (l > S->lmin) {
    rc = accumulate_fine(S, l, dt / S->dtl[l - 1]);
    if (rc != 0) return rc;
  }
  if (l < S->lmax) {
    for (int64_t p = 0; p < mesh->n; ++p)
      if (mesh->leaves[p].level == l + 1)
        memset(&S->psi[p * 4 * m * meqn], 0, sizeof(double) * 4 * m * meqn);
    rc = advance_level(S, l + 1, t);
    if (rc == 0) rc = advance_level(S, l + 1, t + 0.5 * dt);
    if (rc == 0) rc = correct_coarse(S, l);
    if (rc != 0) return rc;
  }
  return 0;
}

int fco_step_subcycled(const fco_mesh *mesh, const fco_params *par, const double *q,
                       double *qn, double dt, double *numax) {
  if (!mesh || !par || !q || !qn || par->m != mesh->m || par->meqn < 1 ||
      par->meqn > FCO_MAXEQ || mesh->sphere || par->physics == FCO_SPHERE ||
      par->physics == FCO_SWIRL)
    return -1;
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t NE = (int64_t)(m + 3) * (m + 2), FR = fco_frame(m);
  const int64_t PS = (int64_t)meqn * FR, n = mesh->n;
  subcycle S;
  memset(&S, 0, sizeof S);
  S.mesh = mesh;
  S.par = par;
  S.lmin = FCO_S;
  S.lmax = 0;
  for (int64_t p = 0; p < n; ++p) {
    const int32_t l = mesh->leaves[p].level;
    if (l < S.lmin) S.lmin = l;
    if (l > S.lmax) S.lmax = l;
  }
  for (int32_t l = S.lmin; l <= S.lmax; ++l) S.dtl[l] = ldexp(dt, -l);
  S.cur = (double *)malloc(sizeof(double) * n * PS);
  S.old = (double *)malloc(sizeof(double) * n * PS);
  S.tmp = (double *)malloc(sizeof(double) * n * PS);
  S.phi = (double *)calloc((size_t)n * 4 * m * meqn, sizeof(double));
  S.psi = (double *)calloc((size_t)n * 4 * m * meqn, sizeof(double));
  S.wk.m = m;
  S.wk.meqn = meqn;
  for (int d = 0; d < 2; ++d) {
    S.wk.F[d] = (double *)malloc(sizeof(double) * NE * meqn);
    S.wk.AM[d] = (double *)malloc(sizeof(double) * NE * meqn);
    S.wk.AP[d] = (double *)malloc(sizeof(double) * NE * meqn);
    S.wk.FL[d] = (double *)calloc(NE, sizeof(double));
  }
  S.wk.W = (double *)malloc(sizeof(double) * (m + 3) * MW * meqn);
  S.wk.S = (double *)malloc(sizeof(double) * (m + 3) * MW);
  S.wk.kap = (double *)malloc(sizeof(double) * FR);
  S.wk.eg = (edge_geom *)malloc(sizeof(edge_geom) * (m + 3));
  S.wk.tg = NULL;
  memcpy(S.cur, q, sizeof(double) * n * PS);
  memcpy(S.tmp, q, sizeof(double) * n * PS);
  const int rc = advance_level(&S, S.lmin, 0.0);
  if (rc == 0) memcpy(qn, S.cur, sizeof(double) * n * PS);
  if (numax) *numax = S.numax;
  for (int d = 0; d < 2; ++d) {
    free(S.wk.F[d]);
    free(S.wk.AM[d]);
    free(S.wk.AP[d]);
    free(S.wk.FL[d]);
  }
  free(S.wk.W);
  free(S.wk.S);
  free(S.wk.kap);
  free(S.wk.eg);
  free(S.cur);
  free(S.old);
  free(S.tmp);
  free(S.phi);
  free(S.psi);
  return rc;
}

/* ---------------- conservation sums ---------------------------------- */
/* M_k = sum over interior cells of kappa Q_k dxi deta, with Neumaier's
 * compensated summation. */
int fco_sums(const fco_mesh *mesh, const fco_params *par, const double *q,
             double *sums) {
  const int32_t m = mesh->m, meqn = par->meqn;
  const int64_t FR = fco_frame(m);
  for (int k = 0; k < meqn; ++k) {
    double s = 0.0, c = 0.0;
    for (int64_t p = 0; p < mesh->n; ++p) {
      const double dx = ldexp(1.0, -mesh->leaves[p].level) / m;
      for (int32_t j = 1; j <= m; ++j)
        for (int32_t i = 1; i <= m; ++i) {
          double kap = mesh->sphere ? fco_sphere_kappa(mesh, p, i, j) : 1.0;
          double v = kap * q[(p * meqn + k) * FR + fco_fidx(m, i, j)] * dx * dx;
          double t = s + v;
          if (fabs(s) >= fabs(v)) c += (s - t) + v;
          else c += (v - t) + s;
          s = t;
        }
    }
    sums[k] = s + c;
  }
  return 0;
}
