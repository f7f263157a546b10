/* fco_sphere.c -- cubed-sphere geometry and solver of the CPU oracle
 * (test infrastructure only).  Placeholder until the mapped path lands. */
#include "fco_internal.h"

#include <math.h>

double fco_sphere_kappa(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j) {
  (void)mesh; (void)p; (void)i; (void)j;
  return NAN;
}
void fco_sphere_edge(const fco_mesh *mesh, int64_t p, int32_t dir, int32_t i,
                     int32_t j, double *gamma, double n[3], double t[3]) {
  (void)mesh; (void)p; (void)dir; (void)i; (void)j;
  *gamma = NAN;
  for (int c = 0; c < 3; ++c) { n[c] = NAN; t[c] = NAN; }
}
void fco_sphere_centre(const fco_mesh *mesh, int64_t p, int32_t i, int32_t j,
                       double r[3]) {
  (void)mesh; (void)p; (void)i; (void)j;
  for (int c = 0; c < 3; ++c) r[c] = NAN;
}

typedef struct { double gamma; double n[3], t[3]; } edge_geom;
int fco_rp_sphere(const fco_params *par, const edge_geom *e, const double *ql,
                  const double *qr, double *W, double *s, double *am,
                  double *ap) {
  return -1;
}
int fco_tsplit_sphere(const fco_params *par, const double *ql,
                      const double *qr, const edge_geom *normal_edge,
                      const edge_geom *tedge, const double *psi, double *bsdq,
                      int up) {
  return -1;
}
void fco_sphere_project(const fco_mesh *mesh, const fco_params *par,
                        double *qn) {}
