// sphere.hpp -- the cubed sphere: geometry of patches and of their ghost
// layers from the gnomonic equiangular map (Sec. 2: six mapped trees), and
// the shallow-water step with 3D Cartesian momentum on mapped cells (the
// capacity form of the wave-propagation method the paper adopts for mapped
// grids, Calhoun, Helzel and LeVeque 2008).
//
// Tree t is cube face t with centre c, axes u, v (u x v = c); reference
// point (xi, eta) -> c + T(xi) u + T(eta) v -> unit sphere, T(s) =
// tan((s - 1/2) pi/2) with T(0) = -1, T(1) = 1, T(1 - s) = -T(s) exactly,
// so points on a cube edge get the same coordinates from either face.
//
// Geometry table of a patch, indexed by frame cell f = (j+1)(m+4) + (i+1),
// i, j = -1 .. m+2 (doubles, kGeoN frames per patch):
//   [kGeoK] capacity kappa = cell area / dxi^2;
//   [kGeoC] cell centre (3 per cell);
//   [kGeoE] low-side edge of the cell in direction 0 (xi) then 1 (eta):
//           gamma = arc length / dxi, normal n (towards higher index),
//           tangent t = r_mid x n (7 per cell and direction).
// Corner points outside the patch's tree are carried into the tree that
// holds them (ghost cells get the geometry of the cells they copy); the
// corner region at a cube vertex, which no tree covers, uses the patch's own
// face mapping extended, for its cells and for edges between two of them.
#pragma once

#include "device.hpp"
#include "step.hpp"

namespace fcx {

constexpr int kGeoK = 0, kGeoC = 1, kGeoE = 4, kGeoN = 18;

__constant__ double kCubeFace[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {0, 1, 0}, {-1, 0, 0}},
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

__device__ __forceinline__ int fidx(int m, int i, int j) { return (j + 1) * (m + 4) + (i + 1); }

__device__ inline double tline(int32_t X) {
  const int64_t d = 2 * int64_t(X) - kSide;
  if (d == 0) return 0.0;
  const int64_t ad = d < 0 ? -d : d;
  const double t = ad == kSide ? 1.0 : tan(ldexp(double(ad), -kS) * 0.78539816339744830962);
  return d < 0 ? -t : t;
}

__device__ inline void face_point(int t, int32_t X, int32_t Y, double* r) {
  const double a = tline(X), b = tline(Y);
  double p[3];
  for (int c = 0; c < 3; ++c) p[c] = kCubeFace[t][0][c] + a * kCubeFace[t][1][c] + b * kCubeFace[t][2][c];
  const double s = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  for (int c = 0; c < 3; ++c) r[c] = p[c] / s;
}

// The pillow sphere (two trees, one per hemisphere): with x = 2 xi - 1,
// y = 2 eta - 1 and d = max(|x|, |y|), the square of half-width d goes to
// the circle of polar angle d pi / 2 about the tree's pole, each point along
// its direction (x, y) / |(x, y)|; tree 1 negates the second and third
// components (both trees right-handed seen from outside).  The boundary
// (d = 1) lands on the equator exactly, and glued faces give identical
// points: faces 0 and 1 meet their namesakes reversed, face 2 meets face 3.
__device__ inline void pillow_point(int t, int32_t X, int32_t Y, double* r) {
  const double x = ldexp(double(2 * int64_t(X) - kSide), -kS);
  const double y = ldexp(double(2 * int64_t(Y) - kSide), -kS);
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

__device__ inline void tree_point(bool pillow, int t, int32_t X, int32_t Y, double* r) {
  if (pillow) pillow_point(t, X, Y, r);
  else face_point(t, X, Y, r);
}

// Sphere point of tree coordinates (X, Y) of patch r's tree, carried into
// the tree that holds it (trees closed; own face extended at a cube vertex;
// beyond a pillow corner, the point mirrored into the own tree).
__device__ inline void patch_point(const PatchRec* __restrict__ rec, const PatchRec& r,
                                   int32_t X, int32_t Y, double* out, bool pillow) {
  const int tree = r.flags >> kTreeShift;
  const int32_t side = int32_t(kSide);
  const bool ox = X < 0 || X > side, oy = Y < 0 || Y > side;
  if (!ox && !oy) { tree_point(pillow, tree, X, Y, out); return; }
  int32_t code, nb;
  if (ox && !oy) {
    const int f = X < 0 ? 0 : 1;
    code = r.xf[f];
    nb = r.nbr[2 * f];
  } else if (oy && !ox) {
    const int f = Y < 0 ? 2 : 3;
    code = r.xf[f];
    nb = r.nbr[2 * f];
  } else {
    const int c = (X > 0) + 2 * (Y > 0);
    nb = r.nbr[8 + c];
    code = r.xf[4 + c];
    if (nb < 0) { tree_point(pillow, tree, X, Y, out); return; }   // cube vertex
  }
  int32_t X2, Y2;
  xf_apply(code, X, Y, X2, Y2);
  tree_point(pillow, rec[nb].flags >> kTreeShift, X2, Y2, out);
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
// solid angle of the counter-clockwise spherical triangle (Van Oosterom and
// Strackee), with the triple product taken over the two short sides,
// a.((b - a) x (c - a)): for a cell of angular size h, a.(b x c) formed
// directly loses relative accuracy to cancellation (an error of order
// eps / h^2, about 1e-9 for the finest cells of a level-7 patch of 32 x 32),
// while the differences of close points are exact and this form keeps it.
__device__ __forceinline__ double tri_area(const double* a, const double* b, const double* c) {
  double u[3], v[3], w[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = b[k] - a[k];
    v[k] = c[k] - a[k];
  }
  cross3(u, v, w);
  return 2.0 * atan2(dot3(a, w), 1.0 + dot3(a, b) + dot3(b, c) + dot3(c, a));
}

// a x b for two close unit vectors as their mean crossed with their
// difference: accurate where a x b cancels, and exactly negated when a and b
// swap, so an edge shared by two cells or patches is the same from either.
__device__ __forceinline__ void cross_near(const double* a, const double* b, double* o) {
  double mid[3], d[3];
  for (int k = 0; k < 3; ++k) {
    mid[k] = 0.5 * (a[k] + b[k]);
    d[k] = b[k] - a[k];
  }
  cross3(mid, d, o);
}

// frame cell (i, j) lies in a corner region at a cube vertex
__device__ __forceinline__ bool vertex_cell(const PatchRec& r, int m, int i, int j) {
  if ((i >= 1 && i <= m) || (j >= 1 && j <= m)) return false;
  return r.nbr[8 + (i > m) + 2 * (j > m)] == kNbrValence3;
}

// One workgroup per patch: the geometry table (dynamic LDS: the canonical
// corner grid of (m+5)^2 points; own-face points are recomputed where a
// cube-vertex region needs them).
__global__ void __launch_bounds__(256)
k_sphere_metrics(const PatchRec* __restrict__ rec, int m, int lm, double* __restrict__ geo,
                 int pillow) {
  extern __shared__ double can[];
  const int NC = m + 5, FR = (m + 4) * (m + 4);
  const int p = blockIdx.x;
  const PatchRec r = rec[p];
  const int tree = r.flags >> kTreeShift;
  const int sh = kS - r.level;
  const int32_t cs = int32_t(1) << (sh - lm);
  const int32_t x0 = r.ix << sh, y0 = r.iy << sh;
  for (int k = threadIdx.x; k < NC * NC; k += blockDim.x) {
    const int32_t X = x0 + (k % NC - 2) * cs, Y = y0 + (k / NC - 2) * cs;
    patch_point(rec, r, X, Y, can + 3 * k, pillow != 0);
  }
  __syncthreads();
  const double dx = ldexp(1.0, -r.level) / m;
  double* g = geo + size_t(p) * kGeoN * FR;
  // corner (I, J): canonical from LDS, or the own face mapping into buf
  auto pt = [&](bool own, int I, int J, double* buf) -> const double* {
    if (!own) return can + 3 * ((J + 2) * NC + (I + 2));
    tree_point(pillow != 0, tree, x0 + I * cs, y0 + J * cs, buf);
    return buf;
  };
  for (int f = threadIdx.x; f < FR; f += blockDim.x) {
    const int i = f % (m + 4) - 1, j = f / (m + 4) - 1;
    const bool vc = vertex_cell(r, m, i, j);
    double ba[3], bb[3], bc[3], bd[3];
    const double *A = pt(vc, i - 1, j - 1, ba), *B = pt(vc, i, j - 1, bb),
                 *C = pt(vc, i, j, bc), *D = pt(vc, i - 1, j, bd);
    g[kGeoK * FR + f] = (tri_area(A, B, C) + tri_area(A, C, D)) / (dx * dx);
    patch_point(rec, r, x0 + (2 * i - 1) * (cs >> 1), y0 + (2 * j - 1) * (cs >> 1),
                g + kGeoC * FR + 3 * f, pillow != 0);
    for (int dir = 0; dir < 2; ++dir) {
      const bool vn = dir == 0 ? vertex_cell(r, m, i - 1, j) : vertex_cell(r, m, i, j - 1);
      const bool own = vc && vn;
      double be[3], bf[3];
      const double* ea = pt(own, i - 1, j - 1, be);
      const double* eb = dir == 0 ? pt(own, i - 1, j, bf) : pt(own, i, j - 1, bf);
      double cr[3], nn[3], rm[3], tt[3];
      cross_near(ea, eb, cr);
      const double len = sqrt(dot3(cr, cr));
      const double sg = dir == 0 ? -1.0 : 1.0;
      for (int c = 0; c < 3; ++c) nn[c] = sg * cr[c] / len;
      for (int c = 0; c < 3; ++c) rm[c] = ea[c] + eb[c];
      const double rl = sqrt(dot3(rm, rm));
      for (int c = 0; c < 3; ++c) rm[c] /= rl;
      cross3(rm, nn, tt);
      double* e = g + kGeoE * FR + (dir * FR + f) * 7;
      e[0] = atan2(len, dot3(ea, eb)) / dx;
      for (int c = 0; c < 3; ++c) e[1 + c] = nn[c];
      for (int c = 0; c < 3; ++c) e[4 + c] = tt[c];
    }
  }
}

// ---------------------------------------------------------------------------
// rotated Roe solver and transverse splitting

template <typename R>
struct SEdge {
  R g, n[3], t[3];
};

template <typename R, typename G>
__device__ __forceinline__ SEdge<R> load_edge(const G* e) {
  SEdge<R> s;
  s.g = R(e[0]);
  for (int c = 0; c < 3; ++c) { s.n[c] = R(e[1 + c]); s.t[c] = R(e[4 + c]); }
  return s;
}

// The step's geometry in FP32 for FP32 state (the FP32 step rounds every
// edge and centre value to FP32 anyway): per patch the two edge frames of
// each frame cell (7 values each, interleaved, direction-major) and the
// centre (3 values per cell).
constexpr int kG32E = 0, kG32C = 14, kG32N = 17;

__global__ void __launch_bounds__(256)
k_sphere_geo32(const double* __restrict__ geo, float* __restrict__ g32, int64_t P, int m) {
  const int FR = (m + 4) * (m + 4);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P * kG32N * FR) return;
  const int64_t p = t / (int64_t(kG32N) * FR);
  const int v = int(t - p * kG32N * FR);
  // frames kGeoE.. of the FP64 table hold the edges in the same order, and
  // frames kGeoC.. the centres
  const double* g = geo + size_t(p) * kGeoN * FR;
  g32[t] = float(v < 14 * FR ? g[kGeoE * FR + v] : g[kGeoC * FR + (v - 14 * FR)]);
}

// waves W[w][k], speeds s[w] (times gamma), fluctuations, mass flux fl;
// false if a depth is not positive
template <typename R>
__device__ bool rp_sphere(R grav, const SEdge<R>& e, const R* ql, const R* qr, R (*W)[4],
                          R* s, R* am, R* ap, R& fl) {
  const R hl = ql[0], hr = qr[0];
  if (!(hl > R(0) && hr > R(0))) return false;
  const R nl = ql[1] * e.n[0] + ql[2] * e.n[1] + ql[3] * e.n[2];
  const R nr = qr[1] * e.n[0] + qr[2] * e.n[1] + qr[3] * e.n[2];
  const R tl = ql[1] * e.t[0] + ql[2] * e.t[1] + ql[3] * e.t[2];
  const R tr = qr[1] * e.t[0] + qr[2] * e.t[1] + qr[3] * e.t[2];
  const R sl = sqrt_(hl), sr = sqrt_(hr);
  const R isl = rcp_(sl), isr = rcp_(sr), iss = rcp_(sl + sr);
  const R u = (nl * isl + nr * isr) * iss;
  const R v = (tl * isl + tr * isr) * iss;
  const R c = sqrt_(grav * R(0.5) * (hl + hr));
  const R i2c = R(0.5) * rcp_(c);
  const R d0 = hr - hl, d1 = nr - nl, d2 = tr - tl;
  const R a1 = ((u + c) * d0 - d1) * i2c;
  const R a2 = d2 - v * d0;
  const R a3 = (d1 - (u - c) * d0) * i2c;
  const R wv[3][3] = {{a1, a1 * (u - c), a1 * v}, {R(0), R(0), a2}, {a3, a3 * (u + c), a3 * v}};
  const R sp[3] = {u - c, u, u + c};
  for (int w = 0; w < 3; ++w) {
    W[w][0] = wv[w][0];
    for (int k = 0; k < 3; ++k) W[w][1 + k] = wv[w][1] * e.n[k] + wv[w][2] * e.t[k];
    s[w] = e.g * sp[w];
  }
  for (int k = 0; k < 4; ++k) {
    R m_ = R(0), p_ = R(0);
    for (int w = 0; w < 3; ++w) {
      m_ += fmin(s[w], R(0)) * W[w][k];
      p_ += fmax(s[w], R(0)) * W[w][k];
    }
    am[k] = m_;
    ap[k] = p_;
  }
  fl = R(0.5) * e.g * (nl + nr) - R(0.5) * (ap[0] - am[0]);
  return true;
}

// Roe averages of an edge's two states (3D velocity and celerity), shared by
// the four transverse splits of that edge; false if a depth is not positive
template <typename R>
struct SRoe {
  R ub[3], c, i2c;
};

template <typename R>
__device__ __forceinline__ bool roe_sphere(R grav, const R* ql, const R* qr, SRoe<R>& rs) {
  const R hl = ql[0], hr = qr[0];
  if (!(hl > R(0) && hr > R(0))) return false;
  const R sl = sqrt_(hl), sr = sqrt_(hr);
  const R isl = rcp_(sl), isr = rcp_(sr), iss = rcp_(sl + sr);
  for (int k = 0; k < 3; ++k) rs.ub[k] = (ql[1 + k] * isl + qr[1 + k] * isr) * iss;
  rs.c = sqrt_(grav * R(0.5) * (hl + hr));
  rs.i2c = R(0.5) * rcp_(rs.c);
  return true;
}

// part of psi crossing the transverse edge te of the receiving cell, down
// (up = false) or up, with the Roe averages rs of the normal edge's states
template <typename R>
__device__ void tsplit_sphere(const SRoe<R>& rs, const SEdge<R>& te, const R* psi, bool up,
                              R* out) {
  const R* ub = rs.ub;
  const R c = rs.c;
  const R un = ub[0] * te.n[0] + ub[1] * te.n[1] + ub[2] * te.n[2];
  const R ut = ub[0] * te.t[0] + ub[1] * te.t[1] + ub[2] * te.t[2];
  const R pn = psi[1] * te.n[0] + psi[2] * te.n[1] + psi[3] * te.n[2];
  const R pt = psi[1] * te.t[0] + psi[2] * te.t[1] + psi[3] * te.t[2];
  const R beta[3] = {((un + c) * psi[0] - pn) * rs.i2c, pt - ut * psi[0],
                     (pn - (un - c) * psi[0]) * rs.i2c};
  const R lam[3] = {te.g * (un - c), te.g * un, te.g * (un + c)};
  R Rv[3][4];
  Rv[0][0] = R(1); Rv[1][0] = R(0); Rv[2][0] = R(1);
  for (int k = 0; k < 3; ++k) {
    Rv[0][1 + k] = (un - c) * te.n[k] + ut * te.t[k];
    Rv[1][1 + k] = te.t[k];
    Rv[2][1 + k] = (un + c) * te.n[k] + ut * te.t[k];
  }
  for (int k = 0; k < 4; ++k) {
    R acc = R(0);
    for (int w = 0; w < 3; ++w) {
      const R l = up ? fmax(lam[w], R(0)) : fmin(lam[w], R(0));
      acc += l * beta[w] * Rv[w][k];
    }
    out[k] = acc;
  }
}

// ---------------------------------------------------------------------------
// the step

template <typename R>
struct SphereArgs {
  const R* q;
  const R* ghost;
  R* qn;
  const double* dt;
  double* numax;
  const PatchRec* __restrict__ rec;
  const int32_t* __restrict__ phislot;
  R* phi;
  int32_t* err;
  const double* __restrict__ geo;
  const float* __restrict__ geo32;   // FP32 state: edges and centres in FP32
  int P, m, lm, limiter, transverse;
  double g;
};

// Edge records of one tile, per direction and edge (e, r) -> e (T+2) + r:
//   W 12 and S 3 (waves and speeds, until every limiter has read them), then
//   in their place T 16 (transverse parts [side][lo/hi][k], already scaled
//   by -dt/(2 kappa dx)); AM 4, AP 4, FL 1, CQ 4 (limited correction; the
//   edge's own correction flux is half of it)
constexpr int kSEw = 0, kSEs = 12, kSEt = 0, kSEam = 16, kSEap = 20, kSEfl = 24,
              kSEcq = 25, kSEn = 29;
// the step works on T x T tiles of a patch, one workgroup each
constexpr int kSphereTile = 8, kSphereThreads = 256;
// LDS of one tile: the state with its 2-cell halo, the capacities, and the
// edge records of both directions
template <typename R>
__host__ __device__ constexpr size_t sphere_lds() {
  return sizeof(R) * 4 * (kSphereTile + 4) * (kSphereTile + 4) +
         sizeof(double) * (kSphereTile + 4) * (kSphereTile + 4) +
         sizeof(R) * 2 * (kSphereTile + 3) * (kSphereTile + 2) * kSEn;
}

// One workgroup per T x T tile of a patch: phase 1 solves the rotated Roe
// problem at every edge of the tile and its halo rows, phase 2 forms the
// limited corrections and then the transverse parts, phase 3 gathers each
// cell's update in a fixed order, projects the momentum and writes the face
// terms.
// Everything between the staged input and the output stays in LDS.
template <typename R>
__global__ void __launch_bounds__(kSphereThreads)
k_sphere_step(SphereArgs<R> A) {
  constexpr int T = kSphereTile, FT = T + 4, FRT = FT * FT, M2 = T + 2,
                NE = (T + 3) * (T + 2);
  extern __shared__ unsigned char smem_raw[];
  R* Qs = reinterpret_cast<R*>(smem_raw);                                  // [4][FRT]
  // dt / (kappa dx) of each frame cell, the only form the step needs kappa in
  double* dtk = reinterpret_cast<double*>(smem_raw + sizeof(R) * 4 * FRT);  // [FRT]
  R* scr = reinterpret_cast<R*>(smem_raw + sizeof(R) * 4 * FRT + sizeof(double) * FRT);
  __shared__ double red[kSphereThreads / 64];
  auto E = [&](int d, int e, int r) { return scr + (size_t(d) * NE + size_t(e) * M2 + r) * kSEn; };
  auto cell_i = [](int d, int n, int r) { return d == 0 ? n : r; };
  auto cell_j = [](int d, int n, int r) { return d == 0 ? r : n; };
  auto lf = [](int i, int j) { return (j + 1) * FT + (i + 1); };   // tile frame
  const int m = A.m, FR = (m + 4) * (m + 4);
  const double dt = *A.dt;
  const R grav = R(A.g);
  const int G = 8 * m + 16;
  const int tps = m / T;
  const int p = blockIdx.x / (tps * tps), tile = blockIdx.x - p * (tps * tps);
  const int i0 = (tile % tps) * T, j0 = (tile / tps) * T;
  auto pf = [&](int i, int j) { return fidx(m, i0 + i, j0 + j); };  // patch frame
  const PatchRec& rp = A.rec[p];
  const double dx = ldexp(1.0, -rp.level) / m;
  const double* geo = A.geo + size_t(p) * kGeoN * FR;
  // edge frames and centres: the FP32 copy for FP32 state
  const float* g32 = sizeof(R) == 4 ? A.geo32 + size_t(p) * kG32N * FR : nullptr;
  auto edge = [&](int d, int f) -> SEdge<R> {
    if constexpr (sizeof(R) == 4) return load_edge<R>(g32 + kG32E * FR + (d * FR + f) * 7);
    else return load_edge<R>(geo + kGeoE * FR + (d * FR + f) * 7);
  };
  for (int f = threadIdx.x; f < FRT; f += blockDim.x) {
    const int i = i0 + f % FT - 1, j = j0 + f / FT - 1;
    const bool outer = (i == -1 || i == m + 2) && (j == -1 || j == m + 2);
    for (int k = 0; k < 4; ++k) {
      R v;
      if (i >= 1 && i <= m && j >= 1 && j <= m)
        v = A.q[(size_t(p * 4 + k) * m + (j - 1)) * m + (i - 1)];
      else
        v = outer ? R(0) : A.ghost[size_t(p * 4 + k) * G + ghost_index(m, i, j)];
      Qs[k * FRT + f] = v;
    }
    dtk[f] = dt / (geo[kGeoK * FR + fidx(m, i, j)] * dx);
  }
  __syncthreads();
  // phase 1: Riemann problems at every edge of rows 0..T+1, both directions
  double nmax = 0.0;
  for (int it = threadIdx.x; it < 2 * NE; it += blockDim.x) {
    const int d = it / NE, er = it % NE, e = er / M2, r = er % M2;
    const int il = cell_i(d, e - 1, r), jl = cell_j(d, e - 1, r);
    const int ir = cell_i(d, e, r), jr = cell_j(d, e, r);
    R ql[4], qr[4];
    for (int k = 0; k < 4; ++k) {
      ql[k] = Qs[k * FRT + lf(il, jl)];
      qr[k] = Qs[k * FRT + lf(ir, jr)];
    }
    const SEdge<R> eg = edge(d, pf(ir, jr));
    R* o = E(d, e, r);
    R W[3][4], s[3], am[4], ap[4], fl;
    if (!rp_sphere<R>(grav, eg, ql, qr, W, s, am, ap, fl)) {
      atomicOr(A.err, kErrNegDepth);
      for (int w = 0; w < 3; ++w) { s[w] = R(0); for (int k = 0; k < 4; ++k) W[w][k] = R(0); }
      for (int k = 0; k < 4; ++k) am[k] = ap[k] = R(0);
      fl = R(0);
    }
    for (int w = 0; w < 3; ++w) {
      for (int k = 0; k < 4; ++k) o[kSEw + 4 * w + k] = W[w][k];
      o[kSEs + w] = s[w];
    }
    for (int k = 0; k < 4; ++k) { o[kSEam + k] = am[k]; o[kSEap + k] = ap[k]; }
    o[kSEfl] = fl;
    // Courant numbers of the edges the patch owns (1..T+1 of the tile; the
    // outer halo edges of a tile on a patch face join two ghost cells)
    if (r >= 1 && r <= T && e >= 1 && e <= T + 1) {
      const double dtdl = dtk[lf(il, jl)], dtdr = dtk[lf(ir, jr)];
      for (int w = 0; w < 3; ++w) {
        nmax = fmax(nmax, dtdr * fmax(double(s[w]), 0.0));
        nmax = fmax(nmax, dtdl * fmax(-double(s[w]), 0.0));
      }
    }
  }
  __syncthreads();
  // phase 2: limited corrections at edges 1..T+1 (reads the waves of the
  // upwind edges) ...
  for (int it = threadIdx.x; it < 2 * NE; it += blockDim.x) {
    const int d = it / NE, er = it % NE, e = er / M2, r = er % M2;
    if (e < 1 || e > T + 1) continue;
    const int il = cell_i(d, e - 1, r), jl = cell_j(d, e - 1, r);
    const int ir = cell_i(d, e, r), jr = cell_j(d, e, r);
    const double dtdl = dtk[lf(il, jl)], dtdr = dtk[lf(ir, jr)];
    const R nu = R(0.5 * (dtdl + dtdr));
    R* o = E(d, e, r);
    R cq[4] = {R(0), R(0), R(0), R(0)};
    for (int w = 0; w < 3; ++w) {
      const R* Wc = o + kSEw + 4 * w;
      const R sw = o[kSEs + w];
      R wn2 = R(0);
      for (int k = 0; k < 4; ++k) wn2 += Wc[k] * Wc[k];
      if (wn2 == R(0)) continue;
      const R* Wu = E(d, sw > R(0) ? e - 1 : e + 1, r) + kSEw + 4 * w;
      R dot = R(0);
      for (int k = 0; k < 4; ++k) dot += Wu[k] * Wc[k];
      const R lim = limiter_phi<R>(A.limiter, dot * rcp_(wn2));
      const R as = fabs(sw);
      for (int k = 0; k < 4; ++k) cq[k] += as * (R(1) - nu * as) * lim * Wc[k];
    }
    for (int k = 0; k < 4; ++k) o[kSEcq + k] = cq[k];
  }
  __syncthreads();
  // ... then the transverse parts, written over the waves
  for (int it = threadIdx.x; it < 2 * NE; it += blockDim.x) {
    const int d = it / NE, er = it % NE, e = er / M2, r = er % M2;
    if (e < 1 || e > T + 1) continue;
    R* o = E(d, e, r);
    if (A.transverse == 0) {
      for (int k = 0; k < 16; ++k) o[kSEt + k] = R(0);
      continue;
    }
    const int il = cell_i(d, e - 1, r), jl = cell_j(d, e - 1, r);
    const int ir = cell_i(d, e, r), jr = cell_j(d, e, r);
    const double dtdl = dtk[lf(il, jl)], dtdr = dtk[lf(ir, jr)];
    R ql[4], qr[4], amt[4], apt[4];
    for (int k = 0; k < 4; ++k) {
      ql[k] = Qs[k * FRT + lf(il, jl)];
      qr[k] = Qs[k * FRT + lf(ir, jr)];
      const R c2 = A.transverse == 2 ? o[kSEcq + k] : R(0);
      amt[k] = o[kSEam + k] + c2;
      apt[k] = o[kSEap + k] - c2;
    }
    SRoe<R> rs;
    const bool ok = roe_sphere<R>(grav, ql, qr, rs);
    if (!ok) atomicOr(A.err, kErrNegDepth);
    for (int side = 0; side < 2; ++side) {
      const int col = side == 0 ? e - 1 : e;
      const R h = R(-0.5 * (side == 0 ? dtdl : dtdr));
      const int ci = cell_i(d, col, r), cj = cell_j(d, col, r);
      const int ui = cell_i(d, col, r + 1), uj = cell_j(d, col, r + 1);
      const SEdge<R> lo = edge(1 - d, pf(ci, cj));
      const SEdge<R> hi = edge(1 - d, pf(ui, uj));
      R bm[4], bp[4];
      const R* psi = side == 0 ? amt : apt;
      if (ok) {
        tsplit_sphere<R>(rs, lo, psi, false, bm);
        tsplit_sphere<R>(rs, hi, psi, true, bp);
      } else {
        for (int k = 0; k < 4; ++k) bm[k] = bp[k] = R(0);
      }
      for (int k = 0; k < 4; ++k) {
        o[kSEt + (side * 2 + 0) * 4 + k] = h * bm[k];
        o[kSEt + (side * 2 + 1) * 4 + k] = h * bp[k];
      }
    }
  }
  __syncthreads();
  // phase 3: update of the tile's cells and face terms
  // total correction flux of edge (e, r) in direction d: own part, then the
  // transverse parts of the other sweep's edges
  auto Ftot = [&](int d, int e, int r, int k) -> R {
    const int o = 1 - d;
    R v = R(0.5) * E(d, e, r)[kSEcq + k];
    v += E(o, r, e - 1)[kSEt + (1 * 2 + 1) * 4 + k];
    v += E(o, r + 1, e - 1)[kSEt + (0 * 2 + 1) * 4 + k];
    v += E(o, r, e)[kSEt + (1 * 2 + 0) * 4 + k];
    v += E(o, r + 1, e)[kSEt + (0 * 2 + 0) * 4 + k];
    return v;
  };
  for (int c = threadIdx.x; c < T * T; c += blockDim.x) {
    const int i = c % T + 1, j = c / T + 1;
    const int f = lf(i, j);
    const R dtd = R(dtk[f]);
    R out[4];
    for (int k = 0; k < 4; ++k) {
      R fx, gy;
      if (k == 0) {
        fx = E(0, i + 1, j)[kSEfl] - E(0, i, j)[kSEfl];
        gy = E(1, j + 1, i)[kSEfl] - E(1, j, i)[kSEfl];
      } else {
        fx = E(0, i, j)[kSEap + k] + E(0, i + 1, j)[kSEam + k];
        gy = E(1, j, i)[kSEap + k] + E(1, j + 1, i)[kSEam + k];
      }
      fx = fx + (Ftot(0, i + 1, j, k) - Ftot(0, i, j, k));
      gy = gy + (Ftot(1, j + 1, i, k) - Ftot(1, j, i, k));
      out[k] = Qs[k * FRT + f] - dtd * fx - dtd * gy;
    }
    // momentum onto the tangent plane at the cell centre
    R rc[3];
    for (int k = 0; k < 3; ++k)
      rc[k] = sizeof(R) == 4 ? R(g32[kG32C * FR + 3 * pf(i, j) + k])
                             : R(geo[kGeoC * FR + 3 * pf(i, j) + k]);
    const R mr = out[1] * rc[0] + out[2] * rc[1] + out[3] * rc[2];
    for (int k = 0; k < 3; ++k) out[1 + k] -= mr * rc[k];
    for (int k = 0; k < 4; ++k)
      A.qn[(size_t(p * 4 + k) * m + (j0 + j - 1)) * m + (i0 + i - 1)] = out[k];
  }
  const int slot = A.phislot[p];
  if (slot >= 0) {
    // face terms of the patch faces this tile lies on
    R* ph = A.phi + size_t(slot) * 4 * m * 4;
    for (int it = threadIdx.x; it < 4 * T * 4; it += blockDim.x) {
      const int k = it % 4, t = (it / 4) % T + 1, fc = it / (4 * T);
      const bool on = fc == 0 ? i0 == 0 : fc == 1 ? i0 + T == m : fc == 2 ? j0 == 0 : j0 + T == m;
      if (!on) continue;
      const int d = fc / 2, e = (fc & 1) ? T + 1 : 1;
      const R* o = E(d, e, t);
      R fluct;
      if (k == 0) fluct = (fc & 1) ? o[kSEfl] : -o[kSEfl];
      else fluct = (fc & 1) ? o[kSEam + k] : o[kSEap + k];
      const R corr = Ftot(d, e, t, k);
      const int tp = (d == 0 ? j0 : i0) + t;
      ph[(fc * m + (tp - 1)) * 4 + k] = R(dx) * ((fc & 1) ? fluct + corr : fluct - corr);
    }
  }
  for (int off = 32; off > 0; off >>= 1) nmax = fmax(nmax, __shfl_xor(nmax, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = red[0];
    for (int w = 1; w < int(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
    atomic_max_pos(A.numax, v);
  }
}

// Coarse-fine correction and cube-edge mass sync (one thread per item and
// coarse cell); momentum corrections are projected like the step's output.
template <typename R>
__global__ void __launch_bounds__(256)
k_sphere_reflux(const R* q, R* qn, const RefluxItem* __restrict__ items, int32_t nitems,
                const PatchRec* __restrict__ rec, const int32_t* __restrict__ phislot,
                const R* phi, const double* __restrict__ geo, const double* dt, double g,
                int m, int32_t* err) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nitems) * 32) return;
  const int ii = int(t >> 5), tc = int(t & 31) + 1;
  if (tc > m) return;
  const int FR = (m + 4) * (m + 4);
  const RefluxItem it = items[ii];
  const int fc = it.face, d = fc >> 1, hi = fc & 1, C = it.coarse;
  const int ic = d == 0 ? (hi ? m : 1) : tc, jc = d == 0 ? tc : (hi ? m : 1);
  const double dxc = ldexp(1.0, -rec[C].level) / m;
  const double kc = geo[size_t(C) * kGeoN * FR + kGeoK * FR + fidx(m, ic, jc)];
  const R* pc = phi + size_t(phislot[C]) * 4 * m * 4 + (fc * m + (tc - 1)) * 4;
  const double fac = *dt / (kc * dxc * dxc);
  if (it.fine[1] == kSyncItem) {
    const int L = it.fine[0], ff = it.fine_face[0];
    const int pos = it.fine_rev[0] ? m + 1 - tc : tc;
    const R* pn = phi + size_t(phislot[L]) * 4 * m * 4 + (ff * m + (pos - 1)) * 4;
    qn[(size_t(C * 4) * m + (jc - 1)) * m + (ic - 1)] -= R(fac) * (-pn[0] - pc[0]);
    return;
  }
  const int k2 = (tc - 1) / (m / 2);
  const int fp = it.fine[k2], ff = it.fine_face[k2];
  R qc[4], corr[4] = {R(0), R(0), R(0), R(0)};
  for (int k = 0; k < 4; ++k) qc[k] = q[(size_t(C * 4 + k) * m + (jc - 1)) * m + (ic - 1)];
  const R* pf = phi + size_t(phislot[fp]) * 4 * m * 4;
  for (int s = 0; s < 2; ++s) {
    int pos = 2 * (tc - 1 - k2 * (m / 2)) + 1 + s;
    if (it.fine_rev[k2]) pos = m + 1 - pos;
    const int fi = ff < 2 ? (ff == 0 ? 1 : m) : pos;
    const int fj = ff < 2 ? pos : (ff == 2 ? 1 : m);
    R qv[4];
    for (int k = 0; k < 4; ++k) qv[k] = q[(size_t(fp * 4 + k) * m + (fj - 1)) * m + (fi - 1)];
    // the fine edge as the fine leaf sees it, normal turned from the left
    // state to the right one
    const int ei = ff == 1 ? fi + 1 : fi, ej = ff == 3 ? fj + 1 : fj;
    SEdge<R> eg = load_edge<R>(geo + size_t(fp) * kGeoN * FR + kGeoE * FR +
                               ((ff / 2) * FR + fidx(m, ei, ej)) * 7);
    if (((ff & 1) == 1) != (hi == 0))
      for (int c = 0; c < 3; ++c) { eg.n[c] = -eg.n[c]; eg.t[c] = -eg.t[c]; }
    R W[3][4], sp[3], am[4], ap[4], fl;
    const bool ok = hi ? rp_sphere<R>(R(g), eg, qc, qv, W, sp, am, ap, fl)
                       : rp_sphere<R>(R(g), eg, qv, qc, W, sp, am, ap, fl);
    if (!ok) {
      atomicOr(err, kErrNegDepth);
      for (int k = 0; k < 4; ++k) am[k] = ap[k] = R(0);
    }
    for (int k = 0; k < 4; ++k)
      corr[k] += (k == 0 ? R(0) : R(0.5 * dxc) * (am[k] + ap[k])) - pf[(ff * m + (pos - 1)) * 4 + k];
  }
  R dq[4];
  for (int k = 0; k < 4; ++k) dq[k] = -R(fac) * (corr[k] - pc[k]);
  const double* rc = geo + size_t(C) * kGeoN * FR + kGeoC * FR + 3 * fidx(m, ic, jc);
  const R mr = dq[1] * R(rc[0]) + dq[2] * R(rc[1]) + dq[3] * R(rc[2]);
  for (int k = 0; k < 3; ++k) dq[1 + k] -= mr * R(rc[k]);
  for (int k = 0; k < 4; ++k) qn[(size_t(C * 4 + k) * m + (jc - 1)) * m + (ic - 1)] += dq[k];
}

// Per-patch FP64 partial sums of kappa q dxi^2.
template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_sphere_sums_patch(const R* __restrict__ q, const PatchRec* __restrict__ rec,
                    const double* __restrict__ geo, int m, double* __restrict__ partial) {
  __shared__ double red[4][MEQN];
  const int p = blockIdx.x, tid = threadIdx.x, FR = (m + 4) * (m + 4);
  const double dx = ldexp(1.0, -rec[p].level) / m;
  const double* kap = geo + size_t(p) * kGeoN * FR + kGeoK * FR;
  double acc[MEQN] = {};
  for (int c = tid; c < m * m; c += 256) {
    const double kk = kap[fidx(m, c % m + 1, c / m + 1)];
    for (int k = 0; k < MEQN; ++k) acc[k] += kk * double(q[size_t(p * MEQN + k) * m * m + c]);
  }
  for (int k = 0; k < MEQN; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid < MEQN)
    partial[size_t(p) * MEQN + tid] =
        ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) * dx * dx;
}

// ---------------------------------------------------------------------------
// the colour equation carried by a rigid rotation (FCX_ROTATION)

struct RotationArgs {
  const void* q;
  const void* ghost;
  void* qn;
  const double* dt;
  double* numax;
  const PatchRec* __restrict__ rec;
  const double* __restrict__ geo;
  const double* __restrict__ flux;   // k_rotation_fluxes' table
  int m, limiter, transverse;
};

// The flux of every edge of a patch's frame over the computational cell
// size, signed towards higher index: per patch two frames of (m+4)^2, the
// low-side xi-edge then the low-side eta-edge of each frame cell.  The flux
// of an edge is Omega w.(b - a) (+ for xi-edges, - for eta-edges, a, b its
// corners in index order) over dx; the chord b - a is 2 sin(theta / 2)
// times the edge's tangent t (+t for xi-edges, -t for eta-edges), with
// theta = gamma dx the arc's angle, so the flux is (2 / dx) sin(theta / 2)
// (Omega w).t for either direction.  Formed in FP64 from the FP64 geometry
// once per forest (the flow is steady).
__global__ void __launch_bounds__(256)
k_rotation_fluxes(const double* __restrict__ geo, double* __restrict__ flux,
                  const PatchRec* __restrict__ rec, int64_t P, int m, double3 w) {
  const int FR = (m + 4) * (m + 4);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= P * 2 * FR) return;
  const int64_t p = t / (2 * FR);
  const int df = int(t - p * 2 * FR), d = df / FR, f = df - d * FR;
  const double dx = ldexp(1.0, -rec[p].level) / m;
  const double* g = geo + size_t(p) * kGeoN * FR + kGeoE * FR + (size_t(d) * FR + f) * 7;
  const double wt = w.x * g[4] + w.y * g[5] + w.z * g[6];
  flux[t] = (2.0 / dx) * sin(0.5 * g[0] * dx) * wt;
}

// One workgroup per T x T tile of a patch, all in LDS:
//   phase 0: the tile's state with its 2-cell halo, dt / (kappa dx) of every
//     frame cell, and the flux of every edge of both directions (edges
//     e = 0 .. T+2 between cells e-1 and e, rows r = 0 .. T+1);
//   phase 1: at edges 1 .. T+1, the waves (jumps of the staged state), the
//     Courant numbers, limited corrections and the transverse parts, which
//     leave the receiving cell through its own transverse edges at their
//     fluxes;
//   phase 2: each cell's update, q - dt / (kappa dx) (fluctuations +
//     differences of the correction fluxes) per direction.
// The edge fluxes come from k_rotation_fluxes' table, rounded to R.
template <typename R, int T, int NT>
__global__ void __launch_bounds__(NT)
k_rotation_step(RotationArgs A) {
  constexpr int FT = T + 4, FRT = FT * FT, M2 = T + 2, NE = (T + 3) * (T + 2);
  __shared__ R Qs[FRT];
  __shared__ double dtk[FRT];
  __shared__ R S[2][NE], CQ[2][NE], TR[2][NE][4];
  __shared__ double red[NT / 64];
  const R* q = static_cast<const R*>(A.q);
  const R* ghost = static_cast<const R*>(A.ghost);
  const int m = A.m, FR = (m + 4) * (m + 4), G = 8 * m + 16, tps = m / T;
  const int p = blockIdx.x / (tps * tps), tile = blockIdx.x - p * (tps * tps);
  const int i0 = (tile % tps) * T, j0 = (tile / tps) * T;
  const double dt = *A.dt;
  const double dx = ldexp(1.0, -A.rec[p].level) / m;
  const double* geo = A.geo + size_t(p) * kGeoN * FR;
  auto lf = [](int i, int j) { return (j + 1) * FT + (i + 1); };   // tile frame
  auto ei = [](int e, int r) { return e * M2 + r; };
  // phase 0
  for (int f = threadIdx.x; f < FRT; f += blockDim.x) {
    const int i = i0 + f % FT - 1, j = j0 + f / FT - 1;
    const bool outer = (i == -1 || i == m + 2) && (j == -1 || j == m + 2);
    R v;
    if (i >= 1 && i <= m && j >= 1 && j <= m)
      v = q[(size_t(p) * m + (j - 1)) * m + (i - 1)];
    else
      v = outer ? R(0) : ghost[size_t(p) * G + ghost_index(m, i, j)];
    Qs[f] = v;
    dtk[f] = dt / (geo[kGeoK * FR + fidx(m, i, j)] * dx);
  }
  const double* fl0 = A.flux + size_t(p) * 2 * FR;
  for (int it = threadIdx.x; it < 2 * NE; it += blockDim.x) {
    const int d = it / NE, er = it % NE, e = er / M2, r = er % M2;
    // the low-side d-edge of the cell on the edge's high side
    const int ir = d == 0 ? e : r, jr = d == 0 ? r : e;
    S[d][er] = R(fl0[d * FR + fidx(m, i0 + ir, j0 + jr)]);
  }
  __syncthreads();
  // phase 1: at edges 1..T+1 of both directions, the wave (the jump, read
  // from the staged state), the Courant numbers, the limited correction and
  // the transverse parts
  double nmax = 0.0;
  auto wave = [&](int d, int e, int r) -> R {
    return d == 0 ? Qs[lf(e, r)] - Qs[lf(e - 1, r)] : Qs[lf(r, e)] - Qs[lf(r, e - 1)];
  };
  constexpr int NI = (T + 1) * M2;
  for (int it = threadIdx.x; it < 2 * NI; it += blockDim.x) {
    const int d = it / NI, ir_ = it % NI, e = 1 + ir_ / M2, r = ir_ % M2;
    const int er = ei(e, r);
    const int il = d == 0 ? e - 1 : r, jl = d == 0 ? r : e - 1;
    const int ir = d == 0 ? e : r, jr = d == 0 ? r : e;
    const double dtdl = dtk[lf(il, jl)], dtdr = dtk[lf(ir, jr)];
    const R sw = S[d][er], wc = Qs[lf(ir, jr)] - Qs[lf(il, jl)];
    if (r >= 1 && r <= T) {
      nmax = fmax(nmax, dtdr * fmax(double(sw), 0.0));
      nmax = fmax(nmax, dtdl * fmax(-double(sw), 0.0));
    }
    R cq = R(0);
    if (wc != R(0)) {
      const R wu = wave(d, sw > R(0) ? e - 1 : e + 1, r);
      const R lim = limiter_phi<R>(A.limiter, (wu * wc) * rcp_(wc * wc));
      const R as = fabs(sw);
      cq = as * (R(1) - R(0.5 * (dtdl + dtdr)) * as) * lim * wc;
    }
    CQ[d][er] = cq;
    const int o = 1 - d;
    if (A.transverse == 0) {
      for (int k = 0; k < 4; ++k) TR[d][er][k] = R(0);
      continue;
    }
    const R c2 = A.transverse == 2 ? cq : R(0);
    const R amt = fmin(sw, R(0)) * wc + c2, apt = fmax(sw, R(0)) * wc - c2;
    for (int side = 0; side < 2; ++side) {
      const int col = side == 0 ? e - 1 : e;
      const R h = R(-0.5 * (side == 0 ? dtdl : dtdr));
      const R ps = side == 0 ? amt : apt;
      // the receiving cell's lower and upper o-edges
      const R slo = S[o][ei(r, col)], shi = S[o][ei(r + 1, col)];
      TR[d][er][side * 2 + 0] = h * (fmin(slo, R(0)) * ps);
      TR[d][er][side * 2 + 1] = h * (fmax(shi, R(0)) * ps);
    }
  }
  __syncthreads();
  // phase 2: total correction flux of edge (e, r) in direction d: its own
  // half correction, then the transverse parts of the other direction's
  // edges whose receiving cells it bounds
  auto Ftot = [&](int d, int e, int r) -> R {
    const int o = 1 - d;
    R v = R(0.5) * CQ[d][ei(e, r)];
    v += TR[o][ei(r, e - 1)][3];
    v += TR[o][ei(r + 1, e - 1)][1];
    v += TR[o][ei(r, e)][2];
    v += TR[o][ei(r + 1, e)][0];
    return v;
  };
  auto fl = [&](int d, int e, int r, bool ap) -> R {
    const R sw = S[d][ei(e, r)], wv = wave(d, e, r);
    return ap ? fmax(sw, R(0)) * wv : fmin(sw, R(0)) * wv;
  };
  R* qn = static_cast<R*>(A.qn);
  for (int c = threadIdx.x; c < T * T; c += blockDim.x) {
    const int i = c % T + 1, j = c / T + 1;
    const int f = lf(i, j);
    const R dtd = R(dtk[f]);
    R fx = fl(0, i, j, true) + fl(0, i + 1, j, false);
    R gy = fl(1, j, i, true) + fl(1, j + 1, i, false);
    fx = fx + (Ftot(0, i + 1, j) - Ftot(0, i, j));
    gy = gy + (Ftot(1, j + 1, i) - Ftot(1, j, i));
    qn[(size_t(p) * m + (j0 + j - 1)) * m + (i0 + i - 1)] = Qs[f] - dtd * fx - dtd * gy;
  }
  for (int off = 32; off > 0; off >>= 1) nmax = fmax(nmax, __shfl_xor(nmax, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = red[0];
    for (int w = 1; w < int(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
    atomic_max_pos(A.numax, v);
  }
}

}  // namespace fcx
