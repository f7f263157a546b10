// device.hpp -- device-side helpers shared by the fcx kernels: patch
// records, coordinate transforms, and the ghost-cell value of a patch frame
// cell (arXiv 1308.1472, Sec. 3: copy from a same-level neighbour, average
// from finer neighbours, limited conservative interpolation from a coarser
// one).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "forest.hpp"

namespace fcx {

// Fast reciprocal / root: the hardware instructions in FP32 (about 1 ulp;
// the FP32 path is held to 1e-5, and a correctly rounded square root costs
// some fifteen instructions more), correctly rounded operations in FP64.
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }

// LDS written by some lanes of a wavefront and read by others (a
// wavefront's LDS accesses are performed in program order; the fences keep
// the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// error bits raised by kernels
constexpr int32_t kErrNegDepth = 2;
constexpr int32_t kErrNested = 4;

struct KPhys {
  double g, ax, ay;
  int32_t limiter, transverse;
  double period;                           // FCX_SWIRL: period of the flow
};

template <int PHYS> struct PhysTraits;
template <> struct PhysTraits<FCX_ADVECTION> { static constexpr int MEQN = 1; };
template <> struct PhysTraits<FCX_SHALLOW> { static constexpr int MEQN = 3; };
template <> struct PhysTraits<FCX_SPHERE> { static constexpr int MEQN = 4; };
template <> struct PhysTraits<FCX_SWIRL> { static constexpr int MEQN = 1; };
template <> struct PhysTraits<FCX_ROTATION> { static constexpr int MEQN = 1; };
// physics on the cubed sphere (capacity-weighted means across levels)
__host__ __device__ constexpr bool sphere_phys(int p) {
  return p == FCX_SPHERE || p == FCX_ROTATION;
}

__device__ __forceinline__ void xf_apply(int32_t code, int32_t x, int32_t y,
                                         int32_t& xo, int32_t& yo) {
  int32_t u = (code & 1) ? y : x;
  int32_t v = (code & 1) ? x : y;
  if (code & 2) u = -u;
  if (code & 4) v = -v;
  xo = u + (((code >> 3) & 7) - 4) * int32_t(kSide);
  yo = v + (((code >> 6) & 7) - 4) * int32_t(kSide);
}

template <typename R>
__device__ __forceinline__ R minmod(R a, R b) {
  if (a * b <= R(0)) return R(0);
  return fabs(a) <= fabs(b) ? a : b;
}

// Compact state: q[((p*MEQN + k)*m + (j-1))*m + (i-1)]
template <typename R, int MEQN>
__device__ __forceinline__ void read_interior(const R* __restrict__ q, int m,
                                              int p, int i, int j,
                                              R (&out)[MEQN]) {
#pragma unroll
  for (int k = 0; k < MEQN; ++k)
    out[k] = q[(size_t(p * MEQN + k) * m + (j - 1)) * m + (i - 1)];
}

// Mirror (i, j) across the physical walls of a patch: xi walls first, then
// eta walls; a reflecting wall flips the normal momentum, an extrapolation
// wall repeats the first interior cell.
__host__ __device__ __forceinline__ void resolve_walls(int32_t flags, int m, int& i,
                                              int& j, bool& negx, bool& negy) {
  if (i < 1 && (flags & 1)) {
    if (flags & 16) i = 1; else { i = 1 - i; negx = !negx; }
  } else if (i > m && (flags & 2)) {
    if (flags & 32) i = m; else { i = 2 * m + 1 - i; negx = !negx; }
  }
  if (j < 1 && (flags & 4)) {
    if (flags & 64) j = 1; else { j = 1 - j; negy = !negy; }
  } else if (j > m && (flags & 8)) {
    if (flags & 128) j = m; else { j = 2 * m + 1 - j; negy = !negy; }
  }
}

// Sub-cycling: where the state of each level is read at the time of one
// level's substep.  By level: the buffer (index into bufs) holding the state
// at the substep's time, or, for a coarser level in the middle of its own
// step (alpha > 0), the buffers of the start (old) and end (cur) of that
// step, mixed (1 - alpha) old + alpha cur.
struct LevelSrc {
  int32_t cur, old;
  double alpha;
};
constexpr int kLevels = 32;

template <typename R>
struct TimeView {
  const R* bufs[3];
  const LevelSrc* src;            // [kLevels], in device memory
};

template <typename R, int MEQN>
struct GhostView {
  const R* __restrict__ q;
  const PatchRec* __restrict__ rec;
  int m, lm;                      // m = 2^lm
  int32_t* err;
  const double* geo = nullptr;    // sphere: per-patch geometry tables
  TimeView<R> tv{};               // sub-cycling (frame_value with TIMED)
};

// Interior cell (i, j) of leaf p: from q, or (TIMED) from the buffer(s) of
// p's level at the time of the current substep.
template <typename R, int MEQN, bool TIMED>
__device__ __forceinline__ void leaf_cell(const GhostView<R, MEQN>& g, int p, int i, int j,
                                          R (&out)[MEQN]) {
  if constexpr (!TIMED) {
    read_interior<R, MEQN>(g.q, g.m, p, i, j, out);
  } else {
    // (1 - alpha) old + alpha cur; alpha = 0 is the step's start (old),
    // and levels read at their own time have old = cur
    const LevelSrc s = g.tv.src[g.rec[p].level];
    read_interior<R, MEQN>(g.tv.bufs[s.old], g.m, p, i, j, out);
    if (s.alpha != 0.0) {
      R c[MEQN];
      read_interior<R, MEQN>(g.tv.bufs[s.cur], g.m, p, i, j, c);
      const R a = R(s.alpha), b = R(1.0 - s.alpha);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) out[k] = b * out[k] + a * c[k];
    }
  }
}

// capacity of interior cell (i, j) of patch p from a sphere geometry table
// (kappa is the first frame of (m+4)^2 values, then 17 more frames)
__device__ __forceinline__ double geo_kappa(const double* geo, int m, int p, int i, int j) {
  const int FR = (m + 4) * (m + 4);
  return geo[size_t(p) * 18 * FR + (j + 1) * (m + 4) + (i + 1)];
}

// centre (unit vector) of frame cell (i, j) of patch p from a sphere
// geometry table (frames 1-3 hold the three coordinates of each cell in turn)
__device__ __forceinline__ void geo_centre(const double* geo, int m, int p, int i, int j,
                                           double r[3]) {
  const int FR = (m + 4) * (m + 4);
  const double* c = geo + size_t(p) * 18 * FR + FR + 3 * ((j + 1) * (m + 4) + (i + 1));
  r[0] = c[0];
  r[1] = c[1];
  r[2] = c[2];
}

// great-circle angle between unit vectors a and b, as atan2(|a x b|, a . b)
__device__ __forceinline__ double arc_between(const double a[3], const double b[3]) {
#pragma clang fp contract(off)
  const double c0 = a[1] * b[2] - a[2] * b[1];
  const double c1 = a[2] * b[0] - a[0] * b[2];
  const double c2 = a[0] * b[1] - a[1] * b[0];
  const double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
  return atan2(sqrt(c0 * c0 + c1 * c1 + c2 * c2), dot);
}

// The leaf that holds the centre of non-interior, non-wall frame cell (i, j)
// of patch p, and that centre in the leaf's tree coordinates.  Returns the
// leaf id, or kNbrValence3.
template <typename R, int MEQN>
__device__ __forceinline__ int32_t holder(const GhostView<R, MEQN>& g,
                                          const PatchRec& r, int i, int j,
                                          int32_t& X, int32_t& Y) {
  const int m = g.m;
  int32_t nb, code;
  if (i >= 1 && i <= m) {
    const int f = j < 1 ? 2 : 3;
    nb = r.nbr[2 * f + (i > (m >> 1))];
    code = r.xf[f];
  } else if (j >= 1 && j <= m) {
    const int f = i < 1 ? 0 : 1;
    nb = r.nbr[2 * f + (j > (m >> 1))];
    code = r.xf[f];
  } else {
    const int c = (i > m) + 2 * (j > m);
    nb = r.nbr[8 + c];
    code = r.xf[4 + c];
  }
  const int sh = kS - r.level;                  // log2 of leaf size
  const int32_t half = int32_t(1) << (sh - g.lm - 1);
  const int32_t x = (r.ix << sh) + (2 * i - 1) * half;
  const int32_t y = (r.iy << sh) + (2 * j - 1) * half;
  xf_apply(code, x, y, X, Y);
  return nb;
}

// Copy or 2x2 average from leaf nb at the point (X, Y); interpolation from a
// coarser leaf if ALLOW_INTERP (its slope stencil uses frame values of the
// coarse leaf, which never need interpolation themselves under full 2:1
// balance with m >= 4).
template <typename R, int MEQN, int PHYS, bool ALLOW_INTERP, bool TIMED = false>
__device__ void from_leaf(const GhostView<R, MEQN>& g, int lev, int32_t nb,
                          int32_t X, int32_t Y, R (&out)[MEQN]);

template <typename R, int MEQN, int PHYS, bool ALLOW_INTERP, bool TIMED = false>
__device__ void frame_value(const GhostView<R, MEQN>& g, int p, int i, int j,
                            R (&out)[MEQN]) {
  const PatchRec& r = g.rec[p];
  bool nx = false, ny = false;
  resolve_walls(r.flags, g.m, i, j, nx, ny);
  if (i >= 1 && i <= g.m && j >= 1 && j <= g.m) {
    leaf_cell<R, MEQN, TIMED>(g, p, i, j, out);
  } else {
    int32_t X, Y;
    const int32_t nb = holder(g, r, i, j, X, Y);
    if (nb == kNbrValence3) {
      // three trees meet: mean of the two mirrored face ghosts
      const int mi = i < 1 ? 1 - i : 2 * g.m + 1 - i;
      const int mj = j < 1 ? 1 - j : 2 * g.m + 1 - j;
      R a[MEQN], b[MEQN];
      int32_t Xa, Ya, Xb, Yb;
      const int32_t na = holder(g, r, i, mj, Xa, Ya);
      const int32_t nb2 = holder(g, r, mi, j, Xb, Yb);
      from_leaf<R, MEQN, PHYS, ALLOW_INTERP, TIMED>(g, r.level, na, Xa, Ya, a);
      from_leaf<R, MEQN, PHYS, ALLOW_INTERP, TIMED>(g, r.level, nb2, Xb, Yb, b);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) out[k] = R(0.5) * (a[k] + b[k]);
    } else {
      from_leaf<R, MEQN, PHYS, ALLOW_INTERP, TIMED>(g, r.level, nb, X, Y, out);
    }
  }
  if (PHYS == FCX_SHALLOW) {
    if (nx) out[1] = -out[1];
    if (ny) out[2 % MEQN] = -out[2 % MEQN];
  }
}

template <typename R, int MEQN, int PHYS, bool ALLOW_INTERP, bool TIMED>
__device__ void from_leaf(const GhostView<R, MEQN>& g, int lev, int32_t nb,
                          int32_t X, int32_t Y, R (&out)[MEQN]) {
  const PatchRec& n = g.rec[nb];
  const int shn = kS - n.level;
  const int csh = shn - g.lm;                    // log2 of n's cell size
  const int32_t u = X - (n.ix << shn), v = Y - (n.iy << shn);
  if (n.level == lev) {
    leaf_cell<R, MEQN, TIMED>(g, nb, (u >> csh) + 1, (v >> csh) + 1, out);
  } else if (n.level == lev + 1) {
    // the centre is the common corner of four cells of the finer leaf
    const int i0 = u >> csh, j0 = v >> csh;
    R a[MEQN], b[MEQN], c[MEQN], d[MEQN];
    leaf_cell<R, MEQN, TIMED>(g, nb, i0, j0, a);
    leaf_cell<R, MEQN, TIMED>(g, nb, i0 + 1, j0, b);
    leaf_cell<R, MEQN, TIMED>(g, nb, i0, j0 + 1, c);
    leaf_cell<R, MEQN, TIMED>(g, nb, i0 + 1, j0 + 1, d);
    if (sphere_phys(PHYS)) {
      // capacity-weighted mean
      const R ka = R(geo_kappa(g.geo, g.m, nb, i0, j0));
      const R kb = R(geo_kappa(g.geo, g.m, nb, i0 + 1, j0));
      const R kc = R(geo_kappa(g.geo, g.m, nb, i0, j0 + 1));
      const R kd = R(geo_kappa(g.geo, g.m, nb, i0 + 1, j0 + 1));
      const R w = ((ka + kb) + kc) + kd;
#pragma unroll
      for (int k = 0; k < MEQN; ++k)
        out[k] = (((ka * a[k] + kb * b[k]) + kc * c[k]) + kd * d[k]) / w;
    } else {
#pragma unroll
      for (int k = 0; k < MEQN; ++k) out[k] = (((a[k] + b[k]) + c[k]) + d[k]) / R(4);
    }
  } else if (ALLOW_INTERP) {
    // coarser leaf: minmod-limited linear interpolation at offset +-1/4
    const int ic = (u >> csh) + 1, jc = (v >> csh) + 1;
    const int32_t cs = int32_t(1) << csh;
    const R dx = (2 * u > (2 * ic - 1) * cs) ? R(0.25) : R(-0.25);
    const R dy = (2 * v > (2 * jc - 1) * cs) ? R(0.25) : R(-0.25);
    R qc[MEQN], qe[MEQN], qw[MEQN], qn[MEQN], qs[MEQN];
    leaf_cell<R, MEQN, TIMED>(g, nb, ic, jc, qc);
    frame_value<R, MEQN, PHYS, false, TIMED>(g, nb, ic + 1, jc, qe);
    frame_value<R, MEQN, PHYS, false, TIMED>(g, nb, ic - 1, jc, qw);
    frame_value<R, MEQN, PHYS, false, TIMED>(g, nb, ic, jc + 1, qn);
    frame_value<R, MEQN, PHYS, false, TIMED>(g, nb, ic, jc - 1, qs);
#pragma unroll
    for (int k = 0; k < MEQN; ++k) {
      const R sx = minmod(qe[k] - qc[k], qc[k] - qw[k]);
      const R sy = minmod(qn[k] - qc[k], qc[k] - qs[k]);
      out[k] = qc[k] + dx * sx + dy * sy;
    }
  } else {
    // a slope stencil reached a coarser leaf: cannot happen on a 2:1
    // balanced forest; flag it and use the coarse cell value
    atomicOr(g.err, kErrNested);
    leaf_cell<R, MEQN, TIMED>(g, nb, (u >> csh) + 1, (v >> csh) + 1, out);
  }
}

// Ghost-buffer index of frame cell (i, j) of an m x m patch.
__device__ __forceinline__ int ghost_index(int m, int i, int j) {
  if (j <= 0) return (j + 1) * (m + 4) + (i + 1);
  if (j > m) return 2 * (m + 4) + (j - m - 1) * (m + 4) + (i + 1);
  const int s = i == -1 ? 0 : i == 0 ? 1 : i == m + 1 ? 2 : 3;
  return 4 * (m + 4) + 4 * (j - 1) + s;
}

__device__ __forceinline__ void ghost_cell(int m, int g, int& i, int& j) {
  const int w = m + 4;
  if (g < 2 * w) { j = g / w - 1; i = g % w - 1; return; }
  if (g < 4 * w) { g -= 2 * w; j = m + 1 + g / w; i = g % w - 1; return; }
  g -= 4 * w;
  j = g / 4 + 1;
  const int s = g % 4;
  i = s == 0 ? -1 : s == 1 ? 0 : s == 2 ? m + 1 : m + 2;
}

__device__ __forceinline__ void atomic_max_pos(double* addr, double v) {
  // Many workgroups update one word: read it first and skip the atomic when
  // it already holds at least v (a stale read is never larger than the
  // true value, so no update is lost).  Non-negative doubles order like
  // their bit patterns.
  unsigned long long* w = reinterpret_cast<unsigned long long*>(addr);
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  if (b <= __atomic_load_n(w, __ATOMIC_RELAXED)) return;
  atomicMax(w, b);
}

}  // namespace fcx
