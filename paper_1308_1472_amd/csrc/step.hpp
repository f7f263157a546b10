// step.hpp -- the wave-propagation patch update on gfx950 (arXiv 1308.1472,
// Sec. 3: Clawpack's wave-propagation algorithm on every leaf patch; LeVeque,
// JCP 1997, for the unsplit method with transverse propagation; Roe's
// approximate solver for shallow water).
//
// One workgroup advances one T x T tile of one patch.  The tile and its
// two-cell halo are staged in LDS -- from the compact state plus the ghost
// buffer (plain path) or straight from neighbouring patches' interiors
// (fused path).  Per-cell primitive quantities (sqrt h, u, v) are formed
// once per staged cell.  Each sweep direction then runs three phases
// separated by barriers:
//   A  one Riemann solve per edge of the (T+2) x (T+3) edge set; compact
//      wave data (strengths and Roe averages) go to LDS;
//   B  per edge: wave limiter from the neighbour edges' waves, second-order
//      correction, transverse splitting of the corrected fluctuations.  The
//      edge's contributions go to per-cell LDS accumulators in two race-free
//      sub-passes: the cell on its left first, then (after a barrier) the
//      cell on its right -- every cell gets exactly one of each;
//   C  per interior cell: the normal flux difference and the difference of
//      the transverse fluxes at its two transverse edges go into a register
//      accumulator.
// After both sweeps q_new = q + dq is written with coalesced stores.
#pragma once

#include "device.hpp"

namespace fcx {

template <typename R>
struct StepArgs {
  const R* __restrict__ q;
  const R* __restrict__ ghost;
  R* __restrict__ qn;
  const double* dt;
  double* numax;
  const PatchRec* __restrict__ rec;
  const int32_t* __restrict__ phislot;
  R* __restrict__ phi;
  int32_t* err;
  int32_t P;
  int32_t m, lm;          // patch size and its log2
  int32_t ntiles;         // total tiles = P * (m / T)^2
  // with one tile per patch, optionally the patch of each launch slot (the
  // dispatch order; null: slot order)
  const int32_t* order = nullptr;
  KPhys ph;
  const double* tsim = nullptr;   // FCX_SWIRL: time of the state q
};

template <int T> struct TileThreads { static constexpr int value = T * T >= 256 ? 256 : T * T; };


// min / max of two finite values: one v_med3 in FP32 (a median with an
// infinity), without the NaN-quieting fmin / fmax need
__device__ __forceinline__ float min_(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, -__builtin_inff());
}
__device__ __forceinline__ float max_(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, __builtin_inff());
}
__device__ __forceinline__ double min_(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double max_(double a, double b) { return fmax(a, b); }

template <typename R>
__device__ __forceinline__ R limiter_phi(int lim, R th) {
  switch (lim) {
    case 0: return R(1);
    case 1: return max_(R(0), min_(R(1), th));
    case 2: return max_(R(0), max_(min_(R(1), R(2) * th), min_(R(2), th)));
    case 3: return (th + fabs(th)) * rcp_(R(1) + fabs(th));
    default: return max_(R(0), min_(min_(R(0.5) * (R(1) + th), R(2)), R(2) * th));
  }
}

// Map a linear block index so that the blocks one XCD receives (the
// dispatcher deals blocks round-robin over the 8 XCDs) form a contiguous
// range of tiles: neighbouring patches in SFC order then share an L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int per = n >> 3, rem = n & 7;
  const int x = b & 7, k = b >> 3;
  // XCD x owns tiles [start(x), start(x) + per + (x < rem))
  const int start = x * per + (x < rem ? x : rem);
  return start + k;
}

// Halo of a patch flagged kSimpleHalo: every neighbour region is a wall or a
// same-level leaf glued by a pure translation, so a ghost cell is a copy of
// cell (i -+ m, j -+ m) of that neighbour.

template <typename R, int MEQN, int PHYS>
__device__ __forceinline__ void simple_halo(const R* __restrict__ q,
                                            const PatchRec& r, int m, int lm,
                                            int p, int i, int j, R (&out)[MEQN]) {
  bool nx = false, ny = false;
  resolve_walls(r.flags, m, i, j, nx, ny);
  int src = p;
  if (i < 1 || i > m || j < 1 || j > m) {
    int slot;
    if (i >= 1 && i <= m) slot = j < 1 ? 4 : 6;
    else if (j >= 1 && j <= m) slot = i < 1 ? 0 : 2;
    else slot = 8 + (i > m) + 2 * (j > m);
    src = r.nbr[slot];
    i = i < 1 ? i + m : (i > m ? i - m : i);
    j = j < 1 ? j + m : (j > m ? j - m : j);
  }
  const uint32_t base = (uint32_t(src) * MEQN << (2 * lm)) + (uint32_t(j - 1) << lm) + (i - 1);
#pragma unroll
  for (int k = 0; k < MEQN; ++k) out[k] = q[base + (uint32_t(k) << (2 * lm))];
  if (PHYS == FCX_SHALLOW) {
    if (nx) out[1] = -out[1];
    if (ny) out[2 % MEQN] = -out[2 % MEQN];
  }
}

// Value of frame cell (i, j) of patch p outside its interior: gathered from
// the neighbours' interiors (fused path) or read from the ghost buffer.
template <typename R, int MEQN, int PHYS, bool FUSED>
__device__ __forceinline__ void halo_value(const StepArgs<R>& A, const PatchRec& rp,
                                           bool simple, int p, int i, int j,
                                           R (&v)[MEQN]) {
  if (FUSED) {
    if (simple) {
      simple_halo<R, MEQN, PHYS>(A.q, rp, A.m, A.lm, p, i, j, v);
    } else {
      GhostView<R, MEQN> gv{A.q, A.rec, A.m, A.lm, A.err};
      frame_value<R, MEQN, PHYS, true>(gv, p, i, j, v);
    }
  } else {
    const int G = 8 * A.m + 16;
    const uint32_t o = uint32_t(p) * MEQN * G + ghost_index(A.m, i, j);
#pragma unroll
    for (int k = 0; k < MEQN; ++k) v[k] = A.ghost[o + uint32_t(k) * G];
  }
}

// LDS layout of one tile update (carved from a caller-provided buffer so that
// kernels handling several physics share one allocation).
template <typename R, int PHYS, int T, int NT>
struct TileLds {
  static constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  static constexpr int WD = PHYS == FCX_SHALLOW ? 7 : 1;     // wave data per edge
  // per-cell primitives (sqrt h, u, v) are kept for FP64 shallow water; in
  // FP32 each edge forms them from the state (an rsqrt and a few products),
  // which leaves room in the LDS for one more resident tile per CU
  static constexpr bool PRIM = PHYS == FCX_SHALLOW && sizeof(R) == 8;
  static constexpr int NPR = PRIM ? 3 : 1;
  static constexpr int F = T + 4, NR = T + 2, NE = T + 3;
  R qs[MEQN][F * F];
  R pr[NPR][PRIM ? F * F : 1];
  R wb[WD][NR * NE];
  R fn[MEQN][T * T];          // normal fluxes, per interior cell
  R tup[MEQN][NR * T];        // transverse flux at a cell's upper
  R tdn[MEQN][NR * T];        //   and lower transverse edge
  R fb[2][MEQN][T];           // normal terms at the tile's two faces
  double red[NT / 64 > 0 ? NT / 64 : 1];
  // FCX_SWIRL: sin^2(pi x) at the tile frame's corner columns -2 .. T+2
  // (x0 + (i0 + a - 2) dx, a = 0 .. T+4), sin^2(pi y) likewise
  double sw[PHYS == FCX_SWIRL ? 2 : 1][PHYS == FCX_SWIRL ? T + 5 : 1];
};

// tid_in: the thread's index when the caller has hidden it from the
// optimizer (a loop over tiles then recomputes what depends on it per tile
// rather than keeping it in registers across tiles); -1: threadIdx.x.
// SPEC: 1 fixes the MC limiter and transverse mode 2 when compiling; 0
// takes the forest's at run time.
template <typename R, int PHYS, int T, int NT, bool FUSED, int SPEC = 0>
__device__ __forceinline__ void tile_step(const StepArgs<R>& A, int p, int tx, int ty,
                                          TileLds<R, PHYS, T, NT>& L, int tid_in = -1) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  constexpr int F = T + 4, NR = T + 2, NE = T + 3;
  constexpr int CPT = (T * T + NT - 1) / NT;
  constexpr int EPT = (NR * (T + 1) + NT - 1) / NT;   // phase-B edges per thread
  auto& qs = L.qs;
  auto& pr = L.pr;
  auto& wb = L.wb;
  auto& fn = L.fn;
  auto& tup = L.tup;
  auto& tdn = L.tdn;
  auto& fb = L.fb;
  auto& red = L.red;

  const int m = A.m, lm = A.lm;
  const int tid = tid_in >= 0 ? tid_in : int(threadIdx.x);
  const PatchRec& rp = A.rec[p];
  const int level = rp.level;
  const double dxd = ldexp(1.0, -level - lm);
  const double dtv = *A.dt;
  const double dtdx_d = dtv / dxd;
  const R dtdx = R(dtdx_d);
  const uint32_t pbase = uint32_t(p) * MEQN << (2 * lm);

  // ---- stage the tile and its halo ----------------------------------
  // interior cells first (coalesced), then the 8T + 12 halo cells strip by
  // strip (bottom, top, left, right), so that the lanes of a wavefront
  // mostly take the same ghost-cell path
  const bool simple = (rp.flags & kSimpleHalo) != 0;
  // face terms are kept only for patches on a coarse-fine face
  const int slot = A.phislot[p];
  const bool faces = slot >= 0;
  const int i0 = tx * T, j0 = ty * T;
  auto stage = [&](int c, const R (&v)[MEQN]) {
#pragma unroll
    for (int k = 0; k < MEQN; ++k) qs[k][c] = v[k];
    if (PHYS == FCX_SHALLOW) {
      // primitives: sqrt(h), u, v (zero for a non-positive depth)
      const R h = v[0];
      if (h > R(0)) {
        if constexpr (TileLds<R, PHYS, T, NT>::PRIM) {
          const R ih = rcp_(h);
          pr[0][c] = sqrt_(h);
          pr[1][c] = v[1] * ih;
          pr[2][c] = v[2 % MEQN] * ih;
        }
      } else {
        if constexpr (TileLds<R, PHYS, T, NT>::PRIM) {
          pr[0][c] = R(0);
          pr[1][c] = R(0);
          pr[2][c] = R(0);
        }
        atomicOr(A.err, kErrNegDepth);
      }
    }
  };
  for (int c = tid; c < T * T; c += NT) {
    const int ci = c % T + 1, cj = c / T + 1;
    const uint32_t o = pbase + (uint32_t(j0 + cj - 1) << lm) + (i0 + ci - 1);
    R v[MEQN];
#pragma unroll
    for (int k = 0; k < MEQN; ++k) v[k] = A.q[o + (uint32_t(k) << (2 * lm))];
    stage((cj + 1) * F + (ci + 1), v);
  }
  for (int h = tid; h < 8 * T + 12; h += NT) {
    int ci, cj;
    if (h < 2 * F - 2) {                     // bottom rows cj = -1, 0
      const int r = h < F - 2 ? 0 : 1;
      ci = r == 0 ? h : h - (F - 2) - 1;
      cj = r == 0 ? -1 : 0;
    } else if (h < 4 * F - 4) {              // top rows cj = T+1, T+2
      const int g = h - (2 * F - 2);
      const int r = g < F ? 0 : 1;
      ci = r == 0 ? g - 1 : g - F;
      cj = r == 0 ? T + 1 : T + 2;
    } else {                                 // side columns, rows 1..T
      const int g = h - (4 * F - 4);
      cj = g / 4 + 1;
      const int s2 = g % 4;
      ci = s2 == 0 ? -1 : s2 == 1 ? 0 : s2 == 2 ? T + 1 : T + 2;
    }
    const int i = i0 + ci, j = j0 + cj;
    R v[MEQN];
    if (i >= 1 && i <= m && j >= 1 && j <= m) {
      const uint32_t o = pbase + (uint32_t(j - 1) << lm) + (i - 1);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) v[k] = A.q[o + (uint32_t(k) << (2 * lm))];
    } else {
      halo_value<R, MEQN, PHYS, FUSED>(A, rp, simple, p, i, j, v);
    }
    stage((cj + 1) * F + (ci + 1), v);
  }
  // FCX_SWIRL: the stream function is separable, psi = k sx(x) sy(y) with
  // k = cos(pi t / T) / pi, so the tile needs sin^2 at its frame's corner
  // lines only (FP64); an edge's normal velocity is then a product and a
  // difference of these (the stream function's difference over the edge)
  double swk = 0;                           // k / dx
  if constexpr (PHYS == FCX_SWIRL) {
    const double pi = 3.14159265358979323846;
    const double tmid = *A.tsim + 0.5 * dtv;
    swk = cos(pi * tmid / A.ph.period) / pi / dxd;
    const double x0 = ldexp(double(rp.ix), -level), y0 = ldexp(double(rp.iy), -level);
    for (int k = tid; k < 2 * (T + 5); k += NT) {
      const int ax = k / (T + 5), a = k % (T + 5);
      const double c = (ax == 0 ? x0 + double(i0 + a - 2) * dxd : y0 + double(j0 + a - 2) * dxd);
      const double sn = sin(pi * c);
      L.sw[ax][a] = sn * sn;
    }
  }
  __syncthreads();

  R dq[CPT][MEQN], phx[CPT][MEQN], phy[CPT][MEQN];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int k = 0; k < MEQN; ++k) dq[c][k] = phx[c][k] = phy[c][k] = R(0);
  // largest |speed| over interior edges; the Courant number is formed once
  // at the end (monotone rounding: the same as the largest product)
  R smax = R(0);
  const int lim = SPEC ? 4 : A.ph.limiter, trans = SPEC ? 2 : A.ph.transverse;
  const R half_dtdx = R(0.5) * dtdx;
  const R ghalf = R(0.5 * A.ph.g);

#pragma unroll
  for (int d = 0; d < 2; ++d) {
    // (normal, transverse) component indices of the momentum
    const int mu = 1 + d, mv = 2 - d;
    const R an = R(d == 0 ? A.ph.ax : A.ph.ay);
    const R at = R(d == 0 ? A.ph.ay : A.ph.ax);
    auto bidx = [&](int r, int e) { return d == 0 ? r * NE + e : e * NR + r; };
    auto qidx = [&](int r, int e) {   // cell (normal e, transverse r)
      return d == 0 ? (r + 1) * F + (e + 1) : (e + 1) * F + (r + 1);
    };
    // per-cell accumulators of cell (normal n in 1..T, transverse r)
    auto nidx = [&](int r, int n) { return d == 0 ? (r - 1) * T + (n - 1)
                                                  : (n - 1) * T + (r - 1); };
    auto uidx = [&](int r, int n) { return d == 0 ? r * T + (n - 1)
                                                  : (n - 1) * NR + r; };
    // FCX_SWIRL: normal velocity of the direction-dd edge between frame
    // cells e - 1 and e (of direction dd) at frame cell r of the other
    // direction: u = psi_y (dd = 0), v = -psi_x (dd = 1)
    auto swirl_vel = [&](int dd, int e, int r) -> R {
      if constexpr (PHYS == FCX_SWIRL) {
        const double* nrm = L.sw[dd];
        const double* trn = L.sw[1 - dd];
        const double v = nrm[e + 1] * (trn[r + 2] - trn[r + 1]) * swk;
        return R(dd == 0 ? v : -v);
      } else {
        return R(0);
      }
    };

    // ---- phase A: Riemann solves ------------------------------------
    // (advection: the wave is the jump of the staged state, which phase B
    // forms where it needs it, so there is no phase A and no barrier after it)
    if (PHYS != FCX_ADVECTION && PHYS != FCX_SWIRL) {
    for (int idx = tid; idx < NR * NE; idx += NT) {
      const int r = d == 0 ? idx / NE : idx % NR;
      const int e = d == 0 ? idx % NE : idx / NR;
      const int cl = qidx(r, e - 1), cr = qidx(r, e);
      {
        const R hl = qs[0][cl], hr = qs[0][cr];
        R a1 = 0, a2 = 0, a3 = 0, u = 0, v = 0, c = 1, i2c_ = R(0.5);
        if (hl > R(0) && hr > R(0)) {
          // Roe averages (sqrt(h_l) u_l + sqrt(h_r) u_r) / (sqrt(h_l) + sqrt(h_r))
          if constexpr (TileLds<R, PHYS, T, NT>::PRIM) {
            const R sl = pr[0][cl], sr = pr[0][cr];
            const R inv = rcp_(sl + sr);
            u = (sl * pr[mu][cl] + sr * pr[mu][cr]) * inv;
            v = (sl * pr[mv][cl] + sr * pr[mv][cr]) * inv;
          } else {
            // sqrt(h) u = (h u) / sqrt(h)
            const R il = rsq_(hl), ir = rsq_(hr);
            const R inv = rcp_(hl * il + hr * ir);
            u = (qs[mu][cl] * il + qs[mu][cr] * ir) * inv;
            v = (qs[mv][cl] * il + qs[mv][cr] * ir) * inv;
          }
          c = sqrt_(ghalf * (hl + hr));
          i2c_ = R(0.5) * rcp_(c);
          const R d0 = hr - hl, d1 = qs[mu][cr] - qs[mu][cl];
          const R d2 = qs[mv][cr] - qs[mv][cl];
          a1 = ((u + c) * d0 - d1) * i2c_;
          a2 = d2 - v * d0;
          a3 = (d1 - (u - c) * d0) * i2c_;
        }
        const int b = bidx(r, e);
        wb[0][b] = a1; wb[1][b] = a2; wb[2][b] = a3;
        wb[3][b] = u; wb[4][b] = v; wb[5][b] = c;
        wb[6][b] = i2c_;
      }
    }
    __syncthreads();
    }

    // ---- phase B: limiter, corrections, transverse splitting ---------
    R keep[EPT][3][MEQN];                  // right-cell terms across the barrier
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int idx = tid + it * NT;
      if (idx >= NR * (T + 1)) break;
      const int r = d == 0 ? idx / (T + 1) : idx % NR;
      const int e = d == 0 ? idx % (T + 1) + 1 : idx / NR + 1;
      const bool inner = (r >= 1 && r <= T);
      R am[MEQN], ap[MEQN], cq[MEQN];
      if (PHYS == FCX_ADVECTION || PHYS == FCX_SWIRL) {
        // the edge's speed: constant, or the prescribed flow's
        const R ae = PHYS == FCX_SWIRL ? swirl_vel(d, e, r) : an;
        auto jump = [&](int ee) { return qs[0][qidx(r, ee)] - qs[0][qidx(r, ee - 1)]; };
        const R w = jump(e);
        am[0] = min_(ae, R(0)) * w;
        ap[0] = max_(ae, R(0)) * w;
        cq[0] = R(0);
        if (inner) smax = max_(smax, fabs(ae));
        if (w != R(0)) {
          const R wu = jump(ae > R(0) ? e - 1 : e + 1);
          const R th = (wu * w) * rcp_(w * w);
          const R s = fabs(ae);
          cq[0] = s * (R(1) - dtdx * s) * limiter_phi(lim, th) * w;
        }
      } else {
        // waves in (h, normal, tangential) order: a1 (1, u - c, v),
        // (0, 0, a2), a3 (1, u + c, v); speeds u - c, u, u + c
        const int b = bidx(r, e);
        const R u = wb[3][b], v = wb[4][b], c = wb[5][b];
        const R a1 = wb[0][b], a2 = wb[1][b], a3 = wb[2][b];
        const R s1 = u - c, s3 = u + c;
        const R b1m = min_(s1, R(0)) * a1, b2m = min_(u, R(0)) * a2, b3m = min_(s3, R(0)) * a3;
        const R b1p = max_(s1, R(0)) * a1, b2p = max_(u, R(0)) * a2, b3p = max_(s3, R(0)) * a3;
        const R m0 = b1m + b3m, p0 = b1p + b3p;
        R amh[3] = {m0, b1m * s1 + b3m * s3, m0 * v + b2m};
        R aph[3] = {p0, b1p * s1 + b3p * s3, p0 * v + b2p};
        // limited corrections: g_w = |s|(1 - dtdx |s|) phi(theta) a_w
        R g[3] = {R(0), R(0), R(0)};
        const R nv = R(1) + v * v;
        const R sp[3] = {s1, u, s3};
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          const R aw = w == 0 ? a1 : (w == 1 ? a2 : a3);
          const R r2 = w == 1 ? R(1) : sp[w] * sp[w] + nv;     // |r_w|^2
          const R wn2 = (aw * aw) * r2;
          if (wn2 != R(0)) {
            const int bu = bidx(r, sp[w] > R(0) ? e - 1 : e + 1);
            R dot;
            if (w == 1) {
              dot = wb[1][bu] * a2;
            } else {
              const R au = wb[w][bu], uu = wb[3][bu], vu = wb[4][bu], cu = wb[5][bu];
              const R nu_ = w == 0 ? uu - cu : uu + cu;
              dot = (au * aw) * (R(1) + nu_ * sp[w] + vu * v);
            }
            const R phi = limiter_phi(lim, dot * rcp_(wn2));
            const R as = fabs(sp[w]);
            g[w] = as * (R(1) - dtdx * as) * phi * aw;
          }
        }
        const R g13 = g[0] + g[2];
        R cqh[3] = {g13, g[0] * s1 + g[2] * s3, g13 * v + g[1]};
        if (inner) smax = max_(smax, max_(fabs(s1), fabs(s3)));
        am[0] = amh[0]; am[mu] = amh[1]; am[mv] = amh[2];
        ap[0] = aph[0]; ap[mu] = aph[1]; ap[mv] = aph[2];
        cq[0] = cqh[0]; cq[mu] = cqh[1]; cq[mv] = cqh[2];
      }
      // transverse: left-going part to the cell left of the edge, right-going
      // part to the cell on its right, each split into down / up parts
      R ldn[MEQN], lup[MEQN], rdn[MEQN], rup[MEQN];
#pragma unroll
      for (int k = 0; k < MEQN; ++k) ldn[k] = lup[k] = rdn[k] = rup[k] = R(0);
      if (trans > 0) {
        R amt[MEQN], apt[MEQN];
#pragma unroll
        for (int k = 0; k < MEQN; ++k) {
          amt[k] = am[k] + (trans == 2 ? cq[k] : R(0));
          apt[k] = ap[k] - (trans == 2 ? cq[k] : R(0));
        }
        if (PHYS == FCX_ADVECTION) {
          const R bm = -half_dtdx * min_(at, R(0)), bp = -half_dtdx * max_(at, R(0));
          ldn[0] = bm * amt[0];
          lup[0] = bp * amt[0];
          rdn[0] = bm * apt[0];
          rup[0] = bp * apt[0];
        } else if (PHYS == FCX_SWIRL) {
          // each part leaves its receiving cell (column e - 1 for the
          // left-going one, e for the right-going one) down through the
          // cell's lower transverse edge and up through its upper one, at
          // those edges' own velocities
          const int od = 1 - d;
          const R vll = swirl_vel(od, r, e - 1), vlh = swirl_vel(od, r + 1, e - 1);
          const R vrl = swirl_vel(od, r, e), vrh = swirl_vel(od, r + 1, e);
          ldn[0] = -half_dtdx * min_(vll, R(0)) * amt[0];
          lup[0] = -half_dtdx * max_(vlh, R(0)) * amt[0];
          rdn[0] = -half_dtdx * min_(vrl, R(0)) * apt[0];
          rup[0] = -half_dtdx * max_(vrh, R(0)) * apt[0];
        } else {
          const int b = bidx(r, e);
          const R u = wb[3][b], v = wb[4][b], c = wb[5][b];
          const R i2c = wb[6][b];
          const R lmn[3] = {-half_dtdx * min_(v - c, R(0)), -half_dtdx * min_(v, R(0)),
                            -half_dtdx * min_(v + c, R(0))};
          const R lmx[3] = {-half_dtdx * max_(v - c, R(0)), -half_dtdx * max_(v, R(0)),
                            -half_dtdx * max_(v + c, R(0))};
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const R* psi = side == 0 ? amt : apt;
            const R ph = psi[0], pn = psi[mu], pt = psi[mv];
            const R b1 = ((v + c) * ph - pt) * i2c, b2 = pn - u * ph;
            const R b3 = (pt - (v - c) * ph) * i2c;
            // eigenvectors (1, u, v - c), (0, 1, 0), (1, u, v + c)
            const R m1 = lmn[0] * b1, m2 = lmn[1] * b2, m3 = lmn[2] * b3;
            const R p1 = lmx[0] * b1, p2 = lmx[1] * b2, p3 = lmx[2] * b3;
            R* dn = side == 0 ? ldn : rdn;
            R* up = side == 0 ? lup : rup;
            dn[0] = m1 + m3;
            dn[mu] = u * (m1 + m3) + m2;
            dn[mv] = (v - c) * m1 + (v + c) * m3;
            up[0] = p1 + p3;
            up[mu] = u * (p1 + p3) + p2;
            up[mv] = (v - c) * p1 + (v + c) * p3;
          }
        }
      }
      // left cell (e - 1) now; right cell (e) after the barrier
      if (e >= 2) {
#pragma unroll
        for (int k = 0; k < MEQN; ++k) {
          tup[k][uidx(r, e - 1)] = lup[k];
          tdn[k][uidx(r, e - 1)] = ldn[k];
          if (inner) fn[k][nidx(r, e - 1)] = am[k] + R(0.5) * cq[k];
        }
      }
      if (faces && inner && (e == 1 || e == T + 1)) {
#pragma unroll
        for (int k = 0; k < MEQN; ++k)
          fb[e == 1 ? 0 : 1][k][r - 1] = e == 1 ? ap[k] - R(0.5) * cq[k]
                                              : am[k] + R(0.5) * cq[k];
      }
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        keep[it][0][k] = ap[k] - R(0.5) * cq[k];
        keep[it][1][k] = rup[k];
        keep[it][2][k] = rdn[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int idx = tid + it * NT;
      if (idx >= NR * (T + 1)) break;
      const int r = d == 0 ? idx / (T + 1) : idx % NR;
      const int e = d == 0 ? idx % (T + 1) + 1 : idx / NR + 1;
      if (e > T) continue;
      const bool inner = (r >= 1 && r <= T);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        tup[k][uidx(r, e)] += keep[it][1][k];
        tdn[k][uidx(r, e)] += keep[it][2][k];
        if (inner) fn[k][nidx(r, e)] += keep[it][0][k];
      }
    }
    __syncthreads();

    // ---- phase C: per-cell gather ------------------------------------
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int cell = tid + c * NT;
      if (cell >= T * T) break;
      const int ci = cell % T + 1, cj = cell / T + 1;
      const int n = d == 0 ? ci : cj;         // normal index
      const int r = d == 0 ? cj : ci;         // transverse index
      const int pn = (d == 0 ? tx : ty) * T + n;   // patch-level indices
      const int prr = (d == 0 ? ty : tx) * T + r;
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        // other-direction flux at the transverse edges r + 1/2 and r - 1/2
        const R gup = tup[k][uidx(r, n)] + tdn[k][uidx(r + 1, n)];
        const R gdn = tup[k][uidx(r - 1, n)] + tdn[k][uidx(r, n)];
        dq[c][k] -= dtdx * (fn[k][nidx(r, n)] + (gup - gdn));
        if (faces) {
          // face terms through the patch faces (for the reflux)
          R& pnrm = d == 0 ? phx[c][k] : phy[c][k];
          R& ptrn = d == 0 ? phy[c][k] : phx[c][k];
          if (pn == 1) pnrm += fb[0][k][r - 1];
          if (pn == m) pnrm += fb[1][k][r - 1];
          if (prr == 1) ptrn -= gdn;
          if (prr == m) ptrn += gup;
        }
      }
    }
    __syncthreads();
  }

  // ---- write q_new and face terms -----------------------------------
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int cell = tid + c * NT;
    if (cell >= T * T) break;
    const int ci = cell % T + 1, cj = cell / T + 1;
    const int i = i0 + ci, j = j0 + cj;
    const uint32_t o = pbase + (uint32_t(j - 1) << lm) + (i - 1);
#pragma unroll
    for (int k = 0; k < MEQN; ++k)
      A.qn[o + (uint32_t(k) << (2 * lm))] = qs[k][(cj + 1) * F + (ci + 1)] + dq[c][k];
    if (faces) {
      R* ph = A.phi + size_t(slot) * 4 * m * MEQN;
      const R dxr = R(dxd);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        if (i == 1) ph[(0 * m + (j - 1)) * MEQN + k] = dxr * phx[c][k];
        if (i == m) ph[(1 * m + (j - 1)) * MEQN + k] = dxr * phx[c][k];
        if (j == 1) ph[(2 * m + (i - 1)) * MEQN + k] = dxr * phy[c][k];
        if (j == m) ph[(3 * m + (i - 1)) * MEQN + k] = dxr * phy[c][k];
      }
    }
  }

  // ---- CFL number: wavefront max, then one atomic per workgroup -----
  double numax = dtdx_d * double(smax);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) numax = fmax(numax, __shfl_xor(numax, off));
  if ((tid & 63) == 0) red[tid >> 6] = numax;
  __syncthreads();
  if (tid == 0) {
    double v = red[0];
    for (int w = 1; w < NT / 64; ++w) v = fmax(v, red[w]);
    atomic_max_pos(A.numax, v);
  }
}

// One workgroup per tile, over all tiles of one forest.  With an order
// table, each XCD's run of slots takes the patches with a general halo (the
// costlier tiles) first, so the last tiles to be dispatched are cheap ones.
template <typename R, int PHYS, int T, int NT, bool FUSED, int SPEC>
__global__ void __launch_bounds__(NT)
k_step(StepArgs<R> A) {
  __shared__ TileLds<R, PHYS, T, NT> lds;
  int t = xcd_tile(blockIdx.x, A.ntiles);
  if (A.order && A.m == T) t = A.order[t];
  const int tps = A.m / T;
  const int p = t / (tps * tps);
  const int tile = t - p * (tps * tps);
  tile_step<R, PHYS, T, NT, FUSED, SPEC>(A, p, tile % tps, tile / tps, lds);
}

// One workgroup per tile of the patches in `list` (one level of a
// sub-cycled step); plain path (ghosts from the ghost buffer).
template <typename R, int PHYS, int T, int NT, int SPEC>
__global__ void __launch_bounds__(NT)
k_step_level(StepArgs<R> A, const int32_t* __restrict__ list) {
  __shared__ TileLds<R, PHYS, T, NT> lds;
  const int t = xcd_tile(blockIdx.x, A.ntiles);
  const int tps = A.m / T;
  const int p = list[t / (tps * tps)];
  const int tile = t % (tps * tps);
  tile_step<R, PHYS, T, NT, false, SPEC>(A, p, tile % tps, tile / tps, lds);
}

}  // namespace fcx
