// advect.hpp -- the patch update of constant-velocity advection (arXiv
// 1308.1472, Sec. 3 and its advection example; LeVeque, JCP 1997, for the
// unsplit wave-propagation method with transverse propagation) as a tile of
// its own, run by one wavefront, and its step kernels.
//
// With a constant velocity (a_x, a_y) every edge carries one wave, the jump
// w of the state across it, moving at a_x or a_y.  The tile is staged in a
// mirrored frame in which both components are non-negative: mirroring an
// axis negates the velocity along it, and the scheme is exactly symmetric
// under that (jumps, fluctuations and correction fluxes change sign, and the
// left- and right-going parts trade places).  In that frame every wave comes
// from the lower neighbour, the limiter's upwind wave is the one below the
// edge, only the up-going transverse parts are non-zero, and the stencil
// needs two halo cells on the lower sides and one on the upper sides
// (6T + 5 cells instead of the general 8T + 12).
//
// Per edge, with g = a w the right-going fluctuation and the limited
// correction c = a (1 - a dt/dx) phi(theta) w (phi(theta) w in a form
// without a division: theta = w_up / w has the sign of w_up w), keep
// Q = c / 2 and P = g - c / 2.  For a cell with lower edge 1 and upper edge 2
// in one sweep direction:
//   normal term      Q_2 + P_1,
//   transverse source U = 2 Q_2 + P_1 - Q_1   (transverse mode 2),
//                     U = P_1 + Q_1            (mode 1), 0 (mode 0),
// and the sweep's contribution to dq / (dt/dx) is
//   -(Q_2 + P_1) - b (U - U_prev),   b = -(dt/dx) a_t / 2,
// with U_prev the source of the neighbour below in the transverse direction
// (the up-going transverse fluxes of LeVeque's method at the cell's two
// transverse edges).
//
// One wavefront per tile (several tiles per workgroup, each with its own
// LDS; a CU holds only so many workgroups and the tile's cost is mostly the
// latency of its loads); each lane owns T*T/64 vertically consecutive cells
// of one column (mirrored frame).  Its cells' values stay in registers; the
// source U of the cell below is its own previous cell's, or the lower lane
// group's (ds_bpermute); the values of the neighbouring columns come through
// DPP row shifts (a tile row of 16 cells is a DPP row of 16 lanes); only the
// 4T + 2 edges on the tile's first row and column and on its upper sides go
// through LDS.  The Courant number dt/dx max(|a_x|, |a_y|) needs no reduction.
#pragma once

#include "step.hpp"

namespace fcx {

// ---- lane exchange within a wavefront --------------------------------
// DPP row shifts move a value one lane along a row of 16 lanes: row_shr:1
// gives lane l the value of lane l - 1, row_shl:1 that of lane l + 1 (lanes
// whose source lies outside the row get 0 here and are overwritten by the
// caller).  ds_bpermute gives lane l the value of any lane (address 4 x lane,
// taken modulo the wavefront).  Doubles move as two 32-bit halves.
constexpr int kDppRowShr1 = 0x111, kDppRowShl1 = 0x101;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__device__ __forceinline__ float lane_fetch(int lane, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(lane << 2, __float_as_int(v)));
}

__device__ __forceinline__ double lane_fetch(int lane, double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(lane << 2, int(b));
  const int hi = __builtin_amdgcn_ds_bpermute(lane << 2, int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// (P, Q) of one edge
template <typename R>
struct alignas(2 * sizeof(R)) EdgePQ {
  R P, Q;
};

// Row stride of a tile's frame (columns -1 .. T+1) in LDS: one more than
// the frame's width, which spreads the lane groups' rows over the LDS banks
// (measured: no slower for 16 x 16 tiles, faster for 8 x 8).
template <int T>
constexpr int adv_frame_stride() {
  return T + 4;
}

template <typename R, int T>
struct AdvLds {
  static constexpr int F = adv_frame_stride<T>();
  R qs[F * (T + 3)];                        // rows -1 .. T+1
  // the edges beside the tile's own, in the order they are computed:
  // x-edges T+1 of rows 1..T, x-edges 1..T+1 of row 0, y-edges T+1 of
  // columns 1..T, y-edges 1..T+1 of column 0
  EdgePQ<R> ext[4 * T + 2];
  R sink[64];                               // stores of lanes past the halo's end
  __device__ const EdgePQ<R>& xt(int r) const { return ext[r]; }       // row r + 1
  __device__ const EdgePQ<R>& x0(int e) const { return ext[T + e]; }   // edge e + 1
  __device__ const EdgePQ<R>& yt(int c) const { return ext[2 * T + 1 + c]; }
  __device__ const EdgePQ<R>& y0(int e) const { return ext[3 * T + 1 + e]; }
};

// phi(theta) w for theta = wu / w, limiter `lim` (0 none, 1 minmod,
// 2 superbee, 3 van Leer, else MC); zero where w wu <= 0 (theta <= 0).
template <typename R>
__device__ __forceinline__ R limited_wave(int lim, R w, R wu) {
  if (lim == 0) return w;
  const R aw = fabs(w), au = fabs(wu);
  R v;
  if (lim == 1) {
    v = min_(aw, au);
  } else if (lim == 2) {
    v = max_(min_(aw, R(2) * au), min_(R(2) * aw, au));
  } else if (lim == 3) {
    // 2 theta / (1 + theta) w = 2 w wu / (w + wu)
    v = R(2) * (aw * au) * rcp_(aw + au);
  } else {
    v = min_(R(0.5) * (aw + au), R(2) * min_(aw, au));
  }
  return (w * wu > R(0)) ? copysign(v, w) : R(0);
}

// In FP32, minmod(x, y) (the one of smaller magnitude where the signs
// agree, else zero) is the median of x, y and 0: one v_med3.  The MC
// limited wave is minmod((w + wu) / 2, 2 w, 2 wu) =
// minmod(2 minmod(w, wu), (w + wu) / 2), and half of
// minmod(4 minmod(w, wu), w + wu): the same value, rounded the same (the
// sum rounds once either way; the scalings are exact), as the form above.
__device__ __forceinline__ float minmod_(float x, float y) {
  return __builtin_amdgcn_fmed3f(x, y, 0.0f);
}

// (P, Q) of the edge between a cell (value q0) and the one below it (q1),
// with q2 below that; kh = a (1 - a dt/dx) / 2.
template <typename R>
__device__ __forceinline__ EdgePQ<R> edge_pq(int lim, R a, R kh, R q0, R q1, R q2) {
  const R w = q0 - q1, wu = q1 - q2;
  R Q;
  if constexpr (sizeof(R) == 4) {
    if (lim == 1)
      Q = kh * minmod_(w, wu);
    else if (lim >= 4)
      Q = (R(0.5) * kh) * minmod_(R(4) * minmod_(w, wu), w + wu);
    else
      Q = kh * limited_wave(lim, w, wu);
  } else {
    Q = kh * limited_wave(lim, w, wu);
  }
  return EdgePQ<R>{a * w - Q, Q};
}

// transverse source of a cell from its lower edge e1 and the Q of its upper
// edge
template <typename R>
__device__ __forceinline__ R trans_source(int trans, const EdgePQ<R>& e1, R q2) {
  return trans == 2 ? (R(2) * q2 + e1.P) - e1.Q : (trans == 1 ? e1.P + e1.Q : R(0));
}

// Halo of a tile of a patch flagged kSimpleHalo, in the mirrored frame: six
// strips of T cells -- 0 row -1, 1 row 0, 2 column -1, 3 column 0, 4 row
// T+1, 5 column T+1 (cell t = 1..T of a row strip at (t, d), of a column
// strip at (c, t)) -- and five corner cells (-1, 0), (0, 0), (T+1, 0),
// (0, -1), (0, T+1).  Every cell is a copy: from the patch itself (inside,
// or mirrored by a wall) or from a same-level neighbour glued by a
// translation.  A strip lies on one side of the tile and inside the patch
// along its length, so its source patch and wall rule are the same for all
// its cells: the state offset of its cell t is base + t * step (step +-1
// for a row strip, +-m for a column strip, the sign that of the mirror).
// Offsets count from the state of patch 0 of the patch's forest, assuming
// all its patches have the patch's size (p m^2 + local offset).
struct AdvHalo {
  int32_t base[6];
  int32_t corner[5];
};

__host__ __device__ constexpr void adv_halo_cell(int T, int h, int& c, int& d) {
  if (h < 6 * T) {
    const int s = h / T, t = h % T + 1;
    c = s == 2 ? -1 : (s == 3 ? 0 : (s == 5 ? T + 1 : t));
    d = s == 0 ? -1 : (s == 1 ? 0 : (s == 4 ? T + 1 : t));
  } else {
    const int e = h - 6 * T;
    c = e == 0 ? -1 : (e == 2 ? T + 1 : 0);
    d = e < 3 ? 0 : (e == 3 ? -1 : T + 1);
  }
}

// The LDS index (frame cell (c, d) at (d + 1) F + c + 1, F the frame stride) of halo cell
// h, without branches (selects only, so that it stays out of loops over
// tiles: it depends on the lane alone).
template <int T>
__host__ __device__ constexpr int adv_halo_lds(int h) {
  constexpr int F = adv_frame_stride<T>();
  const int s = h / T, t = h % T + 1;
  const bool row = s == 0 || s == 1 || s == 4;
  const int rb = s == 0 ? 0 : (s == 1 ? F : (T + 2) * F);
  const int cc = s == 2 ? 0 : (s == 3 ? 1 : T + 2);
  const int rowv = rb + t + 1, colv = (t + 1) * F + cc;     // (both formed, then chosen)
  const int strip = row ? rowv : colv;
  const int e = h - 6 * T;
  const int corner =
      e == 0 ? F : (e == 1 ? F + 1 : (e == 2 ? F + T + 2 : (e == 3 ? 1 : (T + 2) * F + 1)));
  return h < 6 * T ? strip : corner;
}

template <int T>
constexpr bool adv_halo_lds_agrees() {
  for (int h = 0; h < 6 * T + 5; ++h) {
    int c = 0, d = 0;
    adv_halo_cell(T, h, c, d);
    if (adv_halo_lds<T>(h) != (d + 1) * adv_frame_stride<T>() + c + 1) return false;
  }
  return true;
}
static_assert(adv_halo_lds_agrees<8>() && adv_halo_lds_agrees<16>(), "halo LDS index");

// nbr: the patch's 12 neighbour slots (faces two each, then corners).
__host__ __device__ __forceinline__ AdvHalo adv_halo_offsets(int T, int m, int lm, int p,
                                                             int tx, int ty, bool mx,
                                                             bool my, int32_t flags,
                                                             const int32_t* nbr) {
  AdvHalo H;
  auto flip_x = [&](int c) { return mx ? T + 1 - c : c; };
  auto flip_y = [&](int d) { return my ? T + 1 - d : d; };
  const int i0 = tx * T, j0 = ty * T;
  for (int s = 0; s < 6; ++s) {
    const bool row = s == 0 || s == 1 || s == 4;
    const int fixed = (s == 0 || s == 2) ? -1 : ((s == 1 || s == 3) ? 0 : T + 1);
    int x = row ? j0 + flip_y(fixed) : i0 + flip_x(fixed);
    int src = p;
    const int lo_wall = row ? 4 : 1, lo_ext = row ? 64 : 16;
    const int hi_wall = row ? 8 : 2, hi_ext = row ? 128 : 32;
    if (x < 1) {
      if (flags & lo_wall) x = (flags & lo_ext) ? 1 : 1 - x;
      else { src = row ? nbr[4] : nbr[0]; x += m; }
    } else if (x > m) {
      if (flags & hi_wall) x = (flags & hi_ext) ? m : 2 * m + 1 - x;
      else { src = row ? nbr[6] : nbr[2]; x -= m; }
    }
    H.base[s] = int32_t(uint32_t(src) << (2 * lm)) +
                (row ? ((x - 1) << lm) + i0 - 1 + (mx ? T + 1 : 0)
                     : x - 1 + ((j0 - 1 + (my ? T + 1 : 0)) << lm));
  }
  for (int e = 0; e < 5; ++e) {
    int c, d;
    adv_halo_cell(T, 6 * T + e, c, d);
    int i = i0 + flip_x(c), j = j0 + flip_y(d);
    bool nx = false, ny = false;
    resolve_walls(flags, m, i, j, nx, ny);
    const bool lo_x = i < 1, hi_x = i > m, lo_y = j < 1, hi_y = j > m;
    int src = p;
    if (lo_y || hi_y) {
      if (lo_x || hi_x) src = hi_y ? (hi_x ? nbr[11] : nbr[10]) : (hi_x ? nbr[9] : nbr[8]);
      else src = hi_y ? nbr[6] : nbr[4];
    } else if (lo_x || hi_x) {
      src = hi_x ? nbr[2] : nbr[0];
    }
    i = lo_x ? i + m : (hi_x ? i - m : i);
    j = lo_y ? j + m : (hi_y ? j - m : j);
    H.corner[e] = int32_t(uint32_t(src) << (2 * lm)) + ((j - 1) << lm) + (i - 1);
  }
  return H;
}

// Where a tile's halo comes from: the ghost buffer (plain path); copies of
// the patch's and its same-level neighbours' cells, for patches flagged
// kSimpleHalo; the general gather (averages, interpolation, rotated trees);
// or either of the last two, chosen per patch.
// kHaloStripWords: strip halos whose offsets are held one dword per lane
// (base[s] at lane hl0 + s, corner[e] at lane hl0 + 6 + e).
enum AdvHaloSource {
  kHaloGhostBuf = 0,
  kHaloStrips = 1,
  kHaloGeneral = 2,
  kHaloAny = 3,
  kHaloStripWords = 4
};

// A tile's values as loaded: a lane's own cells and its halo cells.
template <typename R, int T>
struct AdvRegs {
  static constexpr int RPL = T * T / 64;
  static constexpr int HPT = (6 * T + 5 + 63) / 64;
  R qv[RPL], vh[HPT];
};

// Loads of one tile into registers (no LDS): every load is issued here and
// nothing waits for them.  desc: the tile's halo offsets formed beforehand
// (strip halos; null: formed here); mirror: bit 0 / bit 1 set where the x /
// y velocity is negative (-1: read from the velocity here); hwords, hl0:
// the offsets held in lanes (kHaloStripWords).
template <typename R, int T, int HALO>
__device__ __forceinline__ void adv_tile_load(const StepArgs<R>& A, int p, int tx, int ty,
                                              int lane, const AdvHalo* desc,
                                              AdvRegs<R, T>& g, int mirror = -1,
                                              int32_t hwords = 0, int hl0 = 0) {
  constexpr int NT = 64, RPL = T * T / NT;   // lanes, own rows per lane
  static_assert(T * T % NT == 0 && RPL >= 1, "one wavefront per tile");
  constexpr int NH = 6 * T + 5;              // halo cells of the mirrored frame
  constexpr int HPT = (NH + NT - 1) / NT;    // halo cells per lane
  const int m = A.m, lm = A.lm;
  const int n = lane % T + 1, grp = lane / T;      // own column, lane group
  const int r0 = RPL * grp + 1;                    // first own row
  const PatchRec& rp = A.rec[p];
  const uint32_t pbase = uint32_t(p) << (2 * lm);
  const int i0 = tx * T, j0 = ty * T;
  const bool mx = mirror >= 0 ? (mirror & 1) != 0 : R(A.ph.ax) < R(0);
  const bool my = mirror >= 0 ? (mirror & 2) != 0 : R(A.ph.ay) < R(0);
  // tile cell (c, d) of the mirrored frame <-> tile cell of the patch
  auto flip_x = [&](int c) { return mx ? T + 1 - c : c; };
  auto flip_y = [&](int d) { return my ? T + 1 - d : d; };
  auto cell = [&](int i, int j) { return pbase + (uint32_t(j - 1) << lm) + (i - 1); };

  // own cells (for each k the lanes read whole tile rows), then the halo
  R* qv = g.qv;
  R* vh = g.vh;
  {
    // a lane's rows are consecutive: one address, then a uniform stride
    const R* qp = A.q + cell(i0 + flip_x(n), j0 + flip_y(r0));
    const int32_t rs = my ? -m : m;
#pragma unroll
    for (int k = 0; k < RPL; ++k) qv[k] = qp[k * rs];
  }
  if constexpr (HALO == kHaloStripWords) {
    // each lane takes its strip's (or corner's) offset from the lane that
    // holds it; lanes past the last corner read the last one again (their
    // value is not used), so that no load is under a branch
    const int32_t step_row = mx ? -1 : 1, step_col = my ? -m : m;
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int h = lane + k * NT;
      const bool strip = h < 6 * T;
      const int s = h / T, t = strip ? h % T + 1 : 0;
      const int wi = strip ? s : 6 + (h - 6 * T < 4 ? h - 6 * T : 4);
      const int32_t b = __builtin_amdgcn_ds_bpermute((hl0 + wi) << 2, hwords);
      const bool row = s == 0 || s == 1 || s == 4;
      vh[k] = A.q[b + t * (row ? step_row : step_col)];
    }
    return;
  }
  const int32_t flags = rp.flags;
  const bool simple = (flags & kSimpleHalo) != 0;
  auto halo_pos = [&](int h, int& c, int& d) { adv_halo_cell(T, h, c, d); };
  const bool strips = HALO == kHaloStrips || (HALO == kHaloAny && simple);
  if constexpr (HALO == kHaloStrips || HALO == kHaloAny) if (strips) {
    // copies (the strip halo above); offsets read with the work item or
    // formed here from the patch's neighbour slots (uniform values)
    AdvHalo H;
    if (desc) {
      H = *desc;
    } else {
      int32_t nbr[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) nbr[k] = __builtin_amdgcn_readfirstlane(rp.nbr[k]);
      H = adv_halo_offsets(T, m, lm, p, tx, ty, mx, my, flags, nbr);
    }
    const int32_t step_row = mx ? -1 : 1, step_col = my ? -m : m;
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int h = lane + k * NT;
      if (h < 6 * T) {
        const int s = h / T, t = h % T + 1;
        // select among the strips this pass can reach (fixed per pass)
        const int s_first = k * NT / T, s_last = (k * NT + NT - 1) / T;
        int32_t b = H.base[s_first < 6 ? s_first : 5];
#pragma unroll
        for (int q = 1; q < 6; ++q)
          if (q > s_first && q <= s_last) b = s == q ? H.base[q] : b;
        const bool row = s == 0 || s == 1 || s == 4;
        vh[k] = A.q[b + t * (row ? step_row : step_col)];
      } else {
        // corners; lanes past the last one read the last one again (their
        // value is not used), so that the load is not under a branch
        const int e = h - 6 * T;
        int32_t b = H.corner[0];
#pragma unroll
        for (int q = 1; q < 5; ++q) b = e == q || (q == 4 && e > 4) ? H.corner[q] : b;
        vh[k] = A.q[b];
      }
    }
  }
  if constexpr (HALO != kHaloStrips) if (!strips) {
    // the ghost buffer (plain path), or the general halo of the fused path:
    // averages and interpolation from other levels, trees glued with
    // rotations
    constexpr bool GATHER = HALO != kHaloGhostBuf;
    for (int k = 0; k < HPT; ++k) {
      const int h = lane + k * NT;
      if (h < NH) {
        int c, d;
        halo_pos(h, c, d);
        const int i = i0 + flip_x(c), j = j0 + flip_y(d);
        R v[1];
        if (i >= 1 && i <= m && j >= 1 && j <= m)
          v[0] = A.q[cell(i, j)];
        else
          halo_value<R, 1, FCX_ADVECTION, GATHER>(A, rp, false, p, i, j, v);
        vh[k] = v[0];
      }
    }
  }
}

// The rest of a tile's update from its loaded values: LDS staging, edges,
// cells, face terms.  LIM and TRANS fix the limiter and transverse mode when
// compiling (-1: the forest's, at run time); slot: the patch's face-term slot
// (-1: none); level: the patch's refinement level; dt: the time step.  With
// NU the tile's Courant number goes into *A.numax here; it is returned
// either way.
template <typename R, int T, int LIM = -1, int TRANS = -1, bool NU = true>
__device__ __forceinline__ double adv_tile_rest(const StepArgs<R>& A, int p, int slot, int tx,
                                                int ty, AdvLds<R, T>& L, int lane,
                                                const AdvRegs<R, T>& g, int level, double dt) {
  constexpr int NT = 64, RPL = T * T / NT;
  constexpr int F = AdvLds<R, T>::F;
  constexpr int NH = 6 * T + 5;              // halo cells of the mirrored frame
  constexpr int NX = 4 * T + 2;              // edges on the first row / column
                                             // and the upper sides
  constexpr int HPT = (NH + NT - 1) / NT;    // halo cells per lane
  const int m = A.m, lm = A.lm;
  const int n = lane % T + 1, grp = lane / T;
  const int r0 = RPL * grp + 1;
  const uint32_t pbase = uint32_t(p) << (2 * lm);
  const int i0 = tx * T, j0 = ty * T;
  const R axr = R(A.ph.ax), ayr = R(A.ph.ay);
  const bool mx = axr < R(0), my = ayr < R(0);
  auto flip_x = [&](int c) { return mx ? T + 1 - c : c; };
  auto flip_y = [&](int d) { return my ? T + 1 - d : d; };
  auto at = [&](int c, int d) { return (d + 1) * F + (c + 1); };
  auto cell = [&](int i, int j) { return pbase + (uint32_t(j - 1) << lm) + (i - 1); };
  const R* qv = g.qv;
  const R* vh = g.vh;
#pragma unroll
  for (int k = 0; k < RPL; ++k) L.qs[at(n, r0 + k)] = qv[k];
  // (lanes past the halo's last cell store into a sink: no branch)
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int h = lane + k * NT;
    R* dst = h < NH ? &L.qs[adv_halo_lds<T>(h)] : &L.sink[lane];
    *dst = vh[k];
  }
  const double dtdx_d = ldexp(dt, level + lm);             // dx = 2^-(level + lm)
  const R dtdx = R(dtdx_d);
  const R ax = fabs(axr), ay = fabs(ayr);
  // the Courant number: the same on every edge of the tile
  const double cfl = dtdx_d * double(fmax(ax, ay));
  if (NU && lane == 0) atomic_max_pos(A.numax, cfl);
  wave_sync();

  // ---- edges -------------------------------------------------------------
  const R kxh = R(0.5) * (ax * (R(1) - dtdx * ax));
  const R kyh = R(0.5) * (ay * (R(1) - dtdx * ay));
  const int lim = LIM >= 0 ? LIM : A.ph.limiter;
  const int trans = TRANS >= 0 ? TRANS : A.ph.transverse;
  EdgePQ<R> ex[RPL], ey[RPL];
  {
    const R b1 = L.qs[at(n, r0 - 1)], b2 = L.qs[at(n, r0 - 2)];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int b = at(n, r0 + k);
      ex[k] = edge_pq(lim, ax, kxh, qv[k], L.qs[b - 1], L.qs[b - 2]);
      const R q1 = k >= 1 ? qv[k - 1] : b1;
      const R q2 = k >= 2 ? qv[k - 2] : (k == 1 ? b1 : b2);
      ey[k] = edge_pq(lim, ay, kyh, qv[k], q1, q2);
    }
  }
  // the extra edges go to the last lanes (the first ones staged more halo);
  // one edge evaluation per pass, its cells and direction chosen per lane
  // by selects: the LDS index of the edge's upper cell is base + x * mul
#pragma unroll
  for (int x = NT - 1 - lane; x < NX; x += NT) {
    const bool s1 = x >= T, s2 = x >= 2 * T + 1, s3 = x >= 3 * T + 1;
    int base = 2 * F + T + 2, mul = F;           // x-edges T+1, rows 1..T: at(T+1, x+1)
    base = s1 ? F - T + 2 : base;                // x-edges 1..T+1 of row 0: at(x-T+1, 0)
    mul = s1 ? 1 : mul;
    base = s2 ? (T + 2) * F - 2 * T + 1 : base;  // y-edges T+1: at(x-2T, T+1)
    base = s3 ? (1 - 3 * T) * F + 1 : base;      // y-edges 1..T+1 of column 0: at(0, x-3T)
    mul = s3 ? F : mul;
    const int b = base + x * mul;
    const int st = s2 ? F : 1;
    L.ext[x] = edge_pq(lim, s2 ? ay : ax, s2 ? kyh : kxh, L.qs[b], L.qs[b - st],
                       L.qs[b - 2 * st]);
  }
  wave_sync();

  // ---- cells ---------------------------------------------------------------
  // (every lane takes part in every exchange; boundary lanes then replace
  // what came from outside the tile by the extra edges)
  const R half_dtdx = R(0.5) * dtdx;
  const R bx = -half_dtdx * ax, by = -half_dtdx * ay;  // transverse factors
  R qx2[RPL], qy2[RPL], U[RPL], V[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const R right = dpp_move<kDppRowShl1>(ex[k].Q);  // x-edge n+1, same row
    const R last = L.xt(r0 + k - 1).Q;               // (read by every lane: no branch)
    qx2[k] = n == T ? last : right;
    U[k] = trans_source(trans, ex[k], qx2[k]);
  }
  {
    const R above = lane_fetch(lane + T, ey[0].Q);   // y-edge of the row above
    const R top = L.yt(n - 1).Q;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      qy2[k] = k + 1 < RPL ? ey[k + 1].Q : (grp == NT / T - 1 ? top : above);
      V[k] = trans_source(trans, ey[k], qy2[k]);
    }
  }
  const R u_low = lane_fetch(lane - T, U[RPL - 1]);  // source of the row below
  const R u_row0 = trans_source(trans, L.x0(n - 1), L.x0(n).Q);
  R u_dn[RPL], v_dn[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int r = r0 + k;
    u_dn[k] = k > 0 ? U[k - 1] : (grp > 0 ? u_low : u_row0);
    const R v_left = dpp_move<kDppRowShr1>(V[k]);     // column n-1, same row
    const R v_first = trans_source(trans, L.y0(r - 1), L.y0(r).Q);   // (every lane)
    v_dn[k] = n > 1 ? v_left : v_first;
    const R X = (qx2[k] + ex[k].P) + by * (U[k] - u_dn[k]);
    const R Y = (qy2[k] + ey[k].P) + bx * (V[k] - v_dn[k]);
    A.qn[cell(i0 + flip_x(n), j0 + flip_y(r))] = (qv[k] - dtdx * X) - dtdx * Y;
  }
  if (slot >= 0) {
    // terms through the patch faces, for the reflux: a face that is the
    // lower side in the mirrored frame takes the lower-edge terms
    R* ph = A.phi + size_t(slot) * 4 * m;
    const R dxr = R(ldexp(1.0, -level - lm));
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int i = i0 + flip_x(n), j = j0 + flip_y(r0 + k);
      const R vxl = ex[k].P - bx * v_dn[k], vxh = qx2[k] + bx * V[k];
      const R vyl = ey[k].P - by * u_dn[k], vyh = qy2[k] + by * U[k];
      if (i == 1) ph[0 * m + (j - 1)] = dxr * (mx ? vxh : vxl);
      if (i == m) ph[1 * m + (j - 1)] = dxr * (mx ? vxl : vxh);
      if (j == 1) ph[2 * m + (i - 1)] = dxr * (my ? vyh : vyl);
      if (j == m) ph[3 * m + (i - 1)] = dxr * (my ? vyl : vyh);
    }
  }
  return cfl;
}

// One wavefront advances one T x T tile (T = 8 or 16) with its own LDS.
template <typename R, int T, int HALO, int LIM = -1, int TRANS = -1>
__device__ __forceinline__ void adv_tile_step(const StepArgs<R>& A, int p, int slot, int tx,
                                              int ty, AdvLds<R, T>& L, int lane,
                                              const AdvHalo* desc = nullptr) {
  AdvRegs<R, T> g;
  adv_tile_load<R, T, HALO>(A, p, tx, ty, lane, desc, g);
  adv_tile_rest<R, T, LIM, TRANS>(A, p, slot, tx, ty, L, lane, g, A.rec[p].level, *A.dt);
}

// Tiles (wavefronts) per workgroup: a CU holds only so many workgroups, and
// the tiles' load latency is hidden by having many of them resident.
constexpr int kAdvWaves = 4;

// Tile slot of wavefront `wv` of this workgroup: consecutive blocks go to
// the XCDs in turn, and each XCD takes a contiguous run of slots.
__device__ __forceinline__ int adv_slot(int ntiles, int wv) {
  const int nblk = (ntiles + kAdvWaves - 1) / kAdvWaves;
  return xcd_tile(blockIdx.x, nblk) * kAdvWaves + wv;
}

// One wavefront per tile, over all tiles of one forest (order: as k_step).
// SPEC: 1 for the MC limiter with transverse mode 2 fixed when compiling,
// 0 for the forest's at run time.
template <typename R, int T, bool FUSED, int SPEC>
__global__ void __launch_bounds__(64 * kAdvWaves, 8)
k_adv_step(StepArgs<R> A) {
  constexpr int HALO = FUSED ? kHaloAny : kHaloGhostBuf;
  __shared__ AdvLds<R, T> lds[kAdvWaves];
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  int t = adv_slot(A.ntiles, wv);
  if (t >= A.ntiles) return;
  if (A.order && A.m == T) t = A.order[t];
  const int tps = A.m / T;
  const int p = t / (tps * tps);
  const int tile = t - p * (tps * tps);
  adv_tile_step<R, T, HALO, SPEC ? 4 : -1, SPEC ? 2 : -1>(A, p, A.phislot[p], tile % tps,
                                                         tile / tps, lds[wv],
                                                         int(threadIdx.x) & 63);
}

// One wavefront per tile of the patches in `list` (one level of a
// sub-cycled step); plain path.
template <typename R, int T, int SPEC>
__global__ void __launch_bounds__(64 * kAdvWaves, 8)
k_adv_step_level(StepArgs<R> A, const int32_t* __restrict__ list) {
  __shared__ AdvLds<R, T> lds[kAdvWaves];
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int t = adv_slot(A.ntiles, wv);
  if (t >= A.ntiles) return;
  const int tps = A.m / T;
  const int p = list[t / (tps * tps)];
  const int tile = t % (tps * tps);
  adv_tile_step<R, T, kHaloGhostBuf, SPEC ? 4 : -1, SPEC ? 2 : -1>(
      A, p, A.phislot[p], tile % tps, tile / tps, lds[wv], int(threadIdx.x) & 63);
}

}  // namespace fcx
