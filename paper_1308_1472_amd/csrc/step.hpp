// step.hpp -- the wave-propagation patch update on gfx950 (arXiv 1308.1472,
// Sec. 3: Clawpack's wave-propagation algorithm on every leaf patch; LeVeque,
// JCP 1997, for the unsplit method with transverse propagation; Roe's
// approximate solver for shallow water).
//
// One workgroup advances one T x T tile of one patch.  The tile and its
// two-cell halo are staged in LDS -- from the compact state plus the ghost
// buffer (plain path) or straight from neighbouring patches' interiors
// (fused path).  Each sweep direction runs three phases separated by
// barriers:
//   A  one Riemann solve per edge of the (T+2) x (T+3) edge set; compact
//      wave data (shallow water: strengths and Roe averages) go to LDS;
//   B  per edge: wave limiter from the neighbour edges' waves, second-order
//      correction, transverse splitting of the corrected fluctuations;
//      results go to LDS per edge;
//   C  per interior cell: gather the normal fluctuations and correction
//      fluxes of its two edges and the transverse fluxes of its two
//      transverse edges into a register accumulator.
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
  KPhys ph;
};

template <int T> struct TileThreads { static constexpr int value = T * T >= 256 ? 256 : T * T; };

template <typename R>
__device__ __forceinline__ R limiter_phi(int lim, R th) {
  switch (lim) {
    case 0: return R(1);
    case 1: return fmax(R(0), fmin(R(1), th));
    case 2: return fmax(R(0), fmax(fmin(R(1), R(2) * th), fmin(R(2), th)));
    case 3: return (th + fabs(th)) / (R(1) + fabs(th));
    default: return fmax(R(0), fmin(fmin(R(0.5) * (R(1) + th), R(2)), R(2) * th));
  }
}

template <typename R, int PHYS, int M, int T, bool FUSED>
__global__ void __launch_bounds__(TileThreads<T>::value)
k_step(StepArgs<R> A) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  constexpr int WD = PHYS == FCX_ADVECTION ? 1 : 6;   // wave data per edge
  constexpr int F = T + 4, NR = T + 2, NE = T + 3;
  constexpr int NT = TileThreads<T>::value;
  constexpr int TPS = M / T;
  constexpr int CPT = (T * T + NT - 1) / NT;
  constexpr int LM = M == 8 ? 3 : M == 16 ? 4 : 5;
  constexpr int G = 8 * M + 16;

  __shared__ R qs[MEQN][F * F];
  __shared__ R wb[WD][NR * NE];
  __shared__ R tl[MEQN][T * (T + 1)];
  __shared__ R tr[MEQN][T * (T + 1)];
  __shared__ R tq[4][MEQN][NR * (T + 1)];
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];

  const int tid = threadIdx.x;
  const int blk = blockIdx.x;
  const int p = blk / (TPS * TPS);
  const int tile = blk - p * (TPS * TPS);
  const int tx = tile % TPS, ty = tile / TPS;
  const PatchRec& rp = A.rec[p];
  const int level = rp.level;
  const double dxd = ldexp(1.0, -level) / M;
  const double dtv = *A.dt;
  const double dtdx_d = dtv / dxd;
  const R dtdx = R(dtdx_d);

  // ---- stage the tile and its halo ----------------------------------
  GhostView<R, MEQN> gv{A.q, A.rec, M, LM, A.err};
  for (int c = tid; c < F * F; c += NT) {
    const int ci = c % F - 1, cj = c / F - 1;
    const int i = tx * T + ci, j = ty * T + cj;
    R v[MEQN];
    const bool outer = (ci == -1 || ci == T + 2) && (cj == -1 || cj == T + 2);
    if (outer) {
#pragma unroll
      for (int k = 0; k < MEQN; ++k) v[k] = R(0);
    } else if (i >= 1 && i <= M && j >= 1 && j <= M) {
      read_interior<R, MEQN>(A.q, M, p, i, j, v);
    } else if (FUSED) {
      frame_value<R, MEQN, PHYS, true>(gv, p, i, j, v);
    } else {
      const int gi = ghost_index(M, i, j);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) v[k] = A.ghost[size_t(p * MEQN + k) * G + gi];
    }
#pragma unroll
    for (int k = 0; k < MEQN; ++k) qs[k][c] = v[k];
  }
  __syncthreads();

  R dq[CPT][MEQN], phx[CPT][MEQN], phy[CPT][MEQN];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int k = 0; k < MEQN; ++k) dq[c][k] = phx[c][k] = phy[c][k] = R(0);
  double numax = 0.0;
  const int lim = A.ph.limiter, trans = A.ph.transverse;
  const R half_dtdx = R(0.5) * dtdx;

#pragma unroll
  for (int d = 0; d < 2; ++d) {
    // (normal, transverse) component indices of the momentum
    const int mu = 1 + d, mv = 2 - d;
    const R an = R(d == 0 ? A.ph.ax : A.ph.ay);
    const R at = R(d == 0 ? A.ph.ay : A.ph.ax);
    auto bidx = [&](int r, int e) { return d == 0 ? r * NE + e : e * NR + r; };
    auto lidx = [&](int r, int e) { return d == 0 ? (r - 1) * (T + 1) + (e - 1)
                                                  : (e - 1) * T + (r - 1); };
    auto qidx = [&](int r, int e) {   // cell (normal e, transverse r)
      return d == 0 ? (r + 1) * F + (e + 1) : (e + 1) * F + (r + 1);
    };
    auto tidx = [&](int r, int e) { return d == 0 ? r * (T + 1) + (e - 1)
                                                  : (e - 1) * NR + r; };

    // ---- phase A: Riemann solves ------------------------------------
    for (int idx = tid; idx < NR * NE; idx += NT) {
      const int r = d == 0 ? idx / NE : idx % NR;
      const int e = d == 0 ? idx % NE : idx / NR;
      const int cl = qidx(r, e - 1), cr = qidx(r, e);
      if (PHYS == FCX_ADVECTION) {
        wb[0][bidx(r, e)] = qs[0][cr] - qs[0][cl];
      } else {
        const R hl = qs[0][cl], hr = qs[0][cr];
        R a1 = 0, a2 = 0, a3 = 0, u = 0, v = 0, c = 1;
        if (hl > R(0) && hr > R(0)) {
          const R sl = sqrt(hl), sr = sqrt(hr);
          const R inv = R(1) / (sl + sr);
          u = (qs[mu][cl] / sl + qs[mu][cr] / sr) * inv;
          v = (qs[mv][cl] / sl + qs[mv][cr] / sr) * inv;
          c = sqrt(R(A.ph.g) * R(0.5) * (hl + hr));
          const R d0 = hr - hl, d1 = qs[mu][cr] - qs[mu][cl];
          const R d2 = qs[mv][cr] - qs[mv][cl];
          const R i2c = R(0.5) / c;
          a1 = ((u + c) * d0 - d1) * i2c;
          a2 = d2 - v * d0;
          a3 = (d1 - (u - c) * d0) * i2c;
        } else {
          atomicOr(A.err, kErrNegDepth);
        }
        const int b = bidx(r, e);
        wb[0][b] = a1; wb[1][b] = a2; wb[2][b] = a3;
        wb[3][b] = u; wb[4][b] = v; wb[5][b] = c;
      }
    }
    __syncthreads();

    // ---- phase B: limiter, corrections, transverse splitting ---------
    for (int idx = tid; idx < NR * (T + 1); idx += NT) {
      const int r = d == 0 ? idx / (T + 1) : idx % NR;
      const int e = d == 0 ? idx % (T + 1) + 1 : idx / NR + 1;
      const bool inner = (r >= 1 && r <= T);
      R am[MEQN], ap[MEQN], cq[MEQN];
      if (PHYS == FCX_ADVECTION) {
        const R w = wb[0][bidx(r, e)];
        am[0] = fmin(an, R(0)) * w;
        ap[0] = fmax(an, R(0)) * w;
        cq[0] = R(0);
        if (inner) numax = fmax(numax, dtdx_d * fabs(double(an)));
        if (w != R(0)) {
          const R wu = wb[0][bidx(r, an > R(0) ? e - 1 : e + 1)];
          const R th = (wu * w) / (w * w);
          const R s = fabs(an);
          cq[0] = s * (R(1) - dtdx * s) * limiter_phi(lim, th) * w;
        }
      } else {
        const int b = bidx(r, e);
        const R u = wb[3][b], v = wb[4][b], c = wb[5][b];
        const R al[3] = {wb[0][b], wb[1][b], wb[2][b]};
        const R s[3] = {u - c, u, u + c};
        // waves in (h, normal, tangential) order
        R W[3][3] = {{al[0], al[0] * (u - c), al[0] * v},
                     {R(0), R(0), al[1]},
                     {al[2], al[2] * (u + c), al[2] * v}};
        R amh[3] = {0, 0, 0}, aph[3] = {0, 0, 0}, cqh[3] = {0, 0, 0};
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          const R smn = fmin(s[w], R(0)), smx = fmax(s[w], R(0));
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            amh[k] += smn * W[w][k];
            aph[k] += smx * W[w][k];
          }
          if (inner) numax = fmax(numax, dtdx_d * fabs(double(s[w])));
          const R wn2 = W[w][0] * W[w][0] + W[w][1] * W[w][1] + W[w][2] * W[w][2];
          if (wn2 != R(0)) {
            const int bu = bidx(r, s[w] > R(0) ? e - 1 : e + 1);
            const R uu = wb[3][bu], vu = wb[4][bu], cu = wb[5][bu];
            R dot;
            if (w == 1) {
              dot = wb[1][bu] * al[1];
            } else {
              const R au = wb[w][bu];
              const R nu_ = w == 0 ? uu - cu : uu + cu;
              dot = au * W[w][0] + au * nu_ * W[w][1] + au * vu * W[w][2];
            }
            const R phi = limiter_phi(lim, dot / wn2);
            const R as = fabs(s[w]);
            const R f = as * (R(1) - dtdx * as) * phi;
#pragma unroll
            for (int k = 0; k < 3; ++k) cqh[k] += f * W[w][k];
          }
        }
        am[0] = amh[0]; am[mu] = amh[1]; am[mv] = amh[2];
        ap[0] = aph[0]; ap[mu] = aph[1]; ap[mv] = aph[2];
        cq[0] = cqh[0]; cq[mu] = cqh[1]; cq[mv] = cqh[2];
      }
      if (inner) {
        const int li = lidx(r, e);
#pragma unroll
        for (int k = 0; k < MEQN; ++k) {
          tl[k][li] = am[k] + R(0.5) * cq[k];
          tr[k][li] = ap[k] - R(0.5) * cq[k];
        }
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
          const R bm = fmin(at, R(0)), bp = fmax(at, R(0));
          ldn[0] = -half_dtdx * bm * amt[0];
          lup[0] = -half_dtdx * bp * amt[0];
          rdn[0] = -half_dtdx * bm * apt[0];
          rup[0] = -half_dtdx * bp * apt[0];
        } else {
          const int b = bidx(r, e);
          const R u = wb[3][b], v = wb[4][b], c = wb[5][b];
          const R i2c = R(0.5) / c;
          const R lam[3] = {v - c, v, v + c};
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const R* psi = side == 0 ? amt : apt;
            const R ph = psi[0], pn = psi[mu], pt = psi[mv];
            const R be[3] = {((v + c) * ph - pt) * i2c, pn - u * ph,
                             (pt - (v - c) * ph) * i2c};
            R bmh[3] = {0, 0, 0}, bph[3] = {0, 0, 0};
#pragma unroll
            for (int w = 0; w < 3; ++w) {
              const R rv[3] = {w == 1 ? R(0) : R(1), w == 1 ? R(1) : u,
                               w == 0 ? v - c : w == 1 ? R(0) : v + c};
              const R fm = fmin(lam[w], R(0)) * be[w];
              const R fp = fmax(lam[w], R(0)) * be[w];
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                bmh[k] += fm * rv[k];
                bph[k] += fp * rv[k];
              }
            }
            R* dn = side == 0 ? ldn : rdn;
            R* up = side == 0 ? lup : rup;
            dn[0] = -half_dtdx * bmh[0]; dn[mu] = -half_dtdx * bmh[1];
            dn[mv] = -half_dtdx * bmh[2];
            up[0] = -half_dtdx * bph[0]; up[mu] = -half_dtdx * bph[1];
            up[mv] = -half_dtdx * bph[2];
          }
        }
      }
      const int ti = tidx(r, e);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        tq[0][k][ti] = ldn[k];
        tq[1][k][ti] = lup[k];
        tq[2][k][ti] = rdn[k];
        tq[3][k][ti] = rup[k];
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
      const int pr = (d == 0 ? ty : tx) * T + r;
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        const R fR = tr[k][lidx(r, n)], fL = tl[k][lidx(r, n + 1)];
        // other-direction flux at the transverse edges r + 1/2 and r - 1/2
        const R gup = tq[1][k][tidx(r, n + 1)] + tq[3][k][tidx(r, n)] +
                      tq[0][k][tidx(r + 1, n + 1)] + tq[2][k][tidx(r + 1, n)];
        const R gdn = tq[1][k][tidx(r - 1, n + 1)] + tq[3][k][tidx(r - 1, n)] +
                      tq[0][k][tidx(r, n + 1)] + tq[2][k][tidx(r, n)];
        dq[c][k] -= dtdx * (fR + fL) + dtdx * (gup - gdn);
        // face terms through the patch faces (for the reflux)
        R& pnrm = d == 0 ? phx[c][k] : phy[c][k];
        R& ptrn = d == 0 ? phy[c][k] : phx[c][k];
        if (pn == 1) pnrm += fR;
        if (pn == M) pnrm += fL;
        if (pr == 1) ptrn -= gdn;
        if (pr == M) ptrn += gup;
      }
    }
    __syncthreads();
  }

  // ---- write q_new and face terms -----------------------------------
  const int slot = A.phislot[p];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int cell = tid + c * NT;
    if (cell >= T * T) break;
    const int ci = cell % T + 1, cj = cell / T + 1;
    const int i = tx * T + ci, j = ty * T + cj;
#pragma unroll
    for (int k = 0; k < MEQN; ++k) {
      const size_t o = (size_t(p * MEQN + k) * M + (j - 1)) * M + (i - 1);
      A.qn[o] = qs[k][(cj + 1) * F + (ci + 1)] + dq[c][k];
    }
    if (slot >= 0) {
      R* ph = A.phi + size_t(slot) * 4 * M * MEQN;
      const R dxr = R(dxd);
#pragma unroll
      for (int k = 0; k < MEQN; ++k) {
        if (i == 1) ph[(0 * M + (j - 1)) * MEQN + k] = dxr * phx[c][k];
        if (i == M) ph[(1 * M + (j - 1)) * MEQN + k] = dxr * phx[c][k];
        if (j == 1) ph[(2 * M + (i - 1)) * MEQN + k] = dxr * phy[c][k];
        if (j == M) ph[(3 * M + (i - 1)) * MEQN + k] = dxr * phy[c][k];
      }
    }
  }

  // ---- CFL number: wavefront max, then one atomic per workgroup -----
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

}  // namespace fcx
