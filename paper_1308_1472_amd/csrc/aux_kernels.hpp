// aux_kernels.hpp -- the kernels around the patch update: ghost fill,
// coarse-fine reflux, next dt, conservation sums, refinement tags and
// regrid transfer (arXiv 1308.1472, Sec. 2-4).
#pragma once

#include "device.hpp"

namespace fcx {

// ---------------------------------------------------------------------------
// Ghost fill: one thread per (patch, frame cell); consecutive threads write
// consecutive ghost-buffer entries of one patch.
template <typename R, int PHYS>
__global__ void __launch_bounds__(256)
k_ghost_fill(const R* __restrict__ q, R* __restrict__ ghost,
             const PatchRec* __restrict__ rec, int32_t P, int m, int lm,
             int32_t* err, const double* __restrict__ geo) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int G = 8 * m + 16;
  // XCD-contiguous block order (see xcd_tile): neighbouring patches' reads
  // then hit the same L2
  const int nb = gridDim.x, b = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, x = b & 7;
  const int blk = x * per + (x < rem ? x : rem) + (b >> 3);
  const int64_t t = int64_t(blk) * blockDim.x + threadIdx.x;
  if (t >= int64_t(P) * G) return;
  const int p = int(t / G), g = int(t - int64_t(p) * G);
  int i, j;
  ghost_cell(m, g, i, j);
  if ((i == -1 || i == m + 2) && (j == -1 || j == m + 2)) return;
  GhostView<R, MEQN> gv{q, rec, m, lm, err, geo};
  R v[MEQN];
  frame_value<R, MEQN, PHYS, true>(gv, p, i, j, v);
#pragma unroll
  for (int k = 0; k < MEQN; ++k) ghost[size_t(p * MEQN + k) * G + g] = v[k];
}

// ---------------------------------------------------------------------------
// Sum of the fluctuations of one Riemann problem, which by Roe's property
// equals f(q_r) - f(q_l) in direction d.
template <typename R, int PHYS>
__device__ void fluct_sum(const KPhys& ph, int d, const R* ql, const R* qr,
                          R* out, int32_t* err) {
  if (PHYS == FCX_ADVECTION) {
    out[0] = R(d == 0 ? ph.ax : ph.ay) * (qr[0] - ql[0]);
    return;
  }
  const int mu = 1 + d, mv = 2 - d;
  const R hl = ql[0], hr = qr[0];
  if (!(hl > R(0) && hr > R(0))) {
    atomicOr(err, kErrNegDepth);
    out[0] = out[1] = out[2] = R(0);
    return;
  }
  R u, v, c, i2c;
  if constexpr (sizeof(R) == 4) {
    // hardware root and reciprocals, as in the patch update
    const R il = rsq_(hl), ir = rsq_(hr);
    const R inv = rcp_(hl * il + hr * ir);
    u = (ql[mu] * il + qr[mu] * ir) * inv;
    v = (ql[mv] * il + qr[mv] * ir) * inv;
    c = sqrt_(R(ph.g) * R(0.5) * (hl + hr));
    i2c = R(0.5) * rcp_(c);
  } else {
    const R sl = sqrt(hl), sr = sqrt(hr), inv = R(1) / (sl + sr);
    u = (ql[mu] / sl + qr[mu] / sr) * inv;
    v = (ql[mv] / sl + qr[mv] / sr) * inv;
    c = sqrt(R(ph.g) * R(0.5) * (hl + hr));
    i2c = R(0.5) / c;
  }
  const R d0 = hr - hl, d1 = qr[mu] - ql[mu], d2 = qr[mv] - ql[mv];
  const R a1 = ((u + c) * d0 - d1) * i2c;
  const R a2 = d2 - v * d0;
  const R a3 = (d1 - (u - c) * d0) * i2c;
  const R s1 = u - c, s3 = u + c;
  out[0] = s1 * a1 + s3 * a3;
  out[mu] = s1 * a1 * s1 + s3 * a3 * s3;
  out[mv] = s1 * a1 * v + u * a2 + s3 * a3 * v;
}

// Per reflux item, built with the plan: the items of the other direction on
// the same coarse patch whose faces meet this one at its low and high end
// (-1: none), the face-term slots of the coarse patch and of the two fine
// patches, and the coarse patch's level.
struct RefluxAux {
  int32_t link[2], slot_c, slot_f[2], level;
};

// Reflux correction of one coarse cell (position tc along the face of item
// it): the coarse face term minus the two fine ones, per component; o is the
// cell's offset in qn (component 0).
template <typename R, int PHYS>
__device__ __forceinline__ void reflux_corr(const R* __restrict__ q, const RefluxItem& it,
                                            const RefluxAux& ax, int tc,
                                            const R* __restrict__ phi, int m,
                                            const KPhys& ph, int32_t* err,
                                            R (&corr)[PhysTraits<PHYS>::MEQN], size_t& o,
                                            double& dxc) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int f = it.face, d = f >> 1, hi = f & 1;
  const int C = it.coarse;
  const int ic = d == 0 ? (hi ? m : 1) : tc, jc = d == 0 ? tc : (hi ? m : 1);
  const int k2 = (tc - 1) / (m / 2);
  const int fp = it.fine[k2], ff = it.fine_face[k2];
  dxc = ldexp(1.0, -ax.level) / m;
  o = (size_t(C * MEQN) * m + (jc - 1)) * m + (ic - 1);
  R qc[MEQN];
  read_interior<R, MEQN>(q, m, C, ic, jc, qc);
  const R* phf = phi + size_t(ax.slot_f[k2]) * 4 * m * MEQN;
  const R* phc = phi + size_t(ax.slot_c) * 4 * m * MEQN;
#pragma unroll
  for (int k = 0; k < MEQN; ++k) corr[k] = -phc[(f * m + (tc - 1)) * MEQN + k];
  R fine[MEQN];
#pragma unroll
  for (int k = 0; k < MEQN; ++k) fine[k] = R(0);
  for (int s = 0; s < 2; ++s) {
    int pos = 2 * (tc - 1 - k2 * (m / 2)) + 1 + s;
    if (it.fine_rev[k2]) pos = m + 1 - pos;
    const int fi = ff < 2 ? (ff == 0 ? 1 : m) : pos;
    const int fj = ff < 2 ? pos : (ff == 2 ? 1 : m);
    R qf[MEQN], fs[MEQN];
    read_interior<R, MEQN>(q, m, fp, fi, fj, qf);
    if (hi) fluct_sum<R, PHYS>(ph, d, qc, qf, fs, err);
    else fluct_sum<R, PHYS>(ph, d, qf, qc, fs, err);
#pragma unroll
    for (int k = 0; k < MEQN; ++k)
      fine[k] += R(0.5 * dxc) * fs[k] - phf[(ff * m + (pos - 1)) * MEQN + k];
  }
#pragma unroll
  for (int k = 0; k < MEQN; ++k) corr[k] = fine[k] + corr[k];
}

// Status bits of the next-dt step (sticky until the caller clears them).
constexpr int32_t kStatCfl = 1;         // nu_max > cfl_max in an accepted step
constexpr int32_t kStatNeg = 2;         // a non-positive depth was met
constexpr int32_t kStatNested = 4;      // a ghost needed nested interpolation
constexpr int32_t kStatRedone = 8;      // an attempt was rejected and is redone

// The CFL rule of the wave-propagation method (LeVeque 2002, Sec. 4.4 and
// the time-step control of Clawpack): with redo on, an attempt whose largest
// Courant number exceeds cfl_max is rejected (the caller's q_new receives q
// unchanged, see copy_state) and the next attempt uses the reduced dt.
__device__ __forceinline__ bool rejected(const double* numax, int f, double cfl_max,
                                         int32_t redo) {
  return redo && numax[f] > cfl_max;
}

// CFL check and next dt of forest f: dt <- dt * cfl_desired / nu_max, the
// status bits above, error word f read and cleared, numax cleared; stats
// (null: none) counts per forest {accepted steps, rejected attempts,
// accepted cell updates}.
__device__ __forceinline__ void next_dt_one(double* numax, double* dt, int32_t* status,
                                            int32_t* err, int64_t* stats, int f,
                                            double cfl_desired, double cfl_max,
                                            int32_t redo, int64_t cells,
                                            double* tsim = nullptr, double tscale = 1.0) {
  const double nu = numax[f];
  if (tsim && !(redo && nu > cfl_max)) tsim[f] += dt[f] * tscale;
  const bool rej = redo && nu > cfl_max;
  int32_t st = 0;
  if (nu > cfl_max) st |= rej ? kStatRedone : kStatCfl;
  const int32_t e = __hip_atomic_load(err + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (e & kErrNegDepth) st |= kStatNeg;
  if (e & kErrNested) st |= kStatNested;
  err[f] = 0;
  status[f] |= st;
  if (nu > 0.0) dt[f] = dt[f] * cfl_desired / nu;
  numax[f] = 0.0;
  if (stats) {
    int64_t* s = stats + 3 * f;
    if (rej) {
      s[1] += 1;
    } else {
      s[0] += 1;
      s[2] += cells;
    }
  }
}

// Copies this workgroup's share (of `parts` equal shares, share `part`) of
// n16 16-byte units from src to dst.
__device__ __forceinline__ void copy_share(const uint4* __restrict__ src,
                                           uint4* __restrict__ dst, int64_t n16, int part,
                                           int parts) {
  const int64_t per = (n16 + parts - 1) / parts;
  const int64_t lo = int64_t(part) * per, hi = lo + per < n16 ? lo + per : n16;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) dst[i] = src[i];
}

// Grid-stride copy of n16 16-byte units (the source may be pinned host
// memory).
__global__ void __launch_bounds__(256)
k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

struct NextDtArgs {
  double* numax;
  double* dt;
  int32_t* status;
  uint32_t* ticket;                          // zero between launches
  int64_t* stats;
  double cfl_desired, cfl_max;
  int32_t redo;
  int64_t cells;                             // cell updates of an accepted step
  int64_t n16;                               // size of the state in 16-byte units
  double* tsim;                              // simulated time of accepted steps
  double tscale;                             //   per unit of dt
};

// Reflux: one thread per (coarse-fine face item, coarse cell along it), all
// items in one launch.  Items of xi faces come first; a coarse corner cell
// that lies on an xi item and an eta item gets both corrections, xi first,
// from the xi item's thread (RefluxAux::link: for an xi item the eta items
// at its low / high end, for an eta item the xi items there), so the result
// does not depend on the order the threads run in; such a thread computes
// both corrections before it updates the cell.
// keep(): whether to write the corrections, asked after the loads are issued
template <typename R, int PHYS, typename Keep>
__device__ __forceinline__ void reflux_cell(const R* __restrict__ q, R* __restrict__ qn,
                                            const RefluxItem* __restrict__ items,
                                            const RefluxAux* __restrict__ aux, int32_t i,
                                            int tc, const R* __restrict__ phi,
                                            const double* dtp, int m, const KPhys& ph,
                                            int32_t* err, Keep keep) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const RefluxItem it = items[i];
  const RefluxAux ax = aux[i];
  const int end = tc == 1 ? 0 : (tc == m ? 1 : -1);
  const int32_t link = end >= 0 ? ax.link[end] : -1;
  if (it.face >= 2 && link >= 0) return;
  R c0[MEQN], c1[MEQN];
  size_t o, o1;          // o1 == o: the second correction is on the same cell
  double dxc, dxc1;
  reflux_corr<R, PHYS>(q, it, ax, tc, phi, m, ph, err, c0, o, dxc);
  const bool two = it.face < 2 && link >= 0;
  if (two)
    reflux_corr<R, PHYS>(q, items[link], aux[link], it.face == 0 ? 1 : m, phi, m, ph, err,
                         c1, o1, dxc1);
  const R fac = R(*dtp / (dxc * dxc));
  R v[MEQN];
#pragma unroll
  for (int k = 0; k < MEQN; ++k) v[k] = qn[o + size_t(k) * m * m];
  if (!keep()) return;
#pragma unroll
  for (int k = 0; k < MEQN; ++k) {
    v[k] -= fac * c0[k];
    if (two) v[k] -= fac * c1[k];
    qn[o + size_t(k) * m * m] = v[k];
  }
}

// All reflux items in one launch.  With NEXT, the workgroup that finishes
// last also takes the CFL check and the next dt; an attempt that the CFL
// rule rejects (redo on) skips the corrections, and every workgroup copies
// its share of q into q_new instead, so that q_new holds the unchanged state.
template <typename R, int PHYS, bool NEXT>
__global__ void __launch_bounds__(256)
k_reflux(const R* __restrict__ q, R* __restrict__ qn,
         const RefluxItem* __restrict__ items, const RefluxAux* __restrict__ aux,
         int32_t nitems, const R* __restrict__ phi, const double* dtp, int m, KPhys ph,
         int32_t* err, NextDtArgs nd) {
  // the CFL check's operand is loaded first and waited for only where a
  // correction is about to be written (its latency overlaps the reflux loads)
  const double nu = NEXT && nd.redo ? *nd.numax : 0.0;
  auto keep = [&]() { return !(NEXT && nd.redo && nu > nd.cfl_max); };
  // grid-stride: with NEXT the grid is kept small (every workgroup takes the
  // ticket)
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < int64_t(nitems) * m;
       t += int64_t(gridDim.x) * blockDim.x)
    reflux_cell<R, PHYS>(q, qn, items, aux, int32_t(t / m), int(t % m) + 1, phi, dtp, m, ph,
                         err, keep);
  if (!keep())
    copy_share(reinterpret_cast<const uint4*>(q), reinterpret_cast<uint4*>(qn), nd.n16,
               blockIdx.x, gridDim.x);
  if (NEXT) {
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      last = atomicAdd(nd.ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
      __threadfence();
      next_dt_one(nd.numax, nd.dt, nd.status, err, nd.stats, 0, nd.cfl_desired, nd.cfl_max,
                  nd.redo, nd.cells, nd.tsim, nd.tscale);
      *nd.ticket = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Next dt of one forest without a rejection copy (the caller decides).
__global__ void k_next_dt(double* numax, double* dt, int32_t* status, int32_t* err,
                          int64_t* stats, double cfl_desired, double cfl_max,
                          int64_t cells, double* tsim) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    next_dt_one(numax, dt, status, err, stats, 0, cfl_desired, cfl_max, 0, cells, tsim);
}

// Next dt of one forest with the CFL rule's rejection: every workgroup
// copies its share of q into q_new if the attempt is rejected; the last one
// takes the next dt.
__global__ void __launch_bounds__(256)
k_next_dt_redo(const uint4* __restrict__ q, uint4* __restrict__ qn, NextDtArgs nd,
               int32_t* err) {
  if (rejected(nd.numax, 0, nd.cfl_max, nd.redo))
    copy_share(q, qn, nd.n16, blockIdx.x, gridDim.x);
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(nd.ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    next_dt_one(nd.numax, nd.dt, nd.status, err, nd.stats, 0, nd.cfl_desired, nd.cfl_max,
                nd.redo, nd.cells, nd.tsim, nd.tscale);
    *nd.ticket = 0;
  }
}

// ---------------------------------------------------------------------------
// Sub-cycling (per-level time steps): the kernels around one level's
// substep.  Level l steps with dt 2^-l; the launches of one coarse step run
// coarse to fine (see fcx_advance_subcycled).

// dt of every level from the level-0 step
__global__ void k_level_dts(const double* __restrict__ dt, double* __restrict__ dtl) {
  const int l = threadIdx.x;
  if (l < kLevels) dtl[l] = ldexp(*dt, -l);
}

// Ghost fill of the patches in `list` (one level) at the time of its
// substep: every leaf is read through the level table of tv.
template <typename R, int PHYS>
__global__ void __launch_bounds__(256)
k_ghost_fill_level(const int32_t* __restrict__ list, int32_t n, R* __restrict__ ghost,
                   const PatchRec* __restrict__ rec, int m, int lm, int32_t* err,
                   TimeView<R> tv) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int G = 8 * m + 16;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * G) return;
  const int slot = int(t / G), g = int(t - int64_t(slot) * G);
  const int p = list[slot];
  int i, j;
  ghost_cell(m, g, i, j);
  if ((i == -1 || i == m + 2) && (j == -1 || j == m + 2)) return;
  GhostView<R, MEQN> gv{nullptr, rec, m, lm, err, nullptr, tv};
  R v[MEQN];
  frame_value<R, MEQN, PHYS, true, true>(gv, p, i, j, v);
#pragma unroll
  for (int k = 0; k < MEQN; ++k) ghost[size_t(p * MEQN + k) * G + g] = v[k];
}

// Fine-side terms of one fine substep at the faces of coarse patches of
// level lc (the reflux items whose coarse patch has that level): per fine
// face cell, psi (=, or += when `add`) w [dx_f (f(q_f) - f(q_c)) - phi_f],
// q_f from qf (the fine states at the substep's start), q_c from qc (the
// coarse states at the start of the coarse level's step).
template <typename R, int PHYS>
__global__ void __launch_bounds__(256)
k_psi_accumulate(const R* __restrict__ qc_buf, const R* __restrict__ qf_buf,
                 const RefluxItem* __restrict__ items, const RefluxAux* __restrict__ aux,
                 int32_t nitems, const R* __restrict__ phi, R* __restrict__ psi, int m,
                 KPhys ph, int32_t lc, double w, int32_t add, int32_t* err) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nitems) * m) return;
  const int32_t ii = int32_t(t / m);
  const int tc = int(t % m) + 1;
  const RefluxAux ax = aux[ii];
  if (ax.level != lc) return;
  const RefluxItem it = items[ii];
  const int f = it.face, d = f >> 1, hi = f & 1;
  const int ic = d == 0 ? (hi ? m : 1) : tc, jc = d == 0 ? tc : (hi ? m : 1);
  const int k2 = (tc - 1) / (m / 2);
  const int fp = it.fine[k2], ff = it.fine_face[k2];
  const double dxc = ldexp(1.0, -ax.level) / m;
  R qc[MEQN];
  read_interior<R, MEQN>(qc_buf, m, it.coarse, ic, jc, qc);
  const R* phf = phi + size_t(ax.slot_f[k2]) * 4 * m * MEQN;
  R* psf = psi + size_t(ax.slot_f[k2]) * 4 * m * MEQN;
  for (int s = 0; s < 2; ++s) {
    int pos = 2 * (tc - 1 - k2 * (m / 2)) + 1 + s;
    if (it.fine_rev[k2]) pos = m + 1 - pos;
    const int fi = ff < 2 ? (ff == 0 ? 1 : m) : pos;
    const int fj = ff < 2 ? pos : (ff == 2 ? 1 : m);
    R qf[MEQN], fs[MEQN];
    read_interior<R, MEQN>(qf_buf, m, fp, fi, fj, qf);
    if (hi) fluct_sum<R, PHYS>(ph, d, qc, qf, fs, err);
    else fluct_sum<R, PHYS>(ph, d, qf, qc, fs, err);
#pragma unroll
    for (int k = 0; k < MEQN; ++k) {
      const size_t o = size_t(ff * m + (pos - 1)) * MEQN + k;
      const R v = R(w) * (R(0.5 * dxc) * fs[k] - phf[o]);
      psf[o] = add ? psf[o] + v : v;
    }
  }
}

// Coarse cells of level lc at faces with level lc + 1, after the finer
// level's two substeps: -dt_lc / dx^2 (psi of the two fine cells - phi_c),
// xi corrections first at corner cells (the links of RefluxAux, as in
// k_reflux).
template <typename R, int MEQN>
__device__ __forceinline__ void subcycle_corr(const RefluxItem& it, const RefluxAux& ax,
                                              int tc, const R* __restrict__ phi,
                                              const R* __restrict__ psi, int m,
                                              R (&corr)[MEQN], size_t& o, double& dxc) {
  const int f = it.face, d = f >> 1, hi = f & 1;
  const int ic = d == 0 ? (hi ? m : 1) : tc, jc = d == 0 ? tc : (hi ? m : 1);
  const int k2 = (tc - 1) / (m / 2);
  const int ff = it.fine_face[k2];
  dxc = ldexp(1.0, -ax.level) / m;
  o = (size_t(it.coarse * MEQN) * m + (jc - 1)) * m + (ic - 1);
  const R* phc = phi + size_t(ax.slot_c) * 4 * m * MEQN;
  const R* psf = psi + size_t(ax.slot_f[k2]) * 4 * m * MEQN;
#pragma unroll
  for (int k = 0; k < MEQN; ++k) corr[k] = -phc[(f * m + (tc - 1)) * MEQN + k];
  R fine[MEQN];
#pragma unroll
  for (int k = 0; k < MEQN; ++k) fine[k] = R(0);
  for (int s = 0; s < 2; ++s) {
    int pos = 2 * (tc - 1 - k2 * (m / 2)) + 1 + s;
    if (it.fine_rev[k2]) pos = m + 1 - pos;
#pragma unroll
    for (int k = 0; k < MEQN; ++k) fine[k] += psf[(ff * m + (pos - 1)) * MEQN + k];
  }
#pragma unroll
  for (int k = 0; k < MEQN; ++k) corr[k] = fine[k] + corr[k];
}

template <typename R, int PHYS>
__global__ void __launch_bounds__(256)
k_subcycle_reflux(R* __restrict__ qn, const RefluxItem* __restrict__ items,
                  const RefluxAux* __restrict__ aux, int32_t nitems,
                  const R* __restrict__ phi, const R* __restrict__ psi,
                  const double* __restrict__ dtl, int m, int32_t lc) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nitems) * m) return;
  const int32_t i = int32_t(t / m);
  const int tc = int(t % m) + 1;
  const RefluxAux ax = aux[i];
  if (ax.level != lc) return;
  const RefluxItem it = items[i];
  const int end = tc == 1 ? 0 : (tc == m ? 1 : -1);
  const int32_t link = end >= 0 ? ax.link[end] : -1;
  if (it.face >= 2 && link >= 0) return;
  R c0[MEQN], c1[MEQN];
  size_t o, o1;
  double dxc, dxc1;
  subcycle_corr<R, MEQN>(it, ax, tc, phi, psi, m, c0, o, dxc);
  const bool two = it.face < 2 && link >= 0;
  if (two)
    subcycle_corr<R, MEQN>(items[link], aux[link], it.face == 0 ? 1 : m, phi, psi, m, c1,
                           o1, dxc1);
  const R fac = R(dtl[lc] / (dxc * dxc));
#pragma unroll
  for (int k = 0; k < MEQN; ++k) {
    const size_t ok = o + size_t(k) * m * m;
    R v = qn[ok];
    v -= fac * c0[k];
    if (two) v -= fac * c1[k];
    qn[ok] = v;
  }
}

// ---------------------------------------------------------------------------
// Conservation sums: per-patch FP64 partials in a fixed thread order, then
// a fixed pairwise reduction over patches.
template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_sums_patch(const R* __restrict__ q, const PatchRec* __restrict__ rec,
             int m, double* __restrict__ partial) {
  __shared__ double red[4][MEQN];
  const int p = blockIdx.x, tid = threadIdx.x;
  const double dx = ldexp(1.0, -rec[p].level) / m;
  double acc[MEQN];
#pragma unroll
  for (int k = 0; k < MEQN; ++k) acc[k] = 0.0;
  for (int c = tid; c < m * m; c += 256)
#pragma unroll
    for (int k = 0; k < MEQN; ++k) acc[k] += double(q[size_t(p * MEQN + k) * m * m + c]);
#pragma unroll
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

template <int MEQN>
__global__ void __launch_bounds__(1024)
k_sums_reduce(const double* __restrict__ partial, const int32_t* __restrict__ first,
              double* __restrict__ sums) {
  __shared__ double red[16][MEQN];
  const int f = blockIdx.x, tid = threadIdx.x;
  const int p0 = first[f], p1 = first[f + 1];
  double acc[MEQN];
#pragma unroll
  for (int k = 0; k < MEQN; ++k) acc[k] = 0.0;
  for (int p = p0 + tid; p < p1; p += 1024)
#pragma unroll
    for (int k = 0; k < MEQN; ++k) acc[k] += partial[size_t(p) * MEQN + k];
#pragma unroll
  for (int k = 0; k < MEQN; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid < MEQN) {
    double v[16];
    for (int w = 0; w < 16; ++w) v[w] = red[w][tid];
    for (int s = 8; s > 0; s >>= 1)
      for (int w = 0; w < s; ++w) v[w] = v[w] + v[w + s];
    sums[size_t(f) * MEQN + tid] = v[0];
  }
}

// ---------------------------------------------------------------------------
// Refinement tags.  Decisions are taken on squared quantities with no fused
// multiply-add so that they reproduce an independent FP64 evaluation.  On
// the sphere (geo given) differences are divided by the great-circle
// distance of the cell centres and a parent value is the capacity-weighted
// average of its four children, its centre their normalised sum.
template <typename R, int MEQN>
__device__ __forceinline__ double frame_q0(const R* q, const R* ghost, int m,
                                           int p, int i, int j) {
  if (i >= 1 && i <= m && j >= 1 && j <= m)
    return double(q[size_t(p * MEQN) * m * m + size_t(j - 1) * m + (i - 1)]);
  return double(ghost[size_t(p * MEQN) * (8 * m + 16) + ghost_index(m, i, j)]);
}

template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_tag_refine(const R* __restrict__ q, const R* __restrict__ ghost,
             const PatchRec* __restrict__ rec, int m, int criterion,
             double thr, int lmax, int8_t* __restrict__ tags,
             const double* __restrict__ geo, int8_t* mirror) {
#pragma clang fp contract(off)
  __shared__ double rlo[4], rhi[4];
  __shared__ int rflag[4];
  const int p = blockIdx.x, tid = threadIdx.x;
  const double dx = ldexp(1.0, -rec[p].level) / m;
  double lo = 1e300, hi = -1e300;
  int flag = 0;
  const double t2 = thr * thr;
  for (int c = tid; c < m * m; c += 256) {
    const int i = c % m + 1, j = c / m + 1;
    const double v = frame_q0<R, MEQN>(q, ghost, m, p, i, j);
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    if (criterion == 1) {
      double sx = 2.0 * dx, sy = 2.0 * dx;
      if (geo) {
        double a[3], b[3];
        geo_centre(geo, m, p, i - 1, j, a);
        geo_centre(geo, m, p, i + 1, j, b);
        sx = arc_between(a, b);
        geo_centre(geo, m, p, i, j - 1, a);
        geo_centre(geo, m, p, i, j + 1, b);
        sy = arc_between(a, b);
      }
      const double gx = (frame_q0<R, MEQN>(q, ghost, m, p, i + 1, j) -
                         frame_q0<R, MEQN>(q, ghost, m, p, i - 1, j)) / sx;
      const double gy = (frame_q0<R, MEQN>(q, ghost, m, p, i, j + 1) -
                         frame_q0<R, MEQN>(q, ghost, m, p, i, j - 1)) / sy;
      double s = gx * gx;
      s = s + gy * gy;
      if (s > t2) flag = 1;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    flag |= __shfl_xor(flag, off);
  }
  if ((tid & 63) == 0) { rlo[tid >> 6] = lo; rhi[tid >> 6] = hi; rflag[tid >> 6] = flag; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = fmin(lo, rlo[w]);
      hi = fmax(hi, rhi[w]);
      flag |= rflag[w];
    }
    lo = fmin(lo, rlo[0]);
    hi = fmax(hi, rhi[0]);
    flag |= rflag[0];
    const bool crit = criterion == 0 ? (hi - lo) > thr : flag != 0;
    tags[p] = (crit && rec[p].level < lmax) ? int8_t(1) : int8_t(0);
    if (mirror) mirror[p] = tags[p];
  }
}

// A complete family of leaf siblings whose first child is p coarsens when
// none of its members is tagged +1 and its averaged parent fails the test.
template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_tag_family(const R* __restrict__ q, const PatchRec* __restrict__ rec,
             const int32_t* __restrict__ family, int m, int criterion,
             double thr, int lmin, int8_t* __restrict__ tags,
             const double* __restrict__ geo, int8_t* mirror) {
#pragma clang fp contract(off)
  // m * m averaged parent values, then (sphere) their 3 m * m centres
  extern __shared__ double par[];
  double* pc = par + m * m;
  __shared__ double rlo[4], rhi[4];
  __shared__ int rflag[4];
  const int p = blockIdx.x, tid = threadIdx.x;
  if (!family[p] || rec[p].level <= lmin) return;
  if (tags[p] == 1 || tags[p + 1] == 1 || tags[p + 2] == 1 || tags[p + 3] == 1)
    return;
  const int h = m / 2;
  for (int c = tid; c < m * m; c += 256) {
    const int I = c % m + 1, J = c / m + 1;
    const int kid = p + ((I - 1) >= h) + 2 * ((J - 1) >= h);
    const int ii = 2 * ((I - 1) % h) + 1, jj = 2 * ((J - 1) % h) + 1;
    const R* b = q + size_t(kid * MEQN) * m * m;
    if (geo) {
      double acc = 0.0, w = 0.0, r[3] = {0.0, 0.0, 0.0};
      for (int e = 0; e < 4; ++e) {
        const int i2 = ii + (e & 1), j2 = jj + (e >> 1);
        const double kap = geo_kappa(geo, m, kid, i2, j2);
        acc = acc + kap * double(b[size_t(j2 - 1) * m + (i2 - 1)]);
        w = w + kap;
        double rc[3];
        geo_centre(geo, m, kid, i2, j2, rc);
        r[0] = r[0] + rc[0];
        r[1] = r[1] + rc[1];
        r[2] = r[2] + rc[2];
      }
      par[c] = acc / w;
      const double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      pc[3 * c] = r[0] / nr;
      pc[3 * c + 1] = r[1] / nr;
      pc[3 * c + 2] = r[2] / nr;
    } else {
      double acc = 0.0;
      acc = acc + double(b[size_t(jj - 1) * m + (ii - 1)]);
      acc = acc + double(b[size_t(jj - 1) * m + ii]);
      acc = acc + double(b[size_t(jj) * m + (ii - 1)]);
      acc = acc + double(b[size_t(jj) * m + ii]);
      par[c] = acc / 4.0;
    }
  }
  __syncthreads();
  const double dxp = ldexp(1.0, -(rec[p].level - 1)) / m;
  const double t2 = thr * thr;
  double lo = 1e300, hi = -1e300;
  int flag = 0;
  for (int c = tid; c < m * m; c += 256) {
    const int I = c % m + 1, J = c / m + 1;
    lo = fmin(lo, par[c]);
    hi = fmax(hi, par[c]);
    if (criterion == 1) {
      const int ia = I > 1 ? I - 1 : I, ib = I < m ? I + 1 : I;
      const int ja = J > 1 ? J - 1 : J, jb = J < m ? J + 1 : J;
      double sx = double(ib - ia) * dxp, sy = double(jb - ja) * dxp;
      if (geo) {
        sx = arc_between(&pc[3 * ((J - 1) * m + (ia - 1))], &pc[3 * ((J - 1) * m + (ib - 1))]);
        sy = arc_between(&pc[3 * ((ja - 1) * m + (I - 1))], &pc[3 * ((jb - 1) * m + (I - 1))]);
      }
      const double gx = (par[(J - 1) * m + (ib - 1)] - par[(J - 1) * m + (ia - 1)]) / sx;
      const double gy = (par[(jb - 1) * m + (I - 1)] - par[(ja - 1) * m + (I - 1)]) / sy;
      double s = gx * gx;
      s = s + gy * gy;
      if (s > t2) flag = 1;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    flag |= __shfl_xor(flag, off);
  }
  if ((tid & 63) == 0) { rlo[tid >> 6] = lo; rhi[tid >> 6] = hi; rflag[tid >> 6] = flag; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 0; w < 4; ++w) {
      lo = fmin(lo, rlo[w]);
      hi = fmax(hi, rhi[w]);
      flag |= rflag[w];
    }
    const bool crit = criterion == 0 ? (hi - lo) > thr : flag != 0;
    if (!crit)
      for (int c = 0; c < 4; ++c) {
        tags[p + c] = int8_t(-1);
        if (mirror) mirror[p + c] = int8_t(-1);
      }
  }
}

// ---------------------------------------------------------------------------
// Regrid transfer: one thread per (new patch, cell, component).
template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_transfer(const R* __restrict__ qo, const R* __restrict__ go,
           R* __restrict__ qn, const PatchRec* __restrict__ rec_new,
           const int32_t* __restrict__ kind, const int32_t* __restrict__ src,
           int32_t P, int m) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(MEQN) * m * m;
  if (t >= int64_t(P) * per) return;
  const int p = int(t / per);
  const int rem = int(t - int64_t(p) * per);
  const int k = rem / (m * m), c = rem % (m * m);
  const int i = c % m + 1, j = c / m + 1;
  const int s = src[p];
  const int G = 8 * m + 16;
  auto oval = [&](int pp, int ii, int jj) -> R {
    if (ii >= 1 && ii <= m && jj >= 1 && jj <= m)
      return qo[(size_t(pp * MEQN + k) * m + (jj - 1)) * m + (ii - 1)];
    return go[size_t(pp * MEQN + k) * G + ghost_index(m, ii, jj)];
  };
  R v;
  if (kind[p] == 0) {
    v = oval(s, i, j);
  } else if (kind[p] == 1) {
    const int cx = rec_new[p].ix & 1, cy = rec_new[p].iy & 1;
    const int ic = cx * (m / 2) + (i - 1) / 2 + 1;
    const int jc = cy * (m / 2) + (j - 1) / 2 + 1;
    const R dx = (i & 1) ? R(-0.25) : R(0.25);
    const R dy = (j & 1) ? R(-0.25) : R(0.25);
    const R qc = oval(s, ic, jc);
    const R sx = minmod(oval(s, ic + 1, jc) - qc, qc - oval(s, ic - 1, jc));
    const R sy = minmod(oval(s, ic, jc + 1) - qc, qc - oval(s, ic, jc - 1));
    v = qc + dx * sx + dy * sy;
  } else {
    const int h = m / 2;
    const int kid = s + ((i - 1) >= h) + 2 * ((j - 1) >= h);
    const int ii = 2 * ((i - 1) % h) + 1, jj = 2 * ((j - 1) % h) + 1;
    v = (((oval(kid, ii, jj) + oval(kid, ii + 1, jj)) + oval(kid, ii, jj + 1)) +
         oval(kid, ii + 1, jj + 1)) / R(4);
  }
  qn[size_t(p) * per + rem] = v;
}

// Regrid transfer on the cubed sphere: one thread per (new patch, component,
// 2 x 2 block of cells).  A merged cell is the capacity-weighted average of
// its four old cells; the four children of a refined cell are interpolated as
// on the plane (limited slopes) and then shifted by one common amount so that
// their capacity-weighted sum equals the old cell's content (a coarse cell
// has four times a child's computational area).  Arithmetic in FP64.
template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_transfer_sphere(const R* __restrict__ qo, const R* __restrict__ go,
                  R* __restrict__ qn, const PatchRec* __restrict__ rec_new,
                  const int32_t* __restrict__ kind, const int32_t* __restrict__ src,
                  const double* __restrict__ geo_old, const double* __restrict__ geo_new,
                  int32_t P, int m) {
#pragma clang fp contract(off)
  const int hb = m / 2, nb = hb * hb;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(P) * MEQN * nb) return;
  const int p = int(t / (MEQN * nb));
  const int rem = int(t - int64_t(p) * MEQN * nb);
  const int k = rem / nb, b = rem % nb;
  const int i0 = 2 * (b % hb) + 1, j0 = 2 * (b / hb) + 1;
  const int s = src[p];
  const int G = 8 * m + 16;
  auto oval = [&](int pp, int ii, int jj) -> double {
    if (ii >= 1 && ii <= m && jj >= 1 && jj <= m)
      return double(qo[(size_t(pp * MEQN + k) * m + (jj - 1)) * m + (ii - 1)]);
    return double(go[size_t(pp * MEQN + k) * G + ghost_index(m, ii, jj)]);
  };
  double v[4];
  if (kind[p] == 0) {
    for (int c = 0; c < 4; ++c) v[c] = oval(s, i0 + (c & 1), j0 + (c >> 1));
  } else if (kind[p] == 1) {
    const int cx = rec_new[p].ix & 1, cy = rec_new[p].iy & 1;
    const int ic = cx * hb + (i0 - 1) / 2 + 1, jc = cy * hb + (j0 - 1) / 2 + 1;
    const double qc = oval(s, ic, jc);
    const double sx = minmod(oval(s, ic + 1, jc) - qc, qc - oval(s, ic - 1, jc));
    const double sy = minmod(oval(s, ic, jc + 1) - qc, qc - oval(s, ic, jc - 1));
    double ksum = 0.0, qsum = 0.0;
    for (int c = 0; c < 4; ++c) {
      const double dx = (c & 1) ? 0.25 : -0.25, dy = (c >> 1) ? 0.25 : -0.25;
      v[c] = qc + dx * sx + dy * sy;
      const double kf = geo_kappa(geo_new, m, p, i0 + (c & 1), j0 + (c >> 1));
      ksum = ksum + kf;
      qsum = qsum + kf * v[c];
    }
    const double kc = geo_kappa(geo_old, m, s, ic, jc);
    const double shift = (4.0 * kc * qc - qsum) / ksum;
    for (int c = 0; c < 4; ++c) v[c] = v[c] + shift;
  } else {
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + (c & 1), j = j0 + (c >> 1);
      const int kid = s + ((i - 1) >= hb) + 2 * ((j - 1) >= hb);
      const int ii = 2 * ((i - 1) % hb) + 1, jj = 2 * ((j - 1) % hb) + 1;
      double acc = 0.0, w = 0.0;
      for (int e = 0; e < 4; ++e) {
        const int i2 = ii + (e & 1), j2 = jj + (e >> 1);
        const double kap = geo_kappa(geo_old, m, kid, i2, j2);
        acc = acc + kap * oval(kid, i2, j2);
        w = w + kap;
      }
      v[c] = acc / w;
    }
  }
  for (int c = 0; c < 4; ++c)
    qn[(size_t(p * MEQN + k) * m + (j0 - 1 + (c >> 1))) * m + (i0 - 1 + (c & 1))] = R(v[c]);
}

}  // namespace fcx
