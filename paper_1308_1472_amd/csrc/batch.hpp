// batch.hpp -- many independent forests advanced together: one fused
// ghost-gather + update launch per tile class over the tiles of every forest,
// then per-forest reflux, dt and conservation sums.
//
// Forests keep their own patch size, physics and parameters.  Their patch
// tables are concatenated (neighbour ids are global) and their states are
// concatenated in one buffer; a small per-forest record gives the bases.
// The work items (global patch, tile) of a class all cost the same, so a
// launch has one workgroup per item, with blocks mapped so that each XCD
// takes a contiguous run of items (SFC neighbours then share an L2).
#pragma once

#include "step.hpp"

namespace fcx {

struct ForestDev {
  int32_t m, lm, meqn, physics;
  int32_t patch_base, slot_base, pad0, pad1;
  int64_t state_base, phi_base;            // in elements
  KPhys ph;
};

template <typename R>
struct BatchArgs {
  const R* q;
  R* qn;
  const double* dt;                        // per forest
  double* numax;                           // per forest
  const PatchRec* __restrict__ rec;        // global patch table
  const int32_t* __restrict__ phislot;     // global slots
  const int32_t* __restrict__ pforest;     // forest of every global patch
  const ForestDev* __restrict__ forests;
  R* phi;
  int32_t* err;
  const uint32_t* __restrict__ items;      // (patch << 4) | tile
  int32_t item0, nitems;                   // this class's items
};

// Step arguments of one forest, with base pointers shifted so that global
// patch ids and global phi slots index them directly.
template <typename R>
__device__ __forceinline__ StepArgs<R> forest_args(const BatchArgs<R>& B, int f,
                                                   const ForestDev& F) {
  StepArgs<R> A;
  const int64_t per = int64_t(F.meqn) << (2 * F.lm);
  A.q = B.q + (F.state_base - int64_t(F.patch_base) * per);
  A.qn = B.qn + (F.state_base - int64_t(F.patch_base) * per);
  A.ghost = nullptr;
  A.dt = B.dt + f;
  A.numax = B.numax + f;
  A.rec = B.rec;
  A.phislot = B.phislot;
  A.phi = B.phi + (F.phi_base - int64_t(F.slot_base) * 4 * F.m * F.meqn);
  A.err = B.err;
  A.P = 0;
  A.m = F.m;
  A.lm = F.lm;
  A.ntiles = 0;
  A.ph = F.ph;
  return A;
}

// One workgroup per work item of one class (tile size and physics).  Each
// tile keeps its registers to itself: a persistent form of this kernel, whose
// loop over items kept the per-item state live across tiles, needed 128
// registers per thread against 71 here and ran the batch a third slower.
template <typename R, int PHYS, int T, int NT>
__global__ void __launch_bounds__(NT)
k_batch_step(BatchArgs<R> B) {
  __shared__ TileLds<R, PHYS, T, NT> lds;
  const int it = B.item0 + xcd_tile(blockIdx.x, B.nitems);
  const uint32_t w = B.items[it];
  const int p = int(w >> 4), tile = int(w & 15);
  const int f = B.pforest[p];
  const ForestDev F = B.forests[f];
  const StepArgs<R> A = forest_args(B, f, F);
  const int tps = F.m / T;
  tile_step<R, PHYS, T, NT, true>(A, p, tile % tps, tile / tps, lds);
}

// Reflux of a batch: one thread per (coarse-fine face item, coarse cell);
// items are grouped by forest, 32 threads per item.
template <typename R>
__global__ void __launch_bounds__(256)
k_batch_reflux(const R* q, R* qn, const RefluxItem* __restrict__ items,
               const int32_t* __restrict__ item_forest, int32_t nitems,
               const PatchRec* __restrict__ rec, const int32_t* __restrict__ phislot,
               const ForestDev* __restrict__ forests, const R* phi,
               const double* dt, int32_t* err) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nitems) * 32) return;
  const int ii = int(t >> 5), tc = int(t & 31) + 1;
  const int f = item_forest[ii];
  const ForestDev F = forests[f];
  const int m = F.m;
  if (tc > m) return;
  const RefluxItem it = items[ii];
  const int64_t per = int64_t(F.meqn) << (2 * F.lm);
  const R* qf = q + (F.state_base - int64_t(F.patch_base) * per);
  R* qnf = qn + (F.state_base - int64_t(F.patch_base) * per);
  const R* phf = phi + (F.phi_base - int64_t(F.slot_base) * 4 * m * F.meqn);
  const int fc = it.face, d = fc >> 1, hi = fc & 1, C = it.coarse;
  const int ic = d == 0 ? (hi ? m : 1) : tc, jc = d == 0 ? tc : (hi ? m : 1);
  const int k2 = (tc - 1) / (m / 2);
  const int fp = it.fine[k2], ff = it.fine_face[k2];
  const double dxc = ldexp(1.0, -rec[C].level) / m;
  R qc[3], corr[3] = {0, 0, 0};
  const int meqn = F.meqn;
  for (int k = 0; k < meqn; ++k)
    qc[k] = qf[(size_t(C * meqn + k) * m + (jc - 1)) * m + (ic - 1)];
  const R* pf = phf + size_t(phislot[fp]) * 4 * m * meqn;
  for (int s = 0; s < 2; ++s) {
    int pos = 2 * (tc - 1 - k2 * (m / 2)) + 1 + s;
    if (it.fine_rev[k2]) pos = m + 1 - pos;
    const int fi = ff < 2 ? (ff == 0 ? 1 : m) : pos;
    const int fj = ff < 2 ? pos : (ff == 2 ? 1 : m);
    R qv[3], fs[3];
    for (int k = 0; k < meqn; ++k)
      qv[k] = qf[(size_t(fp * meqn + k) * m + (fj - 1)) * m + (fi - 1)];
    if (F.physics == FCX_ADVECTION) {
      if (hi) fluct_sum<R, FCX_ADVECTION>(F.ph, d, qc, qv, fs, err);
      else fluct_sum<R, FCX_ADVECTION>(F.ph, d, qv, qc, fs, err);
    } else {
      if (hi) fluct_sum<R, FCX_SHALLOW>(F.ph, d, qc, qv, fs, err);
      else fluct_sum<R, FCX_SHALLOW>(F.ph, d, qv, qc, fs, err);
    }
    for (int k = 0; k < meqn; ++k)
      corr[k] += R(0.5 * dxc) * fs[k] - pf[(ff * m + (pos - 1)) * meqn + k];
  }
  const R* pc = phf + size_t(phislot[C]) * 4 * m * meqn;
  const R fac = R(dt[f] / (dxc * dxc));
  for (int k = 0; k < meqn; ++k)
    qnf[(size_t(C * meqn + k) * m + (jc - 1)) * m + (ic - 1)] -=
        fac * (corr[k] - pc[(fc * m + (tc - 1)) * meqn + k]);
}

// Per-patch FP64 partial sums (stride 4) of a batch, fixed thread order.
template <typename R>
__global__ void __launch_bounds__(256)
k_batch_sums_patch(const R* q, const PatchRec* __restrict__ rec,
                   const int32_t* __restrict__ pforest,
                   const ForestDev* __restrict__ forests, double* partial) {
  __shared__ double red[4][4];
  const int p = blockIdx.x, tid = threadIdx.x;
  const ForestDev F = forests[pforest[p]];
  const int m = F.m, meqn = F.meqn;
  const int64_t per = int64_t(meqn) << (2 * F.lm);
  const R* qf = q + (F.state_base - int64_t(F.patch_base) * per) + int64_t(p) * per;
  const double dx = ldexp(1.0, -rec[p].level) / m;
  double acc[4] = {0, 0, 0, 0};
  for (int c = tid; c < m * m; c += 256)
    for (int k = 0; k < meqn; ++k) acc[k] += double(qf[size_t(k) * m * m + c]);
  for (int k = 0; k < 4; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) red[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid < 4)
    partial[size_t(p) * 4 + tid] =
        ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) * dx * dx;
}

}  // namespace fcx
