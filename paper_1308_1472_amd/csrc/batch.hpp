// batch.hpp -- many independent forests advanced together: one fused
// ghost-gather + update launch per tile class over the tiles of every forest,
// then per-forest reflux, dt and conservation sums.
//
// Forests keep their own patch size, physics and parameters.  Their patch
// tables are concatenated (neighbour ids are global) and their states are
// concatenated in one buffer; a small per-forest record gives the bases.
// The work items (global patch, tile) of a class all cost the same.  A launch
// either has one workgroup per item, with blocks mapped so that each XCD
// takes a contiguous run of items (SFC neighbours then share an L2), or is
// persistent: resident workgroups take items from per-XCD ranges through
// atomic counters and steal from other XCDs' ranges once their own is spent.
// The autotuner picks the form.
#pragma once

#include <cstddef>

#include "advect.hpp"
#include "aux_kernels.hpp"

namespace fcx {

struct ForestDev {
  int32_t m, lm, meqn, physics;
  int32_t patch_base, slot_base, pad0, pad1;
  int64_t state_base, phi_base;            // in elements
  KPhys ph;
};

// One work item: a tile of a patch, with what its loads need (the patch's
// state offset and size) so that they can be issued as soon as the item is
// read; the forest's record is read beside them.
struct alignas(16) BatchItem {
  int32_t patch;                           // global patch id
  uint32_t qoff;                           // patch's state offset, in elements
  int32_t slot;                            // global face-term slot, -1: none
  int32_t info;                            // tile column | row << 4 | log2(m) << 8
                                           // | forest << 12
  __device__ __host__ int tx() const { return info & 15; }
  __device__ __host__ int ty() const { return (info >> 4) & 15; }
  __device__ __host__ int lm() const { return (info >> 8) & 15; }
  __device__ __host__ int forest() const { return info >> 12; }
};

// A work item of an advection class with the tile's halo offsets formed
// when the batch is built (velocity signs and neighbours are fixed then).
constexpr int32_t kAdvReports = 1 << 10;
struct alignas(16) AdvItem {
  BatchItem h;
  AdvHalo halo;                            // simple-halo patches only
  int32_t aux;                             // patch level | x mirror << 8 | y mirror << 9
                                           // | kAdvReports: the item that
                                           // reports its forest's Courant number
  __device__ __host__ int level() const { return aux & 255; }
  __device__ __host__ int mirror() const { return (aux >> 8) & 3; }
};
static_assert(sizeof(AdvItem) == 64, "an advection work item is 16 dwords");

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
  int32_t* err;                            // per forest
  const BatchItem* __restrict__ items;
  const AdvItem* __restrict__ advitems;    // the same items with halo offsets
  int32_t item0, nitems;                   // this class's items
  const int32_t* __restrict__ range;       // persistent: [9] item range of each XCD
  int32_t* counters;                       //   and [8 * kCounterStride] counters, zero at launch
};

// Step arguments of one work item: base pointers shifted so that global
// patch ids and global phi slots index them directly.
template <typename R, int MEQN>
__device__ __forceinline__ StepArgs<R> item_args(const BatchArgs<R>& B, const BatchItem& w) {
  StepArgs<R> A;
  const int f = w.forest(), lm = w.lm(), m = 1 << lm;
  const int64_t shift = int64_t(w.qoff) - (int64_t(w.patch) * MEQN << (2 * lm));
  A.q = B.q + shift;
  A.qn = B.qn + shift;
  A.ghost = nullptr;
  A.dt = B.dt + f;
  A.numax = B.numax + f;
  A.rec = B.rec;
  A.phislot = B.phislot;
  const ForestDev& F = B.forests[f];
  A.phi = B.phi + (F.phi_base - int64_t(F.slot_base) * 4 * m * MEQN);
  A.err = B.err + f;
  A.P = 0;
  A.m = m;
  A.lm = lm;
  A.ntiles = 0;
  A.ph = F.ph;
  return A;
}

// one work counter per XCD, each on a cache line of its own
constexpr int kCounterStride = 32;

// One workgroup per work item of one class (tile size and physics).
template <typename R, int PHYS, int T, int NT, int SPEC>
__global__ void __launch_bounds__(NT)
k_batch_step(BatchArgs<R> B) {
  __shared__ TileLds<R, PHYS, T, NT> lds;
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int it = B.item0 + xcd_tile(blockIdx.x, B.nitems);
  const BatchItem w = B.items[it];
  const StepArgs<R> A = item_args<R, MEQN>(B, w);
  tile_step<R, PHYS, T, NT, true, SPEC>(A, w.patch, w.tx(), w.ty(), lds);
}

// Persistent launch over the work items of one class.  Thread 0 takes items
// through its XCD's counter (stealing from the other XCDs once its own range
// is spent); the ticket for the next item is drawn before the current tile is
// processed, so the atomic's latency overlaps the tile's loads.  The thread
// index is hidden from the optimizer per item: otherwise the index arithmetic
// derived from it is hoisted out of the loop and held in registers across
// tiles (128 registers per thread under a four-wave cap, against 87 so).
template <typename R, int PHYS, int T, int NT, int SPEC>
__global__ void __launch_bounds__(NT)
k_batch_persist(BatchArgs<R> B) {
  __shared__ TileLds<R, PHYS, T, NT> lds;
  __shared__ int item_sh;
  int x = blockIdx.x & 7, tries = 0;
  // resolve a ticket k drawn on counter x into an item, stealing when the
  // range of x is spent; -1 once every range is
  auto resolve = [&](int k) -> int {
    for (;;) {
      if (B.range[x] + k < B.range[x + 1]) return B.range[x] + k;
      if (++tries >= 8) return -1;
      x = (x + 1) & 7;
      k = atomicAdd(&B.counters[x * kCounterStride], 1);
    }
  };
  if (threadIdx.x == 0) item_sh = resolve(atomicAdd(&B.counters[x * kCounterStride], 1));
  __syncthreads();
  for (;;) {
    const int it = __builtin_amdgcn_readfirstlane(item_sh);
    if (it < 0) break;
    int ticket = 0;
    if (threadIdx.x == 0 && tries < 8) ticket = atomicAdd(&B.counters[x * kCounterStride], 1);
    BatchItem w;
    w.patch = __builtin_amdgcn_readfirstlane(B.items[it].patch);
    w.qoff = __builtin_amdgcn_readfirstlane(B.items[it].qoff);
    w.slot = __builtin_amdgcn_readfirstlane(B.items[it].slot);
    w.info = __builtin_amdgcn_readfirstlane(B.items[it].info);
    const StepArgs<R> A = item_args<R, PhysTraits<PHYS>::MEQN>(B, w);
    int tid = int(threadIdx.x);
    asm volatile("" : "+v"(tid));
    tile_step<R, PHYS, T, NT, true, SPEC>(A, w.patch, w.tx(), w.ty(), lds, tid);
    __syncthreads();                     // item_sh and the tile's LDS are free
    if (threadIdx.x == 0) item_sh = tries < 8 ? resolve(ticket) : -1;
    __syncthreads();
  }
}

// Advection: one wavefront per work item, kAdvWaves items per workgroup.
// The items of a class are ordered patches with a simple halo first; the
// two runs are separate launches (HALO kHaloStrips, kHaloGeneral), so that
// the simple tiles' kernel carries none of the general gather.  SPEC: 1 when
// every forest of the class uses the MC limiter and transverse mode 2
// (fixed when compiling), else 0.
template <typename R, int T, int HALO, int SPEC>
__global__ void __launch_bounds__(64 * kAdvWaves, 8)
k_batch_adv(BatchArgs<R> B) {
  __shared__ AdvLds<R, T> lds[kAdvWaves];
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int k = adv_slot(B.nitems, wv);
  if (k >= B.nitems) return;
  const AdvItem& ai = B.advitems[B.item0 + k];
  const BatchItem w = ai.h;
  const StepArgs<R> A = item_args<R, 1>(B, w);
  adv_tile_step<R, T, HALO, SPEC ? 4 : -1, SPEC ? 2 : -1>(
      A, w.patch, w.slot, w.tx(), w.ty(), lds[wv], int(threadIdx.x) & 63,
      HALO == kHaloStrips ? &ai.halo : nullptr);
}

// Strip-halo items walked by resident wavefronts: wavefront w of W takes
// items w, w + W, w + 2W, ... (consecutive wavefronts on one XCD), so that
// the tiles in flight at any time are a compact window of the item order
// (neighbours in space-filling-curve order) and share their halo cells in
// the L2.  The loads of the next item are issued before the current item is
// computed, so that one tile's memory latency overlaps the arithmetic of
// the one before.  Whatever an item needs beside its cells arrives by
// vector loads, one dword per lane: its 16 dwords two items ahead (the halo
// offsets stay there and each lane takes its own by a lane permute), its
// forest's record and time step with its cells; so no wait for the current
// tile's values waits on the scalar cache or on the next tile.  A forest's
// Courant number is the same on all its tiles of one level: one item per
// forest, of its finest level, reports it.
// Resident workgroups per CU a launch is sized for (the register budget:
// two tiles' values live at once).
template <typename R, int T>
struct AdvRunBlocks {
  static constexpr int value = T == 8 ? 6 : (sizeof(R) == 4 ? 4 : 3);
};
template <typename R, int T, int SPEC>
__global__ void __launch_bounds__(64 * kAdvWaves, (AdvRunBlocks<R, T>::value))
k_batch_adv_run(BatchArgs<R> B) {
  constexpr int FW = int(sizeof(ForestDev)) / 4;       // dwords of a forest record
  static_assert(sizeof(ForestDev) % 8 == 0 && FW + 2 <= 64, "forest record layout");
  static_assert(sizeof(AdvItem) == 64 && offsetof(AdvItem, halo) % 4 == 0, "item layout");
  __shared__ AdvLds<R, T> lds[kAdvWaves];
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = int(threadIdx.x) & 63;
  const int nw = int(gridDim.x) * kAdvWaves;
  const int n = B.nitems;
  int it = xcd_tile(blockIdx.x, int(gridDim.x)) * kAdvWaves + wv;
  if (it >= n) return;
  const int32_t* words = reinterpret_cast<const int32_t*>(B.advitems + B.item0);
  // (every lane loads, none under a branch: a wait for one item's values
  // then never counts on a load that may not have been issued; past the
  // walk's end the current item is read again, not used)
  auto fetch = [&](int k, int cur) {
    return words[size_t(k < n ? k : cur) * 16 + (lane & 15)];
  };
  struct Item {
    BatchItem w;
    int aux;
    int32_t fw;                            // lane k < FW: dword k of the forest record;
  };                                       // FW, FW + 1: its time step
  // an item from its dwords (uniform values), and the issue of its loads
  auto start = [&](int32_t d, Item& c, AdvRegs<R, T>& g) {
    c.w.patch = __builtin_amdgcn_readlane(d, 0);
    c.w.qoff = uint32_t(__builtin_amdgcn_readlane(d, 1));
    c.w.slot = __builtin_amdgcn_readlane(d, 2);
    c.w.info = __builtin_amdgcn_readlane(d, 3);
    c.aux = __builtin_amdgcn_readlane(d, offsetof(AdvItem, aux) / 4);
    StepArgs<R> A{};
    const int lm = c.w.lm();
    A.rec = B.rec;
    A.q = B.q + (int64_t(c.w.qoff) - (int64_t(c.w.patch) << (2 * lm)));
    A.m = 1 << lm;
    A.lm = lm;
    adv_tile_load<R, T, kHaloStripWords>(A, c.w.patch, c.w.tx(), c.w.ty(), lane, nullptr, g,
                                         (c.aux >> 8) & 3, d, offsetof(AdvItem, halo) / 4);
    const int f = c.w.forest();
    const int32_t* fr = reinterpret_cast<const int32_t*>(B.forests + f);
    const int32_t* dr = reinterpret_cast<const int32_t*>(B.dt + f);
    c.fw = *(lane < FW ? fr + lane : dr + (lane - FW < 2 ? lane - FW : 1));
  };
  auto word2 = [&](int32_t v, int k) {
    return (int64_t(uint32_t(__builtin_amdgcn_readlane(v, k + 1))) << 32) |
           uint32_t(__builtin_amdgcn_readlane(v, k));
  };
  const int32_t d0 = fetch(it, it);
  int32_t d1 = fetch(it + nw, it);        // the dwords of item it + W
  // one item: issue the next item's loads (into nxt, gn), then compute this
  // one (cur, g); false once the walk ends.  The loop below alternates the
  // two register sets, so that no loaded value is copied between them (a
  // copy would wait for its load).
  auto item = [&](const Item& cur, const AdvRegs<R, T>& g, Item& nxt,
                  AdvRegs<R, T>& gn) -> bool {
    const bool more = it + nw < n;
    const int32_t d2 = fetch(it + 2 * nw, more ? it + nw : it);
    start(d1, nxt, gn);
    d1 = d2;
    // this item's arguments from its forest's record
    constexpr int PH = offsetof(ForestDev, ph) / 4;
    StepArgs<R> A{};
    const int lm = cur.w.lm(), m = 1 << lm;
    A.qn = B.qn + (int64_t(cur.w.qoff) - (int64_t(cur.w.patch) << (2 * lm)));
    const int64_t phi_base = word2(cur.fw, offsetof(ForestDev, phi_base) / 4);
    const int32_t slot_base =
        __builtin_amdgcn_readlane(cur.fw, offsetof(ForestDev, slot_base) / 4);
    A.phi = B.phi + (phi_base - int64_t(slot_base) * 4 * m);
    A.m = m;
    A.lm = lm;
    A.ph.ax = __longlong_as_double(word2(cur.fw, PH + offsetof(KPhys, ax) / 4));
    A.ph.ay = __longlong_as_double(word2(cur.fw, PH + offsetof(KPhys, ay) / 4));
    A.ph.limiter = __builtin_amdgcn_readlane(cur.fw, PH + offsetof(KPhys, limiter) / 4);
    A.ph.transverse = __builtin_amdgcn_readlane(cur.fw, PH + offsetof(KPhys, transverse) / 4);
    const double dt = __longlong_as_double(word2(cur.fw, FW));
    const double nu = adv_tile_rest<R, T, SPEC ? 4 : -1, SPEC ? 2 : -1, false>(
        A, cur.w.patch, cur.w.slot, cur.w.tx(), cur.w.ty(), lds[wv], lane, g,
        cur.aux & 255, dt);
    if ((cur.aux & kAdvReports) && lane == 0) atomic_max_pos(B.numax + cur.w.forest(), nu);
    wave_sync();                           // the tile's LDS is free
    it += nw;
    return more;
  };
  Item ia, ib;
  AdvRegs<R, T> ga, gb;
  start(d0, ia, ga);
  while (item(ia, ga, ib, gb) && item(ib, gb, ia, ga)) {
  }
}

// Persistent form: every wavefront takes items on its own, through the
// counter of its XCD (stealing from the other XCDs' ranges once its own is
// spent), until every range is spent.
template <typename R, int T, int SPEC>
__global__ void __launch_bounds__(64 * kAdvWaves, 8)
k_batch_adv_persist(BatchArgs<R> B) {
  __shared__ AdvLds<R, T> lds[kAdvWaves];
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = int(threadIdx.x) & 63;
  int x = blockIdx.x & 7, tries = 0;
  for (;;) {
    int it = -1;
    while (tries < 8) {
      int k = 0;
      if (lane == 0) k = atomicAdd(&B.counters[x * kCounterStride], 1);
      k = __builtin_amdgcn_readfirstlane(k);
      if (B.range[x] + k < B.range[x + 1]) { it = B.range[x] + k; break; }
      ++tries;
      x = (x + 1) & 7;
    }
    if (it < 0) break;
    BatchItem w;
    w.patch = __builtin_amdgcn_readfirstlane(B.items[it].patch);
    w.qoff = __builtin_amdgcn_readfirstlane(B.items[it].qoff);
    w.slot = __builtin_amdgcn_readfirstlane(B.items[it].slot);
    w.info = __builtin_amdgcn_readfirstlane(B.items[it].info);
    const StepArgs<R> A = item_args<R, 1>(B, w);
    int l = lane;
    asm volatile("" : "+v"(l));
    adv_tile_step<R, T, kHaloAny, SPEC ? 4 : -1, SPEC ? 2 : -1>(A, w.patch, w.slot, w.tx(),
                                                               w.ty(), lds[wv], l);
    wave_sync();                           // the tile's LDS is free
  }
}

__global__ void k_zero_i32(int32_t* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Reflux of a batch: one thread per (coarse-fine face item, coarse cell);
// items are grouped by forest, 32 threads per item.  Items of a forest whose
// attempt the CFL rule rejects are skipped (its state is restored by
// k_batch_next_dt).
template <typename R>
__global__ void __launch_bounds__(256)
k_batch_reflux(const R* q, R* qn, const RefluxItem* __restrict__ items,
               const int32_t* __restrict__ item_forest, int32_t nitems,
               const PatchRec* __restrict__ rec, const int32_t* __restrict__ phislot,
               const ForestDev* __restrict__ forests, const R* phi,
               const double* dt, int32_t* err, const double* numax, double cfl_max,
               int32_t redo) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nitems) * 32) return;
  const int ii = int(t >> 5), tc = int(t & 31) + 1;
  const int f = item_forest[ii];
  if (rejected(numax, f, cfl_max, redo)) return;
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
  int32_t* ef = err + f;
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
      if (hi) fluct_sum<R, FCX_ADVECTION>(F.ph, d, qc, qv, fs, ef);
      else fluct_sum<R, FCX_ADVECTION>(F.ph, d, qv, qc, fs, ef);
    } else {
      if (hi) fluct_sum<R, FCX_SHALLOW>(F.ph, d, qc, qv, fs, ef);
      else fluct_sum<R, FCX_SHALLOW>(F.ph, d, qv, qc, fs, ef);
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

// Per-forest CFL check and next dt of a batch: kBatchRedoParts workgroups
// per forest copy their shares of a rejected forest's q into q_new; the last
// workgroup to finish takes the next dt of every forest.
constexpr int kBatchRedoParts = 8;

template <typename R>
__global__ void __launch_bounds__(256)
k_batch_next_dt(const R* q, R* qn, const ForestDev* __restrict__ forests,
                const int32_t* __restrict__ first, int32_t nforest, NextDtArgs nd,
                int32_t* err) {
  const int f = blockIdx.x / kBatchRedoParts, part = blockIdx.x % kBatchRedoParts;
  if (f < nforest && rejected(nd.numax, f, nd.cfl_max, nd.redo)) {
    const ForestDev F = forests[f];
    const int64_t elems = int64_t(first[f + 1] - first[f]) * F.meqn * F.m * F.m;
    const int64_t units = elems * int64_t(sizeof(R)) / 16;
    copy_share(reinterpret_cast<const uint4*>(q + F.state_base),
               reinterpret_cast<uint4*>(qn + F.state_base), units, part, kBatchRedoParts);
  }
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(nd.ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  for (int g = threadIdx.x; g < nforest; g += blockDim.x) {
    const ForestDev F = forests[g];
    const int64_t cells = int64_t(first[g + 1] - first[g]) * F.m * F.m;
    next_dt_one(nd.numax, nd.dt, nd.status, err, nd.stats, g, nd.cfl_desired, nd.cfl_max,
                nd.redo, cells);
  }
  __syncthreads();
  if (threadIdx.x == 0) *nd.ticket = 0;
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
