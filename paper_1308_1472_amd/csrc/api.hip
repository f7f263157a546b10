// api.hip -- the C ABI of libfcx.so (declared in include/fcx.h): context,
// forest upload, and the launches of the ghost-fill, patch-step, reflux,
// dt, sum, tag and transfer kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "advect.hpp"
#include "aux_kernels.hpp"
#include "batch.hpp"
#include "forest.hpp"
#include "mlp.hpp"
#include "sphere.hpp"
#include "step.hpp"

using namespace fcx;

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(FCX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Owning device buffer: movable, not copyable.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t ensure(size_t count) {
    if (count <= n && p) return hipSuccess;
    // grow geometrically, from at least 256 KiB, so that a mesh that grows
    // step by step does not reallocate (and synchronize) at every regrid
    const size_t c = std::max({count, 2 * n, (size_t(256) << 10) / sizeof(T) + 1});
    release();
    hipError_t e = hipMalloc(&p, c * sizeof(T));
    if (e == hipSuccess) n = c;
    return e;
  }
  hipError_t upload(const std::vector<T>& v) {
    hipError_t e = ensure(v.size());
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  }
};

int log2i(int m) {
  int l = 0;
  while ((1 << l) < m) ++l;
  return l;
}
}  // namespace

// Pinned host staging buffer (grows, never shrinks).
struct HostBuf {
  uint8_t* p = nullptr;
  size_t n = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() { if (p) (void)hipHostFree(p); }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    // pinned allocations are slow: grow by doubling, from 1 MiB
    const size_t c = std::max({bytes, 2 * n, size_t(1) << 20});
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p), c, hipHostMallocDefault);
    n = e == hipSuccess ? c : 0;
    return e;
  }
};

// Device copy of one forest's plan: every array lives in one allocation and
// arrives in one copy.
struct DevForest {
  DevBuf<uint8_t> blob;
  PatchRec* rec = nullptr;
  int32_t* phislot = nullptr;
  int32_t* family = nullptr;
  RefluxItem* reflux = nullptr;
  RefluxAux* aux = nullptr;          // per reflux item: partners, slots, level
  int32_t* counts = nullptr;         // {slots, xi items, eta items} on the device
  int32_t* order = nullptr;          // dispatch order of the step's tiles (null: identity)
  int32_t* bylevel = nullptr;        // patch ids sorted by level (stable)
  std::vector<int32_t> level_first;  // host: level l's ids at [first[l], first[l+1])
  int32_t* first = nullptr;          // {0, P} for the sum reduction
  int32_t* xkind = nullptr;          // transfer plan from the previous forest
  int32_t* xsrc = nullptr;
  int32_t n_reflux_x = 0, n_reflux_y = 0;
  int32_t nslots = 0;
  int64_t P = 0;
  DevBuf<double> geo;                // sphere: per-patch geometry tables
  DevBuf<float> geo32;               //   and, for FP32 state, edges and centres in FP32
  DevBuf<double> flux;               // FCX_ROTATION: the edge fluxes of every patch
};

struct fcx_ctx {
  fcx_config cfg{};
  int meqn = 1;
  int tile = 16;
  std::vector<fcx_tree> trees;
  Forest forest, old_forest;
  bool have_forest = false, have_old = false;
  DevForest cur, old;
  DevBuf<uint8_t> phi;             // face terms of the last patch step
  DevBuf<double> partial;
  DevBuf<int32_t> err;
  DevBuf<uint32_t> ticket;         // last-workgroup ticket of the reflux
  DevBuf<int64_t> stats;           // {accepted steps, rejected attempts, accepted cells}
  DevBuf<double> tsim;             // simulated time of the accepted steps
  DevBuf<uint8_t> psi;             // sub-cycling: fine-side terms per face-term slot
  DevBuf<double> dtl;              //   dt of every level
  DevBuf<LevelSrc> tables;         //   per launch of a coarse step: where levels are read
  int sub_lmin = -1, sub_lmax = -1; //   the level range the tables are for
  HostBuf sub_host;                //   pinned staging of the tables
  DevBuf<uint8_t> sub_work;        //   fcx_run: the work buffer of sub-cycled steps
  HostBuf run_host;                // fcx_run: pinned copies of stats
  HostBuf staging;
  int cus = 256;
  bool threads_auto = false;         // threads per tile left to the library
  bool pillow = false;               // sphere of two trees (else the cube's six)
  int device = 0;                  // the HIP device the context was created on
  size_t lds_per_block = 65536;    // device limit of LDS per workgroup
  Plan plan;                       // host copy of the current forest's plan
  Plan spare;                      // the previous one, its storage reused
  DevBuf<int8_t> tags_dev;         // fcx_regrid: tags on the device
  HostBuf tags_host;               //   and their pinned host copy
  hipEvent_t staged = nullptr;     // end of the last stream-ordered plan upload
  bool staged_pending = false;     //   from `staging`, not yet waited for
  hipEvent_t tags_ready = nullptr; // the tags of a regrid are on the host
  ~fcx_ctx() {
    if (staged) {
      (void)hipEventSynchronize(staged);
      (void)hipEventDestroy(staged);
    }
    if (tags_ready) (void)hipEventDestroy(tags_ready);
  }
};

// Cube faces as (centre, u, v) axis vectors, the same frames as the device
// mapping of sphere.hpp.
static const int kCubeAxes[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},  {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}}, {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {0, 1, 0}, {-1, 0, 0}}, {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

// 1 if the connectivity glues the six cube faces as the cube does: the two
// end points of every glued face coincide, in the stated orientation.
static bool cube_connectivity(const std::vector<fcx_tree>& t) {
  if (t.size() != 6) return false;
  auto ends = [](int tree, int f, int pt[2][3]) {
    const int a = f / 2, s = f % 2;
    for (int e = 0; e < 2; ++e) {
      const int xi = a == 0 ? s : e, eta = a == 0 ? e : s;
      for (int c = 0; c < 3; ++c)
        pt[e][c] = kCubeAxes[tree][0][c] + (2 * xi - 1) * kCubeAxes[tree][1][c] +
                   (2 * eta - 1) * kCubeAxes[tree][2][c];
    }
  };
  for (int tr = 0; tr < 6; ++tr)
    for (int f = 0; f < 4; ++f) {
      const fcx_tree& T = t[tr];
      if (T.bc[f] != 0) return false;
      int a[2][3], b[2][3];
      ends(tr, f, a);
      ends(T.nbr_tree[f], T.nbr_face[f], b);
      const int o = T.orient[f];
      for (int e = 0; e < 2; ++e)
        for (int c = 0; c < 3; ++c)
          if (a[e][c] != b[o ? 1 - e : e][c]) return false;
    }
  return true;
}

// The two trees glued as the pillow sphere (each tree a hemisphere): faces
// 0 and 1 meet their namesakes reversed, face 2 meets face 3 and face 3
// face 2 the same way.
static bool pillow_connectivity(const std::vector<fcx_tree>& t) {
  if (t.size() != 2) return false;
  static const int nf[4] = {0, 1, 3, 2}, orr[4] = {1, 1, 0, 0};
  for (int tr = 0; tr < 2; ++tr)
    for (int f = 0; f < 4; ++f)
      if (t[tr].bc[f] != 0 || t[tr].nbr_tree[f] != 1 - tr || t[tr].nbr_face[f] != nf[f] ||
          t[tr].orient[f] != orr[f])
        return false;
  return true;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free conservation sums: the per-patch FP64
// partials of fcx_conservation_sums_noalloc live in this file-scope device
// array (8 MiB on every device the library runs on, held until the process
// ends).  Host code never passes the array's name to a kernel: each device's
// copy has its own address, resolved once per device (at fcx_create, with
// that device current) and kept in g_scratch.
constexpr int64_t kNoAllocPartials = int64_t(1) << 20;
static __device__ __align__(256) double scratch[kNoAllocPartials];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

static int resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FCX_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return FCX_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(FCX_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[dev] = static_cast<double*>(ptr);
  return FCX_OK;
}

static double* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
}

// The entry points below are declared extern "C" in fcx.h.

const char* fcx_last_error(void) { return g_err.c_str(); }
int32_t fcx_version(void) { return 1; }

int fcx_sfc_sort(int64_t n, fcx_leaf* leaves) {
  if (n < 0 || (n > 0 && !leaves)) return fail(FCX_EINVAL, "bad arguments");
  std::vector<fcx_leaf> v(leaves, leaves + n);
  sort_leaves(v);
  std::copy(v.begin(), v.end(), leaves);
  return FCX_OK;
}

int fcx_balance(int32_t n_trees, const fcx_tree* trees, int64_t n,
                const fcx_leaf* in, int64_t cap, fcx_leaf* out,
                int64_t* n_out) {
  if (n_trees <= 0 || !trees || n < 0 || (n > 0 && !in) || !n_out)
    return fail(FCX_EINVAL, "bad arguments");
  std::vector<fcx_tree> t(trees, trees + n_trees);
  std::vector<fcx_leaf> res;
  std::string err;
  const int rc = balance(t, std::vector<fcx_leaf>(in, in + n), res, err);
  if (rc != FCX_OK) return fail(rc, err);
  *n_out = int64_t(res.size());
  if (int64_t(res.size()) > cap || (!out && !res.empty()))
    return fail(FCX_EINVAL, "output capacity too small");
  std::copy(res.begin(), res.end(), out);
  return FCX_OK;
}

int fcx_regrid_leaves(int32_t n_trees, const fcx_tree* trees, int64_t n,
                      const fcx_leaf* leaves, const int8_t* tags, int32_t lmin,
                      int32_t lmax, int64_t cap, fcx_leaf* out, int64_t* n_out) {
  if (n_trees <= 0 || !trees || n <= 0 || !leaves || !tags || !n_out ||
      lmin < 0 || lmax < lmin || lmax > kMaxLevel)
    return fail(FCX_EINVAL, "bad arguments");
  std::vector<fcx_tree> t(trees, trees + n_trees);
  std::string err;
  Forest f;
  int rc = f.assign(t, std::vector<fcx_leaf>(leaves, leaves + n), err);
  if (rc != FCX_OK) return fail(rc, err);
  std::vector<fcx_leaf> res;
  rc = regrid(f, tags, lmin, lmax, res, err);
  if (rc != FCX_OK) return fail(rc, err);
  *n_out = int64_t(res.size());
  if (int64_t(res.size()) > cap || !out) return fail(FCX_EINVAL, "output capacity too small");
  std::copy(res.begin(), res.end(), out);
  return FCX_OK;
}

int fcx_create(const fcx_config* cfg, int32_t n_trees, const fcx_tree* trees,
               fcx_ctx** out) {
  if (!cfg || !out || n_trees <= 0 || !trees) return fail(FCX_EINVAL, "bad arguments");
  *out = nullptr;
  if (cfg->m != 8 && cfg->m != 16 && cfg->m != 32)
    return fail(FCX_EINVAL, "m must be 8, 16 or 32");
  if (cfg->precision != 32 && cfg->precision != 64)
    return fail(FCX_EINVAL, "precision must be 32 or 64");
  if (cfg->physics != FCX_ADVECTION && cfg->physics != FCX_SHALLOW &&
      cfg->physics != FCX_SPHERE && cfg->physics != FCX_SWIRL &&
      cfg->physics != FCX_ROTATION)
    return fail(FCX_EINVAL, "unknown physics");
  if ((cfg->physics == FCX_SWIRL || cfg->physics == FCX_ROTATION) && !(cfg->period > 0))
    return fail(FCX_EINVAL, "the prescribed flow needs a positive period");
  if (cfg->physics == FCX_ROTATION &&
      !(cfg->axis[0] * cfg->axis[0] + cfg->axis[1] * cfg->axis[1] + cfg->axis[2] * cfg->axis[2] > 0))
    return fail(FCX_EINVAL, "the rotation needs a nonzero axis");
  if (cfg->limiter < 0 || cfg->limiter > 4 || cfg->transverse < 0 ||
      cfg->transverse > 2)
    return fail(FCX_EINVAL, "bad limiter or transverse mode");
  int tile = cfg->tile ? cfg->tile : (cfg->m >= 16 ? 16 : 8);
  if ((tile != 8 && tile != 16) || tile > cfg->m)
    return fail(FCX_EINVAL, "tile must be 8 or 16 and at most m");
  // measured defaults: FP64 16 x 16 tiles run best with two threads per
  // cell (more resident waves at their register count), the rest with one
  const int threads = cfg->threads ? cfg->threads
                                   : (tile == 16 ? (cfg->precision == 64 ? 512 : 256) : 64);
  if (threads != tile * tile && threads != 2 * tile * tile)
    return fail(FCX_EINVAL, "threads must be tile^2 or 2 tile^2");
  if (cfg->redo != 0 && cfg->redo != 1) return fail(FCX_EINVAL, "redo must be 0 or 1");
  std::vector<fcx_tree> t(trees, trees + n_trees);
  std::string err;
  if (check_connectivity(t, err) != FCX_OK) return fail(FCX_EINVAL, err);
  if (cfg->physics == FCX_SHALLOW) {
    // planar momentum is not rotated across trees: only translations
    for (const auto& T : t)
      for (int f = 0; f < 4; ++f)
        if (T.bc[f] == 0 && (T.nbr_face[f] != (f ^ 1) || T.orient[f] != 0))
          return fail(FCX_EINVAL, "shallow water needs axis-aligned tree gluing");
  }
  const bool pillow = cfg->physics == FCX_ROTATION && pillow_connectivity(t);
  if (sphere_phys(cfg->physics) && !pillow && !cube_connectivity(t))
    return fail(FCX_EINVAL, cfg->physics == FCX_ROTATION
                                ? "the rotation needs the cube's six trees or the pillow's two"
                                : "the sphere needs the six cube faces glued as the cube");
  if (sphere_phys(cfg->physics) && cfg->m % kSphereTile != 0)
    return fail(FCX_EINVAL, "the sphere needs m a multiple of 8");
  fcx_ctx* c = new fcx_ctx;
  c->cfg = *cfg;
  c->cfg.tile = tile;
  c->cfg.threads = threads;
  c->threads_auto = cfg->threads == 0;
  c->pillow = pillow;
  c->tile = tile;
  c->meqn = (cfg->physics == FCX_ADVECTION || cfg->physics == FCX_SWIRL ||
             cfg->physics == FCX_ROTATION)
                ? 1
                : (cfg->physics == FCX_SHALLOW ? 3 : 4);
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      c->cus = prop.multiProcessorCount;
      c->lds_per_block = prop.sharedMemPerBlock;
    }
    c->device = dev;
  }
  {
    const int rc = resolve_scratch(c->device);
    if (rc != FCX_OK) {
      delete c;
      return rc;
    }
  }
  c->trees = t;
  if (c->err.ensure(1) != hipSuccess || c->ticket.ensure(1) != hipSuccess ||
      c->stats.ensure(3) != hipSuccess || c->tsim.ensure(1) != hipSuccess) {
    delete c;
    return fail(FCX_ENOMEM, "hipMalloc failed");
  }
  if (hipMemset(c->err.p, 0, sizeof(int32_t)) != hipSuccess ||
      hipMemset(c->ticket.p, 0, sizeof(uint32_t)) != hipSuccess ||
      hipMemset(c->stats.p, 0, 3 * sizeof(int64_t)) != hipSuccess ||
      hipMemset(c->tsim.p, 0, sizeof(double)) != hipSuccess) {
    delete c;
    return fail(FCX_EHIP, "hipMemset failed");
  }
  *out = c;
  return FCX_OK;
}

int fcx_destroy(fcx_ctx* ctx) {
  delete ctx;
  return FCX_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The plan goes to the device in one copy from the pinned staging buffer:
// a blocking copy, or with `s` a copy ordered on that stream (later work on
// the stream sees the new plan; the staging buffer is not written again
// before that copy has ended).
static int upload_plan(fcx_ctx* c, const Forest& f, DevForest& dev,
                       const std::vector<int32_t>* kind = nullptr,
                       const std::vector<int32_t>* src = nullptr,
                       hipStream_t s = nullptr, bool ordered = false) {
  if (c->staged_pending) {
    HIPCHK(hipEventSynchronize(c->staged));
    c->staged_pending = false;
  }
  Plan& plan = c->spare;
  std::string err;
  const bool sync = c->cfg.physics == FCX_SPHERE;
  // after a regrid only the patches next to a change are planned afresh
  int rc = (kind && src && c->plan.recs.size() == c->old_forest.leaves.size())
               ? update_plan(f, c->cfg.m, c->plan, *kind, *src, plan, err, sync)
               : build_plan(f, c->cfg.m, plan, err, sync);
  if (rc != FCX_OK) return fail(rc, err);
  const size_t P = f.leaves.size();
  // reflux items: xi faces first, then eta faces; each item links the items
  // of the other direction on the same coarse patch whose faces meet its own
  // at its low and high end (the corner cell both correct)
  const size_t NI = plan.reflux.size();
  size_t off[10];
  size_t at = 0;
  const size_t sz[9] = {P * sizeof(PatchRec), P * 4, P * 4,
                        NI * sizeof(RefluxItem), 2 * 4,
                        kind ? P * 4 : 0, src ? P * 4 : 0, NI * sizeof(RefluxAux), 3 * 4};
  for (int k = 0; k < 9; ++k) { off[k] = at; at += align256(sz[k]); }
  off[9] = at;
  // dispatch order of the planar step's tiles: within the run of launch
  // slots each XCD takes, patches with a general halo (costlier tiles) come
  // first; left out when every patch or none has a simple halo
  size_t nsimple = 0;
  for (const PatchRec& r : plan.recs) nsimple += (r.flags & kSimpleHalo) != 0;
  const bool reorder = !sphere_phys(c->cfg.physics) && nsimple > 0 && nsimple < P;
  const size_t off_order = at;
  if (reorder) at += align256(P * 4);
  // patches by level, for the launches of a sub-cycled step
  const size_t off_bylevel = at;
  at += align256(P * 4);
  HIPCHK(c->staging.ensure(at));
  uint8_t* h = c->staging.p;
  {
    dev.level_first.assign(kLevels + 1, 0);
    for (const PatchRec& r : plan.recs) dev.level_first[r.level + 1] += 1;
    for (int l = 0; l < kLevels; ++l) dev.level_first[l + 1] += dev.level_first[l];
    std::vector<int32_t> fill(dev.level_first.begin(), dev.level_first.end() - 1);
    int32_t* bl = reinterpret_cast<int32_t*>(h + off_bylevel);
    for (size_t p = 0; p < P; ++p) bl[fill[plan.recs[p].level]++] = int32_t(p);
  }
  {
    RefluxItem* items = reinterpret_cast<RefluxItem*>(h + off[3]);
    RefluxAux* aux = reinterpret_cast<RefluxAux*>(h + off[7]);
    int32_t nx = 0;
    for (const auto& it : plan.reflux) nx += it.face < 2;
    dev.n_reflux_x = nx;
    dev.n_reflux_y = int32_t(NI) - nx;
    int32_t ix = 0, iy = nx;
    for (size_t p = 0; p < P; ++p) {
      const int32_t b = plan.item_first[p], e = plan.item_first[p + 1];
      if (b == e) continue;
      int32_t at_face[4] = {-1, -1, -1, -1}, pos[4];
      for (int32_t t = b; t < e; ++t) {
        const int f = plan.reflux[t].face;
        pos[t - b] = f < 2 ? ix++ : iy++;
        at_face[f] = pos[t - b];
      }
      for (int32_t t = b; t < e; ++t) {
        const int32_t k = pos[t - b];
        const RefluxItem& it = plan.reflux[t];
        const int f = it.face;
        items[k] = it;
        RefluxAux& ax = aux[k];
        ax.link[0] = at_face[f < 2 ? 2 : 0];
        ax.link[1] = at_face[f < 2 ? 3 : 1];
        ax.slot_c = plan.phislot[it.coarse];
        for (int s2 = 0; s2 < 2; ++s2)
          ax.slot_f[s2] = it.fine[s2] >= 0 ? plan.phislot[it.fine[s2]] : -1;
        ax.level = plan.recs[it.coarse].level;
      }
    }
  }
  std::memcpy(h + off[0], plan.recs.data(), sz[0]);
  std::memcpy(h + off[1], plan.phislot.data(), sz[1]);
  std::memcpy(h + off[2], plan.family.data(), sz[2]);
  const int32_t first[2] = {0, int32_t(P)};
  std::memcpy(h + off[4], first, sz[4]);
  if (kind) std::memcpy(h + off[5], kind->data(), sz[5]);
  if (src) std::memcpy(h + off[6], src->data(), sz[6]);
  const int32_t counts[3] = {plan.nslots, dev.n_reflux_x, dev.n_reflux_y};
  std::memcpy(h + off[8], counts, sz[8]);
  if (reorder) {
    int32_t* ord = reinterpret_cast<int32_t*>(h + off_order);
    const size_t per = P >> 3, rem = P & 7;
    for (size_t x = 0; x < 8; ++x) {
      const size_t a = x * per + std::min(x, rem), b = a + per + (x < rem ? 1 : 0);
      size_t k = a;
      for (size_t p = a; p < b; ++p)
        if (!(plan.recs[p].flags & kSimpleHalo)) ord[k++] = int32_t(p);
      for (size_t p = a; p < b; ++p)
        if (plan.recs[p].flags & kSimpleHalo) ord[k++] = int32_t(p);
    }
  }
  HIPCHK(dev.blob.ensure(at));
  if (ordered) {
    // a kernel reads the pinned staging (the runtime's asynchronous copy of
    // a buffer this size kept the calling thread tens of microseconds)
    if (!c->staged) HIPCHK(hipEventCreateWithFlags(&c->staged, hipEventDisableTiming));
    const int64_t n16 = int64_t(at / 16);
    hipLaunchKernelGGL(k_copy16, dim3(unsigned(std::min<int64_t>(1024, (n16 + 255) / 256))),
                       dim3(256), 0, s, reinterpret_cast<const uint4*>(h),
                       reinterpret_cast<uint4*>(dev.blob.p), n16);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->staged, s));
    c->staged_pending = true;
  } else {
    HIPCHK(hipMemcpy(dev.blob.p, h, at, hipMemcpyHostToDevice));
  }
  uint8_t* d = dev.blob.p;
  dev.rec = reinterpret_cast<PatchRec*>(d + off[0]);
  dev.phislot = reinterpret_cast<int32_t*>(d + off[1]);
  dev.family = reinterpret_cast<int32_t*>(d + off[2]);
  dev.reflux = reinterpret_cast<RefluxItem*>(d + off[3]);
  dev.first = reinterpret_cast<int32_t*>(d + off[4]);
  dev.xkind = kind ? reinterpret_cast<int32_t*>(d + off[5]) : nullptr;
  dev.xsrc = src ? reinterpret_cast<int32_t*>(d + off[6]) : nullptr;
  dev.aux = reinterpret_cast<RefluxAux*>(d + off[7]);
  dev.counts = reinterpret_cast<int32_t*>(d + off[8]);
  dev.order = reorder ? reinterpret_cast<int32_t*>(d + off_order) : nullptr;
  dev.bylevel = reinterpret_cast<int32_t*>(d + off_bylevel);
  dev.nslots = plan.nslots;
  dev.P = int64_t(P);
  std::swap(c->plan, c->spare);
  return FCX_OK;
}

// FCX_ROTATION: Omega times the unit axis
static double3 rotation_vector(const fcx_ctx* c) {
  const double* w = c->cfg.axis;
  const double om = 2.0 * 3.14159265358979323846 / c->cfg.period /
                    std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  return make_double3(om * w[0], om * w[1], om * w[2]);
}

// Device tables that follow the plan: face-term slots, sum partials and, on
// the sphere, the geometry of every patch (computed on stream s; without
// `ordered` the call waits for it).
static int finish_upload(fcx_ctx* c, hipStream_t s = nullptr, bool ordered = false) {
  const int64_t P = c->cur.P;
  const size_t esz = c->cfg.precision == 64 ? 8 : 4;
  HIPCHK(c->phi.ensure(size_t(c->cur.nslots) * 4 * c->cfg.m * c->meqn * esz));
  HIPCHK(c->partial.ensure(size_t(P) * c->meqn));
  if (sphere_phys(c->cfg.physics)) {
    const int m = c->cfg.m;
    const size_t FR = size_t(m + 4) * (m + 4);
    HIPCHK(c->cur.geo.ensure(size_t(P) * kGeoN * FR));
    const size_t lds = sizeof(double) * 3 * (m + 5) * (m + 5);
    hipLaunchKernelGGL(k_sphere_metrics, dim3(unsigned(P)), dim3(256), lds, s,
                       c->cur.rec, m, log2i(m), c->cur.geo.p, int(c->pillow));
    HIPCHK(hipGetLastError());
    if (c->cfg.physics == FCX_ROTATION) {
      const int64_t nf = P * 2 * int64_t(FR);
      HIPCHK(c->cur.flux.ensure(size_t(nf)));
      hipLaunchKernelGGL(k_rotation_fluxes, dim3(unsigned((nf + 255) / 256)), dim3(256), 0, s,
                         c->cur.geo.p, c->cur.flux.p, c->cur.rec, P, m, rotation_vector(c));
      HIPCHK(hipGetLastError());
    } else if (c->cfg.precision == 32) {
      const int64_t n32 = P * kG32N * int64_t(FR);
      HIPCHK(c->cur.geo32.ensure(size_t(n32)));
      hipLaunchKernelGGL(k_sphere_geo32, dim3(unsigned((n32 + 255) / 256)), dim3(256), 0, s,
                         c->cur.geo.p, c->cur.geo32.p, P, m);
      HIPCHK(hipGetLastError());
    }
    if (!ordered) HIPCHK(hipDeviceSynchronize());
  }
  return FCX_OK;
}

int fcx_upload_forest(fcx_ctx* c, int64_t n, const fcx_leaf* leaves) {
  if (!c || n <= 0 || !leaves) return fail(FCX_EINVAL, "bad arguments");
  if (n * c->meqn * c->cfg.m * c->cfg.m >=
      (int64_t(1) << 31))
    return fail(FCX_EINVAL, "state larger than 2^31 elements");
  std::vector<fcx_leaf> l(leaves, leaves + n);
  std::string err;
  Forest f;
  int rc = f.assign(c->trees, l, err);
  if (rc != FCX_OK) return fail(rc, err);
  std::vector<fcx_leaf> bal;
  rc = balance(c->trees, l, bal, err);
  if (rc != FCX_OK) return fail(rc, err);
  if (bal.size() != l.size()) return fail(FCX_EBALANCE, "forest is not 2:1 balanced");
  c->forest = std::move(f);
  c->have_forest = true;
  c->have_old = false;
  rc = upload_plan(c, c->forest, c->cur);
  if (rc != FCX_OK) { c->have_forest = false; return rc; }
  return finish_upload(c);
}

int64_t fcx_num_patches(const fcx_ctx* c) {
  return c && c->have_forest ? int64_t(c->forest.leaves.size()) : -1;
}
int64_t fcx_state_elems(const fcx_ctx* c) {
  if (!c || !c->have_forest) return -1;
  return int64_t(c->forest.leaves.size()) * c->meqn * c->cfg.m * c->cfg.m;
}
int64_t fcx_ghost_elems(const fcx_ctx* c) {
  if (!c || !c->have_forest) return -1;
  return int64_t(c->forest.leaves.size()) * c->meqn * (8 * c->cfg.m + 16);
}
int fcx_get_leaves(const fcx_ctx* c, int64_t cap, fcx_leaf* out) {
  if (!c || !c->have_forest) return fail(FCX_ESTATE, "no forest");
  if (cap < int64_t(c->forest.leaves.size()) || !out)
    return fail(FCX_EINVAL, "capacity too small");
  std::copy(c->forest.leaves.begin(), c->forest.leaves.end(), out);
  return FCX_OK;
}

int fcx_patch_table(fcx_ctx* c, int64_t cap_items, void* recs, int32_t* phislot,
                    int32_t* family, int32_t* counts, void* items, void* aux) {
  if (!c || !recs || !phislot || !family || !counts)
    return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  HIPCHK(hipDeviceSynchronize());
  const size_t P = size_t(c->cur.P);
  HIPCHK(hipMemcpy(counts, c->cur.counts, 3 * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(recs, c->cur.rec, P * sizeof(PatchRec), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(phislot, c->cur.phislot, P * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(family, c->cur.family, P * 4, hipMemcpyDeviceToHost));
  const int64_t n = int64_t(counts[1]) + counts[2];
  if (n > 0 && (items || aux)) {
    if (n > cap_items) return fail(FCX_EINVAL, "item capacity too small");
    if (items)
      HIPCHK(hipMemcpy(items, c->cur.reflux, size_t(n) * sizeof(RefluxItem),
                       hipMemcpyDeviceToHost));
    if (aux)
      HIPCHK(hipMemcpy(aux, c->cur.aux, size_t(n) * sizeof(RefluxAux), hipMemcpyDeviceToHost));
  }
  return FCX_OK;
}

// ---------------------------------------------------------------------------
static KPhys kphys(const fcx_ctx* c) {
  return KPhys{c->cfg.g, c->cfg.ax, c->cfg.ay, c->cfg.limiter, c->cfg.transverse,
               c->cfg.period};
}

template <typename R, int PHYS>
static int launch_ghost(fcx_ctx* c, const void* q, void* ghost, hipStream_t s) {
  const int m = c->cfg.m;
  const int64_t tot = c->cur.P * (8 * m + 16);
  const unsigned blocks = unsigned((tot + 255) / 256);
  hipLaunchKernelGGL((k_ghost_fill<R, PHYS>), dim3(blocks), dim3(256), 0, s,
                     static_cast<const R*>(q), static_cast<R*>(ghost),
                     c->cur.rec, int32_t(c->cur.P), m, log2i(m), c->err.p,
                     c->cur.geo.p);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_ghost_fill(fcx_ctx* c, const void* q, void* ghost, void* stream) {
  if (!c || !q || !ghost) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dp = c->cfg.precision == 64;
  // (a scalar either way: the prescribed flow's ghost cells are advection's)
  if (c->cfg.physics == FCX_ADVECTION || c->cfg.physics == FCX_SWIRL)
    return dp ? launch_ghost<double, FCX_ADVECTION>(c, q, ghost, s)
              : launch_ghost<float, FCX_ADVECTION>(c, q, ghost, s);
  if (c->cfg.physics == FCX_SPHERE)
    return dp ? launch_ghost<double, FCX_SPHERE>(c, q, ghost, s)
              : launch_ghost<float, FCX_SPHERE>(c, q, ghost, s);
  if (c->cfg.physics == FCX_ROTATION)
    return dp ? launch_ghost<double, FCX_ROTATION>(c, q, ghost, s)
              : launch_ghost<float, FCX_ROTATION>(c, q, ghost, s);
  return dp ? launch_ghost<double, FCX_SHALLOW>(c, q, ghost, s)
            : launch_ghost<float, FCX_SHALLOW>(c, q, ghost, s);
}

// Two threads per cell of a tile: as configured, or, left to the library,
// for FP64 16 x 16 tiles (more resident waves at their register count) and
// for FP32 16 x 16 tiles of a forest with at most four tiles per CU (a launch
// of one or two rounds of tiles is bound by one tile's latency, which two
// threads per cell shorten; larger forests are bound by instructions).
static bool wide_tiles(const fcx_ctx* c, int64_t patches) {
  if (!c->threads_auto) return c->cfg.threads == 2 * c->tile * c->tile;
  if (c->tile != 16) return false;
  const int64_t tiles = patches * (c->cfg.m / 16) * (c->cfg.m / 16);
  return c->cfg.precision == 64 || tiles <= 4 * int64_t(c->cus);
}

template <typename R, int PHYS, int T, int NT, bool FUSED>
static int launch_step_t(fcx_ctx* c, const void* q, const void* ghost, void* qn,
                         const double* dt, double* numax, hipStream_t s) {
  StepArgs<R> a;
  a.q = static_cast<const R*>(q);
  a.ghost = static_cast<const R*>(ghost);
  a.qn = static_cast<R*>(qn);
  a.dt = dt;
  a.numax = numax;
  a.rec = c->cur.rec;
  a.phislot = c->cur.phislot;
  a.phi = reinterpret_cast<R*>(c->phi.p);
  a.err = c->err.p;
  a.P = int32_t(c->cur.P);
  a.m = c->cfg.m;
  a.lm = log2i(c->cfg.m);
  const int tps = c->cfg.m / T;
  a.ntiles = int32_t(c->cur.P * tps * tps);
  a.ph = kphys(c);
  a.order = c->cur.order;
  a.tsim = c->tsim.p;
  if constexpr (PHYS == FCX_ADVECTION) {
    // advection tiles: one wavefront each, kAdvWaves per workgroup
    const dim3 grid(unsigned((a.ntiles + kAdvWaves - 1) / kAdvWaves));
    if (c->cfg.limiter == 4 && c->cfg.transverse == 2)
      hipLaunchKernelGGL((k_adv_step<R, T, FUSED, 1>), grid, dim3(64 * kAdvWaves), 0, s, a);
    else
      hipLaunchKernelGGL((k_adv_step<R, T, FUSED, 0>), grid, dim3(64 * kAdvWaves), 0, s, a);
  } else if (c->cfg.limiter == 4 && c->cfg.transverse == 2) {
    hipLaunchKernelGGL((k_step<R, PHYS, T, NT, FUSED, 1>), dim3(unsigned(a.ntiles)),
                       dim3(NT), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_step<R, PHYS, T, NT, FUSED, 0>), dim3(unsigned(a.ntiles)),
                       dim3(NT), 0, s, a);
  }
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

template <typename R, int PHYS, bool FUSED>
static int launch_step_m(fcx_ctx* c, const void* q, const void* ghost, void* qn,
                         const double* dt, double* numax, hipStream_t s) {
  const bool wide = wide_tiles(c, c->cur.P);
  if (c->tile == 8)
    return wide ? launch_step_t<R, PHYS, 8, 128, FUSED>(c, q, ghost, qn, dt, numax, s)
                : launch_step_t<R, PHYS, 8, 64, FUSED>(c, q, ghost, qn, dt, numax, s);
  return wide ? launch_step_t<R, PHYS, 16, 512, FUSED>(c, q, ghost, qn, dt, numax, s)
              : launch_step_t<R, PHYS, 16, 256, FUSED>(c, q, ghost, qn, dt, numax, s);
}

template <typename R>
static int launch_sphere_step(fcx_ctx* c, const void* q, const void* ghost, void* qn,
                              const double* dt, double* numax, hipStream_t s) {
  const size_t lds = sphere_lds<R>();
  if (lds > c->lds_per_block)
    return fail(FCX_EINVAL, "sphere step tile does not fit this device's LDS");
  SphereArgs<R> a;
  a.q = static_cast<const R*>(q);
  a.ghost = static_cast<const R*>(ghost);
  a.qn = static_cast<R*>(qn);
  a.dt = dt;
  a.numax = numax;
  a.rec = c->cur.rec;
  a.phislot = c->cur.phislot;
  a.phi = reinterpret_cast<R*>(c->phi.p);
  a.err = c->err.p;
  a.geo = c->cur.geo.p;
  a.geo32 = c->cur.geo32.p;
  a.P = int32_t(c->cur.P);
  a.m = c->cfg.m;
  a.lm = log2i(c->cfg.m);
  a.limiter = c->cfg.limiter;
  a.transverse = c->cfg.transverse;
  a.g = c->cfg.g;
  const int tps = a.m / kSphereTile;
  const int64_t grid = c->cur.P * tps * tps;
  hipLaunchKernelGGL((k_sphere_step<R>), dim3(unsigned(grid)), dim3(kSphereThreads), lds, s,
                     a);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

template <typename R, int T, int NT>
static int launch_rotation_step(fcx_ctx* c, const void* q, const void* ghost, void* qn,
                                const double* dt, double* numax, hipStream_t s) {
  RotationArgs a;
  a.q = q;
  a.ghost = ghost;
  a.qn = qn;
  a.dt = dt;
  a.numax = numax;
  a.rec = c->cur.rec;
  a.geo = c->cur.geo.p;
  a.flux = c->cur.flux.p;
  a.m = c->cfg.m;
  a.limiter = c->cfg.limiter;
  a.transverse = c->cfg.transverse;
  const int tps = a.m / T;
  const int64_t grid = c->cur.P * tps * tps;
  hipLaunchKernelGGL((k_rotation_step<R, T, NT>), dim3(unsigned(grid)), dim3(NT), 0, s, a);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

template <bool FUSED>
static int step_dispatch(fcx_ctx* c, const void* q, const void* ghost, void* qn,
                         const double* dt, double* numax, void* stream) {
  if (!c || !q || !qn || !dt || !numax || (!FUSED && !ghost))
    return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  if (q == qn) return fail(FCX_EINVAL, "q_new must not alias q");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dp = c->cfg.precision == 64;
  if (c->cfg.physics == FCX_SPHERE) {
    if (FUSED) return fail(FCX_EINVAL, "no fused step on the sphere");
    return dp ? launch_sphere_step<double>(c, q, ghost, qn, dt, numax, s)
              : launch_sphere_step<float>(c, q, ghost, qn, dt, numax, s);
  }
  if (c->cfg.physics == FCX_ROTATION) {
    if (FUSED) return fail(FCX_EINVAL, "no fused step on the sphere");
    if (c->cfg.m % 16 == 0)
      return dp ? launch_rotation_step<double, 16, 256>(c, q, ghost, qn, dt, numax, s)
                : launch_rotation_step<float, 16, 256>(c, q, ghost, qn, dt, numax, s);
    return dp ? launch_rotation_step<double, 8, 128>(c, q, ghost, qn, dt, numax, s)
              : launch_rotation_step<float, 8, 128>(c, q, ghost, qn, dt, numax, s);
  }
  if (c->cfg.physics == FCX_ADVECTION)
    return dp ? launch_step_m<double, FCX_ADVECTION, FUSED>(c, q, ghost, qn, dt, numax, s)
              : launch_step_m<float, FCX_ADVECTION, FUSED>(c, q, ghost, qn, dt, numax, s);
  if (c->cfg.physics == FCX_SWIRL)
    return dp ? launch_step_m<double, FCX_SWIRL, FUSED>(c, q, ghost, qn, dt, numax, s)
              : launch_step_m<float, FCX_SWIRL, FUSED>(c, q, ghost, qn, dt, numax, s);
  return dp ? launch_step_m<double, FCX_SHALLOW, FUSED>(c, q, ghost, qn, dt, numax, s)
            : launch_step_m<float, FCX_SHALLOW, FUSED>(c, q, ghost, qn, dt, numax, s);
}

int fcx_patch_step(fcx_ctx* c, const void* q, const void* ghost, void* qn,
                   const double* dt, double* numax, void* stream) {
  return step_dispatch<false>(c, q, ghost, qn, dt, numax, stream);
}

int fcx_fused_step(fcx_ctx* c, const void* q, void* qn, const double* dt,
                   double* numax, void* stream) {
  return step_dispatch<true>(c, q, nullptr, qn, dt, numax, stream);
}

// Workgroups that copy a rejected attempt's state (256 threads, a few
// 16-byte units each, at most one per CU).
// Workgroups of a launch that ends in the last-workgroup ticket (reflux +
// next dt, next dt with redo): every one of them takes the ticket with an
// agent-scope fence and atomic, so they are few (a rejected attempt's copy,
// rare, then runs on fewer workgroups).
static int64_t redo_grid(const fcx_ctx* c, int64_t n16) {
  (void)c;
  return std::max<int64_t>(1, std::min<int64_t>(32, (n16 + 1023) / 1024));
}

static NextDtArgs next_args(fcx_ctx* c, double* numax, double* dt, int32_t* status,
                            int32_t redo) {
  NextDtArgs nd{};
  nd.numax = numax;
  nd.dt = dt;
  nd.status = status;
  nd.ticket = c->ticket.p;
  nd.stats = c->stats.p;
  nd.cfl_desired = c->cfg.cfl_desired;
  nd.cfl_max = c->cfg.cfl_max;
  nd.redo = redo;
  nd.cells = c->cur.P * c->cfg.m * c->cfg.m;
  nd.n16 = c->cur.P * c->meqn * c->cfg.m * c->cfg.m * (c->cfg.precision / 8) / 16;
  nd.tsim = c->tsim.p;
  nd.tscale = 1.0;
  return nd;
}

// All reflux items in one launch; with NEXT the launch also takes the CFL
// check and next dt (then it runs even without items) and, with redo on,
// the copy of a rejected attempt's state.
template <typename R, int PHYS, bool NEXT>
static int launch_reflux(fcx_ctx* c, const void* q, void* qn, const double* dt,
                         hipStream_t s, NextDtArgs nd = {}) {
  const int m = c->cfg.m;
  // (the prescribed-flow advection is not in conservation form: no items)
  const int32_t n =
      c->cfg.physics == FCX_SWIRL ? 0 : c->cur.n_reflux_x + c->cur.n_reflux_y;
  if (n == 0 && !NEXT) return FCX_OK;
  const int64_t tot = int64_t(n) * m;
  int64_t g = std::max<int64_t>(1, (tot + 255) / 256);
  // with NEXT every workgroup takes the last-workgroup ticket: a small grid
  // (the reflux loops over its cells)
  if (NEXT) g = std::max(std::min<int64_t>(g, 32), nd.redo ? redo_grid(c, nd.n16) : 1);
  const unsigned grid = unsigned(g);
  hipLaunchKernelGGL((k_reflux<R, PHYS, NEXT>), dim3(grid), dim3(256), 0, s,
                     static_cast<const R*>(q), static_cast<R*>(qn), c->cur.reflux,
                     c->cur.aux, n, reinterpret_cast<const R*>(c->phi.p), dt, m, kphys(c),
                     c->err.p, nd);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

template <typename R>
static int launch_sphere_reflux(fcx_ctx* c, const void* q, void* qn, const double* dt,
                                hipStream_t s) {
  const int m = c->cfg.m;
  for (int axis = 0; axis < 2; ++axis) {
    const int32_t n = axis == 0 ? c->cur.n_reflux_x : c->cur.n_reflux_y;
    if (n == 0) continue;
    const RefluxItem* items = c->cur.reflux + (axis == 0 ? 0 : c->cur.n_reflux_x);
    const int64_t tot = int64_t(n) * 32;
    hipLaunchKernelGGL((k_sphere_reflux<R>), dim3(unsigned((tot + 255) / 256)), dim3(256),
                       0, s, static_cast<const R*>(q), static_cast<R*>(qn), items, n,
                       c->cur.rec, c->cur.phislot, reinterpret_cast<const R*>(c->phi.p),
                       c->cur.geo.p, dt, c->cfg.g, m, c->err.p);
    HIPCHK(hipGetLastError());
  }
  return FCX_OK;
}

int fcx_reflux(fcx_ctx* c, const void* q, void* qn, const double* dt, void* stream) {
  if (!c || !q || !qn || !dt) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  // (the rotation's colour equation is not in conservation form)
  if (c->cfg.physics == FCX_ROTATION) return FCX_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dp = c->cfg.precision == 64;
  if (c->cfg.physics == FCX_SPHERE)
    return dp ? launch_sphere_reflux<double>(c, q, qn, dt, s)
              : launch_sphere_reflux<float>(c, q, qn, dt, s);
  if (c->cfg.physics == FCX_ADVECTION || c->cfg.physics == FCX_SWIRL)
    return dp ? launch_reflux<double, FCX_ADVECTION, false>(c, q, qn, dt, s)
              : launch_reflux<float, FCX_ADVECTION, false>(c, q, qn, dt, s);
  return dp ? launch_reflux<double, FCX_SHALLOW, false>(c, q, qn, dt, s)
            : launch_reflux<float, FCX_SHALLOW, false>(c, q, qn, dt, s);
}

int fcx_next_dt(fcx_ctx* c, double* numax, double* dt, int32_t* status, void* stream) {
  if (!c || !numax || !dt || !status) return fail(FCX_EINVAL, "bad arguments");
  hipLaunchKernelGGL(k_next_dt, dim3(1), dim3(64), 0,
                     static_cast<hipStream_t>(stream), numax, dt, status, c->err.p,
                     c->stats.p, c->cfg.cfl_desired, c->cfg.cfl_max,
                     int64_t(c->cur.P) * c->cfg.m * c->cfg.m, c->tsim.p);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

// fcx_next_dt with the CFL rule's rejection (redo on): a rejected attempt's
// q_new receives q.
static int next_dt_redo(fcx_ctx* c, const void* q, void* qn, double* numax, double* dt,
                        int32_t* status, hipStream_t s) {
  const NextDtArgs nd = next_args(c, numax, dt, status, 1);
  hipLaunchKernelGGL(k_next_dt_redo, dim3(unsigned(redo_grid(c, nd.n16))), dim3(256), 0, s,
                     static_cast<const uint4*>(q), static_cast<uint4*>(qn), nd, c->err.p);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_step_stats(const fcx_ctx* c, int64_t* out) {
  if (!c || !out) return fail(FCX_EINVAL, "bad arguments");
  HIPCHK(hipMemcpy(out, c->stats.p, 3 * sizeof(int64_t), hipMemcpyDeviceToHost));
  return FCX_OK;
}

int fcx_sim_time(const fcx_ctx* c, double* t) {
  if (!c || !t) return fail(FCX_EINVAL, "bad arguments");
  HIPCHK(hipMemcpy(t, c->tsim.p, sizeof(double), hipMemcpyDeviceToHost));
  return FCX_OK;
}

template <typename R, int MEQN>
static int launch_sums(fcx_ctx* c, const void* q, double* sums, hipStream_t s,
                       double* partial) {
  hipLaunchKernelGGL((k_sums_patch<R, MEQN>), dim3(unsigned(c->cur.P)), dim3(256),
                     0, s, static_cast<const R*>(q), c->cur.rec, c->cfg.m, partial);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL((k_sums_reduce<MEQN>), dim3(1), dim3(1024), 0, s,
                     partial, c->cur.first, sums);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

// Per-patch partials (P * meqn doubles) into `partial`, then the fixed-order
// reduction.
static int sums_with(fcx_ctx* c, const void* q, double* sums, hipStream_t s,
                     double* partial) {
  const bool dp = c->cfg.precision == 64;
  if (c->cfg.physics == FCX_SPHERE) {
    if (dp)
      hipLaunchKernelGGL((k_sphere_sums_patch<double, 4>), dim3(unsigned(c->cur.P)), dim3(256),
                         0, s, static_cast<const double*>(q), c->cur.rec, c->cur.geo.p,
                         c->cfg.m, partial);
    else
      hipLaunchKernelGGL((k_sphere_sums_patch<float, 4>), dim3(unsigned(c->cur.P)), dim3(256),
                         0, s, static_cast<const float*>(q), c->cur.rec, c->cur.geo.p,
                         c->cfg.m, partial);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((k_sums_reduce<4>), dim3(1), dim3(1024), 0, s, partial,
                       c->cur.first, sums);
    HIPCHK(hipGetLastError());
    return FCX_OK;
  }
  if (c->cfg.physics == FCX_ROTATION) {
    if (dp)
      hipLaunchKernelGGL((k_sphere_sums_patch<double, 1>), dim3(unsigned(c->cur.P)), dim3(256),
                         0, s, static_cast<const double*>(q), c->cur.rec, c->cur.geo.p,
                         c->cfg.m, partial);
    else
      hipLaunchKernelGGL((k_sphere_sums_patch<float, 1>), dim3(unsigned(c->cur.P)), dim3(256),
                         0, s, static_cast<const float*>(q), c->cur.rec, c->cur.geo.p,
                         c->cfg.m, partial);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((k_sums_reduce<1>), dim3(1), dim3(1024), 0, s, partial,
                       c->cur.first, sums);
    HIPCHK(hipGetLastError());
    return FCX_OK;
  }
  if (c->meqn == 1)
    return dp ? launch_sums<double, 1>(c, q, sums, s, partial)
              : launch_sums<float, 1>(c, q, sums, s, partial);
  return dp ? launch_sums<double, 3>(c, q, sums, s, partial)
            : launch_sums<float, 3>(c, q, sums, s, partial);
}

int fcx_conservation_sums(fcx_ctx* c, const void* q, double* sums, void* stream) {
  if (!c || !q || !sums) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  return sums_with(c, q, sums, static_cast<hipStream_t>(stream), c->partial.p);
}

int fcx_conservation_sums_noalloc(fcx_ctx* c, const void* q, double* sums, void* stream) {
  if (!c || !q || !sums) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  if (c->cur.P * c->meqn > kNoAllocPartials)
    return fail(FCX_EINVAL, "fcx_conservation_sums_noalloc: patches x components exceeds "
                            "its scratch of 1048576 partial sums");
  double* part = scratch_of(c->device);
  if (!part) return fail(FCX_ESTATE, "scratch of this device not resolved");
  return sums_with(c, q, sums, static_cast<hipStream_t>(stream), part);
}

template <typename R, int MEQN>
// mirror: pinned host memory that receives the final tags as well (null:
// none); the kernels write it directly, so no copy follows them
static int launch_tags(fcx_ctx* c, const void* q, const void* ghost, int criterion,
                       double thr, int lmin, int lmax, int8_t* tags, hipStream_t s,
                       int8_t* mirror = nullptr) {
  const int m = c->cfg.m;
  const double* geo = sphere_phys(c->cfg.physics) ? c->cur.geo.p : nullptr;
  hipLaunchKernelGGL((k_tag_refine<R, MEQN>), dim3(unsigned(c->cur.P)), dim3(256),
                     0, s, static_cast<const R*>(q), static_cast<const R*>(ghost),
                     c->cur.rec, m, criterion, thr, lmax, tags, geo, mirror);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL((k_tag_family<R, MEQN>), dim3(unsigned(c->cur.P)), dim3(256),
                     size_t(m) * m * sizeof(double) * (geo ? 4 : 1), s,
                     static_cast<const R*>(q), c->cur.rec, c->cur.family, m, criterion,
                     thr, lmin, tags, geo, mirror);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

static int regrid_tags(fcx_ctx* c, const void* q, const void* ghost, int32_t criterion,
                       double thr, int32_t lmin, int32_t lmax, int8_t* tags, void* stream,
                       int8_t* mirror) {
  if (!c || !q || !tags || (criterion != 0 && criterion != 1) ||
      (criterion == 1 && !ghost))
    return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dp = c->cfg.precision == 64;
  int8_t* mi = mirror;
  if (c->meqn == 1)
    return dp ? launch_tags<double, 1>(c, q, ghost, criterion, thr, lmin, lmax, tags, s, mi)
              : launch_tags<float, 1>(c, q, ghost, criterion, thr, lmin, lmax, tags, s, mi);
  if (c->meqn == 4)
    return dp ? launch_tags<double, 4>(c, q, ghost, criterion, thr, lmin, lmax, tags, s, mi)
              : launch_tags<float, 4>(c, q, ghost, criterion, thr, lmin, lmax, tags, s, mi);
  return dp ? launch_tags<double, 3>(c, q, ghost, criterion, thr, lmin, lmax, tags, s, mi)
            : launch_tags<float, 3>(c, q, ghost, criterion, thr, lmin, lmax, tags, s, mi);
}

int fcx_regrid_tags(fcx_ctx* c, const void* q, const void* ghost, int32_t criterion,
                    double thr, int32_t lmin, int32_t lmax, int8_t* tags,
                    void* stream) {
  return regrid_tags(c, q, ghost, criterion, thr, lmin, lmax, tags, stream, nullptr);
}

// old_to_new of every old leaf from the transfer plan of the new ones
// (kind 0: copy of old src, 1: child of old src, 2: parent of the four old
// leaves from src): >= 0 kept at that index, -2 - k refined with its first
// child at k, -1 merged into a parent.
static int fill_old_to_new(const std::vector<int32_t>& kind, const std::vector<int32_t>& src,
                           int64_t n_old, int64_t* o2n) {
  const int64_t unset = INT64_MIN;
  for (int64_t i = 0; i < n_old; ++i) o2n[i] = unset;
  for (size_t p = 0; p < kind.size(); ++p) {
    const int64_t s = src[p];
    if (s < 0 || s >= n_old) return fail(FCX_EINVAL, "transfer plan out of range");
    if (kind[p] == 0) {
      o2n[s] = int64_t(p);
    } else if (kind[p] == 1) {
      if (o2n[s] == unset) o2n[s] = -2 - int64_t(p);
    } else {
      if (s + 3 >= n_old) return fail(FCX_EINVAL, "transfer plan out of range");
      for (int k = 0; k < 4; ++k) o2n[s + k] = -1;
    }
  }
  for (int64_t i = 0; i < n_old; ++i)
    if (o2n[i] == unset) return fail(FCX_EINVAL, "an old leaf has no image in the new forest");
  return FCX_OK;
}

static int regrid_apply(fcx_ctx* c, const int8_t* tags, int32_t lmin, int32_t lmax,
                        int64_t* n_new, int64_t* old_to_new, hipStream_t s, bool ordered) {
  if (!c || !tags || !n_new || lmin < 0 || lmax < lmin || lmax > kMaxLevel)
    return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  std::vector<fcx_leaf> out;
  std::vector<int32_t> kind, src;
  std::string err;
  int rc = regrid(c->forest, tags, lmin, lmax, out, err, &kind, &src);
  if (rc != FCX_OK) return fail(rc, err);
  for (int32_t k : kind)
    if (k < 0) return fail(FCX_EINVAL, "new leaf is not a copy, child or parent of old leaves");
  if (old_to_new) {
    rc = fill_old_to_new(kind, src, int64_t(c->forest.leaves.size()), old_to_new);
    if (rc != FCX_OK) return rc;
  }
  Forest nf;
  nf.adopt(c->trees, std::move(out));
  // the current device forest becomes the old one
  std::swap(c->cur, c->old);
  c->old_forest = std::move(c->forest);
  c->forest = std::move(nf);
  c->have_old = true;
  rc = upload_plan(c, c->forest, c->cur, &kind, &src, s, ordered);
  if (rc != FCX_OK) return rc;
  rc = finish_upload(c, s, ordered);
  if (rc != FCX_OK) return rc;
  *n_new = int64_t(c->forest.leaves.size());
  return FCX_OK;
}

int fcx_regrid_apply(fcx_ctx* c, const int8_t* tags, int32_t lmin, int32_t lmax,
                     int64_t* n_new, int64_t* old_to_new) {
  return regrid_apply(c, tags, lmin, lmax, n_new, old_to_new, nullptr, false);
}

template <typename R, int MEQN>
static int launch_transfer(fcx_ctx* c, const void* qo, const void* go, void* qn,
                           hipStream_t s) {
  const int m = c->cfg.m;
  const int64_t tot = c->cur.P * MEQN * m * m;
  hipLaunchKernelGGL((k_transfer<R, MEQN>), dim3(unsigned((tot + 255) / 256)),
                     dim3(256), 0, s, static_cast<const R*>(qo),
                     static_cast<const R*>(go), static_cast<R*>(qn), c->cur.rec,
                     c->cur.xkind, c->cur.xsrc, int32_t(c->cur.P), m);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

template <typename R, int MEQN>
static int launch_transfer_sphere(fcx_ctx* c, const void* qo, const void* go, void* qn,
                                  hipStream_t s) {
  const int m = c->cfg.m;
  const int64_t tot = c->cur.P * MEQN * (m / 2) * (m / 2);
  hipLaunchKernelGGL((k_transfer_sphere<R, MEQN>), dim3(unsigned((tot + 255) / 256)), dim3(256),
                     0, s, static_cast<const R*>(qo), static_cast<const R*>(go),
                     static_cast<R*>(qn), c->cur.rec, c->cur.xkind, c->cur.xsrc,
                     c->old.geo.p, c->cur.geo.p, int32_t(c->cur.P), m);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_regrid_transfer(fcx_ctx* c, const void* qo, const void* go, void* qn,
                        void* stream) {
  if (!c || !qo || !go || !qn) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_old) return fail(FCX_ESTATE, "no regrid applied");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dp = c->cfg.precision == 64;
  if (c->cfg.physics == FCX_SPHERE)
    return dp ? launch_transfer_sphere<double, 4>(c, qo, go, qn, s)
              : launch_transfer_sphere<float, 4>(c, qo, go, qn, s);
  if (c->cfg.physics == FCX_ROTATION)
    return dp ? launch_transfer_sphere<double, 1>(c, qo, go, qn, s)
              : launch_transfer_sphere<float, 1>(c, qo, go, qn, s);
  if (c->meqn == 1)
    return dp ? launch_transfer<double, 1>(c, qo, go, qn, s)
              : launch_transfer<float, 1>(c, qo, go, qn, s);
  return dp ? launch_transfer<double, 3>(c, qo, go, qn, s)
            : launch_transfer<float, 3>(c, qo, go, qn, s);
}


// ===========================================================================
// Batches of independent forests
// ===========================================================================
struct fcx_batch {
  int32_t n = 0;
  int precision = 64;
  double cfl_desired = 0.9, cfl_max = 1.0;
  int32_t redo = 0;
  std::vector<fcx_ctx*> ctx;
  std::vector<ForestDev> fh;
  std::vector<int64_t> state_off;
  int64_t state_elems = 0, P = 0;
  // tuning: tile used by forests with m >= 16, threads per tile class, and
  // the launch form (0: a workgroup per tile; 1: persistent workgroups)
  int32_t tile_big = 16, threads8 = 64, threads16 = 256, persistent = 0;
  // device data
  DevBuf<uint8_t> blob;
  PatchRec* rec = nullptr;
  int32_t* phislot = nullptr;
  int32_t* pforest = nullptr;
  ForestDev* forests = nullptr;
  BatchItem* items = nullptr;
  AdvItem* advitems = nullptr;        // [item index], advection classes only
  int32_t* range = nullptr;           // [class][9]: item range of each XCD
  RefluxItem* reflux = nullptr;
  int32_t* reflux_forest = nullptr;
  int32_t* first = nullptr;           // [n + 1] patch offsets
  int32_t n_reflux_x = 0, n_reflux_y = 0;
  // work classes: 8 x 8 or large tiles, times advection or shallow water
  int32_t nitems[4] = {0, 0, 0, 0}, item0[4] = {0, 0, 0, 0};
  int32_t nsimple[4] = {0, 0, 0, 0};  // advection classes: simple-halo items first
  bool mc2[4] = {true, true, true, true};  // every forest: MC limiter, transverse 2
  DevBuf<uint8_t> phi;
  DevBuf<double> partial;
  DevBuf<int32_t> counters, err;    // counters: persistent launches; err: per forest
  DevBuf<uint32_t> ticket;          // last-workgroup ticket of the next-dt launch
  DevBuf<int64_t> stats;            // per forest {accepted, rejected, accepted cells}
  HostBuf staging;
  int cus = 256;
  // captured graph
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the general-halo advection tiles of a class run on `side`, beside the
  // strip walk of the same class (fork before the walk, join before the
  // reflux): the walk leaves registers free for one of their wavefronts per
  // SIMD, and their launch is latency-bound
  hipStream_t side = nullptr;
  hipEvent_t fork[4] = {}, join[4] = {};
  bool joined[4] = {};
  ~fcx_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    for (int k = 0; k < 4; ++k) {
      if (fork[k]) (void)hipEventDestroy(fork[k]);
      if (join[k]) (void)hipEventDestroy(join[k]);
    }
    if (side) (void)hipStreamDestroy(side);
  }
};

static int batch_build(fcx_batch* b) {
  // concatenated tables, items per tile class, cost-balanced XCD ranges
  std::vector<PatchRec> recs;
  std::vector<int32_t> phislot, pforest, first(1, 0);
  std::vector<RefluxItem> rx, ry;
  std::vector<int32_t> rfx, rfy;
  std::vector<BatchItem> items[4];
  int64_t phi_elems = 0, slot_base = 0;
  for (int k = 0; k < 4; ++k) b->mc2[k] = true;
  b->fh.clear();
  b->state_off.clear();
  int64_t sbase = 0, pbase = 0;
  for (int f = 0; f < b->n; ++f) {
    fcx_ctx* c = b->ctx[f];
    Plan plan;
    std::string err;
    int rc = build_plan(c->forest, c->cfg.m, plan, err);
    if (rc != FCX_OK) return fail(rc, err);
    const int64_t P = int64_t(c->forest.leaves.size());
    ForestDev F{};
    F.m = c->cfg.m;
    F.lm = log2i(c->cfg.m);
    F.meqn = c->meqn;
    F.physics = c->cfg.physics;
    F.patch_base = int32_t(pbase);
    F.slot_base = int32_t(slot_base);
    F.state_base = sbase;
    F.phi_base = phi_elems;
    F.ph = kphys(c);
    b->fh.push_back(F);
    b->state_off.push_back(sbase);
    for (int64_t p = 0; p < P; ++p) {
      PatchRec r = plan.recs[p];
      for (int k = 0; k < 12; ++k)
        if (r.nbr[k] >= 0) r.nbr[k] += int32_t(pbase);
      recs.push_back(r);
      phislot.push_back(plan.phislot[p] >= 0 ? plan.phislot[p] + int32_t(slot_base) : -1);
      pforest.push_back(f);
      const int T = F.m == 8 ? 8 : b->tile_big;
      const int cls = (T == 8 ? 0 : 2) + (F.physics == FCX_SHALLOW ? 1 : 0);
      if (c->cfg.limiter != 4 || c->cfg.transverse != 2) b->mc2[cls] = false;
      const int tps = F.m / T;
      const int64_t qoff = sbase + p * F.meqn * F.m * F.m;
      for (int t = 0; t < tps * tps; ++t)
        items[cls].push_back(BatchItem{int32_t(pbase + p), uint32_t(qoff), phislot.back(),
                                       (t % tps) | ((t / tps) << 4) | (F.lm << 8) |
                                           (f << 12)});
    }
    for (auto it : plan.reflux) {
      it.coarse += int32_t(pbase);
      for (int s2 = 0; s2 < 2; ++s2) it.fine[s2] += int32_t(pbase);
      if (it.face < 2) { rx.push_back(it); rfx.push_back(f); }
      else { ry.push_back(it); rfy.push_back(f); }
    }
    slot_base += plan.nslots;
    phi_elems += int64_t(plan.nslots) * 4 * F.m * F.meqn;
    sbase += P * F.meqn * F.m * F.m;
    pbase += P;
    first.push_back(int32_t(pbase));
  }
  // 32-bit element offsets: every forest's patches are addressed as
  // (global patch id) x (patch size) from a shifted base
  bool fits = sbase < (int64_t(1) << 31) && pbase < (int64_t(1) << 27);
  for (const ForestDev& F : b->fh)
    fits = fits && int64_t(pbase) * F.meqn * F.m * F.m < (int64_t(1) << 31);
  if (!fits) return fail(FCX_EINVAL, "batch too large");
  b->P = pbase;
  b->state_elems = sbase;
  b->n_reflux_x = int32_t(rx.size());
  b->n_reflux_y = int32_t(ry.size());
  rx.insert(rx.end(), ry.begin(), ry.end());
  rfx.insert(rfx.end(), rfy.begin(), rfy.end());
  // the items of the four classes, one after the other; for persistent
  // launches each class is cut into eight equal runs, one per XCD (the
  // items of a class cost the same)
  std::vector<BatchItem> all;
  std::vector<int32_t> ranges(4 * 9, 0);
  for (int cls = 0; cls < 4; ++cls) {
    if (cls == 0 || cls == 2) {
      // advection: the tiles of simple-halo patches first (own launch)
      auto simple = [&](const BatchItem& it) {
        return (recs[size_t(it.patch)].flags & kSimpleHalo) != 0;
      };
      std::stable_partition(items[cls].begin(), items[cls].end(), simple);
      b->nsimple[cls] = int32_t(std::count_if(items[cls].begin(), items[cls].end(), simple));
    }
    b->item0[cls] = int32_t(all.size());
    b->nitems[cls] = int32_t(items[cls].size());
    for (int x = 0; x <= 8; ++x)
      ranges[cls * 9 + x] =
          b->item0[cls] + int32_t(int64_t(b->nitems[cls]) * x / 8);
    all.insert(all.end(), items[cls].begin(), items[cls].end());
  }
  // advection items with their tiles' halo offsets (simple-halo patches;
  // the mirror of each axis is the sign of the velocity in the precision
  // the kernels compute in)
  std::vector<AdvItem> adv(all.size());
  for (int cls = 0; cls < 4; cls += 2) {
    for (int32_t k = b->item0[cls]; k < b->item0[cls] + b->nitems[cls]; ++k) {
      const BatchItem& it = all[size_t(k)];
      const ForestDev& F = b->fh[size_t(it.forest())];
      const PatchRec& r = recs[size_t(it.patch)];
      AdvItem& a = adv[size_t(k)];
      a.h = it;
      a.aux = 0;
      a.halo = AdvHalo{};
      if (!(r.flags & kSimpleHalo)) continue;
      const bool mx = b->precision == 64 ? F.ph.ax < 0.0 : float(F.ph.ax) < 0.0f;
      const bool my = b->precision == 64 ? F.ph.ay < 0.0 : float(F.ph.ay) < 0.0f;
      a.aux = r.level | int(mx) << 8 | int(my) << 9;
      const int T = F.m == 8 ? 8 : b->tile_big;
      a.halo = adv_halo_offsets(T, F.m, F.lm, it.patch, it.tx(), it.ty(), mx, my, r.flags,
                                r.nbr);
    }
    // one simple-halo item per forest reports the forest's Courant number:
    // the first of its finest level (the number is the same on every tile
    // of a level and grows with the level)
    std::vector<int32_t> best(b->fh.size(), -1);
    for (int32_t k = b->item0[cls]; k < b->item0[cls] + b->nsimple[cls]; ++k) {
      const int f = all[size_t(k)].forest();
      const int32_t cur = best[size_t(f)];
      if (cur < 0 || adv[size_t(k)].level() > adv[size_t(cur)].level()) best[size_t(f)] = k;
    }
    for (int32_t k : best)
      if (k >= 0) adv[size_t(k)].aux |= kAdvReports;
  }
  // one packed upload
  const size_t sz[10] = {recs.size() * sizeof(PatchRec), phislot.size() * 4,
                         pforest.size() * 4, b->fh.size() * sizeof(ForestDev),
                         all.size() * sizeof(BatchItem), rx.size() * sizeof(RefluxItem),
                         rfx.size() * 4, first.size() * 4, ranges.size() * 4,
                         adv.size() * sizeof(AdvItem)};
  const void* src[10] = {recs.data(), phislot.data(), pforest.data(), b->fh.data(),
                         all.data(), rx.data(), rfx.data(), first.data(), ranges.data(),
                         adv.data()};
  size_t off[10], at = 0;
  for (int k = 0; k < 10; ++k) { off[k] = at; at += align256(sz[k]); }
  HIPCHK(b->staging.ensure(at));
  for (int k = 0; k < 10; ++k)
    if (sz[k]) std::memcpy(b->staging.p + off[k], src[k], sz[k]);
  HIPCHK(b->blob.ensure(at));
  HIPCHK(hipMemcpy(b->blob.p, b->staging.p, at, hipMemcpyHostToDevice));
  uint8_t* d = b->blob.p;
  b->rec = reinterpret_cast<PatchRec*>(d + off[0]);
  b->phislot = reinterpret_cast<int32_t*>(d + off[1]);
  b->pforest = reinterpret_cast<int32_t*>(d + off[2]);
  b->forests = reinterpret_cast<ForestDev*>(d + off[3]);
  b->items = reinterpret_cast<BatchItem*>(d + off[4]);
  b->advitems = reinterpret_cast<AdvItem*>(d + off[9]);
  b->reflux = reinterpret_cast<RefluxItem*>(d + off[5]);
  b->reflux_forest = reinterpret_cast<int32_t*>(d + off[6]);
  b->first = reinterpret_cast<int32_t*>(d + off[7]);
  b->range = reinterpret_cast<int32_t*>(d + off[8]);
  HIPCHK(b->counters.ensure(4 * 8 * kCounterStride));
  const size_t esz = b->precision == 64 ? 8 : 4;
  HIPCHK(b->phi.ensure(size_t(phi_elems) * esz));
  HIPCHK(b->partial.ensure(size_t(pbase) * 4));
  return FCX_OK;
}

int fcx_batch_create(int32_t n, fcx_ctx* const* forests, fcx_batch** out) {
  if (n <= 0 || !forests || !out) return fail(FCX_EINVAL, "bad arguments");
  if (n >= (1 << 19)) return fail(FCX_EINVAL, "too many forests in one batch");
  *out = nullptr;
  for (int f = 0; f < n; ++f) {
    if (!forests[f] || !forests[f]->have_forest)
      return fail(FCX_ESTATE, "every context needs an uploaded forest");
    if (forests[f]->cfg.precision != forests[0]->cfg.precision)
      return fail(FCX_EINVAL, "all forests of a batch share one precision");
    if (sphere_phys(forests[f]->cfg.physics) || forests[f]->cfg.physics == FCX_SWIRL)
      return fail(FCX_EINVAL, "sphere and prescribed-flow forests are not batched");
  }
  fcx_batch* b = new fcx_batch;
  b->n = n;
  b->ctx.assign(forests, forests + n);
  b->precision = forests[0]->cfg.precision;
  b->cfl_desired = forests[0]->cfg.cfl_desired;
  b->cfl_max = forests[0]->cfg.cfl_max;
  b->redo = forests[0]->cfg.redo;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->cus = prop.multiProcessorCount;
  int rc = batch_build(b);
  if (rc == FCX_OK && (b->err.ensure(size_t(n)) != hipSuccess ||
                       b->ticket.ensure(1) != hipSuccess ||
                       b->stats.ensure(3 * size_t(n)) != hipSuccess))
    rc = fail(FCX_ENOMEM, "hipMalloc failed");
  if (rc == FCX_OK && (hipMemset(b->err.p, 0, 4 * size_t(n)) != hipSuccess ||
                       hipMemset(b->ticket.p, 0, 4) != hipSuccess ||
                       hipMemset(b->stats.p, 0, 24 * size_t(n)) != hipSuccess))
    rc = fail(FCX_EHIP, "hipMemset failed");
  if (rc != FCX_OK) { delete b; return rc; }
  *out = b;
  return FCX_OK;
}

int fcx_batch_destroy(fcx_batch* b) {
  delete b;
  return FCX_OK;
}

int64_t fcx_batch_state_elems(const fcx_batch* b) { return b ? b->state_elems : -1; }
int64_t fcx_batch_state_offset(const fcx_batch* b, int32_t f) {
  return (b && f >= 0 && f < b->n) ? b->state_off[f] : -1;
}
int64_t fcx_batch_num_patches(const fcx_batch* b) { return b ? b->P : -1; }

int fcx_batch_set_tuning(fcx_batch* b, int32_t tile_big, int32_t threads8,
                         int32_t threads16, int32_t persistent) {
  if (!b || (tile_big != 8 && tile_big != 16) || (threads8 != 64 && threads8 != 128) ||
      (threads16 != 256 && threads16 != 512) || (persistent != 0 && persistent != 1))
    return fail(FCX_EINVAL, "bad tuning");
  const bool rebuild = tile_big != b->tile_big;
  b->tile_big = tile_big;
  b->threads8 = threads8;
  b->threads16 = threads16;
  b->persistent = persistent;
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return rebuild ? batch_build(b) : FCX_OK;
}

template <typename R, int PHYS, int T, int NT>
static int launch_batch_class(fcx_batch* b, int cls, const void* q, void* qn,
                              const double* dt, double* numax, hipStream_t s) {
  if (b->nitems[cls] == 0) return FCX_OK;
  BatchArgs<R> B;
  B.q = static_cast<const R*>(q);
  B.qn = static_cast<R*>(qn);
  B.dt = dt;
  B.numax = numax;
  B.rec = b->rec;
  B.phislot = b->phislot;
  B.pforest = b->pforest;
  B.forests = b->forests;
  B.phi = reinterpret_cast<R*>(b->phi.p);
  B.err = b->err.p;
  B.items = b->items;
  B.advitems = b->advitems;
  B.item0 = b->item0[cls];
  B.nitems = b->nitems[cls];
  B.range = b->range + cls * 9;
  B.counters = b->counters.p + cls * 8 * kCounterStride;
  // advection: one wavefront per item, kAdvWaves per workgroup
  constexpr bool ADV = PHYS == FCX_ADVECTION;
  constexpr int threads = ADV ? 64 * kAdvWaves : NT;
  if (b->persistent) {
    // about as many workgroups as the LDS lets be resident (at most one per
    // item), a multiple of 8 so that every XCD starts on its own counter;
    // any beyond residency start late, find the ranges spent and exit
    const int lds = ADV ? int(kAdvWaves * sizeof(AdvLds<R, T>))
                        : int(sizeof(TileLds<R, PHYS, T, NT>));
    const int per_cu = std::max(1, std::min(160 * 1024 / (lds + 64), 32 * 64 / threads));
    const int per_wg = ADV ? kAdvWaves : 1;
    int grid = std::min(b->cus * per_cu, (b->nitems[cls] + per_wg * 8 - 1) / (per_wg * 8) * 8);
    grid = std::max(8, (grid + 7) / 8 * 8);
    // a fill kernel, not a memset: the launch may be captured into a graph
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(8 * kCounterStride), 0, s, B.counters,
                       8 * kCounterStride);
    if constexpr (ADV) {
      if (b->mc2[cls])
        hipLaunchKernelGGL((k_batch_adv_persist<R, T, 1>), dim3(unsigned(grid)),
                           dim3(threads), 0, s, B);
      else
        hipLaunchKernelGGL((k_batch_adv_persist<R, T, 0>), dim3(unsigned(grid)),
                           dim3(threads), 0, s, B);
    } else if (b->mc2[cls]) {
      hipLaunchKernelGGL((k_batch_persist<R, PHYS, T, NT, 1>), dim3(unsigned(grid)), dim3(NT),
                         0, s, B);
    } else {
      hipLaunchKernelGGL((k_batch_persist<R, PHYS, T, NT, 0>), dim3(unsigned(grid)), dim3(NT),
                         0, s, B);
    }
  } else if constexpr (ADV) {
    const int32_t ns = b->nsimple[cls], ng = b->nitems[cls] - ns;
    const dim3 gs(unsigned((ns + kAdvWaves - 1) / kAdvWaves));
    const dim3 gg(unsigned((ng + kAdvWaves - 1) / kAdvWaves));
    const bool spec = b->mc2[cls];
    // both runs present: the general tiles go to the side stream, forked
    // here (after the work before this class) and joined before the reflux
    const bool fork = ns > 0 && ng > 0;
    if (fork) {
      if (!b->side) HIPCHK(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
      if (!b->fork[cls]) HIPCHK(hipEventCreateWithFlags(&b->fork[cls], hipEventDisableTiming));
      if (!b->join[cls]) HIPCHK(hipEventCreateWithFlags(&b->join[cls], hipEventDisableTiming));
      HIPCHK(hipEventRecord(b->fork[cls], s));
      HIPCHK(hipStreamWaitEvent(b->side, b->fork[cls], 0));
    }
    if (ns > 0) {
      // the strip-halo items: resident wavefronts walking runs of items
      B.nitems = ns;
      const dim3 gr(
          unsigned(std::min<int64_t>(int64_t(b->cus) * AdvRunBlocks<R, T>::value, gs.x)));
      if (spec)
        hipLaunchKernelGGL((k_batch_adv_run<R, T, 1>), gr, dim3(threads), 0, s, B);
      else
        hipLaunchKernelGGL((k_batch_adv_run<R, T, 0>), gr, dim3(threads), 0, s, B);
    }
    if (ng > 0) {
      B.item0 = b->item0[cls] + ns;
      B.nitems = ng;
      hipStream_t sg = fork ? b->side : s;
      if (spec)
        hipLaunchKernelGGL((k_batch_adv<R, T, kHaloGeneral, 1>), gg, dim3(threads), 0, sg, B);
      else
        hipLaunchKernelGGL((k_batch_adv<R, T, kHaloGeneral, 0>), gg, dim3(threads), 0, sg, B);
      if (fork) {
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(b->join[cls], b->side));
        b->joined[cls] = true;
      }
    }
  } else if (b->mc2[cls]) {
    hipLaunchKernelGGL((k_batch_step<R, PHYS, T, NT, 1>), dim3(unsigned(b->nitems[cls])),
                       dim3(NT), 0, s, B);
  } else {
    hipLaunchKernelGGL((k_batch_step<R, PHYS, T, NT, 0>), dim3(unsigned(b->nitems[cls])),
                       dim3(NT), 0, s, B);
  }
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

template <typename R>
static int batch_step_t(fcx_batch* b, const void* q, void* qn, double* dt,
                        double* numax, int32_t* status, hipStream_t s) {
  const bool t8 = b->threads8 == 128, t16 = b->threads16 == 512;
  int rc = t8 ? launch_batch_class<R, FCX_ADVECTION, 8, 128>(b, 0, q, qn, dt, numax, s)
              : launch_batch_class<R, FCX_ADVECTION, 8, 64>(b, 0, q, qn, dt, numax, s);
  if (rc == FCX_OK)
    rc = t8 ? launch_batch_class<R, FCX_SHALLOW, 8, 128>(b, 1, q, qn, dt, numax, s)
            : launch_batch_class<R, FCX_SHALLOW, 8, 64>(b, 1, q, qn, dt, numax, s);
  if (rc == FCX_OK)
    rc = t16 ? launch_batch_class<R, FCX_ADVECTION, 16, 512>(b, 2, q, qn, dt, numax, s)
             : launch_batch_class<R, FCX_ADVECTION, 16, 256>(b, 2, q, qn, dt, numax, s);
  if (rc == FCX_OK)
    rc = t16 ? launch_batch_class<R, FCX_SHALLOW, 16, 512>(b, 3, q, qn, dt, numax, s)
             : launch_batch_class<R, FCX_SHALLOW, 16, 256>(b, 3, q, qn, dt, numax, s);
  if (rc != FCX_OK) return rc;
  for (int k = 0; k < 4; ++k)
    if (b->joined[k]) {
      HIPCHK(hipStreamWaitEvent(s, b->join[k], 0));
      b->joined[k] = false;
    }
  for (int axis = 0; axis < 2; ++axis) {
    const int32_t n = axis == 0 ? b->n_reflux_x : b->n_reflux_y;
    if (n == 0) continue;
    const int32_t o = axis == 0 ? 0 : b->n_reflux_x;
    const int64_t tot = int64_t(n) * 32;
    hipLaunchKernelGGL((k_batch_reflux<R>), dim3(unsigned((tot + 255) / 256)), dim3(256),
                       0, s, static_cast<const R*>(q), static_cast<R*>(qn),
                       b->reflux + o, b->reflux_forest + o, n, b->rec, b->phislot,
                       b->forests, reinterpret_cast<const R*>(b->phi.p), dt, b->err.p,
                       numax, b->cfl_max, b->redo);
    HIPCHK(hipGetLastError());
  }
  NextDtArgs nd{};
  nd.numax = numax;
  nd.dt = dt;
  nd.status = status;
  nd.ticket = b->ticket.p;
  nd.stats = b->stats.p;
  nd.cfl_desired = b->cfl_desired;
  nd.cfl_max = b->cfl_max;
  nd.redo = b->redo;
  hipLaunchKernelGGL((k_batch_next_dt<R>), dim3(unsigned(b->n * kBatchRedoParts)), dim3(256),
                     0, s, static_cast<const R*>(q), static_cast<R*>(qn), b->forests,
                     b->first, b->n, nd, b->err.p);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_batch_class_items(const fcx_batch* b, int32_t* items, int32_t* simple) {
  if (!b || !items || !simple) return fail(FCX_EINVAL, "bad arguments");
  for (int c = 0; c < 4; ++c) {
    items[c] = b->nitems[c];
    simple[c] = (c == 0 || c == 2) ? b->nsimple[c] : 0;
  }
  return FCX_OK;
}

int fcx_batch_step_stats(const fcx_batch* b, int64_t* out) {
  if (!b || !out) return fail(FCX_EINVAL, "bad arguments");
  HIPCHK(hipMemcpy(out, b->stats.p, 3 * sizeof(int64_t) * size_t(b->n),
                   hipMemcpyDeviceToHost));
  return FCX_OK;
}

int fcx_batch_step(fcx_batch* b, const void* q, void* qn, double* dt, double* numax,
                   int32_t* status, void* stream) {
  if (!b || !q || !qn || q == qn || !dt || !numax || !status)
    return fail(FCX_EINVAL, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return b->precision == 64 ? batch_step_t<double>(b, q, qn, dt, numax, status, s)
                            : batch_step_t<float>(b, q, qn, dt, numax, status, s);
}

int fcx_batch_capture(fcx_batch* b, int32_t steps, void* qa, void* qb, double* dt,
                      double* numax, int32_t* status) {
  if (!b || steps <= 0 || !qa || !qb || qa == qb || !dt || !numax || !status)
    return fail(FCX_EINVAL, "bad arguments");
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  int rc = FCX_OK;
  for (int k = 0; k < steps && rc == FCX_OK; ++k) {
    void* src = (k & 1) ? qb : qa;
    void* dst = (k & 1) ? qa : qb;
    rc = fcx_batch_step(b, src, dst, dt, numax, status, b->cap);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc != FCX_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
  HIPCHK(e);
  b->graph = g;
  HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return FCX_OK;
}

int fcx_batch_replay(fcx_batch* b, void* stream) {
  if (!b || !b->exec) return fail(FCX_ESTATE, "nothing captured");
  HIPCHK(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return FCX_OK;
}

template <typename R>
static int batch_sums_t(fcx_batch* b, const void* q, double* sums, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_sums_patch<R>), dim3(unsigned(b->P)), dim3(256), 0, s,
                     static_cast<const R*>(q), b->rec, b->pforest, b->forests,
                     b->partial.p);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL((k_sums_reduce<4>), dim3(unsigned(b->n)), dim3(1024), 0, s,
                     b->partial.p, b->first, sums);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_batch_sums(fcx_batch* b, const void* q, double* sums, void* stream) {
  if (!b || !q || !sums) return fail(FCX_EINVAL, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return b->precision == 64 ? batch_sums_t<double>(b, q, sums, s)
                            : batch_sums_t<float>(b, q, sums, s);
}

// ---- learned tagging ----------------------------------------------------

int fcx_features(fcx_ctx* c, const void* q, const void* ghost, float* feats,
                 void* stream) {
  if (!c || !q || !ghost || !feats) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  if (sphere_phys(c->cfg.physics)) return fail(FCX_EINVAL, "no features on the sphere");
  if (c->cur.P == 0) return FCX_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned grid = unsigned(c->cur.P);
  const int m = c->cfg.m;
  const bool dp = c->cfg.precision == 64;
  if (c->meqn == 1) {
    if (dp)
      hipLaunchKernelGGL((k_features<double, 1>), dim3(grid), dim3(256), 0, s,
                         static_cast<const double*>(q), static_cast<const double*>(ghost),
                         c->cur.rec, m, feats);
    else
      hipLaunchKernelGGL((k_features<float, 1>), dim3(grid), dim3(256), 0, s,
                         static_cast<const float*>(q), static_cast<const float*>(ghost),
                         c->cur.rec, m, feats);
  } else {
    if (dp)
      hipLaunchKernelGGL((k_features<double, 3>), dim3(grid), dim3(256), 0, s,
                         static_cast<const double*>(q), static_cast<const double*>(ghost),
                         c->cur.rec, m, feats);
    else
      hipLaunchKernelGGL((k_features<float, 3>), dim3(grid), dim3(256), 0, s,
                         static_cast<const float*>(q), static_cast<const float*>(ghost),
                         c->cur.rec, m, feats);
  }
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

static unsigned mlp_grid(int64_t rows, int64_t blocks_per_wave, unsigned cap) {
  const int64_t blocks = (rows + 15) / 16;
  const int64_t wg = (blocks + 4 * blocks_per_wave - 1) / (4 * blocks_per_wave);
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(wg, cap)));
}

int fcx_mlp_forward(const float* params, const float* norm, int64_t rows,
                    const float* x, float* logits, void* stream) {
  if (!params || !norm || rows < 0 || (rows > 0 && (!x || !logits)) ||
      rows > (int64_t(1) << 40))
    return fail(FCX_EINVAL, "bad arguments");
  if (rows == 0) return FCX_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_grid(rows, 1, 2048)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), params, norm, x, rows, logits);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_mlp_backward(const float* params, const float* norm, int64_t rows,
                     const float* x, const int32_t* labels, const float* class_weight,
                     float scale, float* grad, float* loss, void* stream) {
  if (!params || !norm || !class_weight || !grad || !loss || rows < 0 ||
      (rows > 0 && (!x || !labels)) || rows > (int64_t(1) << 40))
    return fail(FCX_EINVAL, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_zero_f32, dim3((kMlpParams + 255) / 256), dim3(256), 0, s,
                     grad, int64_t(kMlpParams));
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, loss, int64_t(1));
  HIPCHK(hipGetLastError());
  if (rows == 0) return FCX_OK;
  hipLaunchKernelGGL(k_mlp_backward, dim3(mlp_grid(rows, 4, 256)), dim3(256), 0, s,
                     params, norm, x, labels, class_weight, scale, rows, grad, loss);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_adam_step(int64_t n, float* params, const float* grad, float* m1, float* m2,
                  int32_t t, float lr, float beta1, float beta2, float eps,
                  void* stream) {
  if (n < 0 || t < 1 || (n > 0 && (!params || !grad || !m1 || !m2)) ||
      !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps >= 0.0f))
    return fail(FCX_EINVAL, "bad arguments");
  if (n == 0) return FCX_OK;
  hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), params, grad, m1, m2, n, t, lr,
                     beta1, beta2, eps);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_learned_tags(int64_t rows, const float* logits, const int8_t* plain,
                     float confidence, int8_t* tags, void* stream) {
  if (rows < 0 || (rows > 0 && (!logits || !plain || !tags)))
    return fail(FCX_EINVAL, "bad arguments");
  if (rows == 0) return FCX_OK;
  hipLaunchKernelGGL(k_learned_tags, dim3(unsigned((rows + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), logits, plain, rows, confidence,
                     tags);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_dilate_tags(fcx_ctx* c, const int8_t* in, int32_t lmax, int8_t* out,
                    void* stream) {
  if (!c || !in || !out || in == out) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  const int64_t P = c->cur.P;
  if (P == 0) return FCX_OK;
  hipLaunchKernelGGL(k_dilate_tags, dim3(unsigned((P + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), in, c->cur.rec, P, lmax, out);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

// ---- cubed sphere ---------------------------------------------------------

int fcx_sphere_geometry(fcx_ctx* c, double* geo, void* stream) {
  if (!c || !geo) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  if (!sphere_phys(c->cfg.physics)) return fail(FCX_EINVAL, "not a sphere context");
  const size_t FR = size_t(c->cfg.m + 4) * (c->cfg.m + 4);
  HIPCHK(hipMemcpyAsync(geo, c->cur.geo.p, sizeof(double) * c->cur.P * kGeoN * FR,
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return FCX_OK;
}

// ---- one whole step --------------------------------------------------------

int fcx_advance(fcx_ctx* c, const void* q, void* qn, double* dt, double* numax,
                int32_t* status, void* stream) {
  if (!c || !status) return fail(FCX_EINVAL, "bad arguments");
  int rc = fcx_fused_step(c, q, qn, dt, numax, stream);
  if (rc != FCX_OK) return rc;
  // reflux and next dt (and the copy of a rejected attempt) in one launch
  hipStream_t s = static_cast<hipStream_t>(stream);
  const NextDtArgs nd = next_args(c, numax, dt, status, c->cfg.redo);
  const bool dp = c->cfg.precision == 64;
  if (c->cfg.physics == FCX_ADVECTION || c->cfg.physics == FCX_SWIRL)
    return dp ? launch_reflux<double, FCX_ADVECTION, true>(c, q, qn, dt, s, nd)
              : launch_reflux<float, FCX_ADVECTION, true>(c, q, qn, dt, s, nd);
  return dp ? launch_reflux<double, FCX_SHALLOW, true>(c, q, qn, dt, s, nd)
            : launch_reflux<float, FCX_SHALLOW, true>(c, q, qn, dt, s, nd);
}

// ---- sub-cycled step ----------------------------------------------------------
// One step of the coarsest level with per-level time steps (level l: dt 2^-l),
// coarse to fine: for each substep of a level, a ghost fill of that level's
// patches at the substep's time (coarser levels read in the middle of their
// own steps, interpolated in time), the step of those patches, and the
// fine-side terms of their faces with the next coarser level; after the two
// substeps of the next finer level, the correction of this level's cells at
// faces with it.  Buffers: q (state at the start, never written), q_new
// (result) and w (work): level lmin steps q -> q_new; a finer level's i-th
// substep goes q -> w (i = 1), w -> q_new (i even), q_new -> w (i odd > 1),
// so every level ends in q_new and q stays available for a redo.
namespace {

struct SubPlan {
  int lmin, lmax;
  // the actions of one coarse step, in order: a substep of a level (ghost
  // fill, step, fine-side terms) or the correction of a level's cells
  struct Action {
    int correct;                    // 0: substep of `level`; 1: correct `level`
    int level, sub, src, dst;       // buffers: 0 q, 1 q_new, 2 w (dst: corrected)
    int qc_old;                     // coarse level's step-start buffer (psi)
    int add;                        // psi: accumulate (second fine substep)
    int table;                      // substeps: index of its level table
  };
  std::vector<Action> actions;
  std::vector<LevelSrc> tables;     // kLevels per substep
};

struct SubState {
  int cur[kLevels], old[kLevels];
  double t0[kLevels];
};

void sub_recurse(SubPlan& sp, SubState& st, int l, double t, int sub) {
  const double dtr = std::ldexp(1.0, -(l - sp.lmin));   // in coarse steps
  const int src = l == sp.lmin ? 0 : (sub == 1 ? 0 : (sub % 2 == 0 ? 2 : 1));
  const int dst = l == sp.lmin ? 1 : (sub % 2 == 1 ? 2 : 1);
  // where each level is read at time t
  const int table = int(sp.tables.size() / kLevels);
  for (int v = 0; v < kLevels; ++v) {
    LevelSrc e{st.cur[v], st.cur[v], 0.0};
    if (v >= sp.lmin && v < l) {
      const double dv = std::ldexp(1.0, -(v - sp.lmin));
      e = LevelSrc{st.cur[v], st.old[v], (t - st.t0[v]) / dv};
    } else if (v == l) {
      e = LevelSrc{src, src, 0.0};
    }
    sp.tables.push_back(e);
  }
  sp.actions.push_back(SubPlan::Action{0, l, sub, src, dst, l > sp.lmin ? st.old[l - 1] : -1,
                                       sub % 2 == 0, table});
  st.old[l] = src;
  st.cur[l] = dst;
  st.t0[l] = t;
  if (l < sp.lmax) {
    sub_recurse(sp, st, l + 1, t, 2 * sub - 1);
    sub_recurse(sp, st, l + 1, t + 0.5 * dtr, 2 * sub);
    sp.actions.push_back(SubPlan::Action{1, l, sub, -1, st.cur[l], -1, 0, -1});
  }
}

}  // namespace

template <typename R, int PHYS, int T, int NT>
static void launch_step_level(fcx_ctx* c, const R* q, const R* ghost, R* qn, const double* dt,
                              double* numax, const int32_t* list, int32_t n, hipStream_t s) {
  StepArgs<R> a;
  a.q = q;
  a.ghost = ghost;
  a.qn = qn;
  a.dt = dt;
  a.numax = numax;
  a.rec = c->cur.rec;
  a.phislot = c->cur.phislot;
  a.phi = reinterpret_cast<R*>(c->phi.p);
  a.err = c->err.p;
  a.P = int32_t(c->cur.P);
  a.m = c->cfg.m;
  a.lm = log2i(c->cfg.m);
  const int tps = c->cfg.m / T;
  a.ntiles = n * tps * tps;
  a.ph = kphys(c);
  // the limiter and transverse mode fixed when compiling exactly where the
  // global-dt step fixes them (the two then round alike)
  const bool spec = c->cfg.limiter == 4 && c->cfg.transverse == 2;
  const dim3 agrid(unsigned((a.ntiles + kAdvWaves - 1) / kAdvWaves));
  if constexpr (PHYS == FCX_ADVECTION) {
    if (spec)
      hipLaunchKernelGGL((k_adv_step_level<R, T, 1>), agrid, dim3(64 * kAdvWaves), 0, s, a,
                         list);
    else
      hipLaunchKernelGGL((k_adv_step_level<R, T, 0>), agrid, dim3(64 * kAdvWaves), 0, s, a,
                         list);
  } else if (spec) {
    hipLaunchKernelGGL((k_step_level<R, PHYS, T, NT, 1>), dim3(unsigned(a.ntiles)), dim3(NT),
                       0, s, a, list);
  } else {
    hipLaunchKernelGGL((k_step_level<R, PHYS, T, NT, 0>), dim3(unsigned(a.ntiles)), dim3(NT),
                       0, s, a, list);
  }
}

template <typename R, int PHYS>
static int subcycled_t(fcx_ctx* c, const void* q, void* qn, void* w, void* ghost, double* dt,
                       double* numax, int32_t* status, hipStream_t s) {
  constexpr int MEQN = PhysTraits<PHYS>::MEQN;
  const int m = c->cfg.m, lm = log2i(m), G = 8 * m + 16;
  const auto& lf = c->cur.level_first;
  int lmin = -1, lmax = -1;
  for (int l = 0; l < kLevels; ++l)
    if (lf[l + 1] > lf[l]) {
      if (lmin < 0) lmin = l;
      lmax = l;
    }
  if (lmin < 0) return fail(FCX_ESTATE, "empty forest");
  SubPlan sp;
  sp.lmin = lmin;
  sp.lmax = lmax;
  SubState st;
  for (int v = 0; v < kLevels; ++v) { st.cur[v] = 0; st.old[v] = 0; st.t0[v] = 0.0; }
  sub_recurse(sp, st, lmin, 0.0, 1);
  // the tables depend on the level range only: upload when it changes
  if (c->sub_lmin != lmin || c->sub_lmax != lmax) {
    const size_t bytes = sp.tables.size() * sizeof(LevelSrc);
    HIPCHK(hipStreamSynchronize(s));          // the pinned copy may be in use
    HIPCHK(c->sub_host.ensure(bytes));
    std::memcpy(c->sub_host.p, sp.tables.data(), bytes);
    HIPCHK(c->tables.ensure(sp.tables.size()));
    HIPCHK(hipMemcpyAsync(c->tables.p, c->sub_host.p, bytes, hipMemcpyHostToDevice, s));
    c->sub_lmin = lmin;
    c->sub_lmax = lmax;
  }
  const size_t esz = sizeof(R);
  HIPCHK(c->psi.ensure(size_t(c->cur.nslots) * 4 * m * MEQN * esz + 256));
  HIPCHK(c->dtl.ensure(kLevels));
  hipLaunchKernelGGL(k_level_dts, dim3(1), dim3(kLevels), 0, s, dt, c->dtl.p);
  R* bufs[3] = {const_cast<R*>(static_cast<const R*>(q)), static_cast<R*>(qn),
                static_cast<R*>(w)};
  TimeView<R> tv;
  for (int b = 0; b < 3; ++b) tv.bufs[b] = bufs[b];
  const int32_t nitems = c->cur.n_reflux_x + c->cur.n_reflux_y;
  const bool wide = wide_tiles(c, c->cur.P);   // as the global-dt step
  R* psi = reinterpret_cast<R*>(c->psi.p);
  const R* phi = reinterpret_cast<const R*>(c->phi.p);
  int64_t cells = 0;
  const unsigned ig = unsigned(std::max<int64_t>(1, (int64_t(nitems) * m + 255) / 256));
  for (const SubPlan::Action& A : sp.actions) {
    if (A.correct) {
      if (nitems > 0) {
        hipLaunchKernelGGL((k_subcycle_reflux<R, PHYS>), dim3(ig), dim3(256), 0, s,
                           bufs[A.dst], c->cur.reflux, c->cur.aux, nitems, phi, psi,
                           c->dtl.p, m, int32_t(A.level));
        HIPCHK(hipGetLastError());
      }
      continue;
    }
    const int32_t n = lf[A.level + 1] - lf[A.level];
    const int32_t* list = c->cur.bylevel + lf[A.level];
    if (n > 0) {
      tv.src = c->tables.p + size_t(A.table) * kLevels;
      hipLaunchKernelGGL((k_ghost_fill_level<R, PHYS>),
                         dim3(unsigned((int64_t(n) * G + 255) / 256)), dim3(256), 0, s, list, n,
                         static_cast<R*>(ghost), c->cur.rec, m, lm, c->err.p, tv);
      const R* gq = static_cast<const R*>(ghost);
      const double* dtlev = c->dtl.p + A.level;
      if (c->tile == 8)
        wide ? launch_step_level<R, PHYS, 8, 128>(c, bufs[A.src], gq, bufs[A.dst], dtlev, numax,
                                                  list, n, s)
             : launch_step_level<R, PHYS, 8, 64>(c, bufs[A.src], gq, bufs[A.dst], dtlev, numax,
                                                 list, n, s);
      else
        wide ? launch_step_level<R, PHYS, 16, 512>(c, bufs[A.src], gq, bufs[A.dst], dtlev,
                                                   numax, list, n, s)
             : launch_step_level<R, PHYS, 16, 256>(c, bufs[A.src], gq, bufs[A.dst], dtlev,
                                                   numax, list, n, s);
      HIPCHK(hipGetLastError());
      cells += int64_t(n) * m * m;
    }
    if (A.level > lmin && nitems > 0) {
      hipLaunchKernelGGL((k_psi_accumulate<R, PHYS>), dim3(ig), dim3(256), 0, s,
                         bufs[A.qc_old], bufs[A.src], c->cur.reflux, c->cur.aux, nitems, phi,
                         psi, m, kphys(c), int32_t(A.level - 1), 0.5, int32_t(A.add),
                         c->err.p);
      HIPCHK(hipGetLastError());
    }
  }
  // CFL check, next dt and (redo on) the copy of a rejected attempt
  NextDtArgs nd = next_args(c, numax, dt, status, c->cfg.redo);
  nd.cells = cells;
  nd.tscale = std::ldexp(1.0, -lmin);       // a coarse step lasts dt 2^-lmin
  hipLaunchKernelGGL(k_next_dt_redo, dim3(unsigned(redo_grid(c, nd.n16))), dim3(256), 0, s,
                     static_cast<const uint4*>(q), static_cast<uint4*>(qn), nd, c->err.p);
  HIPCHK(hipGetLastError());
  return FCX_OK;
}

int fcx_advance_subcycled(fcx_ctx* c, const void* q, void* q_new, void* work, void* ghost,
                          double* dt, double* nu_max, int32_t* status, void* stream) {
  if (!c || !q || !q_new || !work || !ghost || !dt || !nu_max || !status ||
      q == q_new || q == work || q_new == work)
    return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  if (sphere_phys(c->cfg.physics)) return fail(FCX_EINVAL, "no sub-cycled step on the sphere");
  if (c->cfg.physics == FCX_SWIRL)
    return fail(FCX_EINVAL, "no sub-cycled step for the prescribed flow");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dp = c->cfg.precision == 64;
  if (c->cfg.physics == FCX_ADVECTION)
    return dp ? subcycled_t<double, FCX_ADVECTION>(c, q, q_new, work, ghost, dt, nu_max, status, s)
              : subcycled_t<float, FCX_ADVECTION>(c, q, q_new, work, ghost, dt, nu_max, status, s);
  return dp ? subcycled_t<double, FCX_SHALLOW>(c, q, q_new, work, ghost, dt, nu_max, status, s)
            : subcycled_t<float, FCX_SHALLOW>(c, q, q_new, work, ghost, dt, nu_max, status, s);
}

// ---- tags and mesh change in one call ---------------------------------------

int fcx_regrid(fcx_ctx* c, const void* q, void* ghost, int32_t criterion, double threshold,
               int32_t lmin, int32_t lmax, int64_t* n_new, int64_t* old_to_new,
               void* stream) {
  if (!c || !q || !ghost || !n_new) return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  const int64_t P = c->cur.P;
  HIPCHK(c->tags_dev.ensure(size_t(P)));
  HIPCHK(c->tags_host.ensure(size_t(P)));
  int rc = fcx_ghost_fill(c, q, ghost, stream);
  if (rc != FCX_OK) return rc;
  // the tag kernels write the tags into pinned host memory as well (no copy
  // after them)
  rc = regrid_tags(c, q, ghost, criterion, threshold, lmin, lmax, c->tags_dev.p, stream,
                   reinterpret_cast<int8_t*>(c->tags_host.p));
  if (rc != FCX_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the host planner is the next step of the critical path: poll for the
  // tags rather than sleep until the runtime wakes this thread
  if (!c->tags_ready) HIPCHK(hipEventCreateWithFlags(&c->tags_ready, hipEventDisableTiming));
  HIPCHK(hipEventRecord(c->tags_ready, s));
  for (;;) {
    const hipError_t e = hipEventQuery(c->tags_ready);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) HIPCHK(e);
  }
  return regrid_apply(c, reinterpret_cast<const int8_t*>(c->tags_host.p), lmin, lmax, n_new,
                      old_to_new, s, true);
}

// ---- a run of many steps ----------------------------------------------------

int fcx_run(fcx_ctx* c, int32_t fused, void* q0, void* q1, int64_t cap, void* ghost,
            int64_t ghost_cap, int32_t steps, int32_t step0, int32_t regrid_every,
            int32_t criterion,
            double threshold, int32_t lmin, int32_t lmax, double* dt, double* nu_max,
            int32_t* status, int32_t* which, int64_t* cell_updates, void* stream) {
  if (!c || !q0 || !q1 || !ghost || !dt || !nu_max || !status || !which || !cell_updates ||
      steps < 0 || step0 < 0 || regrid_every < 0 || q0 == q1)
    return fail(FCX_EINVAL, "bad arguments");
  if (!c->have_forest) return fail(FCX_ESTATE, "no forest uploaded");
  if (fused < 0 || fused > 2) return fail(FCX_EINVAL, "mode must be 0, 1 or 2");
  if (sphere_phys(c->cfg.physics) && fused)
    return fail(FCX_EINVAL, "no fused or sub-cycled run on the sphere");
  void* buf[2] = {q0, q1};
  int cur = 0;
  int64_t cells = 0;
  const int64_t mm = int64_t(c->cfg.m) * c->cfg.m;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool redo = c->cfg.redo != 0;
  // with redo on, the accepted cell updates are counted on the device: a
  // copy of the counters before the run and one after it
  int64_t* counts = nullptr;
  if (redo) {
    HIPCHK(c->run_host.ensure(6 * sizeof(int64_t)));
    counts = reinterpret_cast<int64_t*>(c->run_host.p);
    HIPCHK(hipMemcpyAsync(counts, c->stats.p, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  }
  for (int32_t k = 0; k < steps; ++k) {
    const int64_t n = int64_t(step0) + k;
    if (regrid_every > 0 && n > 0 && n % regrid_every == 0) {
      if (fcx_ghost_elems(c) > ghost_cap) return fail(FCX_ENOMEM, "ghost capacity exceeded");
      int64_t pn = 0;
      int rc = fcx_regrid(c, buf[cur], ghost, criterion, threshold, lmin, lmax, &pn, nullptr,
                          stream);
      if (rc != FCX_OK) return rc;
      if (fcx_state_elems(c) > cap) return fail(FCX_ENOMEM, "state capacity exceeded");
      rc = fcx_regrid_transfer(c, buf[cur], ghost, buf[1 - cur], stream);
      if (rc != FCX_OK) return rc;
      cur = 1 - cur;
    }
    if (fcx_state_elems(c) > cap) return fail(FCX_ENOMEM, "state capacity exceeded");
    int rc;
    if (fused == 2) {
      if (fcx_ghost_elems(c) > ghost_cap) return fail(FCX_ENOMEM, "ghost capacity exceeded");
      const size_t wbytes = size_t(fcx_state_elems(c)) * (c->cfg.precision / 8);
      HIPCHK(c->sub_work.ensure(wbytes));
      rc = fcx_advance_subcycled(c, buf[cur], buf[1 - cur], c->sub_work.p, ghost, dt, nu_max,
                                 status, stream);
    } else if (fused) {
      rc = fcx_advance(c, buf[cur], buf[1 - cur], dt, nu_max, status, stream);
    } else {
      if (fcx_ghost_elems(c) > ghost_cap) return fail(FCX_ENOMEM, "ghost capacity exceeded");
      rc = fcx_ghost_fill(c, buf[cur], ghost, stream);
      if (rc == FCX_OK) rc = fcx_patch_step(c, buf[cur], ghost, buf[1 - cur], dt, nu_max, stream);
      if (rc == FCX_OK) rc = fcx_reflux(c, buf[cur], buf[1 - cur], dt, stream);
      if (rc == FCX_OK)
        rc = redo ? next_dt_redo(c, buf[cur], buf[1 - cur], nu_max, dt, status, s)
                  : fcx_next_dt(c, nu_max, dt, status, stream);
    }
    if (rc != FCX_OK) return rc;
    cur = 1 - cur;
    if (fused == 2) {
      const auto& lf = c->cur.level_first;
      int lmin = -1;
      for (int l = 0; l < kLevels && lmin < 0; ++l)
        if (lf[l + 1] > lf[l]) lmin = l;
      for (int l = lmin; l < kLevels; ++l)
        cells += int64_t(lf[l + 1] - lf[l]) * mm << (l - lmin);
    } else {
      cells += c->cur.P * mm;
    }
  }
  if (redo) {
    HIPCHK(hipMemcpyAsync(counts + 3, c->stats.p, 3 * sizeof(int64_t), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    cells = counts[5] - counts[2];
  }
  *which = cur;
  *cell_updates = cells;
  return FCX_OK;
}
