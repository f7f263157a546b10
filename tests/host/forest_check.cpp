// Host check of the forest code: random forests on one walled tree, one
// periodic tree and two trees glued with a reversed face go through balance,
// regrid, the transfer plan, plan updates and fresh plan builds, with lookups
// that hit and miss.  It prints one digest per forest (the caller compares
// builds with different lookup structures) and exits non-zero if an updated
// plan, written over the storage of an older one, differs from a fresh build,
// or if the transfer plan the regrid emits differs from transfer_plan's.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "forest.hpp"

using namespace fcx;

static uint64_t H = 1469598103934665603ull;
static void mix(const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  for (size_t i = 0; i < n; ++i) { H ^= b[i]; H *= 1099511628211ull; }
}
template <class T> static void mixv(const std::vector<T>& v) {
  const size_t n = v.size();
  mix(&n, sizeof n);
  if (n) mix(v.data(), n * sizeof(T));
}
static void mixplan(const Plan& p) {
  mixv(p.recs); mixv(p.phislot); mixv(p.family); mixv(p.item_first); mixv(p.reflux);
  mix(&p.nslots, sizeof p.nslots);
}
static bool same(const Plan& a, const Plan& b) {
  return a.recs.size() == b.recs.size() && a.nslots == b.nslots &&
         std::memcmp(a.recs.data(), b.recs.data(), a.recs.size() * sizeof(PatchRec)) == 0 &&
         a.phislot == b.phislot && a.family == b.family && a.item_first == b.item_first &&
         a.reflux.size() == b.reflux.size() &&
         std::memcmp(a.reflux.data(), b.reflux.data(), a.reflux.size() * sizeof(RefluxItem)) == 0;
}

int main() {
  std::mt19937 rng(7);
  int mismatches = 0;
  for (int trial = 0; trial < 60; ++trial) {
    std::vector<fcx_tree> trees;
    const int shape = trial % 3;
    if (shape < 2) {
      trees.resize(1);
      for (int f = 0; f < 4; ++f) {
        trees[0].nbr_tree[f] = shape ? 0 : -1;
        trees[0].nbr_face[f] = shape ? (f ^ 1) : -1;
        trees[0].orient[f] = 0;
        trees[0].bc[f] = shape ? 0 : 1;
      }
    } else {
      trees.resize(2);
      for (int t = 0; t < 2; ++t)
        for (int f = 0; f < 4; ++f) {
          trees[t].nbr_tree[f] = -1; trees[t].nbr_face[f] = -1;
          trees[t].orient[f] = 0; trees[t].bc[f] = 1;
        }
      for (int t = 0; t < 2; ++t) {
        trees[t].nbr_tree[1] = 1 - t; trees[t].nbr_face[1] = 1;
        trees[t].orient[1] = 1; trees[t].bc[1] = 0;
      }
    }
    const int maxl = 4 + trial % 7;      // shallow and deep forests
    std::vector<fcx_leaf> lv;
    std::string err;
    for (int t = 0; t < int(trees.size()); ++t)
      for (int y = 0; y < 4; ++y)
        for (int x = 0; x < 4; ++x) lv.push_back({t, 2, x, y});
    for (int s = 0; s < 10 + trial * 3; ++s) {
      const int k = int(rng() % lv.size());
      const fcx_leaf a = lv[k];
      if (a.level >= maxl) continue;
      lv.erase(lv.begin() + k);
      for (int c = 0; c < 4; ++c)
        lv.push_back({a.tree, a.level + 1, 2 * a.ix + (c & 1), 2 * a.iy + (c >> 1)});
    }
    std::vector<fcx_leaf> bl;
    int rc = balance(trees, lv, bl, err);
    mix(&rc, 4); mixv(bl);
    Forest f;
    rc = f.assign(trees, bl, err);
    mix(&rc, 4);
    Plan p, pu;    // pu: the plan before p, its storage reused as the library does
    rc = build_plan(f, 16, p, err, trial % 2);
    mix(&rc, 4); mixplan(p);
    for (int step = 0; step < 4; ++step) {
      std::vector<int8_t> tags(f.leaves.size());
      for (auto& t : tags) { const int r = int(rng() % 10); t = r < 1 ? 1 : (r < 5 ? -1 : 0); }
      std::vector<fcx_leaf> out;
      std::vector<int32_t> rkind, rsrc;
      rc = regrid(f, tags.data(), 1, maxl + 1, out, err, &rkind, &rsrc);
      mix(&rc, 4); mixv(out);
      Forest nf;
      rc = nf.assign(trees, out, err);
      mix(&rc, 4);
      if (rc != FCX_OK) ++mismatches;   // regrid output must validate
      Forest na;                        // what the library keeps: no re-validation
      na.adopt(trees, out);
      if (na.maxlevel != nf.maxlevel) ++mismatches;
      std::vector<int32_t> kind, src;
      rc = transfer_plan(f, nf, kind, src, err);
      mix(&rc, 4); mixv(kind); mixv(src);
      if (kind != rkind || src != rsrc) ++mismatches;   // the regrid's own plan
      Plan pb;
      rc = update_plan(nf, 16, p, kind, src, pu, err, trial % 2);
      mix(&rc, 4); mixplan(pu);
      rc = build_plan(nf, 16, pb, err, trial % 2);
      mix(&rc, 4);
      if (!same(pu, pb)) ++mismatches;
      for (int k = 0; k < 200; ++k) {
        const int l = int(rng() % (maxl + 3)) - 1;
        int64_t ix = int64_t(rng() % 4096) - 8, iy = int64_t(rng() % 4096) - 8;
        if (l >= 0 && l < 12) { ix >>= (12 - l); iy >>= (12 - l); }
        const int32_t tf = int32_t(rng() % (trees.size() + 1));
        const int64_t r1 = nf.find(tf, l, ix, iy);
        mix(&r1, 8);
        if (na.find(tf, l, ix, iy) != r1) ++mismatches;
        const int64_t x = int64_t(rng()) % (kSide + 100) - 50;
        const int64_t y = int64_t(rng()) % (kSide + 100) - 50;
        const int32_t tl = int32_t(rng() % trees.size());
        const int hint = (k & 1) ? -1 : int(rng() % (maxl + 1));
        const int64_t r2 = nf.leaf_at(tl, x, y, hint);
        mix(&r2, 8);
        if (na.leaf_at(tl, x, y, hint) != r2) ++mismatches;
      }
      f = std::move(nf);
      std::swap(p, pu);
    }
    std::printf("%d %zu %016llx\n", trial, f.leaves.size(), (unsigned long long)H);
  }
  return mismatches ? 1 : 0;
}
