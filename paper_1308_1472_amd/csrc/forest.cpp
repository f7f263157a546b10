// forest.cpp -- host-side forest: SFC order, validation, point location
// through the connectivity, 2:1 balance by ripple propagation, neighbour
// records for the kernels, regrid and transfer plans.  Integer work only.
#include "forest.hpp"

#include <algorithm>
#include <deque>
#include <thread>

namespace fcx {

// ---------------------------------------------------------------------------
void Xform::apply(int64_t x, int64_t y, int64_t& xo, int64_t& yo) const {
  int64_t u = (code & 1) ? y : x;
  int64_t v = (code & 1) ? x : y;
  if (code & 2) u = -u;
  if (code & 4) v = -v;
  xo = u + int64_t(((code >> 3) & 7) - 4) * kSide;
  yo = v + int64_t(((code >> 6) & 7) - 4) * kSide;
}

// spread the low 32 bits of v to the even bit positions
static inline uint64_t spread(uint64_t v) {
  v &= 0xffffffffull;
  v = (v | (v << 16)) & 0x0000ffff0000ffffull;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

uint64_t morton_key(const fcx_leaf& a) {
  const int sh = kS - a.level;
  return spread(uint64_t(a.ix) << sh) | (spread(uint64_t(a.iy) << sh) << 1);
}

bool leaf_less(const fcx_leaf& a, const fcx_leaf& b) {
  if (a.tree != b.tree) return a.tree < b.tree;
  const uint64_t ka = morton_key(a), kb = morton_key(b);
  if (ka != kb) return ka < kb;
  return a.level < b.level;
}

void sort_leaves(std::vector<fcx_leaf>& v) {
  // (tree, Morton key, level) computed once per leaf
  std::vector<std::pair<std::pair<uint64_t, uint64_t>, uint32_t>> k(v.size());
  for (size_t i = 0; i < v.size(); ++i)
    k[i] = {{(uint64_t(uint32_t(v[i].tree)) << 8) | uint64_t(v[i].level), morton_key(v[i])},
            uint32_t(i)};
  std::sort(k.begin(), k.end(), [](const auto& a, const auto& b) {
    if ((a.first.first >> 8) != (b.first.first >> 8)) return a.first.first < b.first.first;
    if (a.first.second != b.first.second) return a.first.second < b.first.second;
    return (a.first.first & 255) < (b.first.first & 255);
  });
  std::vector<fcx_leaf> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = v[k[i].second];
  v.swap(o);
}

static inline uint64_t pack_key(int32_t tree, int32_t level, int64_t ix,
                                int64_t iy) {
  return (uint64_t(tree) << 53) | (uint64_t(level) << 48) |
         (uint64_t(ix) << 24) | uint64_t(iy);
}

// ---------------------------------------------------------------------------
static inline uint64_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

void LeafIndex::reset(size_t expected) {
  size_t cap = 64;
  while (cap < 2 * expected + 16) cap <<= 1;
  keys_.assign(cap, kEmpty);
  vals_.assign(cap, -1);
  mask_ = cap - 1;
  live_ = used_ = 0;
}

void LeafIndex::grow() {
  std::vector<uint64_t> k = std::move(keys_);
  std::vector<int32_t> v = std::move(vals_);
  reset(live_ * 2 + 16);
  for (size_t s = 0; s < k.size(); ++s)
    if (k[s] != kEmpty && k[s] != kTomb) put(k[s], v[s]);
}

void LeafIndex::put(uint64_t key, int32_t val) {
  if (keys_.empty() || 2 * (used_ + 1) > keys_.size()) grow();
  size_t s = mix64(key) & mask_, tomb = SIZE_MAX;
  for (;; s = (s + 1) & mask_) {
    if (keys_[s] == key) { vals_[s] = val; return; }
    if (keys_[s] == kTomb && tomb == SIZE_MAX) tomb = s;
    if (keys_[s] == kEmpty) break;
  }
  if (tomb != SIZE_MAX) s = tomb; else ++used_;
  keys_[s] = key;
  vals_[s] = val;
  ++live_;
}

int32_t LeafIndex::get(uint64_t key) const {
  if (keys_.empty()) return -1;
  for (size_t s = mix64(key) & mask_;; s = (s + 1) & mask_) {
    if (keys_[s] == key) return vals_[s];
    if (keys_[s] == kEmpty) return -1;
  }
}

bool LeafIndex::erase(uint64_t key) {
  if (keys_.empty()) return false;
  for (size_t s = mix64(key) & mask_;; s = (s + 1) & mask_) {
    if (keys_[s] == key) { keys_[s] = kTomb; --live_; return true; }
    if (keys_[s] == kEmpty) return false;
  }
}

// ---------------------------------------------------------------------------
int check_connectivity(const std::vector<fcx_tree>& trees, std::string& err) {
  const int n = int(trees.size());
  if (n <= 0 || n > 64) { err = "tree count must be 1..64"; return FCX_EINVAL; }
  for (int t = 0; t < n; ++t)
    for (int f = 0; f < 4; ++f) {
      const fcx_tree& T = trees[t];
      if (T.bc[f] < 0 || T.bc[f] > 2) { err = "bad bc"; return FCX_EINVAL; }
      if (T.bc[f] != 0) continue;
      const int t2 = T.nbr_tree[f], f2 = T.nbr_face[f];
      if (t2 < 0 || t2 >= n || f2 < 0 || f2 > 3 || T.orient[f] < 0 ||
          T.orient[f] > 1) {
        err = "bad face connection";
        return FCX_EINVAL;
      }
      const fcx_tree& U = trees[t2];
      if (U.bc[f2] != 0 || U.nbr_tree[f2] != t || U.nbr_face[f2] != f ||
          U.orient[f2] != T.orient[f]) {
        err = "face connections are not symmetric";
        return FCX_EINVAL;
      }
    }
  return FCX_OK;
}

#ifndef FCX_DENSE_FACTOR
#define FCX_DENSE_FACTOR 4     // dense map when cells <= factor * (leaves + 1024)
#endif

int Forest::assign(const std::vector<fcx_tree>& t, std::vector<fcx_leaf> l,
                   std::string& err) {
  int rc = check_connectivity(t, err);
  if (rc != FCX_OK) return rc;
  trees = t;
  leaves = std::move(l);
  maxlevel = 0;
  size_t k = 0;
  for (int32_t tr = 0; tr < int32_t(trees.size()); ++tr) {
    uint64_t next = 0;
    for (; k < leaves.size() && leaves[k].tree == tr; ++k) {
      const fcx_leaf& a = leaves[k];
      if (a.level < 0 || a.level > kMaxLevel || a.ix < 0 || a.iy < 0 ||
          a.ix >= (1 << a.level) || a.iy >= (1 << a.level)) {
        err = "leaf coordinates out of range";
        return FCX_EINVAL;
      }
      if (morton_key(a) != next) {
        err = "leaves are not SFC-sorted or do not tile the tree";
        return FCX_EINVAL;
      }
      next += uint64_t(1) << (2 * (kS - a.level));
      maxlevel = std::max(maxlevel, int(a.level));
    }
    if (next != (uint64_t(1) << (2 * kS))) {
      err = "leaves do not tile every tree";
      return FCX_EINVAL;
    }
  }
  if (k != leaves.size()) {
    err = "leaf with an unknown tree";
    return FCX_EINVAL;
  }
  build_index();
  return FCX_OK;
}

void Forest::adopt(const std::vector<fcx_tree>& t, std::vector<fcx_leaf> l) {
  trees = t;
  leaves = std::move(l);
  maxlevel = 0;
  for (const fcx_leaf& a : leaves) maxlevel = std::max(maxlevel, int(a.level));
  build_index();
}

void Forest::build_index() {
  const uint64_t cells = uint64_t(trees.size()) << (2 * maxlevel);
  if (cells <= uint64_t(FCX_DENSE_FACTOR) * (leaves.size() + 1024)) {
    dense_level_ = maxlevel;
    index_.reset(0);
    const int64_t side = int64_t(1) << maxlevel;
    dense_.resize(size_t(cells));
    for (size_t q = 0; q < leaves.size(); ++q) {
      const fcx_leaf& a = leaves[q];
      const int64_t s = int64_t(1) << (maxlevel - a.level);
      int32_t* row = dense_.data() + (int64_t(a.tree) * side + int64_t(a.iy) * s) * side +
                     int64_t(a.ix) * s;
      for (int64_t r = 0; r < s; ++r, row += side) std::fill(row, row + s, int32_t(q));
    }
  } else {
    dense_level_ = -1;
    dense_.clear();
    index_.reset(leaves.size());
    for (size_t q = 0; q < leaves.size(); ++q) {
      const fcx_leaf& a = leaves[q];
      index_.put(pack_key(a.tree, a.level, a.ix, a.iy), int32_t(q));
    }
  }
}

int64_t Forest::find(int32_t tree, int32_t level, int64_t ix, int64_t iy) const {
  if (dense_level_ < 0) return index_.get(pack_key(tree, level, ix, iy));
  if (tree < 0 || tree >= int32_t(trees.size()) || level < 0 || level > dense_level_ ||
      ix < 0 || iy < 0 || ix >= (int64_t(1) << level) || iy >= (int64_t(1) << level))
    return -1;
  const int sh = dense_level_ - level;
  const int64_t side = int64_t(1) << dense_level_;
  const int32_t q = dense_[size_t((int64_t(tree) * side + (iy << sh)) * side + (ix << sh))];
  return leaves[q].level == level ? q : -1;
}

int64_t Forest::leaf_at(int32_t tree, int64_t x, int64_t y, int hint) const {
  if (x < 0 || y < 0 || x >= kSide || y >= kSide) return -1;
  if (dense_level_ >= 0) {
    if (tree < 0 || tree >= int32_t(trees.size())) return -1;
    const int sh = kS - dense_level_;
    const int64_t side = int64_t(1) << dense_level_;
    return dense_[size_t((int64_t(tree) * side + (y >> sh)) * side + (x >> sh))];
  }
  if (hint >= 0) {
    // 2:1 balance puts every neighbour within one level of the asker
    const int cand[3] = {hint, hint + 1, hint - 1};
    for (int l : cand) {
      if (l < 0 || l > maxlevel) continue;
      const int64_t s = find(tree, l, x >> (kS - l), y >> (kS - l));
      if (s >= 0) return s;
    }
  }
  for (int l = maxlevel; l >= 0; --l) {
    const int64_t s = find(tree, l, x >> (kS - l), y >> (kS - l));
    if (s >= 0) return s;
  }
  return -1;
}

bool Forest::wall_face(int64_t p, int f) const {
  const fcx_leaf& a = leaves[p];
  const int32_t last = (1 << a.level) - 1;
  const bool on = (f == 0 && a.ix == 0) || (f == 1 && a.ix == last) ||
                  (f == 2 && a.iy == 0) || (f == 3 && a.iy == last);
  return on && trees[a.tree].bc[f] != 0;
}

// ---------------------------------------------------------------------------
// Crossing face f of tree t maps a point beyond the face into the glued tree:
// its depth beyond face f becomes its depth inside face f2; the tangential
// coordinate is kept or reversed by the orientation.
static void cross_point(const fcx_tree& T, int f, int64_t x, int64_t y,
                        int64_t& xo, int64_t& yo) {
  const int f2 = T.nbr_face[f];
  const int64_t n = (f < 2) ? x : y, tg = (f < 2) ? y : x;
  const int64_t depth = (f & 1) ? n - kSide : -n;
  const int64_t n2 = (f2 & 1) ? kSide - depth : depth;
  const int64_t t2 = T.orient[f] ? kSide - tg : tg;
  if (f2 < 2) { xo = n2; yo = t2; } else { xo = t2; yo = n2; }
}

struct Path {
  int n = 0;
  int tree[3];
  int face[3];
};

static void run_path(const std::vector<fcx_tree>& trees, const Path& p,
                     int64_t x, int64_t y, int64_t& xo, int64_t& yo) {
  for (int k = 0; k < p.n; ++k) {
    int64_t a, b;
    cross_point(trees[p.tree[k]], p.face[k], x, y, a, b);
    x = a;
    y = b;
  }
  xo = x;
  yo = y;
}

static Xform xform_of(const std::vector<fcx_tree>& trees, const Path& p) {
  int64_t bx, by, ax, ay, cx, cy;
  run_path(trees, p, 0, 0, bx, by);
  run_path(trees, p, kSide, 0, ax, ay);
  run_path(trees, p, 0, kSide, cx, cy);
  const int64_t c0x = (ax - bx) / kSide, c0y = (ay - by) / kSide;
  const int64_t c1x = (cx - bx) / kSide, c1y = (cy - by) / kSide;
  Xform xf;
  int code = 0;
  if (c0x == 0) {                 // x feeds y': axes swap
    code |= 1;
    if (c1x < 0) code |= 2;
    if (c0y < 0) code |= 4;
  } else {
    if (c0x < 0) code |= 2;
    if (c1y < 0) code |= 4;
  }
  code |= int((bx / kSide) + 4) << 3;
  code |= int((by / kSide) + 4) << 6;
  xf.code = code;
  return xf;
}

static int outside_axis_face(int64_t v, int axis) {
  if (v < 0) return 2 * axis;
  if (v >= kSide) return 2 * axis + 1;
  return -1;
}

// follow faces, preferring `axis` when the point is outside in both
static int follow(const std::vector<fcx_tree>& trees, int32_t t, int64_t x,
                  int64_t y, int axis, Path& path, int32_t& tout, int64_t& xo,
                  int64_t& yo) {
  path.n = 0;
  for (int hop = 0; hop < 3; ++hop) {
    const int fx = outside_axis_face(x, 0), fy = outside_axis_face(y, 1);
    if (fx < 0 && fy < 0) {
      tout = t;
      xo = x;
      yo = y;
      return 0;
    }
    if (hop == 2) return 3;
    const int f = (fx >= 0 && fy >= 0) ? (axis == 0 ? fx : fy)
                                       : (fx >= 0 ? fx : fy);
    const fcx_tree& T = trees[t];
    if (T.bc[f] != 0) return 1;
    path.tree[path.n] = t;
    path.face[path.n] = f;
    ++path.n;
    int64_t a, b;
    cross_point(T, f, x, y, a, b);
    x = a;
    y = b;
    t = T.nbr_tree[f];
    axis ^= 1;
  }
  return 3;
}

int Forest::locate(int32_t tree, int64_t x, int64_t y, int32_t& tout,
                   int64_t& xo, int64_t& yo, Xform& xf) const {
  if (x >= 0 && y >= 0 && x < kSide && y < kSide) {   // inside: identity
    tout = tree;
    xo = x;
    yo = y;
    xf = Xform();
    return 0;
  }
  Path pa, pb;
  int32_t ta, tb;
  int64_t xa, ya, xb, yb;
  const int ra = follow(trees, tree, x, y, 0, pa, ta, xa, ya);
  const bool corner = outside_axis_face(x, 0) >= 0 && outside_axis_face(y, 1) >= 0;
  if (!corner) {
    if (ra != 0) return ra == 1 ? 1 : 3;
    tout = ta;
    xo = xa;
    yo = ya;
    xf = xform_of(trees, pa);
    return 0;
  }
  const int rb = follow(trees, tree, x, y, 1, pb, tb, xb, yb);
  if (ra == 0 && rb == 0) {
    if (ta != tb || xa != xb || ya != yb) return 2;   // three trees meet
    tout = ta;
    xo = xa;
    yo = ya;
    xf = xform_of(trees, pa);
    return 0;
  }
  if (ra == 1 && rb == 1) return 1;
  return 3;
}

// ---------------------------------------------------------------------------
// The tentative leaves of a balance or regrid; they tile every tree at all
// times.  has(): is (tree, level, ix, iy) a leaf; covering(): level of the
// leaf holding the point (x, y) if it is at most maxlev, else -1; add():
// insert a leaf; split(): replace a leaf by its four children.
struct HashLeafSet {
  LeafIndex idx;
  explicit HashLeafSet(size_t n) { idx.reset(n); }
  bool has(int32_t t, int l, int64_t ix, int64_t iy) const {
    return idx.get(pack_key(t, l, ix, iy)) >= 0;
  }
  int covering(int32_t t, int64_t x, int64_t y, int maxlev) const {
    for (int l = maxlev; l >= 0; --l)
      if (has(t, l, x >> (kS - l), y >> (kS - l))) return l;
    return -1;
  }
  void add(int32_t t, int l, int64_t ix, int64_t iy) { idx.put(pack_key(t, l, ix, iy), 1); }
  void split(int32_t t, int l, int64_t ix, int64_t iy) {
    idx.erase(pack_key(t, l, ix, iy));
    for (int c = 0; c < 4; ++c) add(t, l + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1));
  }
  size_t size() const { return idx.size(); }
};

// Dense form for shallow forests: the level of the leaf holding each cell of
// level L (rows of 2^L cells, tree-major).  Leaves are at most level L.
struct DenseLeafSet {
  std::vector<int8_t> lev;
  int L;
  int64_t side;
  size_t count = 0;
  DenseLeafSet(int ntrees, int L_) : L(L_), side(int64_t(1) << L_) {
    lev.assign(size_t(ntrees) * size_t(side) * size_t(side), int8_t(-1));
  }
  int8_t* at(int32_t t, int64_t cx, int64_t cy) {
    return lev.data() + (int64_t(t) * side + cy) * side + cx;
  }
  int8_t get(int32_t t, int64_t cx, int64_t cy) const {
    return lev[size_t((int64_t(t) * side + cy) * side + cx)];
  }
  bool has(int32_t t, int l, int64_t ix, int64_t iy) const {
    return l <= L && get(t, ix << (L - l), iy << (L - l)) == l;
  }
  int covering(int32_t t, int64_t x, int64_t y, int maxlev) const {
    const int v = get(t, x >> (kS - L), y >> (kS - L));
    return v <= maxlev ? v : -1;
  }
  void fill(int32_t t, int l, int64_t ix, int64_t iy, int8_t v) {
    const int64_t s = int64_t(1) << (L - l);
    int8_t* row = at(t, ix * s, iy * s);
    for (int64_t r = 0; r < s; ++r, row += side) std::fill(row, row + s, v);
  }
  void add(int32_t t, int l, int64_t ix, int64_t iy) { fill(t, l, ix, iy, int8_t(l)); ++count; }
  void split(int32_t t, int l, int64_t ix, int64_t iy) {
    fill(t, l, ix, iy, int8_t(l + 1));
    count += 3;
  }
  size_t size() const { return count; }
};

// Balance by ripple propagation.  A leaf L of level l needs the leaf holding
// each of its eight same-size neighbour boxes to have level >= l - 1; when
// that leaf is coarser it is split (and its children queued), until every
// leaf reachable from the worklist satisfies this.  Only forced splits are
// made, so the result is the coarsest balanced refinement.
template <class Set>
static void ripple(const Forest& geo, Set& set, std::deque<fcx_leaf>& work) {
  while (!work.empty()) {
    const fcx_leaf L = work.front();
    work.pop_front();
    if (!set.has(L.tree, L.level, L.ix, L.iy)) continue;
    if (L.level < 2) continue;
    const int64_t size = kSide >> L.level;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        const int64_t px = (int64_t(L.ix + dx) * 2 + 1) * (size / 2);
        const int64_t py = (int64_t(L.iy + dy) * 2 + 1) * (size / 2);
        int32_t t2;
        int64_t x2, y2;
        Xform xf;
        if (geo.locate(L.tree, px, py, t2, x2, y2, xf) != 0) continue;
        for (;;) {
          // leaf among the ancestors of the neighbour box (level <= L.level)
          const int found = set.covering(t2, x2, y2, L.level);
          if (found < 0 || found >= L.level - 1) break;
          const int64_t ax = x2 >> (kS - found), ay = y2 >> (kS - found);
          set.split(t2, found, ax, ay);
          for (int c = 0; c < 4; ++c)
            work.push_back({t2, found + 1, int32_t(2 * ax + (c & 1)),
                            int32_t(2 * ay + (c >> 1))});
        }
      }
  }
}

static void collect(const HashLeafSet& set, std::vector<fcx_leaf>& out) {
  out.clear();
  out.reserve(set.size());
  set.idx.for_each([&](uint64_t k, int32_t) {
    fcx_leaf a;
    a.tree = int32_t(k >> 53);
    a.level = int32_t((k >> 48) & 31);
    a.ix = int32_t((k >> 24) & 0xffffff);
    a.iy = int32_t(k & 0xffffff);
    out.push_back(a);
  });
  sort_leaves(out);
}

// Coarsest balanced refinement of arbitrary leaves: the ripple seeded with
// every leaf.
int balance(const std::vector<fcx_tree>& trees, std::vector<fcx_leaf> in,
            std::vector<fcx_leaf>& out, std::string& err) {
  int rc = check_connectivity(trees, err);
  if (rc != FCX_OK) return rc;
  HashLeafSet set(in.size() * 2);
  std::deque<fcx_leaf> work;
  for (const auto& a : in) {
    if (a.tree < 0 || a.tree >= int32_t(trees.size()) || a.level < 0 ||
        a.level > kMaxLevel) {
      err = "leaf out of range";
      return FCX_EINVAL;
    }
    set.add(a.tree, a.level, a.ix, a.iy);
    work.push_back(a);
  }
  Forest geo;            // connectivity only (for locate)
  geo.trees = trees;
  ripple(geo, set, work);
  collect(set, out);
  return FCX_OK;
}

// ---------------------------------------------------------------------------
// Neighbour records of one patch; coarse-fine faces are reported in items.
static int plan_one(const Forest& f, int m, int64_t p, PatchRec& r,
                    bool& mixed, int32_t& family, RefluxItem* items,
                    int& nitems, bool sync, std::string& err) {
  {
    const fcx_leaf& a = f.leaves[p];
    r.level = a.level;
    r.ix = a.ix;
    r.iy = a.iy;
    r.flags = a.tree << kTreeShift;
    const int64_t size = kSide >> a.level, half = size / (2 * m);
    const int64_t x0 = int64_t(a.ix) * size, y0 = int64_t(a.iy) * size;
    auto centre = [&](int i, int j, int64_t& x, int64_t& y) {
      x = x0 + (2 * i - 1) * half;
      y = y0 + (2 * j - 1) * half;
    };
    mixed = false;
    nitems = 0;
    for (int fc = 0; fc < 4; ++fc) {
      if (f.wall_face(p, fc)) {
        r.flags |= 1 << fc;
        if (f.trees[a.tree].bc[fc] == 2) r.flags |= 16 << fc;
        r.nbr[2 * fc] = r.nbr[2 * fc + 1] = kNbrWall;
        r.xf[fc] = Xform().code;
        continue;
      }
      int32_t ids[2];
      Xform xf;
      for (int s = 0; s < 2; ++s) {
        // a same-level or coarser neighbour holds both halves of the face
        if (s == 1 && f.leaves[ids[0]].level <= a.level) { ids[1] = ids[0]; break; }
        const int t = s == 0 ? 1 : m;
        int64_t x, y;
        if (fc < 2) centre(fc == 0 ? 0 : m + 1, t, x, y);
        else centre(t, fc == 2 ? 0 : m + 1, x, y);
        int32_t t2;
        int64_t x2, y2;
        if (f.locate(a.tree, x, y, t2, x2, y2, xf) != 0) {
          err = "face neighbour not found";
          return FCX_EINVAL;
        }
        ids[s] = int32_t(f.leaf_at(t2, x2, y2, a.level));
        if (ids[s] < 0) { err = "face neighbour missing"; return FCX_EINVAL; }
      }
      const int l0 = f.leaves[ids[0]].level, l1 = f.leaves[ids[1]].level;
      if (ids[0] != ids[1] ? (l0 != a.level + 1 || l1 != a.level + 1)
                           : (l0 > a.level || l0 < a.level - 1)) {
        err = "forest is not 2:1 balanced";
        return FCX_EBALANCE;
      }
      if (l0 != a.level) mixed = true;
      r.nbr[2 * fc] = ids[0];
      r.nbr[2 * fc + 1] = ids[1];
      r.xf[fc] = xf.code;
      // same-level face across trees, kept consistent by a face sync
      const bool synced = sync && ids[0] == ids[1] && l0 == a.level &&
                          f.leaves[ids[0]].tree != a.tree;
      if (synced) mixed = true;
      if (ids[0] != ids[1] || (synced && ids[0] < p)) {
        RefluxItem it{};
        it.coarse = int32_t(p);
        it.face = fc;
        // linear part of the map, applied to directions
        Xform lin = xf;
        lin.code = (xf.code & 7) | (4 << 3) | (4 << 6);
        int64_t dx = 0, dy = 0, tx = 0, ty = 0;
        if (fc < 2) { dx = (fc == 1) ? -1 : 1; ty = 1; } else { dy = (fc == 3) ? -1 : 1; tx = 1; }
        int64_t ddx, ddy, tdx, tdy;
        lin.apply(dx, dy, ddx, ddy);
        lin.apply(tx, ty, tdx, tdy);
        // the direction towards the coarse patch names the fine face
        int ff = ddx > 0 ? 1 : ddx < 0 ? 0 : ddy > 0 ? 3 : 2;
        int rev = (ff < 2) ? (tdy < 0) : (tdx < 0);
        for (int s = 0; s < 2; ++s) {
          it.fine[s] = ids[s];
          it.fine_face[s] = ff;
          it.fine_rev[s] = rev;
        }
        if (ids[0] == ids[1]) it.fine[1] = kSyncItem;
        items[nitems++] = it;
      }
    }
    for (int c = 0; c < 4; ++c) {
      const int fx = c & 1, fy = 2 + (c >> 1);
      if ((r.flags >> fx & 1) || (r.flags >> fy & 1)) {
        r.nbr[8 + c] = kNbrWall;
        r.xf[4 + c] = Xform().code;
        continue;
      }
      int64_t x, y;
      centre((c & 1) ? m + 1 : 0, (c >> 1) ? m + 1 : 0, x, y);
      int32_t t2;
      int64_t x2, y2;
      Xform xf;
      const int st = f.locate(a.tree, x, y, t2, x2, y2, xf);
      if (st == 2) {
        r.nbr[8 + c] = kNbrValence3;
        r.xf[4 + c] = Xform().code;
        continue;
      }
      if (st != 0) { err = "corner neighbour not found"; return FCX_EINVAL; }
      const int64_t id = f.leaf_at(t2, x2, y2, a.level);
      if (id < 0) { err = "corner neighbour missing"; return FCX_EINVAL; }
      const int lc = f.leaves[id].level;
      if (lc < a.level - 1 || lc > a.level + 1) {
        err = "forest is not 2:1 balanced at a corner";
        return FCX_EBALANCE;
      }
      r.nbr[8 + c] = int32_t(id);
      r.xf[4 + c] = xf.code;
    }
    bool simple = true;
    for (int s2 = 0; s2 < 12 && simple; ++s2) {
      const int32_t nb = r.nbr[s2];
      if (nb == kNbrWall) continue;
      const int32_t code = s2 < 8 ? r.xf[s2 / 2] : r.xf[4 + (s2 - 8)];
      if (nb < 0 || f.leaves[nb].level != a.level || (code & 7) != 0) simple = false;
    }
    if (simple) r.flags |= kSimpleHalo;
    // first child of a complete family of leaf siblings
    if (a.level > 0 && !(a.ix & 1) && !(a.iy & 1)) {
      bool all = true;
      for (int c = 1; c < 4; ++c)
        if (f.find(a.tree, a.level, a.ix + (c & 1), a.iy + (c >> 1)) != p + c)
          all = false;
      family = all ? 1 : 0;
    }
  }
  return FCX_OK;
}

// Slots and reflux items numbered in patch order.
static void finish_plan(Plan& plan, const std::vector<uint8_t>& mixed,
                        const std::vector<RefluxItem>& items,
                        const std::vector<uint8_t>& nitems) {
  const int64_t n = int64_t(mixed.size());
  plan.item_first.assign(n + 1, 0);
  for (int64_t p = 0; p < n; ++p) {
    if (mixed[p]) plan.phislot[p] = plan.nslots++;
    plan.item_first[p] = int32_t(plan.reflux.size());
    for (int k = 0; k < nitems[p]; ++k) plan.reflux.push_back(items[size_t(p) * 4 + k]);
  }
  plan.item_first[n] = int32_t(plan.reflux.size());
}

// Records for all patches, computed in parallel chunks; slots and reflux
// items are then numbered in patch order.
int build_plan(const Forest& f, int m, Plan& plan, std::string& err, bool sync) {
  const int64_t n = int64_t(f.leaves.size());
  plan.recs.assign(n, PatchRec{});
  plan.phislot.assign(n, -1);
  plan.family.assign(n, 0);
  plan.reflux.clear();
  plan.nslots = 0;
  std::vector<uint8_t> mixed(n, 0);
  std::vector<RefluxItem> items(size_t(n) * 4);
  std::vector<uint8_t> nitems(n, 0);
  const int hw = int(std::max(1u, std::thread::hardware_concurrency()));
  const int nth = int(std::max<int64_t>(1, std::min<int64_t>(std::min(hw, 16), n / 512)));
  std::vector<int> rcs(nth, FCX_OK);
  std::vector<std::string> errs(nth);
  auto work = [&](int t) {
    const int64_t lo = n * t / nth, hi = n * (t + 1) / nth;
    for (int64_t p = lo; p < hi; ++p) {
      bool mx = false;
      int ni = 0;
      int32_t fam = 0;
      const int rc = plan_one(f, m, p, plan.recs[p], mx, fam, &items[size_t(p) * 4],
                              ni, sync, errs[t]);
      if (rc != FCX_OK) { rcs[t] = rc; return; }
      mixed[p] = mx;
      nitems[p] = uint8_t(ni);
      plan.family[p] = fam;
    }
  };
  if (nth == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  for (int t = 0; t < nth; ++t)
    if (rcs[t] != FCX_OK) { err = errs[t]; return rcs[t]; }
  finish_plan(plan, mixed, items, nitems);
  return FCX_OK;
}

int update_plan(const Forest& f, int m, const Plan& old,
                const std::vector<int32_t>& kind, const std::vector<int32_t>& src,
                Plan& plan, std::string& err, bool sync) {
  const int64_t n = int64_t(f.leaves.size());
  const int64_t no = int64_t(old.recs.size());
  if (int64_t(kind.size()) != n || int64_t(src.size()) != n ||
      int64_t(old.item_first.size()) != no + 1) {
    err = "plan update: inconsistent inputs";
    return FCX_EINVAL;
  }
  std::vector<int32_t> o2n(no, -1);
  for (int64_t p = 0; p < n; ++p)
    if (kind[p] == 0) o2n[src[p]] = int32_t(p);
  plan.recs.resize(n);
  plan.phislot.resize(n);
  plan.family.resize(n);
  plan.item_first.resize(n + 1);
  plan.reflux.clear();
  plan.reflux.reserve(old.reflux.size() + 64);
  plan.nslots = 0;
  RefluxItem fresh[4];
  for (int64_t p = 0; p < n; ++p) {
    bool reuse = kind[p] == 0;
    const int32_t o = src[p];
    PatchRec& r = plan.recs[p];
    if (reuse) {
      r = old.recs[o];
      for (int s2 = 0; s2 < 12 && reuse; ++s2) {
        const int32_t nb = r.nbr[s2];
        if (nb < 0) continue;
        if (o2n[nb] < 0) reuse = false;
        else r.nbr[s2] = o2n[nb];
      }
    }
    plan.item_first[p] = int32_t(plan.reflux.size());
    bool mixed;
    if (reuse) {
      mixed = old.phislot[o] >= 0;
      plan.family[p] = old.family[o];
      for (int32_t t = old.item_first[o]; t < old.item_first[o + 1]; ++t) {
        RefluxItem it = old.reflux[t];
        it.coarse = int32_t(p);
        for (int s2 = 0; s2 < 2; ++s2)
          if (it.fine[s2] >= 0) it.fine[s2] = o2n[it.fine[s2]];
        plan.reflux.push_back(it);
      }
    } else {
      int ni = 0;
      int32_t fam = 0;
      const int rc = plan_one(f, m, p, r, mixed, fam, fresh, ni, sync, err);
      if (rc != FCX_OK) return rc;
      plan.family[p] = fam;
      for (int k = 0; k < ni; ++k) plan.reflux.push_back(fresh[k]);
    }
    plan.phislot[p] = mixed ? plan.nslots++ : -1;
  }
  plan.item_first[n] = int32_t(plan.reflux.size());
  return FCX_OK;
}

// ---------------------------------------------------------------------------
// Regrid of a balanced forest.  The tentative forest refines +1 leaves and
// merges complete families tagged -1.  A merged parent P (level l - 1) that
// touches a tentative leaf of level >= l + 1 must be split again in every
// balanced refinement, so that merge is cancelled up front.  After that, only
// new leaves can break balance, and the ripple is seeded with the refined
// children alone; the result is the coarsest balanced refinement of the
// tentative forest, as a full ripple would give.
template <class Set>
static int regrid_with(const Forest& f, const int8_t* tags, int lmin, int lmax, Set& set,
                       std::vector<fcx_leaf>& out, std::string& err,
                       std::vector<int32_t>* kind, std::vector<int32_t>* src) {
  const int64_t n = int64_t(f.leaves.size());
  std::deque<fcx_leaf> work;
  std::vector<int64_t> merged;                 // first child of each merge
  for (int64_t p = 0; p < n; ++p) {
    const fcx_leaf& a = f.leaves[p];
    if (tags[p] > 0 && a.level < lmax) {
      for (int c = 0; c < 4; ++c) {
        fcx_leaf ch{a.tree, a.level + 1, 2 * a.ix + (c & 1), 2 * a.iy + (c >> 1)};
        set.add(ch.tree, ch.level, ch.ix, ch.iy);
        work.push_back(ch);
      }
      continue;
    }
    if (tags[p] < 0 && a.level > lmin) {
      const int32_t bx = a.ix & ~1, by = a.iy & ~1;
      bool all = true;
      for (int c = 0; c < 4; ++c) {
        const int64_t s2 = f.find(a.tree, a.level, bx + (c & 1), by + (c >> 1));
        if (s2 < 0 || tags[s2] >= 0) { all = false; break; }
      }
      if (all) {
        if (a.ix == bx && a.iy == by) {
          set.add(a.tree, a.level - 1, a.ix >> 1, a.iy >> 1);
          merged.push_back(p);
        }
        continue;
      }
    }
    set.add(a.tree, a.level, a.ix, a.iy);
  }
  // cancel merges whose parent would touch a leaf two levels finer; a
  // cancellation restores finer leaves and can force others, so repeat
  // until no merge changes
  std::vector<uint8_t> cancelled(merged.size(), 0);
  for (bool again = true; again;) {
  again = false;
  for (size_t mi = 0; mi < merged.size(); ++mi) {
    if (cancelled[mi]) continue;
    const int64_t p = merged[mi];
    const fcx_leaf& a = f.leaves[p];                 // child level l
    const int l = a.level, pl = l - 1;
    const int32_t pix = a.ix >> 1, piy = a.iy >> 1;
    const int64_t psize = kSide >> pl, csz = kSide >> l;
    bool bad = false;
    for (int dy = -1; dy <= 1 && !bad; ++dy)
      for (int dx = -1; dx <= 1 && !bad; ++dx) {
        if (!dx && !dy) continue;
        // level-l boxes of the neighbour region that touch P
        for (int s1 = 0; s1 < 2 && !bad; ++s1) {
          if ((dx != 0 && dy != 0) && s1 == 1) break;
          int64_t cx, cy;                            // box centre, P's tree
          const int64_t x0 = int64_t(pix) * psize, y0 = int64_t(piy) * psize;
          if (dx == 0) cx = x0 + s1 * csz + csz / 2;
          else cx = dx < 0 ? x0 - csz / 2 : x0 + psize + csz / 2;
          if (dy == 0) cy = y0 + s1 * csz + csz / 2;
          else cy = dy < 0 ? y0 - csz / 2 : y0 + psize + csz / 2;
          int32_t t2;
          int64_t x2, y2;
          Xform xf;
          if (f.locate(a.tree, cx, cy, t2, x2, y2, xf) != 0) continue;
          if (set.covering(t2, x2, y2, l) < 0) bad = true;
        }
      }
    if (bad) {
      set.split(a.tree, pl, pix, piy);
      cancelled[mi] = 1;
      again = true;
    }
  }
  }
  ripple(f, set, work);
  // the new leaves in SFC order, by walking the old ones in order: an old
  // leaf is kept, the first child of a merged family, or the root of a
  // subtree of new leaves (refined, possibly split further by the ripple)
  // with kind / src: the transfer plan of each new leaf (0 kept, 1 child of
  // a refined old leaf, 2 parent of a merged family; -1 a leaf the transfer
  // cannot fill) and its old leaf (the first child for a merge)
  out.clear();
  out.reserve(set.size());
  if (kind) { kind->clear(); kind->reserve(set.size()); }
  if (src) { src->clear(); src->reserve(set.size()); }
  auto plan = [&](int32_t k, int64_t p) {
    if (kind) kind->push_back(k);
    if (src) src->push_back(int32_t(p));
  };
  std::vector<fcx_leaf> stack;
  for (int64_t p = 0; p < n; ++p) {
    const fcx_leaf& a = f.leaves[p];
    if (set.has(a.tree, a.level, a.ix, a.iy)) { out.push_back(a); plan(0, p); continue; }
    if (a.level > 0 && set.has(a.tree, a.level - 1, a.ix >> 1, a.iy >> 1)) {
      if (!(a.ix & 1) && !(a.iy & 1)) {
        out.push_back({a.tree, a.level - 1, a.ix >> 1, a.iy >> 1});
        plan(2, p);
      }
      continue;
    }
    stack.assign(1, a);
    while (!stack.empty()) {
      const fcx_leaf b = stack.back();
      stack.pop_back();
      // children pushed in reverse Morton order so they pop in order
      for (int c = 3; c >= 0; --c) {
        const fcx_leaf ch{b.tree, b.level + 1, 2 * b.ix + (c & 1), 2 * b.iy + (c >> 1)};
        if (set.has(ch.tree, ch.level, ch.ix, ch.iy)) {
          stack.push_back({-1 - ch.tree, ch.level, ch.ix, ch.iy});   // marked: emit
        } else {
          stack.push_back(ch);
        }
      }
      while (!stack.empty() && stack.back().tree < 0) {
        fcx_leaf e = stack.back();
        stack.pop_back();
        e.tree = -1 - e.tree;
        out.push_back(e);
        plan(e.level == a.level + 1 ? 1 : -1, p);
      }
    }
  }
  if (out.size() != set.size()) {
    err = "regrid: new leaves do not tile the forest";
    return FCX_EINVAL;
  }
  return FCX_OK;
}

int regrid(const Forest& f, const int8_t* tags, int lmin, int lmax,
           std::vector<fcx_leaf>& out, std::string& err, std::vector<int32_t>* kind,
           std::vector<int32_t>* src) {
  const size_t n = f.leaves.size();
  // the finest level the tentative leaves can reach
  const int L = std::max(f.maxlevel, std::min(lmax, f.maxlevel + 1));
  const uint64_t cells = uint64_t(f.trees.size()) << (2 * L);
  if (L <= kMaxLevel && cells <= uint64_t(FCX_DENSE_FACTOR) * (n + 1024)) {
    DenseLeafSet set(int(f.trees.size()), L);
    return regrid_with(f, tags, lmin, lmax, set, out, err, kind, src);
  }
  HashLeafSet set(n * 2 + 64);
  return regrid_with(f, tags, lmin, lmax, set, out, err, kind, src);
}

int transfer_plan(const Forest& old_f, const Forest& new_f,
                  std::vector<int32_t>& kind, std::vector<int32_t>& src,
                  std::string& err) {
  const int64_t n = int64_t(new_f.leaves.size());
  kind.assign(n, 0);
  src.assign(n, -1);
  for (int64_t p = 0; p < n; ++p) {
    const fcx_leaf& a = new_f.leaves[p];
    int64_t s = old_f.find(a.tree, a.level, a.ix, a.iy);
    if (s >= 0) { kind[p] = 0; src[p] = int32_t(s); continue; }
    if (a.level > 0) {
      s = old_f.find(a.tree, a.level - 1, a.ix >> 1, a.iy >> 1);
      if (s >= 0) { kind[p] = 1; src[p] = int32_t(s); continue; }
    }
    s = old_f.find(a.tree, a.level + 1, 2 * a.ix, 2 * a.iy);
    bool all = s >= 0;
    for (int c = 1; c < 4 && all; ++c)
      all = old_f.find(a.tree, a.level + 1, 2 * a.ix + (c & 1),
                       2 * a.iy + (c >> 1)) == s + c;
    if (!all) {
      err = "new leaf is not a copy, child or parent of old leaves";
      return FCX_EINVAL;
    }
    kind[p] = 2;
    src[p] = int32_t(s);
  }
  return FCX_OK;
}

}  // namespace fcx
