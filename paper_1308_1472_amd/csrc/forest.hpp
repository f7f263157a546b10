// forest.hpp -- host-side forest of quadtrees for the fcx library.
//
// A forest is a set of trees (each the reference square [0,1]^2, glued by a
// face connectivity) whose leaves tile every tree; each leaf houses one
// m x m patch (arXiv 1308.1472, Sec. 2: one leaf <-> one patch).  Leaves
// are stored in space-filling-curve order (Sec. 4): tree-major, then Morton
// order of the lower-left corner.  All work here is integer work.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fcx.h"

namespace fcx {

constexpr int kS = 24;                       // tree side = 2^24 units
constexpr int64_t kSide = int64_t(1) << kS;
constexpr int kMaxLevel = 18;

// Affine map between tree coordinate systems: x' = A x + b, A a signed
// permutation (bit 0 swap, bit 1 negate first, bit 2 negate second), b in
// units of the tree side (bits 3..5 and 6..8, biased by 4).
struct Xform {
  int32_t code = 4 << 3 | 4 << 6;            // identity
  void apply(int64_t x, int64_t y, int64_t& xo, int64_t& yo) const;
};

// Open-addressing hash map from packed leaf keys to leaf indices (linear
// probing, power-of-two capacity, no deletion except clear).
class LeafIndex {
 public:
  void reset(size_t expected);
  void put(uint64_t key, int32_t val);
  int32_t get(uint64_t key) const;
  bool erase(uint64_t key);            // tombstone
  size_t size() const { return live_; }
  template <typename F> void for_each(F f) const {
    for (size_t s = 0; s < keys_.size(); ++s)
      if (keys_[s] != kEmpty && keys_[s] != kTomb) f(keys_[s], vals_[s]);
  }

 private:
  static constexpr uint64_t kEmpty = ~uint64_t(0), kTomb = ~uint64_t(0) - 1;
  std::vector<uint64_t> keys_;
  std::vector<int32_t> vals_;
  size_t mask_ = 0, live_ = 0, used_ = 0;
  void grow();
};

uint64_t morton_key(const fcx_leaf& a);
bool leaf_less(const fcx_leaf& a, const fcx_leaf& b);
void sort_leaves(std::vector<fcx_leaf>& v);          // SFC order

class Forest {
 public:
  std::vector<fcx_tree> trees;
  std::vector<fcx_leaf> leaves;              // SFC order
  int maxlevel = 0;

  // Validates connectivity and leaves (sorted, exact tiling); builds the
  // leaf index.  Returns FCX_OK or an error code with a message in err.
  int assign(const std::vector<fcx_tree>& t, std::vector<fcx_leaf> l,
             std::string& err);
  // Leaves that regrid() made from a forest over the same trees: they are
  // SFC-sorted and tile every tree by construction, so only the leaf index
  // is built.
  void adopt(const std::vector<fcx_tree>& t, std::vector<fcx_leaf> l);
  int64_t find(int32_t tree, int32_t level, int64_t ix, int64_t iy) const;
  // leaf containing an in-tree point, -1 if none; levels near `hint` are
  // probed first
  int64_t leaf_at(int32_t tree, int64_t x, int64_t y, int hint = -1) const;

  // Map a point (possibly outside its tree) into the tree containing it.
  // Returns 0 (found), 1 (beyond a physical boundary), 2 (valence-3
  // corner: no tree contains it), 3 (inconsistent connectivity).  The map
  // used is returned in xf.
  int locate(int32_t tree, int64_t x, int64_t y, int32_t& tout, int64_t& xo,
             int64_t& yo, Xform& xf) const;
  bool wall_face(int64_t p, int f) const;

 private:
  // Leaf lookup: a dense map from the cells of the finest level present to
  // leaf ids (rows of 2^dense_level_ cells, tree-major) when it is not much
  // larger than the leaf set, otherwise a hash of (tree, level, ix, iy).
  LeafIndex index_;
  std::vector<int32_t> dense_;
  int dense_level_ = -1;
  void build_index();
};

int check_connectivity(const std::vector<fcx_tree>& trees, std::string& err);

// Coarsest 2:1 (face + corner) balanced forest refining `in` (any order).
int balance(const std::vector<fcx_tree>& trees, std::vector<fcx_leaf> in,
            std::vector<fcx_leaf>& out, std::string& err);

// Per-patch neighbour records consumed by the kernels.
struct PatchRec {
  int32_t level, ix, iy, flags;              // flags: bit f wall on face f,
                                             // bit 4+f extrapolation wall,
                                             // kSimpleHalo, tree << kTreeShift
  int32_t nbr[12];                           // faces 2 slots each, corners
  int32_t xf[8];                             // face / corner transforms
};
static_assert(sizeof(PatchRec) == 96, "PatchRec layout");

constexpr int32_t kNbrWall = -1;
// PatchRec.flags bit: every neighbour region is a wall or a same-level leaf
// glued by a pure translation (ghost cells are plain copies)
constexpr int32_t kSimpleHalo = 1 << 8;
constexpr int32_t kNbrValence3 = -2;
// PatchRec.flags bits 16.. hold the patch's tree
constexpr int kTreeShift = 16;

// One coarse patch face with two finer neighbours (reflux work item), or,
// with fine[1] == kSyncItem, a same-level face across trees whose face
// terms the patch `coarse` takes over from its neighbour fine[0].
struct RefluxItem {
  int32_t coarse, face, fine[2], fine_face[2], fine_rev[2];
};
constexpr int32_t kSyncItem = -3;

struct Plan {
  std::vector<PatchRec> recs;
  std::vector<int32_t> phislot;              // -1 or slot of the patch
  int32_t nslots = 0;
  std::vector<RefluxItem> reflux;            // in patch order
  std::vector<int32_t> item_first;           // items of patch p: [first[p], first[p+1])
  std::vector<int32_t> family;               // 1 at the first child of a
                                             // complete leaf family
};

// sync: also emit face-sync items for same-level faces across trees (used
// by the cubed sphere, whose mass face terms must agree there).
int build_plan(const Forest& f, int m, Plan& plan, std::string& err,
               bool sync = false);

// Plan of forest f obtained by a regrid of the forest whose plan is `old`
// (kind / src from transfer_plan): a kept patch whose twelve neighbour
// regions are all held by kept leaves keeps its record, renumbered; every
// other patch is planned afresh.  Same result as build_plan.
int update_plan(const Forest& f, int m, const Plan& old,
                const std::vector<int32_t>& kind, const std::vector<int32_t>& src,
                Plan& plan, std::string& err, bool sync = false);

// Regrid: refine +1, merge complete families tagged -1, then balance.  With
// kind and src, also the transfer plan of the new leaves (as transfer_plan
// gives it; kind -1 marks a leaf the transfer cannot fill).
int regrid(const Forest& f, const int8_t* tags, int lmin, int lmax,
           std::vector<fcx_leaf>& out, std::string& err,
           std::vector<int32_t>* kind = nullptr, std::vector<int32_t>* src = nullptr);

// Transfer plan from an old to a new forest: per new patch kind
// (0 copy, 1 refined from an old coarser patch, 2 merged from four old
// children) and the old patch index (first child for kind 2).
int transfer_plan(const Forest& old_f, const Forest& new_f,
                  std::vector<int32_t>& kind, std::vector<int32_t>& src,
                  std::string& err);

}  // namespace fcx
