// Host-side structure of an H^2 matrix and the symbolic phase of the
// product (pure C++, no device calls).
//
// The cluster tree is complete and binary (2^l clusters at level l, leaves
// at level L, Section II).  The block tree lists per level its admissible (R),
// dense (F, leaf level only) and non-leaf (NL) nodes.  Every node below the
// root has a non-leaf parent whose four children are all nodes, so
// per-node blocks that the next level reads as a 2x2 "collected" block
// (equations nonleafA / nonleafB / NL_col) are stored grouped by that parent.
#pragma once
#include <stdint.h>

#include <string>
#include <unordered_map>
#include <vector>

namespace h2 {

enum NodeType { kR = 0, kF = 1, kNL = 2, kBlue = 3 };

struct LevelNodes {
  std::vector<int> row, col, type;
  std::vector<int> nl_index;   // per node: index among NL nodes of this level, -1 otherwise
  std::vector<int> tile_loc;   // per node (level >= 1): (parent NL index << 3) | sub
  int n_nl = 0;
  std::unordered_map<uint64_t, int> index;
  int find(int r, int c) const {
    auto it = index.find(((uint64_t)(uint32_t)r << 32) | (uint32_t)c);
    return it == index.end() ? -1 : it->second;
  }
  int size() const { return (int)row.size(); }
};

struct Structure {
  int64_t n = 0;
  int L = 0;
  int lmin = 0;
  int npad = 16;  // leaf size padded to a multiple of 16
  std::vector<int64_t> leaf_off, perm;
  std::vector<int> leaf_size;
  std::vector<LevelNodes> lev;
  std::vector<int64_t> node_base;  // global index of the first node of each level
  bool same_as(const Structure& o) const;
  int sparsity_constant() const;
};

// Builds and validates; returns "" or an error message.
std::string build_structure(Structure& s, int64_t n, int64_t L, const int64_t* leaf_off,
                            const int64_t* perm, const int64_t* node_off, const int32_t* row,
                            const int32_t* col, const int32_t* type);

// A batch task list: outputs with [seg[o], seg[o+1]) task ranges.
struct TaskList {
  std::vector<int> out, seg, a, b;
  TaskList() { seg.push_back(0); }
  void add_task(int av, int bv) { a.push_back(av); b.push_back(bv); }
  void close(int ov) { out.push_back(ov); seg.push_back((int)a.size()); }
  int nout() const { return (int)out.size(); }
  int ntask() const { return (int)a.size(); }
};

inline int enc(int idx, int half_r = 0, int half_c = 0, int sel = 0) {
  return (idx << 3) | (sel << 2) | (half_c << 1) | half_r;
}

// Symbolic phase of the product C = A B over one shared structure
// (derived from Sections III-IV): triples of every level, target classes,
// temporary ("blue") accumulator sets and the Gram contributor lists.
struct LeafPlan {
  TaskList H, X1, G1, G2, G3;        // row Gram pieces
  TaskList Hc, X1c, G1c, G2c, G3c;   // column Gram pieces
  TaskList Z, Zc, gB, hA;            // per dense block products
  TaskList PA, PB;
  TaskList LA_F, PS, LA_R, RB_F, SP, RB_R, Ahat, Bhat;
  TaskList adm_R, adm_B, dense;      // triples by target class
  TaskList densA1, densA2, densB1, densB2;
  int n_blue_tiles = 0;              // number of case-1 parents at level L-1
};

struct LevelPlan {
  // case-1 targets of this level (parents of blue accumulators one level down)
  int n_case1 = 0;
  TaskList G1, G1c, Y, G2, Yc, G2c, D, G3, Q, G3c;
  TaskList PA, PB, AhatNL, PAS, AhatR, BhatNL, SBP, BhatR;
  TaskList c1X, c1_R, c1_B;
  // triples by A-type and target class, re-associated.  NL x R: W_o = sum_J Ahat_IJ S^B_JK
  // (w_nl_*, output o = slot), then target += W_o P^B_K (f_nl_*); R x NL:
  // W_o = sum_J S^A_IJ Bhat_JK (w_r_*), then target += P^A_I W_o (f_r_*)
  TaskList w_nl_R, w_nl_B, w_nl_NL, f_nl_R, f_nl_B, f_nl_NL;
  TaskList w_r_R, w_r_B, w_r_NL, f_r_R, f_r_B, f_r_NL;
  // both second stages of a target class in one list (when the two inner
  // dimensions agree): per target W_nl P^B (selector 0) and P^A W_r (selector 1)
  TaskList f_R, f_B, f_NL;
  int n_blue_tiles = 0;              // case-1 parents at level l-1 (tiles of Acc_l)
};

struct SplitPlan {
  TaskList X, toR, toNL, toF, F1, F2;
};

struct PiPlan {
  TaskList leaf;
  std::vector<TaskList> X, S;  // per level l < L
};

struct Plan {
  LeafPlan leaf;
  std::vector<LevelPlan> lev;     // index l, used for lmin <= l < L
  std::vector<SplitPlan> split;   // index l, lmin <= l < L
  PiPlan pi;
  int64_t n_triples = 0;
  std::vector<int64_t> triples_per_level;
  std::vector<int64_t> n_case1, n_blue;
};

std::string build_plan(const Structure& s, Plan& p);

}  // namespace h2
