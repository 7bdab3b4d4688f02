// Structure validation and the symbolic phase of the H^2 product.
//
// Triples of level l (derived from Sections III-IV): every pair of an A node
// (I,J) and a B node (J,K) of level l that are not both non-leaf; non-leaf x
// non-leaf pairs descend to their children.  The target (I,K) of a triple is
// a node of C (admissible, dense or non-leaf) or lies inside an admissible
// block of an upper level ("blue" block of Fig. 3(c)), in which case the
// result is kept as a temporary coupling and merged 2x2 into its parent at
// the next level (equation nonleafA, "case-1" of the non-leaf level).
#include "structure.h"

#include <algorithm>
#include <map>
#include <set>

namespace h2 {

static inline uint64_t key(int r, int c) { return ((uint64_t)(uint32_t)r << 32) | (uint32_t)c; }

std::string build_structure(Structure& s, int64_t n, int64_t L, const int64_t* leaf_off,
                            const int64_t* perm, const int64_t* node_off, const int32_t* row,
                            const int32_t* col, const int32_t* type) {
  if (n < 1 || L < 0 || L > 30) return "n must be >= 1 and 0 <= L <= 30";
  if (!leaf_off || !perm || !node_off || !row || !col || !type) return "null structure array";
  const int64_t nleaf = 1LL << L;
  s.n = n;
  s.L = (int)L;
  s.leaf_off.assign(leaf_off, leaf_off + nleaf + 1);
  if (s.leaf_off[0] != 0 || s.leaf_off[nleaf] != n) return "leaf_off must run from 0 to n";
  int maxleaf = 0;
  s.leaf_size.resize(nleaf);
  for (int64_t c = 0; c < nleaf; ++c) {
    const int64_t sz = s.leaf_off[c + 1] - s.leaf_off[c];
    if (sz < 1) return "every leaf must hold at least one point";
    s.leaf_size[c] = (int)sz;
    maxleaf = std::max(maxleaf, (int)sz);
  }
  s.npad = ((maxleaf + 15) / 16) * 16;
  s.perm.assign(perm, perm + n);
  {
    std::vector<char> seen(n, 0);
    for (int64_t p = 0; p < n; ++p) {
      if (perm[p] < 0 || perm[p] >= n || seen[perm[p]]) return "perm is not a permutation";
      seen[perm[p]] = 1;
    }
  }
  if (node_off[0] != 0) return "node_off[0] must be 0";
  s.lev.assign(L + 1, LevelNodes());
  s.node_base.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) {
    const int64_t a = node_off[l], b = node_off[l + 1];
    if (b < a) return "node_off must be non-decreasing";
    s.node_base[l] = a;
    LevelNodes& ln = s.lev[l];
    const int nc = 1 << l;
    for (int64_t q = a; q < b; ++q) {
      if (row[q] < 0 || row[q] >= nc || col[q] < 0 || col[q] >= nc) return "node cluster out of range";
      if (type[q] < 0 || type[q] > 2) return "node type must be 0, 1 or 2";
      if (type[q] == kF && l != L) return "dense nodes are only allowed at the leaf level";
      if (type[q] == kNL && l == L) return "non-leaf nodes are not allowed at the leaf level";
      const int idx = (int)(q - a);
      if (!ln.index.emplace(key(row[q], col[q]), idx).second) return "duplicate node";
      ln.row.push_back(row[q]);
      ln.col.push_back(col[q]);
      ln.type.push_back(type[q]);
      ln.nl_index.push_back(type[q] == kNL ? ln.n_nl++ : -1);
    }
  }
  s.node_base[L + 1] = node_off[L + 1];
  if (s.lev[0].size() != 1 || s.lev[0].row[0] != 0 || s.lev[0].col[0] != 0)
    return "level 0 must hold exactly the root block";
  for (int l = 1; l <= L; ++l) {
    LevelNodes& ln = s.lev[l];
    const LevelNodes& up = s.lev[l - 1];
    ln.tile_loc.resize(ln.size());
    for (int q = 0; q < ln.size(); ++q) {
      const int p = up.find(ln.row[q] >> 1, ln.col[q] >> 1);
      if (p < 0 || up.type[p] != kNL) return "node without a non-leaf parent";
      ln.tile_loc[q] = enc(up.nl_index[p], ln.row[q] & 1, ln.col[q] & 1);
    }
    // every non-leaf parent has its four children
    int64_t children = 0;
    for (int q = 0; q < up.size(); ++q) children += up.type[q] == kNL ? 4 : 0;
    if (children != ln.size()) return "non-leaf node without four children";
  }
  if (L == 0) s.lev[0].tile_loc.assign(1, 0);
  s.lmin = L;
  for (int l = 0; l <= L; ++l) {
    bool any = false;
    for (int t : s.lev[l].type) any |= t == kR;
    if (any) {
      s.lmin = l;
      break;
    }
  }
  return "";
}

bool Structure::same_as(const Structure& o) const {
  if (n != o.n || L != o.L || leaf_off != o.leaf_off || perm != o.perm) return false;
  for (int l = 0; l <= L; ++l) {
    if (lev[l].row != o.lev[l].row || lev[l].col != o.lev[l].col || lev[l].type != o.lev[l].type)
      return false;
  }
  return true;
}

int Structure::sparsity_constant() const {
  int best = 0;
  for (int l = 0; l <= L; ++l) {
    std::vector<int> cr(1 << l, 0), cc(1 << l, 0);
    for (int q = 0; q < lev[l].size(); ++q) {
      best = std::max(best, ++cr[lev[l].row[q]]);
      best = std::max(best, ++cc[lev[l].col[q]]);
    }
  }
  return best;
}

namespace {

// Target class of (i,k) at level l: a node type of C, or kBlue when (i,k)
// lies inside an admissible block of an upper level.
int target_of(const Structure& s, int l, int i, int k, int* node) {
  const int q = s.lev[l].find(i, k);
  if (q >= 0) {
    *node = q;
    return s.lev[l].type[q];
  }
  *node = -1;
  return kBlue;
}

struct Seg {
  std::map<std::pair<int, int>, std::vector<std::pair<int, int>>> byout;
  std::map<std::pair<int, int>, int> pcl;  // per output: cluster of its projection factor
  void add(int sortkey, int outv, int av, int bv, int pc = -1) {
    byout[{sortkey, outv}].push_back({av, bv});
    pcl[{sortkey, outv}] = pc;
  }
  void emit(TaskList& t) const {
    for (const auto& kv : byout) {
      for (const auto& ab : kv.second) t.add_task(ab.first, ab.second);
      t.close(kv.first.second);
    }
  }
  // two-stage form: stage 1 sums the tasks of output o into slot o; stage 2
  // applies the output's projection factor (cluster pcl) to slot o and adds
  // into the target; pfirst: the factor is the left operand of stage 2
  void emit2(TaskList& w, TaskList& f, bool pfirst) const {
    int o = 0;
    for (const auto& kv : byout) {
      for (const auto& ab : kv.second) w.add_task(ab.first, ab.second);
      w.close(enc(o));
      const int pc = pcl.at(kv.first);
      if (pfirst)
        f.add_task(enc(pc), enc(o));
      else
        f.add_task(enc(o), enc(pc));
      f.close(kv.first.second);
      ++o;
    }
  }
};

// One second-stage list over the targets of both forms, in target order:
// W_nl[o] P^B_K with selector 0 on both operands, P^A_I W_r[o] with selector 1.
void merge_second_stage(const Seg& nl, const Seg& r, TaskList& f) {
  std::map<std::pair<int, int>, std::pair<int, int>> onl, orr;  // key -> (slot, cluster)
  int o = 0;
  for (const auto& kv : nl.byout) onl[kv.first] = {o++, nl.pcl.at(kv.first)};
  o = 0;
  for (const auto& kv : r.byout) orr[kv.first] = {o++, r.pcl.at(kv.first)};
  std::map<std::pair<int, int>, int> keys;
  for (const auto& kv : onl) keys[kv.first] = 1;
  for (const auto& kv : orr) keys[kv.first] = 1;
  for (const auto& kv : keys) {
    auto a = onl.find(kv.first);
    if (a != onl.end()) f.add_task(enc(a->second.first), enc(a->second.second));
    auto b = orr.find(kv.first);
    if (b != orr.end()) f.add_task(enc(b->second.second, 0, 0, 1), enc(b->second.first, 0, 0, 1));
    f.close(kv.first.second);
  }
}

}  // namespace

std::string build_plan(const Structure& s, Plan& p) {
  const int L = s.L;
  const int lmin = s.lmin;
  p.lev.assign(L + 1, LevelPlan());
  p.split.assign(L + 1, SplitPlan());
  p.triples_per_level.assign(L + 1, 0);
  p.n_case1.assign(L + 1, 0);
  p.n_blue.assign(L + 1, 0);

  // ---- triples of every level
  struct Tri {
    int i, j, k, qa, qb, ta, tb, tg, qc;
  };
  std::vector<std::vector<Tri>> tri(L + 1);
  for (int l = lmin; l <= L; ++l) {
    const LevelNodes& ln = s.lev[l];
    std::vector<std::vector<int>> byrow(1 << l);
    for (int q = 0; q < ln.size(); ++q) byrow[ln.row[q]].push_back(q);
    for (int qa = 0; qa < ln.size(); ++qa) {
      const int i = ln.row[qa], j = ln.col[qa], ta = ln.type[qa];
      for (int qb : byrow[j]) {
        const int tb = ln.type[qb];
        if (ta == kNL && tb == kNL) continue;
        const int k = ln.col[qb];
        int qc;
        const int tg = target_of(s, l, i, k, &qc);
        tri[l].push_back({i, j, k, qa, qb, ta, tb, tg, qc});
      }
    }
    p.triples_per_level[l] = (int64_t)tri[l].size();
    p.n_triples += (int64_t)tri[l].size();
  }

  // ---- blue accumulators and case-1 targets, bottom-up
  std::vector<std::map<std::pair<int, int>, int>> blue(L + 2), case1(L + 1);
  for (int l = L; l >= lmin; --l) {
    std::set<std::pair<int, int>> bl;
    for (const Tri& t : tri[l])
      if (t.tg == kBlue) bl.insert({t.i, t.k});
    if (l < L) {
      for (const auto& kv : case1[l]) {
        int qc;
        if (target_of(s, l, kv.first.first, kv.first.second, &qc) == kBlue) bl.insert(kv.first);
      }
    }
    int idx = 0;
    for (const auto& b : bl) blue[l][b] = idx++;
    p.n_blue[l] = (int64_t)bl.size();
    if (l - 1 >= 0) {
      std::set<std::pair<int, int>> par;
      for (const auto& b : bl) par.insert({b.first >> 1, b.second >> 1});
      int ci = 0;
      for (const auto& pr : par) case1[l - 1][pr] = ci++;
      p.n_case1[l - 1] = (int64_t)par.size();
    }
  }
  if (lmin >= 0 && !blue[lmin].empty()) return "internal: blue accumulator above the top level";
  auto acc_loc = [&](int l, int i, int k) -> int {
    // tile of Acc_l = index of the parent among the case-1 targets of l-1
    const int t = case1[l - 1].at({i >> 1, k >> 1});
    return enc(t, i & 1, k & 1);
  };

  const LevelNodes& lf = s.lev[L];
  const int nleaf = 1 << L;
  // ================================================================ Pi
  for (int j = 0; j < nleaf; ++j) {
    p.pi.leaf.add_task(enc(j), enc(j));
    p.pi.leaf.close(enc(j));
  }
  p.pi.X.assign(L + 1, TaskList());
  p.pi.S.assign(L + 1, TaskList());
  for (int l = L - 1; l >= lmin; --l) {
    for (int c = 0; c < (2 << l); ++c) {
      p.pi.X[l].add_task(enc(c), enc(c >> 1, c & 1));
      p.pi.X[l].close(enc(c));
    }
    for (int J = 0; J < (1 << l); ++J) {
      for (int a = 0; a < 2; ++a) p.pi.S[l].add_task(enc(J, a), enc(2 * J + a));
      p.pi.S[l].close(enc(J));
    }
  }

  // ================================================================ leaf
  LeafPlan& P = p.leaf;
  {
    std::vector<std::vector<int>> arow(nleaf), bcol(nleaf), brow(nleaf);
    for (int q = 0; q < lf.size(); ++q) {
      arow[lf.row[q]].push_back(q);
      bcol[lf.col[q]].push_back(q);
      brow[lf.row[q]].push_back(q);
    }
    auto adm = [&](int i, int k) {
      int qc;
      const int tg = target_of(s, L, i, k, &qc);
      return tg == kR || tg == kBlue;
    };
    // per dense-block Gram pieces
    std::vector<int> hasK1(lf.size(), 0), hasI1(lf.size(), 0);
    for (int q = 0; q < lf.size(); ++q) {
      if (lf.type[q] != kF) continue;
      P.gB.add_task(enc(q), enc(q));
      P.gB.close(enc(q));
      P.hA.add_task(enc(q), enc(q));
      P.hA.close(enc(q));
      const int i = lf.row[q], j = lf.col[q];
      // K1: dense B blocks (j,k) whose product with this block targets an admissible block
      int cnt = 0;
      for (int qb : brow[j])
        if (lf.type[qb] == kF && adm(i, lf.col[qb])) {
          P.H.add_task(enc(qb), 0);
          ++cnt;
        }
      if (cnt) {
        P.H.close(enc(q));
        P.X1.add_task(enc(q), enc(q));
        P.X1.close(enc(q));
        hasK1[q] = 1;
      }
      // I1: dense A blocks (i',i) ... for the column side of block q as a B block (j,k)=(i,j)
      const int jj = lf.row[q], kk = lf.col[q];
      int cnt2 = 0;
      for (int qa : bcol[jj])
        if (lf.type[qa] == kF && adm(lf.row[qa], kk)) {
          P.Hc.add_task(enc(qa), 0);
          ++cnt2;
        }
      if (cnt2) {
        P.Hc.close(enc(q));
        P.X1c.add_task(enc(q), enc(q));
        P.X1c.close(enc(q));
        hasI1[q] = 1;
      }
      P.Z.add_task(enc(q), enc(j));
      P.Z.close(enc(q));
      P.Zc.add_task(enc(q), enc(jj));
      P.Zc.close(enc(q));
    }
    for (int i = 0; i < nleaf; ++i) {
      for (int q : arow[i])
        if (lf.type[q] == kF && hasK1[q]) P.G1.add_task(enc(q), enc(q));
      P.G1.close(enc(i));
      for (int q : arow[i])
        if (lf.type[q] == kF) P.G2.add_task(enc(q), enc(q));
      P.G2.close(enc(i));
      P.G3.add_task(enc(i), enc(i));
      P.G3.close(enc(i));
      for (int q : bcol[i])
        if (lf.type[q] == kF && hasI1[q]) P.G1c.add_task(enc(q), enc(q));
      P.G1c.close(enc(i));
      for (int q : bcol[i])
        if (lf.type[q] == kF) P.G2c.add_task(enc(q), enc(q));
      P.G2c.close(enc(i));
      P.G3c.add_task(enc(i), enc(i));
      P.G3c.close(enc(i));
      P.PA.add_task(enc(i), enc(i));
      P.PA.close(enc(i));
      P.PB.add_task(enc(i), enc(i));
      P.PB.close(enc(i));
    }
    for (int q = 0; q < lf.size(); ++q) {
      const int i = lf.row[q], j = lf.col[q];
      if (lf.type[q] == kF) {
        P.LA_F.add_task(enc(i), enc(q));
        P.LA_F.close(enc(q));
        P.RB_F.add_task(enc(q), enc(j));
        P.RB_F.close(enc(q));
      } else {
        P.PS.add_task(enc(i), enc(q));
        P.PS.close(enc(q));
        P.LA_R.add_task(enc(q), enc(j));
        P.LA_R.close(enc(q));
        P.SP.add_task(enc(q), enc(j));
        P.SP.close(enc(q));
        P.RB_R.add_task(enc(i), enc(q));
        P.RB_R.close(enc(q));
        P.densA1.add_task(enc(i), enc(q));
        P.densA1.close(enc(q));
        P.densA2.add_task(enc(q), enc(j));
        P.densA2.close(enc(q));
        P.densB1.add_task(enc(i), enc(q));
        P.densB1.close(enc(q));
        P.densB2.add_task(enc(q), enc(j));
        P.densB2.close(enc(q));
      }
      if (L >= 1) {
        P.Ahat.add_task(enc(q), enc(j));
        P.Ahat.close(lf.tile_loc[q]);
        P.Bhat.add_task(enc(i), enc(q));
        P.Bhat.close(lf.tile_loc[q]);
      }
    }
    Seg sR, sB, sD;
    for (const Tri& t : tri[L]) {
      if (t.tg == kF) {
        sD.add(t.qc, enc(t.qc), enc(t.qa, 0, 0, t.ta == kR), enc(t.qb, 0, 0, t.tb == kR));
      } else if (t.tg == kR) {
        sR.add(t.qc, enc(t.qc), enc(t.qa), enc(t.qb));
      } else {
        sB.add(blue[L].at({t.i, t.k}), acc_loc(L, t.i, t.k), enc(t.qa), enc(t.qb));
      }
    }
    sR.emit(P.adm_R);
    sB.emit(P.adm_B);
    sD.emit(P.dense);
    P.n_blue_tiles = L >= 1 ? (int)p.n_case1[L - 1] : 0;
  }

  // ============================================================ non-leaf
  for (int l = L - 1; l >= lmin; --l) {
    LevelPlan& Q = p.lev[l];
    const LevelNodes& ln = s.lev[l];
    const int ncl = 1 << l;
    Q.n_case1 = (int)p.n_case1[l];
    Q.n_blue_tiles = l >= 1 ? (int)p.n_case1[l - 1] : 0;
    std::vector<std::vector<int>> c1row(ncl), c1col(ncl), arow(ncl), bcol(ncl);
    std::vector<std::pair<int, int>> c1list(Q.n_case1);
    for (const auto& kv : case1[l]) {
      c1list[kv.second] = kv.first;
      c1row[kv.first.first].push_back(kv.second);
      c1col[kv.first.second].push_back(kv.second);
    }
    for (int q = 0; q < ln.size(); ++q) {
      arow[ln.row[q]].push_back(q);
      bcol[ln.col[q]].push_back(q);
    }
    for (int I = 0; I < ncl; ++I) {
      for (int t : c1row[I]) Q.G1.add_task(enc(t), enc(t));
      Q.G1.close(enc(I));
      for (int t : c1col[I]) Q.G1c.add_task(enc(t), enc(t));
      Q.G1c.close(enc(I));
      for (int q : arow[I])
        if (ln.type[q] == kNL) Q.G2.add_task(enc(q), enc(q));
      Q.G2.close(enc(I));
      for (int q : bcol[I])
        if (ln.type[q] == kNL) Q.G2c.add_task(enc(q), enc(q));
      Q.G2c.close(enc(I));
      for (int a = 0; a < 2; ++a) {
        Q.D.add_task(enc(2 * I + a), enc(I, a));
        Q.D.close(enc(I, a));
        Q.Q.add_task(enc(2 * I + a), enc(I, a));
        Q.Q.close(enc(I, a));
      }
      Q.G3.add_task(enc(I), enc(I));
      Q.G3.close(enc(I));
      Q.G3c.add_task(enc(I), enc(I));
      Q.G3c.close(enc(I));
      Q.PA.add_task(enc(I), enc(I));
      Q.PA.close(enc(I));
      Q.PB.add_task(enc(I), enc(I));
      Q.PB.close(enc(I));
    }
    for (int q = 0; q < ln.size(); ++q) {
      const int I = ln.row[q], J = ln.col[q];
      if (ln.type[q] == kNL) {
        Q.Y.add_task(enc(ln.nl_index[q]), enc(J));
        Q.Y.close(enc(q));
        Q.Yc.add_task(enc(I), enc(ln.nl_index[q]));
        Q.Yc.close(enc(q));
        Q.AhatNL.add_task(enc(I), enc(q));
        Q.AhatNL.close(ln.tile_loc[q]);
        Q.BhatNL.add_task(enc(q), enc(J));
        Q.BhatNL.close(ln.tile_loc[q]);
      } else {  // admissible (no dense nodes above the leaves)
        Q.PAS.add_task(enc(I), enc(q));
        Q.PAS.close(enc(q));
        Q.AhatR.add_task(enc(q), enc(J));
        Q.AhatR.close(ln.tile_loc[q]);
        Q.SBP.add_task(enc(q), enc(J));
        Q.SBP.close(enc(q));
        Q.BhatR.add_task(enc(I), enc(q));
        Q.BhatR.close(ln.tile_loc[q]);
      }
    }
    for (int t = 0; t < Q.n_case1; ++t) {
      const int I = c1list[t].first, K = c1list[t].second;
      Q.c1X.add_task(enc(I), enc(t));
      Q.c1X.close(enc(t));
      int qc;
      const int tg = target_of(s, l, I, K, &qc);
      if (tg == kR) {
        Q.c1_R.add_task(enc(t), enc(K));
        Q.c1_R.close(enc(qc));
      } else if (tg == kBlue) {
        Q.c1_B.add_task(enc(t), enc(K));
        Q.c1_B.close(acc_loc(l, I, K));
      } else {
        return "internal: case-1 target is neither admissible nor blue";
      }
    }
    Seg s_nl[3], s_r[3];
    for (const Tri& t : tri[l]) {
      int cls, outv, sk;
      if (t.tg == kR) {
        cls = 0;
        outv = enc(t.qc);
        sk = t.qc;
      } else if (t.tg == kBlue) {
        cls = 1;
        sk = blue[l].at({t.i, t.k});
        outv = acc_loc(l, t.i, t.k);
      } else if (t.tg == kNL) {
        cls = 2;
        outv = enc(t.qc);
        sk = t.qc;
      } else {
        return "internal: dense target above the leaf level";
      }
      if (t.ta == kNL)
        s_nl[cls].add(sk, outv, ln.tile_loc[t.qa], enc(t.qb), t.k);
      else
        s_r[cls].add(sk, outv, enc(t.qa), ln.tile_loc[t.qb], t.i);
    }
    s_nl[0].emit2(Q.w_nl_R, Q.f_nl_R, false);
    s_nl[1].emit2(Q.w_nl_B, Q.f_nl_B, false);
    s_nl[2].emit2(Q.w_nl_NL, Q.f_nl_NL, false);
    s_r[0].emit2(Q.w_r_R, Q.f_r_R, true);
    s_r[1].emit2(Q.w_r_B, Q.f_r_B, true);
    s_r[2].emit2(Q.w_r_NL, Q.f_r_NL, true);
    merge_second_stage(s_nl[0], s_r[0], Q.f_R);
    merge_second_stage(s_nl[1], s_r[1], Q.f_B);
    merge_second_stage(s_nl[2], s_r[2], Q.f_NL);

    // ---- split of couplings attached to non-leaf nodes (top-down later)
    SplitPlan& SP = p.split[l];
    const LevelNodes& ch = s.lev[l + 1];
    for (int q = 0; q < ln.size(); ++q) {
      if (ln.type[q] != kNL) continue;
      const int I = ln.row[q], K = ln.col[q];
      SP.X.add_task(enc(I), enc(q));
      SP.X.close(enc(q));
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          const int qq = ch.find(2 * I + a, 2 * K + b);
          if (qq < 0) return "internal: missing child of a non-leaf node";
          TaskList* tl = ch.type[qq] == kR ? &SP.toR : (ch.type[qq] == kNL ? &SP.toNL : &SP.toF);
          tl->add_task(enc(q, a), enc(K, b));
          tl->close(enc(qq));
          if (ch.type[qq] == kF) {
            SP.F1.add_task(enc(2 * I + a), enc(qq));
            SP.F1.close(enc(qq));
            SP.F2.add_task(enc(qq), enc(2 * K + b));
            SP.F2.close(enc(qq));
          }
        }
    }
  }
  return "";
}

}  // namespace h2
