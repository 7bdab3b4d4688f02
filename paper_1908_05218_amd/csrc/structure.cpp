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
#include <iterator>
#include <thread>

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

// Nodes of one level grouped by row (or column) cluster, node indices
// ascending within a group: group g is idx[ptr[g] .. ptr[g+1]).
struct Groups {
  std::vector<int> ptr, idx;
  Groups(const LevelNodes& ln, int ncl, bool by_col) : ptr(ncl + 1, 0), idx(ln.size()) {
    const std::vector<int>& g = by_col ? ln.col : ln.row;
    for (int q = 0; q < ln.size(); ++q) ++ptr[g[q] + 1];
    for (int c = 0; c < ncl; ++c) ptr[c + 1] += ptr[c];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int q = 0; q < ln.size(); ++q) idx[fill[g[q]]++] = q;
  }
  const int* begin(int g) const { return idx.data() + ptr[g]; }
  const int* end(int g) const { return idx.data() + ptr[g + 1]; }
};

// Dense map over the clusters of a level, filled for one row (or column) at
// a time and cleared through the list of entries it set.
struct ClusterMap {
  std::vector<int> v, set_;
  explicit ClusterMap(int n) : v(n, -1) {}
  void put(int k, int x) {
    if (v[k] < 0) set_.push_back(k);
    v[k] = x;
  }
  int operator[](int k) const { return v[k]; }
  void clear() {
    for (int k : set_) v[k] = -1;
    set_.clear();
  }
};

inline uint64_t pkey(int r, int c) { return ((uint64_t)(uint32_t)r << 32) | (uint32_t)c; }
inline int key_row(uint64_t k) { return (int)(k >> 32); }
inline int key_col(uint64_t k) { return (int)(k & 0xffffffffu); }

// Sorted (row, column) keys of one level with a per-row index: the keys of
// row r are keys[rp[r] .. rp[r+1]).
struct KeySet {
  std::vector<uint64_t> keys;
  std::vector<int> rp;
  void index(int ncl) {
    rp.assign(ncl + 1, 0);
    for (uint64_t k : keys) ++rp[key_row(k) + 1];
    for (int r = 0; r < ncl; ++r) rp[r + 1] += rp[r];
  }
  // fill m with column -> position for the keys of row r
  void load_row(int r, ClusterMap& m) const {
    for (int x = rp[r]; x < rp[r + 1]; ++x) m.put(key_col(keys[x]), x);
  }
};

// The triples of row i of level l (A node (i,j) x B node (j,k), not both
// non-leaf), bucketed by target column k; targets visited in ascending k.
// A target's tasks are in ascending A-node order, the order in which the
// product sums them.
struct RowTriples {
  struct T {
    int qa, qb;
  };
  std::vector<std::vector<T>> bucket;
  std::vector<int> cols;
  explicit RowTriples(int ncl) : bucket(ncl) {}
  void gather(const LevelNodes& ln, const Groups& rows, int i) {
    for (int k : cols) bucket[k].clear();
    cols.clear();
    for (const int* pa = rows.begin(i); pa != rows.end(i); ++pa) {
      const int qa = *pa, j = ln.col[qa], ta = ln.type[qa];
      for (const int* pb = rows.begin(j); pb != rows.end(j); ++pb) {
        const int qb = *pb;
        if (ta == kNL && ln.type[qb] == kNL) continue;
        const int k = ln.col[qb];
        if (bucket[k].empty()) cols.push_back(k);
        bucket[k].push_back({qa, qb});
      }
    }
    std::sort(cols.begin(), cols.end());
  }
};

// Host threads for the row walks of the symbolic phase.
int plan_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return h < 1 ? 1 : (h > 16 ? 16 : (int)h);
}

// Runs fn(t, r0, r1) for t < nt over contiguous row ranges [r0, r1) of about
// equal total weight, thread t = 0 on the caller's thread.
template <class F>
void parallel_rows(const std::vector<int64_t>& w, int nt, F fn) {
  const int n = (int)w.size();
  int64_t tot = 0;
  for (int64_t x : w) tot += x;
  std::vector<int> cut(nt + 1, n);
  cut[0] = 0;
  int t = 1;
  int64_t acc = 0;
  for (int r = 0; r < n && t < nt; ++r) {
    acc += w[r];
    while (t < nt && acc * nt >= tot * t) cut[t++] = r + 1;
  }
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(fn, i, cut[i], cut[i + 1]);
  fn(0, cut[0], cut[1]);
  for (auto& x : th) x.join();
}

// Appends fragment f to t.  Slot numbers that a fragment counted from zero
// are shifted: outputs by out_add, first / second operands by a_add / b_add
// (in encoded units).
void add_shifted(std::vector<int>& t, const std::vector<int>& f, size_t from, int add) {
  const size_t n0 = t.size();
  t.resize(n0 + f.size() - from);
  int* d = t.data() + n0;
  for (size_t x = from; x < f.size(); ++x) *d++ = f[x] + add;
}

void append(TaskList& t, const TaskList& f, int out_add = 0, int a_add = 0, int b_add = 0) {
  const int base = t.ntask();
  add_shifted(t.out, f.out, 0, out_add);
  add_shifted(t.seg, f.seg, 1, base);
  add_shifted(t.a, f.a, 0, a_add);
  add_shifted(t.b, f.b, 0, b_add);
}

// room for n more tasks and outputs
void reserve_more(TaskList& t, size_t tasks, size_t outs) {
  t.a.reserve(t.a.size() + tasks);
  t.b.reserve(t.b.size() + tasks);
  t.out.reserve(t.out.size() + outs);
  t.seg.reserve(t.seg.size() + outs);
}

// The merged second stage holds two task forms: W_nl[o] x P^B (selector 0,
// slot in the first operand) and P^A x W_r[o] (selector 1, slot in the
// second operand).
void append_merged(TaskList& t, const TaskList& f, int n_add, int r_add) {
  const int base = t.ntask();
  for (int o : f.out) t.out.push_back(o);
  for (size_t x = 1; x < f.seg.size(); ++x) t.seg.push_back(f.seg[x] + base);
  for (size_t x = 0; x < f.a.size(); ++x) {
    const bool r = (f.a[x] >> 2) & 1;
    t.a.push_back(f.a[x] + (r ? 0 : n_add));
    t.b.push_back(f.b[x] + (r ? r_add : 0));
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

  std::vector<Groups> rows, cols;
  rows.reserve(L + 1);
  cols.reserve(L + 1);
  for (int l = 0; l <= L; ++l) {
    rows.emplace_back(s.lev[l], 1 << l, false);
    cols.emplace_back(s.lev[l], 1 << l, true);
  }

  // ---- triple counts, blue accumulators and case-1 targets, bottom-up.
  // blue[l]: targets of level l inside an upper admissible block (from the
  // triples of level l, and the case-1 targets of level l that are not nodes);
  // case1[l-1]: the parents of blue[l], merged 2x2 at level l-1
  std::vector<KeySet> blue(L + 2), case1(L + 1);
  // per row: the pairs of an A node of the row with a B node (the row walks'
  // work, used to split rows over threads)
  std::vector<std::vector<int64_t>> work(L + 1);
  // triples per thread of each level's row walk (same split in both walks)
  std::vector<std::vector<int64_t>> thread_tri(L + 1);
  const int max_threads = plan_threads();
  auto nthreads = [&](const std::vector<int64_t>& w) {
    int64_t tot = 0;
    for (int64_t x : w) tot += x;
    const int64_t by_work = tot / 200000 + 1;  // threads only for large levels
    return (int)std::min<int64_t>(max_threads, std::min<int64_t>(by_work, (int64_t)w.size()));
  };
  for (int l = L; l >= lmin; --l) {
    const LevelNodes& ln = s.lev[l];
    const int ncl = 1 << l;
    std::vector<int64_t>& w = work[l];
    w.assign(ncl, 0);
    for (int i = 0; i < ncl; ++i)
      for (const int* pa = rows[l].begin(i); pa != rows[l].end(i); ++pa)
        w[i] += rows[l].ptr[ln.col[*pa] + 1] - rows[l].ptr[ln.col[*pa]];
    const int nt = nthreads(w);
    std::vector<std::vector<uint64_t>> blt(nt);
    std::vector<int64_t> ntt(nt, 0);
    parallel_rows(w, nt, [&](int t, int r0, int r1) {
      ClusterMap node(ncl), seen(ncl);
      std::vector<uint64_t>& bl = blt[t];
      int64_t ntri = 0;
      for (int i = r0; i < r1; ++i) {
        for (const int* pc = rows[l].begin(i); pc != rows[l].end(i); ++pc) node.put(ln.col[*pc], *pc);
        const size_t first = bl.size();
        for (const int* pa = rows[l].begin(i); pa != rows[l].end(i); ++pa) {
          const int qa = *pa, j = ln.col[qa], ta = ln.type[qa];
          for (const int* pb = rows[l].begin(j); pb != rows[l].end(j); ++pb) {
            const int qb = *pb;
            if (ta == kNL && ln.type[qb] == kNL) continue;
            ++ntri;
            const int k = ln.col[qb];
            if (node[k] < 0 && seen[k] < 0) {
              seen.put(k, 1);
              bl.push_back(pkey(i, k));
            }
          }
        }
        std::sort(bl.begin() + first, bl.end());
        node.clear();
        seen.clear();
      }
      ntt[t] = ntri;
    });
    std::vector<uint64_t>& bl = blue[l].keys;
    int64_t ntri = 0;
    for (int t = 0; t < nt; ++t) {
      bl.insert(bl.end(), blt[t].begin(), blt[t].end());
      ntri += ntt[t];
    }
    p.triples_per_level[l] = ntri;
    thread_tri[l] = ntt;
    p.n_triples += ntri;
    if (l < L) {
      std::vector<uint64_t> extra;
      for (uint64_t k : case1[l].keys)
        if (ln.find(key_row(k), key_col(k)) < 0) extra.push_back(k);
      std::vector<uint64_t> merged;
      merged.reserve(bl.size() + extra.size());
      std::merge(bl.begin(), bl.end(), extra.begin(), extra.end(), std::back_inserter(merged));
      merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
      bl.swap(merged);
    }
    blue[l].index(ncl);
    p.n_blue[l] = (int64_t)bl.size();
    if (l >= 1) {
      std::vector<uint64_t>& par = case1[l - 1].keys;
      par.reserve(bl.size());
      for (uint64_t k : bl) par.push_back(pkey(key_row(k) >> 1, key_col(k) >> 1));
      std::sort(par.begin(), par.end());
      par.erase(std::unique(par.begin(), par.end()), par.end());
      case1[l - 1].index(ncl >> 1);
      p.n_case1[l - 1] = (int64_t)par.size();
    }
  }
  if (lmin >= 0 && !blue[lmin].keys.empty()) return "internal: blue accumulator above the top level";

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
    const Groups& lrow = rows[L];
    const Groups& lcol = cols[L];
    // adm: the product of two leaf blocks with target (i,k) lands in an
    // admissible block (a node of type R, or inside an upper R block)
    ClusterMap tmap(nleaf);
    std::vector<int> hasK1(lf.size(), 0), hasI1(lf.size(), 0);
    // K1 (row side): for a dense block (i,j), the dense B blocks (j,k) whose
    // product with it targets an admissible block; by rows of the target
    for (int i = 0; i < nleaf; ++i) {
      for (const int* pc = lrow.begin(i); pc != lrow.end(i); ++pc) tmap.put(lf.col[*pc], lf.type[*pc]);
      for (const int* pa = lrow.begin(i); pa != lrow.end(i); ++pa) {
        const int q = *pa;
        if (lf.type[q] != kF) continue;
        const int j = lf.col[q];
        int cnt = 0;
        for (const int* pb = lrow.begin(j); pb != lrow.end(j); ++pb) {
          const int tk = tmap[lf.col[*pb]];
          if (lf.type[*pb] == kF && (tk < 0 || tk == kR)) {
            P.H.add_task(enc(*pb), 0);
            ++cnt;
          }
        }
        if (cnt) {
          P.H.close(enc(q));
          P.X1.add_task(enc(q), enc(q));
          P.X1.close(enc(q));
          hasK1[q] = 1;
        }
      }
      tmap.clear();
    }
    // I1 (column side): for a dense block (j,k) as a B factor, the dense A
    // blocks (i,j) whose product with it targets an admissible block; by
    // columns of the target
    {
      // collected per block, emitted in block order
      std::vector<std::vector<int>> i1(lf.size());
      for (int k = 0; k < nleaf; ++k) {
        for (const int* pc = lcol.begin(k); pc != lcol.end(k); ++pc) tmap.put(lf.row[*pc], lf.type[*pc]);
        for (const int* pb = lcol.begin(k); pb != lcol.end(k); ++pb) {
          const int q = *pb;
          if (lf.type[q] != kF) continue;
          const int jj = lf.row[q];
          for (const int* pa = lcol.begin(jj); pa != lcol.end(jj); ++pa) {
            const int ti = tmap[lf.row[*pa]];
            if (lf.type[*pa] == kF && (ti < 0 || ti == kR)) i1[q].push_back(*pa);
          }
        }
        tmap.clear();
      }
      for (int q = 0; q < lf.size(); ++q) {
        if (i1[q].empty()) continue;
        for (int qa : i1[q]) P.Hc.add_task(enc(qa), 0);
        P.Hc.close(enc(q));
        P.X1c.add_task(enc(q), enc(q));
        P.X1c.close(enc(q));
        hasI1[q] = 1;
      }
    }
    for (int q = 0; q < lf.size(); ++q) {
      if (lf.type[q] != kF) continue;
      P.gB.add_task(enc(q), enc(q));
      P.gB.close(enc(q));
      P.hA.add_task(enc(q), enc(q));
      P.hA.close(enc(q));
      P.Z.add_task(enc(q), enc(lf.col[q]));
      P.Z.close(enc(q));
      P.Zc.add_task(enc(q), enc(lf.row[q]));
      P.Zc.close(enc(q));
    }
    auto arow_of = [&](int i) { return std::make_pair(lrow.begin(i), lrow.end(i)); };
    auto bcol_of = [&](int i) { return std::make_pair(lcol.begin(i), lcol.end(i)); };
    for (int i = 0; i < nleaf; ++i) {
      const auto ar = arow_of(i), bc = bcol_of(i);
      for (const int* x = ar.first; x != ar.second; ++x)
        if (lf.type[*x] == kF && hasK1[*x]) P.G1.add_task(enc(*x), enc(*x));
      P.G1.close(enc(i));
      for (const int* x = ar.first; x != ar.second; ++x)
        if (lf.type[*x] == kF) P.G2.add_task(enc(*x), enc(*x));
      P.G2.close(enc(i));
      P.G3.add_task(enc(i), enc(i));
      P.G3.close(enc(i));
      for (const int* x = bc.first; x != bc.second; ++x)
        if (lf.type[*x] == kF && hasI1[*x]) P.G1c.add_task(enc(*x), enc(*x));
      P.G1c.close(enc(i));
      for (const int* x = bc.first; x != bc.second; ++x)
        if (lf.type[*x] == kF) P.G2c.add_task(enc(*x), enc(*x));
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
    // triples of the leaf level by target class: dense targets (densified R
    // factors on selector 1), admissible targets, blue accumulators
    const int nt = nthreads(work[L]);
    struct Frag {
      TaskList dense, adm_R, adm_B;
      bool bad = false;
    };
    std::vector<Frag> fr(nt);
    parallel_rows(work[L], nt, [&](int th, int r0, int r1) {
      Frag& F = fr[th];
      const size_t nt_tri = (size_t)thread_tri[L][th];
      for (TaskList* t : {&F.dense, &F.adm_R, &F.adm_B}) reserve_more(*t, nt_tri, nt_tri);
      RowTriples rt(nleaf);
      ClusterMap node(nleaf), c1(nleaf >= 2 ? nleaf / 2 : 1);
      for (int i = r0; i < r1; ++i) {
        for (const int* pc = lrow.begin(i); pc != lrow.end(i); ++pc) node.put(lf.col[*pc], *pc);
        if (L >= 1) case1[L - 1].load_row(i >> 1, c1);
        rt.gather(lf, lrow, i);
        for (int k : rt.cols) {
          const int qc = node[k];
          const auto& ts = rt.bucket[k];
          if (qc >= 0 && lf.type[qc] == kF) {
            for (const auto& t : ts)
              F.dense.add_task(enc(t.qa, 0, 0, lf.type[t.qa] == kR),
                               enc(t.qb, 0, 0, lf.type[t.qb] == kR));
            F.dense.close(enc(qc));
          } else if (qc >= 0) {
            for (const auto& t : ts) F.adm_R.add_task(enc(t.qa), enc(t.qb));
            F.adm_R.close(enc(qc));
          } else if (L < 1 || c1[k >> 1] < 0) {
            F.bad = true;
          } else {
            for (const auto& t : ts) F.adm_B.add_task(enc(t.qa), enc(t.qb));
            F.adm_B.close(enc(c1[k >> 1], i & 1, k & 1));
          }
        }
        c1.clear();
        node.clear();
      }
    });
    {
      size_t td = 0, od = 0, tr = 0, orr = 0, tb = 0, ob = 0;
      for (const Frag& F : fr) {
        td += F.dense.a.size(), od += F.dense.out.size();
        tr += F.adm_R.a.size(), orr += F.adm_R.out.size();
        tb += F.adm_B.a.size(), ob += F.adm_B.out.size();
      }
      reserve_more(P.dense, td, od);
      reserve_more(P.adm_R, tr, orr);
      reserve_more(P.adm_B, tb, ob);
    }
    for (const Frag& F : fr) {
      if (F.bad) return "internal: blue target without a case-1 parent";
      append(P.dense, F.dense);
      append(P.adm_R, F.adm_R);
      append(P.adm_B, F.adm_B);
    }
    P.n_blue_tiles = L >= 1 ? (int)p.n_case1[L - 1] : 0;
  }

  // ============================================================ non-leaf
  for (int l = L - 1; l >= lmin; --l) {
    LevelPlan& Q = p.lev[l];
    const LevelNodes& ln = s.lev[l];
    const int ncl = 1 << l;
    Q.n_case1 = (int)p.n_case1[l];
    Q.n_blue_tiles = l >= 1 ? (int)p.n_case1[l - 1] : 0;
    const std::vector<uint64_t>& c1keys = case1[l].keys;
    std::vector<std::vector<int>> c1col(ncl);
    for (int t = 0; t < (int)c1keys.size(); ++t) c1col[key_col(c1keys[t])].push_back(t);
    for (int I = 0; I < ncl; ++I) {
      for (int t = case1[l].rp[I]; t < case1[l].rp[I + 1]; ++t) Q.G1.add_task(enc(t), enc(t));
      Q.G1.close(enc(I));
      for (int t : c1col[I]) Q.G1c.add_task(enc(t), enc(t));
      Q.G1c.close(enc(I));
      for (const int* x = rows[l].begin(I); x != rows[l].end(I); ++x)
        if (ln.type[*x] == kNL) Q.G2.add_task(enc(*x), enc(*x));
      Q.G2.close(enc(I));
      for (const int* x = cols[l].begin(I); x != cols[l].end(I); ++x)
        if (ln.type[*x] == kNL) Q.G2c.add_task(enc(*x), enc(*x));
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
    // position of the case-1 parent of (i,k) among the case-1 targets of
    // level l-1 (the tile of Acc_l that accumulates it)
    auto parent_tile = [&](int i, int k) -> int {
      const std::vector<uint64_t>& pk = case1[l - 1].keys;
      const uint64_t key = pkey(i >> 1, k >> 1);
      const auto it = std::lower_bound(pk.begin(), pk.end(), key);
      return (l >= 1 && it != pk.end() && *it == key) ? (int)(it - pk.begin()) : -1;
    };
    for (int t = 0; t < Q.n_case1; ++t) {
      const int I = key_row(c1keys[t]), K = key_col(c1keys[t]);
      Q.c1X.add_task(enc(I), enc(t));
      Q.c1X.close(enc(t));
      const int qc = ln.find(I, K);
      if (qc >= 0 && ln.type[qc] == kR) {
        Q.c1_R.add_task(enc(t), enc(K));
        Q.c1_R.close(enc(qc));
      } else if (qc < 0) {
        const int pt = parent_tile(I, K);
        if (pt < 0) return "internal: blue target without a case-1 parent";
        Q.c1_B.add_task(enc(t), enc(K));
        Q.c1_B.close(enc(pt, I & 1, K & 1));
      } else {
        return "internal: case-1 target is neither admissible nor blue";
      }
    }
    // triples of this level, re-associated by the A factor's type and routed
    // by target class (R, blue, NL).  NL x R: slot o of W_nl holds
    // sum_J Ahat_IJ S^B_JK and the second stage adds W_nl[o] P^B_K; R x NL:
    // W_r[o] = sum_J S^A_IJ Bhat_JK, then P^A_I W_r[o].  Per target the
    // merged second stage f_* lists both forms (selector 1 for P^A W_r)
    {
      struct Frag {
        TaskList wn[3], fn[3], wr[3], fr[3], fb[3];
        int slot_n[3] = {0, 0, 0}, slot_r[3] = {0, 0, 0};
        const char* err = nullptr;
      };
      const int nt = nthreads(work[l]);
      std::vector<Frag> fg(nt);
      parallel_rows(work[l], nt, [&](int th, int r0, int r1) {
        Frag& F = fg[th];
        const size_t nt_tri = (size_t)thread_tri[l][th];
        for (int c = 0; c < 3; ++c) {
          reserve_more(F.wn[c], nt_tri, nt_tri);
          reserve_more(F.wr[c], nt_tri, nt_tri);
        }
        RowTriples rt(ncl);
        ClusterMap node(ncl), c1(ncl >= 2 ? ncl / 2 : 1);
        for (int i = r0; i < r1 && !F.err; ++i) {
          for (const int* pc = rows[l].begin(i); pc != rows[l].end(i); ++pc)
            node.put(ln.col[*pc], *pc);
          if (l >= 1) case1[l - 1].load_row(i >> 1, c1);
          rt.gather(ln, rows[l], i);
          for (int k : rt.cols) {
            const int qc = node[k];
            int cls, outv;
            if (qc < 0) {
              if (l < 1 || c1[k >> 1] < 0) {
                F.err = "internal: blue target without a case-1 parent";
                break;
              }
              cls = 1;
              outv = enc(c1[k >> 1], i & 1, k & 1);
            } else if (ln.type[qc] == kR) {
              cls = 0;
              outv = enc(qc);
            } else if (ln.type[qc] == kNL) {
              cls = 2;
              outv = enc(qc);
            } else {
              F.err = "internal: dense target above the leaf level";
              break;
            }
            int on = -1, orr = -1;
            TaskList &wn = F.wn[cls], &wr = F.wr[cls];
            for (const auto& t : rt.bucket[k])
              if (ln.type[t.qa] == kNL) wn.add_task(ln.tile_loc[t.qa], enc(t.qb));
            if (wn.ntask() > wn.seg.back()) {
              on = F.slot_n[cls]++;
              wn.close(enc(on));
              F.fn[cls].add_task(enc(on), enc(k));
              F.fn[cls].close(outv);
            }
            for (const auto& t : rt.bucket[k])
              if (ln.type[t.qa] != kNL) wr.add_task(enc(t.qa), ln.tile_loc[t.qb]);
            if (wr.ntask() > wr.seg.back()) {
              orr = F.slot_r[cls]++;
              wr.close(enc(orr));
              F.fr[cls].add_task(enc(i), enc(orr));
              F.fr[cls].close(outv);
            }
            if (on >= 0) F.fb[cls].add_task(enc(on), enc(k));
            if (orr >= 0) F.fb[cls].add_task(enc(i, 0, 0, 1), enc(orr, 0, 0, 1));
            F.fb[cls].close(outv);
          }
          c1.clear();
          node.clear();
        }
      });
      TaskList* wn[3] = {&Q.w_nl_R, &Q.w_nl_B, &Q.w_nl_NL};
      TaskList* fn[3] = {&Q.f_nl_R, &Q.f_nl_B, &Q.f_nl_NL};
      TaskList* wr[3] = {&Q.w_r_R, &Q.w_r_B, &Q.w_r_NL};
      TaskList* fr[3] = {&Q.f_r_R, &Q.f_r_B, &Q.f_r_NL};
      TaskList* fb[3] = {&Q.f_R, &Q.f_B, &Q.f_NL};
      int base_n[3] = {0, 0, 0}, base_r[3] = {0, 0, 0};
      for (const Frag& F : fg) {
        if (F.err) return F.err;
        for (int c = 0; c < 3; ++c) {
          const int sn = enc(base_n[c]), sr = enc(base_r[c]);
          append(*wn[c], F.wn[c], sn);
          append(*fn[c], F.fn[c], 0, sn);
          append(*wr[c], F.wr[c], sr);
          append(*fr[c], F.fr[c], 0, 0, sr);
          append_merged(*fb[c], F.fb[c], sn, sr);
          base_n[c] += F.slot_n[c];
          base_r[c] += F.slot_r[c];
        }
      }
    }

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
