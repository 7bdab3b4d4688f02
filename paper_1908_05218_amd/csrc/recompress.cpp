// Recompression of an H^2 matrix: new orthonormal nested bases of the
// smallest ranks that keep every cluster's whole far field (its admissible
// blocks and those of its ancestors, restricted to its rows) to a relative
// accuracy, and the couplings projected onto them; partition and dense
// blocks unchanged.  The paper builds its inputs with a construction it cites
// without describing (Section VI); this is a standard algebraic compression,
// level by level on the device with the product's batched GEMM and
// eigensolver:
//  1. basis Grams bottom-up, B_t = X_t^T X_t^* through the transfers;
//  2. far-field weights top-down, K_t = sum_(t,s) S_ts B^other_s S_ts^H +
//     E_t K_parent E_t^H (the far field's Gram is X_t K_t X_t^H);
//  3. bottom-up truncation: at the leaves the dominant eigenvectors of
//     V_t K_t V_t^H; above them of Z_t K_t Z_t^H with Z_t = [P_t1 E_t1;
//     P_t2 E_t2] the old basis in the children's new ones; P_t = U_t^H Z_t;
//  4. couplings S'_ts = P^row_t S_ts (P^col_s)^T.
// The column side is the row side of the transpose.  Truncation: eigenvalues
// above (theta eps / n_t)^2 lambda_1 (the product's ACCURACY rule), at most
// the old rank.  FP64 (complex128 through the planes) throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace h2 {

namespace {

inline long long cidx(int l, int c) { return (1LL << l) - 1 + c; }

// task lists uploaded to one device buffer; the host copy is kept until the
// stream has passed the upload
struct Lists {
  Buf mem;
  std::vector<int> host;
  std::vector<DevList> d;
};

void upload(h2_ctx ctx, const std::vector<TaskList>& ls, Lists& out, hipStream_t st) {
  size_t total = 0;
  for (const TaskList& t : ls) total += t.out.size() + t.seg.size() + t.a.size() + t.b.size();
  out.host.assign(total + 1, 0);
  out.mem = Buf(ctx, (total + 1) * sizeof(int));
  int* base = out.mem.as<int>();
  size_t off = 0;
  for (const TaskList& t : ls) {
    DevList d;
    d.nout = t.nout();
    d.ntask = t.ntask();
    auto put = [&](const std::vector<int>& v) -> const int* {
      std::copy(v.begin(), v.end(), out.host.begin() + off);
      const int* r = base + off;
      off += v.size();
      return r;
    };
    d.out = put(t.out);
    d.seg = put(t.seg);
    d.a = put(t.a);
    d.b = put(t.b);
    scan_limits(t, d);
    out.d.push_back(d);
  }
  H2_HIP(hipMemcpyAsync(base, out.host.data(), total * sizeof(int), hipMemcpyHostToDevice, st));
}

// the per-level task lists of the recompression (indices into Lists::d)
struct LevelLists {
  int id = -1;      // out c: (c, c)
  int up = -1;      // out child c: (c, half of parent's stacked transfer)
  int sum = -1;     // out parent p: (half a of p's stacked transfer, child 2p+a), a = 0, 1
  int down1 = -1;   // out t: (half of parent's stacked transfer, parent)
  int down2 = -1;   // out t: (t, half of parent's stacked transfer)
  int admT_r = -1;  // out node q: (q, col q)
  int admK_r = -1;  // out row t: (q, q) over its admissible nodes
  int admT_c = -1;  // out node q: (q, row q)
  int admK_c = -1;  // out col s: (q, q) over its admissible nodes
  int zst = -1;     // out (parent, half a): (child 2p+a, (parent, half a))
  int S1 = -1;      // out node q: (row q, q)
  int S2 = -1;      // out node q: (q, col q)
};

}  // namespace

h2_mat recompress_impl(h2_ctx ctx, h2_mat M, double eps) {
  ActiveCtx active(ctx);
  hipStream_t st = ctx->stream;
  const Structure& s = M->st();
  const int L = s.L, lmin = s.lmin, np = s.npad, nleaf = 1 << L;
  const long long nn2 = (long long)np * np;
  const bool cplx = M->cplx;
  const size_t eb = cplx ? 2 * sizeof(double) : sizeof(double);
  const int n_trunc = std::max(1, L - lmin + 1);
  const double sv = kTheta * eps / n_trunc;
  Profiler prof;  // off: the recompression is not timed per kernel class
  Buf status(ctx, 4 * sizeof(int));
  H2_HIP(hipMemsetAsync(status.as<int>(), 0, 4 * sizeof(int), st));
  const EigLevel eg{ctx, st, &prof, status.as<int>(), cplx, sv * sv, false,
                    ctx->readback(2 * (size_t)nleaf + 4), ctx->rb_ev};
  const std::vector<int>&rr = M->rr, &rc = M->rc;

  // ---------------------------------------------------------- task lists
  std::vector<TaskList> tl;
  std::vector<LevelLists> ix(L + 1);
  auto add = [&](TaskList&& t) {
    tl.push_back(std::move(t));
    return (int)tl.size() - 1;
  };
  for (int l = lmin; l <= L; ++l) {
    const int ncl = 1 << l;
    const LevelNodes& ln = s.lev[l];
    LevelLists& x = ix[l];
    {
      TaskList t;
      for (int c = 0; c < ncl; ++c) {
        t.add_task(enc(c), enc(c));
        t.close(enc(c));
      }
      x.id = add(std::move(t));
    }
    if (l < L) {
      TaskList up, sum, zst;
      for (int c = 0; c < 2 * ncl; ++c) {
        up.add_task(enc(c), enc(c >> 1, c & 1));
        up.close(enc(c));
        zst.add_task(enc(c), enc(c >> 1, c & 1));
        zst.close(enc(c >> 1, c & 1));
      }
      for (int p = 0; p < ncl; ++p) {
        for (int a = 0; a < 2; ++a) sum.add_task(enc(p, a), enc(2 * p + a));
        sum.close(enc(p));
      }
      x.up = add(std::move(up));
      x.sum = add(std::move(sum));
      x.zst = add(std::move(zst));
    }
    if (l > lmin) {
      TaskList d1, d2;
      for (int t = 0; t < ncl; ++t) {
        d1.add_task(enc(t >> 1, t & 1), enc(t >> 1));
        d1.close(enc(t));
        d2.add_task(enc(t), enc(t >> 1, t & 1));
        d2.close(enc(t));
      }
      x.down1 = add(std::move(d1));
      x.down2 = add(std::move(d2));
    }
    TaskList tr, kr, tc, kc, s1, s2;
    std::vector<std::vector<int>> byrow(ncl), bycol(ncl);
    for (int q = 0; q < ln.size(); ++q) {
      if (ln.type[q] != kR) continue;
      byrow[ln.row[q]].push_back(q);
      bycol[ln.col[q]].push_back(q);
      tr.add_task(enc(q), enc(ln.col[q]));
      tr.close(enc(q));
      tc.add_task(enc(q), enc(ln.row[q]));
      tc.close(enc(q));
      s1.add_task(enc(ln.row[q]), enc(q));
      s1.close(enc(q));
      s2.add_task(enc(q), enc(ln.col[q]));
      s2.close(enc(q));
    }
    for (int c = 0; c < ncl; ++c) {
      if (!byrow[c].empty()) {
        for (int q : byrow[c]) kr.add_task(enc(q), enc(q));
        kr.close(enc(c));
      }
      if (!bycol[c].empty()) {
        for (int q : bycol[c]) kc.add_task(enc(q), enc(q));
        kc.close(enc(c));
      }
    }
    x.admT_r = add(std::move(tr));
    x.admK_r = add(std::move(kr));
    x.admT_c = add(std::move(tc));
    x.admK_c = add(std::move(kc));
    x.S1 = add(std::move(s1));
    x.S2 = add(std::move(s2));
  }
  Lists lists;
  upload(ctx, tl, lists, st);
  auto dl = [&](int i) -> const DevList& { return lists.d[i]; };

  // old ranks (the cap of the new ones) and leaf sizes
  const long long ncl_all = (2LL << L) - 1;
  std::vector<int> hk(2 * ncl_all + nleaf);
  for (long long i = 0; i < ncl_all; ++i) {
    hk[i] = (int)M->krow[i];
    hk[ncl_all + i] = (int)M->kcol[i];
  }
  for (int c = 0; c < nleaf; ++c) hk[2 * ncl_all + c] = s.leaf_size[c];
  Buf dk(ctx, hk.size() * sizeof(int));
  H2_HIP(hipMemcpyAsync(dk.as<int>(), hk.data(), hk.size() * sizeof(int), hipMemcpyHostToDevice, st));
  const int* kmax_r = dk.as<int>();
  const int* kmax_c = dk.as<int>() + ncl_all;
  const int* leaf_sizes = dk.as<int>() + 2 * ncl_all;

  // ---------------------------------------------- 1. basis Grams, bottom-up
  std::vector<Buf> BV(L + 1), BW(L + 1);
  for (int side = 0; side < 2; ++side) {
    std::vector<Buf>& B = side ? BW : BV;
    const std::vector<int>& k = side ? rc : rr;
    const Buf& X = side ? M->W : M->V;
    const long long xs = side ? M->W_stride : M->V_stride;
    const std::vector<Buf>& T = side ? M->Tc : M->Tr;
    const std::vector<long long>& ts = side ? M->Tc_stride : M->Tr_stride;
    B[L] = Buf(ctx, (size_t)nleaf * k[L] * k[L] * eb, false, cplx);
    gemm(st, nullptr, kKindOther, dl(ix[L].id), k[L], k[L], np, Op{X.p(), nullptr, xs, 0, np}, true,
         Op{X.p(), nullptr, xs, 0, np}, false, B[L].p(), (long long)k[L] * k[L], k[L], 0, 0, 1, 0,
         kConjB);
    for (int l = L - 1; l >= lmin; --l) {
      const int kc = k[l + 1], kp = k[l];
      const Op E{T[l].p(), nullptr, ts[l], 0, 2 * kc, kc, 0};
      Buf Y(ctx, (size_t)(2 << l) * kc * kp * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[l].up), kc, kp, kc,
           Op{B[l + 1].p(), nullptr, (long long)kc * kc, 0, kc}, false, E, false, Y.p(),
           (long long)kc * kp, kc, 0, 0, 1, 0, kConjB);
      B[l] = Buf(ctx, (size_t)(1 << l) * kp * kp * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[l].sum), kp, kp, kc, E, true,
           Op{Y.p(), nullptr, (long long)kc * kp, 0, kc}, false, B[l].p(), (long long)kp * kp, kp,
           0, 0, 1, 0);
    }
  }

  // ------------------------------------------- 2. far-field weights, top-down
  std::vector<Buf> KR(L + 1), KC(L + 1);
  for (int l = lmin; l <= L; ++l) {
    const int ncl = 1 << l, nn = s.lev[l].size();
    const LevelLists& x = ix[l];
    for (int side = 0; side < 2; ++side) {
      std::vector<Buf>& K = side ? KC : KR;
      const std::vector<int>& k = side ? rc : rr;
      const std::vector<Buf>& T = side ? M->Tc : M->Tr;
      const std::vector<long long>& ts = side ? M->Tc_stride : M->Tr_stride;
      K[l] = Buf(ctx, (size_t)ncl * k[l] * k[l] * eb, false, cplx);
      zero(st, K[l].p(), (long long)ncl * k[l] * k[l]);
      if (l > lmin) {
        const int kt = k[l], kp = k[l - 1];
        const Op E{T[l - 1].p(), nullptr, ts[l - 1], 0, 2 * kt, kt, 0};
        Buf Z(ctx, (size_t)ncl * kt * kp * eb, false, cplx);
        gemm(st, nullptr, kKindOther, dl(x.down1), kt, kp, kp, E, false,
             Op{K[l - 1].p(), nullptr, (long long)kp * kp, 0, kp}, false, Z.p(), (long long)kt * kp,
             kt, 0, 0, 1, 0);
        gemm(st, nullptr, kKindOther, dl(x.down2), kt, kt, kp,
             Op{Z.p(), nullptr, (long long)kt * kp, 0, kt}, false, E, true, K[l].p(),
             (long long)kt * kt, kt, 0, 0, 1, 1, kConjB);
      }
    }
    if (dl(x.admT_r).nout == 0) continue;
    const int a = rr[l], b = rc[l];
    const Op So{M->S[l].p(), nullptr, (long long)a * b, 0, a};
    // row side: K_t += (S_q B^W_s) S_q^H
    {
      Buf T1(ctx, (size_t)nn * a * b * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(x.admT_r), a, b, b, So, false,
           Op{BW[l].p(), nullptr, (long long)b * b, 0, b}, false, T1.p(), (long long)a * b, a, 0, 0,
           1, 0);
      gemm(st, nullptr, kKindOther, dl(x.admK_r), a, a, b, Op{T1.p(), nullptr, (long long)a * b, 0, a},
           false, So, true, KR[l].p(), (long long)a * a, a, 0, 0, 1, 1, kConjB);
    }
    // column side: K^c_s += (S_q^T B^V_t) S_q^*
    {
      Buf T1(ctx, (size_t)nn * a * b * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(x.admT_c), b, a, a, So, true,
           Op{BV[l].p(), nullptr, (long long)a * a, 0, a}, false, T1.p(), (long long)b * a, b, 0, 0,
           1, 0);
      gemm(st, nullptr, kKindOther, dl(x.admK_c), b, b, a, Op{T1.p(), nullptr, (long long)b * a, 0, b},
           false, So, false, KC[l].p(), (long long)b * b, b, 0, 0, 1, 1, kConjB);
    }
  }
  for (Buf& b : BV) b.reset();
  for (Buf& b : BW) b.reset();

  // --------------------------------------------- 3. truncation, bottom-up
  auto X = std::make_unique<h2_mat_s>();
  X->ctx = ctx;
  X->shape = M->shape;
  X->product = true;
  X->cplx = cplx;
  X->rr.assign(L + 1, 16);
  X->rc.assign(L + 1, 16);
  X->krow.assign(ncl_all, 0);
  X->kcol.assign(ncl_all, 0);
  X->Tr.resize(L);
  X->Tc.resize(L);
  X->Tr_stride.assign(L, 0);
  X->Tc_stride.assign(L, 0);
  X->S.resize(L + 1);
  std::vector<int> cpad(L + 1, 16);
  std::vector<Buf> Ur(L + 1), Uc(L + 1), rank_r(L + 1), rank_c(L + 1), PR(L + 1), PC(L + 1);
  auto read_ranks = [&](int l) {
    const int ncl = 1 << l;
    const int* h = wait_ranks(eg, l);
    int mx = 1;
    for (int c = 0; c < ncl; ++c) {
      X->krow[cidx(l, c)] = h[c];
      X->kcol[cidx(l, c)] = h[ncl + c];
      mx = std::max(mx, std::max(h[c], h[ncl + c]));
    }
    return pad16(mx);
  };
  // leaves: Gram V_t K_t V_t^H (np x np)
  {
    Buf G[2][3];
    for (int side = 0; side < 2; ++side) {
      const int k = side ? rc[L] : rr[L];
      const Buf& Xb = side ? M->W : M->V;
      const Op Xo{Xb.p(), nullptr, side ? M->W_stride : M->V_stride, 0, np};
      Buf Y(ctx, (size_t)nleaf * np * k * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[L].id), np, k, k, Xo, false,
           Op{(side ? KC : KR)[L].p(), nullptr, (long long)k * k, 0, k}, false, Y.p(),
           (long long)np * k, np, 0, 0, 1, 0);
      G[side][0] = Buf(ctx, (size_t)nleaf * nn2 * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[L].id), np, np, k, Op{Y.p(), nullptr, (long long)np * k, 0, np},
           false, Xo, true, G[side][0].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
    }
    eig_level(eg, L, np, G[0], G[1], Ur[L], Uc[L], rank_r[L], rank_c[L], leaf_sizes, nullptr,
              leaf_sizes, nullptr, 1, np, kmax_r + cidx(L, 0), kmax_c + cidx(L, 0));
  }
  cpad[L] = read_ranks(L);
  for (int side = 0; side < 2; ++side) {
    const int k = side ? rc[L] : rr[L], c = cpad[L];
    const Buf& Xb = side ? M->W : M->V;
    Buf& P = side ? PC[L] : PR[L];
    P = Buf(ctx, (size_t)nleaf * c * k * eb, false, cplx);
    gemm(st, nullptr, kKindOther, dl(ix[L].id), c, k, np, Op{(side ? Uc : Ur)[L].p(), nullptr, nn2, 0, np},
         true, Op{Xb.p(), nullptr, side ? M->W_stride : M->V_stride, 0, np}, false, P.p(),
         (long long)c * k, c, 0, 0, 1, 0, kConjA);
  }
  KR[L].reset();
  KC[L].reset();
  // above the leaves: Gram Z_t K_t Z_t^H (D x D, D = 2 cpad[l+1])
  for (int l = L - 1; l >= lmin; --l) {
    const int ncl = 1 << l, cc = cpad[l + 1], D = 2 * cc;
    Buf G[2][3], Z[2];
    for (int side = 0; side < 2; ++side) {
      const std::vector<int>& k = side ? rc : rr;
      const std::vector<Buf>& T = side ? M->Tc : M->Tr;
      const std::vector<long long>& ts = side ? M->Tc_stride : M->Tr_stride;
      const int kc = k[l + 1], kp = k[l];
      Z[side] = Buf(ctx, (size_t)ncl * D * kp * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[l].zst), cc, kp, kc,
           Op{(side ? PC : PR)[l + 1].p(), nullptr, (long long)cc * kc, 0, cc}, false,
           Op{T[l].p(), nullptr, ts[l], 0, 2 * kc, kc, 0}, false, Z[side].p(), (long long)D * kp, D,
           cc, 0, 1, 0);
      Buf Y(ctx, (size_t)ncl * D * kp * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[l].id), D, kp, kp, Op{Z[side].p(), nullptr, (long long)D * kp, 0, D},
           false, Op{(side ? KC : KR)[l].p(), nullptr, (long long)kp * kp, 0, kp}, false, Y.p(),
           (long long)D * kp, D, 0, 0, 1, 0);
      G[side][0] = Buf(ctx, (size_t)ncl * D * D * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[l].id), D, D, kp, Op{Y.p(), nullptr, (long long)D * kp, 0, D},
           false, Op{Z[side].p(), nullptr, (long long)D * kp, 0, D}, true, G[side][0].p(),
           (long long)D * D, D, 0, 0, 1, 0, kConjB | kLowerOnly);
    }
    eig_level(eg, l, D, G[0], G[1], Ur[l], Uc[l], rank_r[l], rank_c[l], rank_r[l + 1].as<int>(),
              rank_r[l + 1].as<int>() + 1, rank_c[l + 1].as<int>(), rank_c[l + 1].as<int>() + 1, 2,
              cc, kmax_r + cidx(l, 0), kmax_c + cidx(l, 0));
    cpad[l] = read_ranks(l);
    for (int side = 0; side < 2; ++side) {
      const int kp = side ? rc[l] : rr[l], c = cpad[l];
      Buf& P = side ? PC[l] : PR[l];
      P = Buf(ctx, (size_t)ncl * c * kp * eb, false, cplx);
      gemm(st, nullptr, kKindOther, dl(ix[l].id), c, kp, D,
           Op{(side ? Uc : Ur)[l].p(), nullptr, (long long)D * D, 0, D}, true,
           Op{Z[side].p(), nullptr, (long long)D * kp, 0, D}, false, P.p(), (long long)c * kp, c, 0,
           0, 1, 0, kConjA);
    }
    KR[l].reset();
    KC[l].reset();
  }

  // ---------------------------------------------- 4. projected couplings
  for (int l = lmin; l <= L; ++l) {
    const int nn = s.lev[l].size(), c = cpad[l], a = rr[l], b = rc[l];
    X->S[l] = Buf(ctx, (size_t)nn * c * c * eb, false, cplx);
    zero(st, X->S[l].p(), (long long)nn * c * c);
    if (dl(ix[l].S1).nout == 0) continue;
    Buf Y(ctx, (size_t)nn * c * b * eb, false, cplx);
    gemm(st, nullptr, kKindOther, dl(ix[l].S1), c, b, a, Op{PR[l].p(), nullptr, (long long)c * a, 0, c},
         false, Op{M->S[l].p(), nullptr, (long long)a * b, 0, a}, false, Y.p(), (long long)c * b, c, 0,
         0, 1, 0);
    gemm(st, nullptr, kKindOther, dl(ix[l].S2), c, c, b, Op{Y.p(), nullptr, (long long)c * b, 0, c},
         false, Op{PC[l].p(), nullptr, (long long)c * b, 0, c}, true, X->S[l].p(), (long long)c * c, c,
         0, 0, 1, 0);
  }

  // ---------------------------------------------------------- assemble
  for (int l = lmin; l <= L; ++l) {
    X->rr[l] = cpad[l];
    X->rc[l] = cpad[l];
  }
  X->V = std::move(Ur[L]);
  X->W = std::move(Uc[L]);
  X->V_stride = nn2;
  X->W_stride = nn2;
  for (int l = lmin; l < L; ++l) {
    X->Tr[l] = std::move(Ur[l]);
    X->Tc[l] = std::move(Uc[l]);
    X->Tr_stride[l] = 4LL * cpad[l + 1] * cpad[l + 1];
    X->Tc_stride[l] = X->Tr_stride[l];
  }
  if (M->F.bytes()) {
    X->F = Buf(ctx, M->F.bytes(), false, cplx);
    H2_HIP(hipMemcpyAsync(X->F.p(), M->F.p(), M->F.bytes(), hipMemcpyDeviceToDevice, st));
  }
  h2_stats_t& S = X->stats;
  S.L = L;
  S.lmin = lmin;
  for (int l = 0; l <= L && l < H2_MAX_LEVELS; ++l) {
    long long mr = 0, mc = 0;
    double sr = 0, sc = 0;
    for (int c2 = 0; c2 < (1 << l); ++c2) {
      mr = std::max<long long>(mr, X->krow[cidx(l, c2)]);
      mc = std::max<long long>(mc, X->kcol[cidx(l, c2)]);
      sr += X->krow[cidx(l, c2)];
      sc += X->kcol[cidx(l, c2)];
    }
    S.rank_max_r[l] = mr;
    S.rank_max_c[l] = mc;
    S.rank_mean_r[l] = sr / (1 << l);
    S.rank_mean_c[l] = sc / (1 << l);
  }
  S.sparsity_constant = s.sparsity_constant();
  S.bytes_device = (int64_t)ctx->peak_live;
  build_matvec_plan(ctx, X.get());
  H2_HIP(hipStreamSynchronize(st));
  return X.release();
}

}  // namespace h2

extern "C" {

h2_status h2_recompress(h2_ctx ctx, h2_mat M, double eps, h2_mat* out) {
  using namespace h2;
  if (!ctx || !M || !out) return set_error(H2_ERR_ARG, "null argument");
  if (!(eps >= H2_RECOMPRESS_EPS_MIN) || !std::isfinite(eps))
    return set_error(H2_ERR_ARG, "eps must be finite and >= 1e-8");
  ctx = home_of(ctx, M);
  if (!ctx) return set_error(H2_ERR_ARG, "M belongs to another context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  const size_t start = ctx->live_bytes;
  ctx->mark();
  h2_status r = H2_OK;
  try {
    hipSetDevice(ctx->device);
    M->finish();
    *out = recompress_impl(ctx, M, eps);
  } catch (const Error& e) {
    (void)hipGetLastError();
    r = set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    r = set_error(H2_ERR_INTERNAL, e.what());
  }
  // keep in the pool at most twice the call's peak temporaries
  ctx->end_call(start);
  return r;
}

}  // extern "C"
