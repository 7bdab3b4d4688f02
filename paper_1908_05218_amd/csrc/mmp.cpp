// Level scheduler of the H^2 matrix-matrix product C = A B (Ma & Jiao,
// Sections III and IV).  Every step is a batch of uniform small products over
// the task lists of the symbolic phase; ranks of C are data-dependent, so
// after each level's eigen-decompositions the kept ranks are read back and the
// next launches use the level's padded rank.
//
// Data layout (all column-major, FP64):
//  * per-cluster blocks: flat by cluster index, fixed stride;
//  * stacked transfers T_I = [E_I1; E_I2] per parent cluster;
//  * per-node blocks: flat by node index within the level, except the
//    collected blocks A^_l, B^_l (equations Fcollect / NLcollect) and the
//    temporary couplings of blue targets, which are stored 2x2-grouped by the
//    parent so the next level reads them as one (NL)_coll block in place.
//
// The leaf-level admissible-target products use the leaf-coordinate form
//   S_ik += (V^C_i^T A_ij)(B_jk W^C_k)
// with V^C_i^T A_ij equal to V^C_i^T F_ij (dense) or P^A_i S^A_ij W^A_j^T
// (admissible) and B_jk W^C_k equal to F_jk W^C_k or V^B_j S^B_jk P^B_k: an
// exact rewriting of the four cases of equation leafcoup_simple that gives
// every leaf triple the same shape (one batched launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <unordered_map>
#include <unordered_set>

#include "internal.h"

namespace h2 {

namespace {

inline long long cidx(int l, int c) { return (1LL << l) - 1 + c; }

struct Dims {
  int m, n, k;
};


}  // namespace

// Algorithmic work of a product at the actual ranks (unpadded), in four parts
// (Sections III-IV; run on the first h2_stats call for a product, not inside
// it):
//  triple: one contraction per evaluated block product (A node (I,J), B node
//    (J,K) of one level): 2 n_i n_j n_k for a dense target; at the leaves
//    2 kC_i n_j kC_k for dense x dense, 2 kC_i kB_j kB_k (Ahat S^B),
//    2 kA_i kA_j kC_k (S^A Bhat) and 2 kA_i kB_j kB_k ((S^A Pi) S^B) for the
//    other pairs (equation leafcoup_simple); above the leaves the
//    re-associated single contraction 2 kC_I kB_J kB_K for NL x R and
//    2 kA_I kA_J kC_K otherwise (equation nonleafcoup_simple);
//  target: per target the products that apply the projections once
//    (X2 P^B, P^A X3, P^A X4 P^B at the leaves; W P^B, P^A W and
//    T^C_I^H M_IK T^C_K above them);
//  gram: 2 d^2 per contributed column of each row and column Gram sum
//    (equations Gr1L-case3-ch and case1-ch-nl-case3-ch-nl);
//  eig: 9 d^3 per Gram matrix.
FlopCounts flop_counts(const Structure& s, const FlopRanks& r) {
  FlopCounts f;
  const int L = s.L, lmin = s.lmin;
  auto n_ = [&](int c) { return (double)s.leaf_size[c]; };
  auto at = [](const std::vector<int64_t>& v, int l, int c) { return (double)v[cidx(l, c)]; };
  auto key = [](int i, int k) { return ((uint64_t)(uint32_t)i << 32) | (uint32_t)k; };
  std::unordered_set<uint64_t> acc;  // blue accumulators of the level below
  for (int l = L; l >= lmin; --l) {
    const LevelNodes& ln = s.lev[l];
    const int ncl = 1 << l;
    std::vector<std::vector<int>> byrow(ncl);
    for (int q = 0; q < ln.size(); ++q) byrow[ln.row[q]].push_back(q);
    std::vector<double> rcols(ncl, 0.0), ccols(ncl, 0.0), dr(ncl), dc(ncl);
    for (int c = 0; c < ncl; ++c) {
      dr[c] = l == L ? n_(c) : at(r.cr, l + 1, 2 * c) + at(r.cr, l + 1, 2 * c + 1);
      dc[c] = l == L ? n_(c) : at(r.cc, l + 1, 2 * c) + at(r.cc, l + 1, 2 * c + 1);
      rcols[c] = at(r.ar, l, c);  // the old bases (Gr3L / case3-ch-nl)
      ccols[c] = at(r.bc, l, c);
    }
    // merged targets of this level: parents of the blue accumulators below
    std::unordered_set<uint64_t> case1;
    if (l < L)
      for (uint64_t v : acc) case1.insert(key((int)(v >> 32) >> 1, (int)(uint32_t)v >> 1));
    std::unordered_set<uint64_t> next;
    // per target: bit 0 NL x R (or dense x admissible at the leaves),
    // bit 1 admissible x dense, bit 2 admissible x admissible
    std::unordered_map<uint64_t, int> tgt;
    for (int qa = 0; qa < ln.size(); ++qa) {
      const int i = ln.row[qa], j = ln.col[qa], ta = ln.type[qa];
      if (ta == kF) rcols[i] += at(r.br, l, j);  // F^A_ij V^B_j (Gr2L)
      if (ta == kNL) rcols[i] += at(r.br, l, j);  // Acoll_IJ T^B_J (case2-ch-nl)
      if (ta == kF || ta == kNL) ccols[j] += at(r.ac, l, i);  // mirror on B's node (i, j)
      for (int qb : byrow[j]) {
        const int tb = ln.type[qb];
        if (ta == kNL && tb == kNL) continue;
        const int k = ln.col[qb];
        const int qc = ln.find(i, k);
        const int tg = qc < 0 ? kBlue : ln.type[qc];
        if (tg == kF) {
          f.triple += 2.0 * n_(i) * n_(j) * n_(k);
          continue;
        }
        if (tg == kBlue) next.insert(key(i, k));
        int bit = 0;
        if (l == L) {
          if (ta == kF && tb == kF) {
            f.triple += 2.0 * at(r.cr, l, i) * n_(j) * at(r.cc, l, k);
            rcols[i] += n_(k);  // F^A_ij F^B_jk (Gr1L)
            ccols[k] += n_(i);
          } else if (ta == kF) {
            f.triple += 2.0 * at(r.cr, l, i) * at(r.br, l, j) * at(r.bc, l, k);
            bit = 1;
          } else if (tb == kF) {
            f.triple += 2.0 * at(r.ar, l, i) * at(r.ac, l, j) * at(r.cc, l, k);
            bit = 2;
          } else {
            f.triple += 2.0 * at(r.ar, l, i) * at(r.br, l, j) * at(r.bc, l, k);
            bit = 4;
          }
        } else if (ta == kNL) {
          f.triple += 2.0 * at(r.cr, l, i) * at(r.br, l, j) * at(r.bc, l, k);
          bit = 1;
        } else {
          f.triple += 2.0 * at(r.ar, l, i) * at(r.ac, l, j) * at(r.cc, l, k);
          bit = 2;
        }
        if (bit) tgt[key(i, k)] |= bit;
      }
    }
    for (const auto& kv : tgt) {
      const int i = (int)(kv.first >> 32), k = (int)(uint32_t)kv.first;
      const double ci = at(r.cr, l, i), ck = at(r.cc, l, k), ai = at(r.ar, l, i),
                   bk = at(r.bc, l, k);
      if (kv.second & 1) f.target += 2.0 * ci * bk * ck;           // X2 P^B / W_nl P^B
      if (kv.second & 4) f.target += 2.0 * ai * bk * ck;           // X4 P^B
      if (kv.second & 6) f.target += 2.0 * ci * ai * ck;           // P^A (X3 + X4 P^B) / P^A W_r
    }
    for (uint64_t v : case1) {
      const int i = (int)(v >> 32), k = (int)(uint32_t)v;
      f.target += 2.0 * at(r.cr, l, i) * dr[i] * dc[k] + 2.0 * at(r.cr, l, i) * dc[k] * at(r.cc, l, k);
      rcols[i] += dc[k];  // M_IK (case1-ch-nl)
      ccols[k] += dr[i];
      if (ln.find(i, k) < 0) next.insert(v);  // a blue merged target moves up
    }
    for (int c = 0; c < ncl; ++c) {
      f.gram += 2.0 * dr[c] * dr[c] * rcols[c] + 2.0 * dc[c] * dc[c] * ccols[c];
      f.eig += 9.0 * (dr[c] * dr[c] * dr[c] + dc[c] * dc[c] * dc[c]);
      f.eig_tri += (4.0 / 3.0) * (dr[c] * dr[c] * dr[c] + dc[c] * dc[c] * dc[c]);
      f.eig_vec += 6.0 * (dr[c] * dr[c] * at(r.cr, l, c) + dc[c] * dc[c] * at(r.cc, l, c));
    }
    acc.swap(next);
  }
  return f;
}

// the level's ranks and flags to pinned host memory, then the event
static void post_ranks(const EigLevel& e, int ncl, const int* rr, const int* rc) {
  H2_HIP(hipMemcpyAsync(e.host, rr, ncl * sizeof(int), hipMemcpyDeviceToHost, e.st));
  H2_HIP(hipMemcpyAsync(e.host + ncl, rc, ncl * sizeof(int), hipMemcpyDeviceToHost, e.st));
  H2_HIP(hipMemcpyAsync(e.host + 2 * ncl, e.status, 4 * sizeof(int), hipMemcpyDeviceToHost, e.st));
  H2_HIP(hipEventRecord(e.ready, e.st));
}

const int* wait_ranks(const EigLevel& e, int l) {
  H2_HIP(hipEventSynchronize(e.ready));
  const int* stv = e.host + 2 * (1 << l);
  if (stv[0]) throw Error(H2_ERR_NUMERIC, "non-finite Gram matrix at level " + std::to_string(l));
  if (stv[1])
    throw Error(H2_ERR_UNSUPPORTED, "a Gram matrix at level " + std::to_string(l) +
                                        " exceeds the eigensolver limit of " +
                                        std::to_string(h2k::kEigNmax));
  return e.host;
}

// the three eigensolver phases, each timed as its own kernel class; with
// rank arrays given, their read-back is posted between the eigenvalue phase
// (which fixes the ranks) and the eigenvector phase, so the host sizes and
// enqueues the next launches while the eigenvectors are computed
static void run_eig(const EigLevel& e, const h2k::EigArgs* ea, int ncl, const int* rr = nullptr,
                    const int* rc = nullptr) {
  const int phase[3] = {h2k::kEigPhaseTri, h2k::kEigPhaseVal, h2k::kEigPhaseVec};
  const int kind[3] = {kKindEig, kKindEigVal, kKindEigVec};
  for (int ph = 0; ph < 3; ++ph) {
    if (ph == 2 && rr) post_ranks(e, ncl, rr, rc);
    hipEvent_t ev = nullptr;
    e.prof->begin(kind[ph], 0, &ev);
    H2_HIP(h2k::launch_eig(ea[0], ea[1], ncl, e.st, phase[ph]));
    e.prof->end(ev, kind[ph], 0);
  }
}

void eig_level(const EigLevel& e, int l, int D, const Buf* Gr, const Buf* Gc, Buf& Ur_, Buf& Uc_,
               Buf& rank_r_, Buf& rank_c_, const int* k1r, const int* k2r, const int* k1c,
               const int* k2c, int kstride, int half, const int* kmax_r, const int* kmax_c) {
  h2_ctx ctx = e.ctx;
  hipStream_t st = e.st;
  const bool cplx = e.cplx;
  const size_t gb = cplx ? 2 * sizeof(double) : sizeof(double);
  const int ncl = 1 << l;
  if ((cplx ? 2 * D : D) > h2k::kEigNmax)
    throw Error(H2_ERR_UNSUPPORTED, "the Gram matrices at level " + std::to_string(l) +
                                        " have dimension " + std::to_string(D) +
                                        (cplx ? " (complex)" : "") +
                                        ", beyond the eigensolver limit of " +
                                        std::to_string(cplx ? h2k::kEigNmax / 2 : h2k::kEigNmax));
  if (cplx) {
    // Hermitian Grams through their real embedding (dimension 2D)
    const int D2 = 2 * D;
    Buf E[2] = {Buf(ctx, (size_t)ncl * D2 * D2 * sizeof(double)),
                Buf(ctx, (size_t)ncl * D2 * D2 * sizeof(double))};
    Buf Ue[2] = {Buf(ctx, (size_t)ncl * D2 * D2 * sizeof(double)),
                 Buf(ctx, (size_t)ncl * D2 * D2 * sizeof(double))};
    Buf nlive(ctx, (size_t)2 * ncl * sizeof(int)), rank_e(ctx, (size_t)2 * ncl * sizeof(int));
    Ur_ = Buf(ctx, (size_t)ncl * D * D * gb, false, true);
    Uc_ = Buf(ctx, (size_t)ncl * D * D * gb, false, true);
    rank_r_ = Buf(ctx, (size_t)ncl * sizeof(int));
    rank_c_ = Buf(ctx, (size_t)ncl * sizeof(int));
    h2k::CEigArgs ca[2];
    for (int side = 0; side < 2; ++side) {
      h2k::CEigArgs& a = ca[side];
      a = h2k::CEigArgs{};
      for (int c = 0; c < 3; ++c) a.G[c] = (side ? Gc : Gr)[c].d();
      a.gplane = ctx->plane((side ? Gc : Gr)[0].p());
      a.D = D;
      a.half = half;
      a.k1 = side ? k1c : k1r;
      a.k2 = side ? k2c : k2r;
      a.kstride = kstride;
      a.E = E[side].d();
      a.nlive = nlive.as<int>() + side * ncl;
      a.Ue = Ue[side].d();
      a.rank_e = rank_e.as<int>() + side * ncl;
      a.U = (side ? Uc_ : Ur_).d();
      a.uplane = ctx->plane((side ? Uc_ : Ur_).p());
      a.rank = (side ? rank_c_ : rank_r_).as<int>();
      a.kmax = side ? kmax_c : kmax_r;
      a.status = e.status;
    }
    H2_HIP(h2k::launch_ceig_embed(ca[0], ca[1], ncl, st));
    const long long ss = h2k::eig_scratch_doubles(D2);
    Buf scratch(ctx, (size_t)2 * ncl * ss * sizeof(double));
    h2k::EigArgs ea[2];
    for (int side = 0; side < 2; ++side) {
      h2k::EigArgs& x = ea[side];
      x = h2k::EigArgs{};
      x.G = E[side].d();
      x.gstride = (long long)D2 * D2;
      x.D = D2;
      x.U = Ue[side].d();
      x.ustride = (long long)D2 * D2;
      x.rank = rank_e.as<int>() + side * ncl;
      x.k1 = nlive.as<int>() + side * ncl;
      x.k2 = nlive.as<int>() + side * ncl;
      x.kstride = 1;
      x.half = D;
      x.scratch = scratch.d() + (size_t)side * ncl * ss;
      x.sstride = ss;
      x.tau = e.tau;
      x.exact = e.exact ? 1 : 0;
      x.status = e.status;
    }
    run_eig(e, ea, ncl);
    hipEvent_t ev = nullptr;
    e.prof->begin(kKindEigVec, 0, &ev);
    H2_HIP(h2k::launch_ceig_extract(ca[0], ca[1], ncl, st));
    e.prof->end(ev, kKindEigVec, 0);
    post_ranks(e, ncl, rank_r_.as<int>(), rank_c_.as<int>());  // fixed by the extraction
    return;
  }
  Buf Gnr(ctx, (size_t)ncl * D * D * sizeof(double)), Gnc(ctx, (size_t)ncl * D * D * sizeof(double));
  for (int side = 0; side < 2; ++side) {
    h2k::GramNormArgs ga{};
    for (int c = 0; c < 3; ++c) ga.G[c] = (side ? Gc : Gr)[c].d();
    ga.stride = (long long)D * D;
    ga.D = D;
    ga.out = (side ? Gnc : Gnr).d();
    ga.status = e.status;
    H2_HIP(h2k::launch_gram_norm(ga, ncl, st));
  }
  Ur_ = Buf(ctx, (size_t)ncl * D * D * sizeof(double));
  Uc_ = Buf(ctx, (size_t)ncl * D * D * sizeof(double));
  rank_r_ = Buf(ctx, (size_t)ncl * sizeof(int));
  rank_c_ = Buf(ctx, (size_t)ncl * sizeof(int));
  const long long ss = h2k::eig_scratch_doubles(D);
  Buf scratch(ctx, (size_t)2 * ncl * ss * sizeof(double));
  h2k::EigArgs ea[2];
  for (int side = 0; side < 2; ++side) {
    h2k::EigArgs& x = ea[side];
    x = h2k::EigArgs{};
    x.G = (side ? Gnc : Gnr).d();
    x.gstride = (long long)D * D;
    x.D = D;
    x.U = (side ? Uc_ : Ur_).d();
    x.ustride = (long long)D * D;
    x.rank = (side ? rank_c_ : rank_r_).as<int>();
    x.k1 = side ? k1c : k1r;
    x.k2 = side ? k2c : k2r;
    x.kstride = kstride;
    x.half = half;
    x.scratch = scratch.d() + (size_t)side * ncl * ss;
    x.sstride = ss;
    x.tau = e.tau;
    x.exact = e.exact ? 1 : 0;
    x.kmax = side ? kmax_c : kmax_r;
    x.status = e.status;
  }
  run_eig(e, ea, ncl, rank_r_.as<int>(), rank_c_.as<int>());
}

h2_status mmp_impl(h2_ctx ctx, h2_mat A, h2_mat B, double eps, int mode, int prec, h2_mat* C_out) {
  ActiveCtx active(ctx);
  // FP32-bulk: block products on FP32 MFMA over float copies of the operands;
  // Gram sums accumulate in FP64 (the truncation thresholds eigenvalues at
  // eps^2 lambda_1, far below FP32 rounding of a squared quantity), and the
  // eigen-decompositions and bases stay FP64
  const bool bulk = prec == H2_PREC_FP32_BULK;
  // complex128 (Section II allows complex kernels): every block buffer holds a
  // real and an imaginary plane; products run as four real products and the
  // new bases come from the Hermitian Gram sums
  const bool cplx = A->cplx;
  if (B->cplx != cplx) throw Error(H2_ERR_ARG, "A and B must both be real or both complex");
  if (cplx && bulk) throw Error(H2_ERR_UNSUPPORTED, "complex products run in FP64 only");
  const size_t eb = cplx ? 2 * sizeof(double) : bulk ? sizeof(float) : sizeof(double);
  const size_t gb = cplx ? 2 * sizeof(double) : sizeof(double);  // Gram-side element
  BulkScope bulk_scope(bulk);
  const auto t_sym0 = std::chrono::steady_clock::now();
  Shape& sh = *A->shape;
  const Structure& s = sh.s;
  if (!sh.plan || !sh.dplan) {
    // both or neither: a failed upload leaves the structure without a plan
    auto plan = std::make_unique<Plan>();
    std::string err = build_plan(s, *plan);
    if (!err.empty()) throw Error(H2_ERR_INTERNAL, err);
    auto dplan = upload_plan(ctx, *plan);
    sh.plan = std::move(plan);
    sh.dplan = std::move(dplan);
  }
  const double sym_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_sym0).count();
  const Plan& P = *sh.plan;
  const DevPlan& DP = *sh.dplan;
  auto dl = [&](const TaskList& t) -> const DevList& { return DP.get(t); };
  hipStream_t st = ctx->stream;
  const h2_mat_s* Ad = bulk ? &f32_shadow(ctx, A, st) : A;
  const h2_mat_s* Bd = bulk ? (B == A ? Ad : &f32_shadow(ctx, B, st)) : B;
  const int L = s.L, lmin = s.lmin, np = s.npad, nleaf = 1 << L;
  const bool exact = mode == H2_TRUNC_EXACT || (eps == 0.0 && mode != H2_TRUNC_FIXED);
  // ACCURACY: singular values of the stacked normalised contributions above
  // theta eps / n_t, n_t = number of truncated levels (each level's
  // truncation adds its own error to C, so the budget eps is split evenly);
  // PAPER: the Gram's own values above eps (Section III-C)
  const int n_trunc = std::max(1, L - lmin + 1);
  const double sv = kTheta * eps / n_trunc;
  // FIXED: the fixed-basis ("formatted") product of Section I and Table IV:
  // each new basis is the numerical range of the old basis alone (the third
  // Gram component), so C keeps A's row and B's column bases, orthonormalised
  const bool fixed = mode == H2_TRUNC_FIXED;
  const double tau = fixed ? kFixedTau
                           : exact ? 0.0 : (mode == H2_TRUNC_PAPER ? eps : sv * sv);
  Profiler prof;
  prof.on = ctx->profiling;
  prof.stream = st;
  prof.pool = &ctx->prof_events;
  Profiler* pp = &prof;

  // events around the numeric phase; handed to C at the end (destroyed here
  // when the product fails)
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) hipEventDestroy(a);
      if (b) hipEventDestroy(b);
    }
  } ev;
  H2_HIP(hipEventCreate(&ev.a));
  H2_HIP(hipEventCreate(&ev.b));
  H2_HIP(hipEventRecord(ev.a, st));

  const std::vector<int>&rrA = A->rr, &rcA = A->rc, &rrB = B->rr, &rcB = B->rc;
  Buf status(ctx, 4 * sizeof(int));
  H2_HIP(hipMemsetAsync(status.as<int>(), 0, 4 * sizeof(int), st));

  // ---------------------------------------------------------- output C
  auto C = std::make_unique<h2_mat_s>();
  C->ctx = ctx;
  C->shape = A->shape;
  C->product = true;
  C->rr.assign(L + 1, 16);
  C->rc.assign(L + 1, 16);
  C->krow.assign((2LL << L) - 1, 0);
  C->kcol.assign((2LL << L) - 1, 0);
  C->Tr.resize(L);
  C->Tc.resize(L);
  C->Tr_stride.assign(L, 0);
  C->Tc_stride.assign(L, 0);
  C->S.resize(L + 1);
  std::vector<int> cpad(L + 1, 16);
  std::vector<Buf> rank_r(L + 1), rank_c(L + 1);

  // ---------------------------------------------------------- step 0: Pi
  std::vector<Buf> Pi(L + 1);
  Pi[L] = Buf(ctx, (size_t)nleaf * rcA[L] * rrB[L] * eb, bulk, cplx);
  gemm(st, pp, kKindOther, dl(P.pi.leaf), rcA[L], rrB[L], np,
       Op{Ad->W.p(), nullptr, A->W_stride, 0, np}, true, Op{Bd->V.p(), nullptr, B->V_stride, 0, np},
       false, Pi[L].p(), (long long)rcA[L] * rrB[L], rcA[L], 0, 0, 1.0, 0.0);
  for (int l = L - 1; l >= lmin; --l) {
    const int ch = l + 1;
    Buf X(ctx, (size_t)(2 << l) * rcA[ch] * rrB[l] * eb, bulk, cplx);
    gemm(st, pp, kKindOther, dl(P.pi.X[l]), rcA[ch], rrB[l], rrB[ch],
         Op{Pi[ch].p(), nullptr, (long long)rcA[ch] * rrB[ch], 0, rcA[ch]}, false,
         Op{Bd->Tr[l].p(), nullptr, B->Tr_stride[l], 0, 2 * rrB[ch], rrB[ch], 0}, false, X.p(),
         (long long)rcA[ch] * rrB[l], rcA[ch], 0, 0, 1.0, 0.0);
    Pi[l] = Buf(ctx, (size_t)(1 << l) * rcA[l] * rrB[l] * eb, bulk, cplx);
    gemm(st, pp, kKindOther, dl(P.pi.S[l]), rcA[l], rrB[l], rcA[ch],
         Op{Ad->Tc[l].p(), nullptr, A->Tc_stride[l], 0, 2 * rcA[ch], rcA[ch], 0}, true,
         Op{X.p(), nullptr, (long long)rcA[ch] * rrB[l], 0, rcA[ch]}, false, Pi[l].p(),
         (long long)rcA[l] * rrB[l], rcA[l], 0, 0, 1.0, 0.0);
  }

  // the three eigensolver phases, each timed as its own kernel class
  const EigLevel eg{ctx, st, &prof, status.as<int>(), cplx, tau, exact,
                    ctx->readback(2 * (size_t)nleaf + 4), ctx->rb_ev};
  auto eig_level = [&](int l, int D, Buf Gr[3], Buf Gc[3], Buf& Ur_, Buf& Uc_, Buf& rank_r_,
                       Buf& rank_c_, const int* k1r, const int* k2r, const int* k1c,
                       const int* k2c, int kstride, int half) {
    h2::eig_level(eg, l, D, Gr, Gc, Ur_, Uc_, rank_r_, rank_c_, k1r, k2r, k1c, k2c, kstride, half);
  };
  auto read_ranks = [&](int l) {
    const int ncl = 1 << l;
    const int* h = wait_ranks(eg, l);
    int mx = 1;
    for (int c = 0; c < ncl; ++c) {
      C->krow[cidx(l, c)] = h[c];
      C->kcol[cidx(l, c)] = h[ncl + c];
      mx = std::max(mx, std::max(h[c], h[ncl + c]));
    }
    return pad16(mx);
  };

  // Products whose targets nothing later in the upward pass reads (the
  // admissible couplings of C, the non-leaf targets kept for the top-down
  // split, the dense leaf blocks) wait in `later`.  They are enqueued on a
  // helper stream once the main stream reaches the eigen-decompositions of
  // a level with at most kFewClusters clusters: those launches (one
  // workgroup per cluster and side, 64 workgroups on 256 compute units)
  // leave most of the chip idle, while at the levels below the products
  // would slow the main stream's Gram sums and eigensolvers about as much
  // as they gain.  The streams join before the top-down split.  Every
  // buffer such a product touches stays in `held` until the join, so no
  // block returns to the pool while the helper stream may still use it.
  constexpr int kFewClusters = 32;
  hipStream_t ax = ctx->aux[0];
  Profiler prof_ax;
  prof_ax.on = prof.on;
  prof_ax.stream = ax;
  prof_ax.pool = &ctx->prof_events;
  Profiler* pax = &prof_ax;
  std::vector<std::function<void()>> later;
  std::vector<Buf> held;
  // a failed product waits for the helper stream before the buffers its
  // deferred products use are released: guards declared after `held` and
  // after the non-leaf operands below
  struct AuxWait {
    hipStream_t s;
    const bool* armed;
    ~AuxWait() {
      if (*armed) (void)hipStreamSynchronize(s);
    }
  };
  bool ax_armed = false;
  const AuxWait ax_wait{ax, &ax_armed};
  auto flush = [&]() {
    if (later.empty()) return;
    H2_HIP(hipEventRecord(ctx->fork_ev, st));
    H2_HIP(hipStreamWaitEvent(ax, ctx->fork_ev, 0));
    ax_armed = true;
    for (auto& f : later) f();
    later.clear();
  };

  // ============================================================== leaf level
  const LeafPlan& LP = P.leaf;
  const int nnL = s.lev[L].size();
  const long long nn2 = (long long)np * np;
  Buf leaf_sizes(ctx, nleaf * sizeof(int));
  H2_HIP(hipMemcpyAsync(leaf_sizes.as<int>(), s.leaf_size.data(), nleaf * sizeof(int),
                        hipMemcpyHostToDevice, st));
  Buf Ur_L, Uc_L;
  // FP32-bulk products read the new bases through float copies: the values
  // their FP32 arithmetic rounds the FP64 bases to anyway, at half the bytes
  std::vector<Buf> Urf(L + 1), Ucf(L + 1);
  auto narrow = [&](const Buf& src, Buf& dst) {
    const long long n = (long long)(src.bytes() / sizeof(double));
    if (!bulk || n <= 0) return;
    dst = Buf(ctx, (size_t)n * sizeof(float), true);
    H2_HIP(h2k::launch_d2f(src.as<double>(), dst.as<float>(), n, st));
  };
  auto bas = [&](const Buf& f, const Buf& d) { return bulk ? f.p() : d.p(); };
  Buf PA_L, PB_L;       // projections at the leaves
  Buf Ahat_L, Bhat_L;   // collected leaf blocks, 2x2 grouped
  Buf Acc_L;            // blue accumulators of the leaf level
  Buf FC;
  int c = 16;
  {
    Buf G[3], Gc[3];
    for (int k = 0; k < 3; ++k) {
      G[k] = Buf(ctx, (size_t)nleaf * nn2 * gb, false, cplx);
      Gc[k] = Buf(ctx, (size_t)nleaf * nn2 * gb, false, cplx);
    }
    if (fixed) {
      for (Buf* g : {&G[0], &G[1], &Gc[0], &Gc[1]}) zero(st, g->p(), (long long)nleaf * nn2);
    } else {
      Buf b1(ctx, nnL * nn2 * gb, false, cplx), b2(ctx, nnL * nn2 * gb, false, cplx),
          b3(ctx, nnL * nn2 * gb, false, cplx);
      const Op FA{Ad->F.p(), nullptr, nn2, 0, np}, FB{Bd->F.p(), nullptr, nn2, 0, np};
      const Op o1{b1.p(), nullptr, nn2, 0, np}, o2{b2.p(), nullptr, nn2, 0, np},
          o3{b3.p(), nullptr, nn2, 0, np};
      // row Gram, case 1: sum_j F^A_ij (sum_k F^B_jk F^B_jk^T) F^A_ij^T over
      // dense products with an admissible or blue target (equation Gr1L)
      gemm(st, pp, kKindGram, dl(LP.gB), np, np, np, FB, false, FB, true, b1.p(), nn2, np, 0, 0, 1, 0, kConjB);
      segsum(st, dl(LP.H), np, np, o1, b2.p(), nn2, np, 0, 0, 0.0);
      gemm(st, pp, kKindGram, dl(LP.X1), np, np, np, FA, false, o2, false, b3.p(), nn2, np, 0, 0, 1, 0);
      gemm(st, pp, kKindGram, dl(LP.G1), np, np, np, o3, false, FA, true, G[0].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
      // column Gram, case 1 (equation case1-ch)
      gemm(st, pp, kKindGram, dl(LP.hA), np, np, np, FA, true, FA, false, b1.p(), nn2, np, 0, 0, 1, 0, kConjB);
      segsum(st, dl(LP.Hc), np, np, o1, b2.p(), nn2, np, 0, 0, 0.0);
      gemm(st, pp, kKindGram, dl(LP.X1c), np, np, np, FB, true, o2, false, b3.p(), nn2, np, 0, 0, 1, 0);
      gemm(st, pp, kKindGram, dl(LP.G1c), np, np, np, o3, false, FB, false, Gc[0].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
      // case 2: F^A_ij V^B_j (Gr2L) and (W^A_j^T F^B_jk)^T (case2-ch)
      Buf Z(ctx, (size_t)nnL * np * std::max(rrB[L], rcA[L]) * gb, false, cplx);
      const long long zs = (long long)np * rrB[L], zcs = (long long)np * rcA[L];
      gemm(st, pp, kKindGram, dl(LP.Z), np, rrB[L], np, FA, false,
           Op{Bd->V.p(), nullptr, B->V_stride, 0, np}, false, Z.p(), zs, np, 0, 0, 1, 0);
      gemm(st, pp, kKindGram, dl(LP.G2), np, np, rrB[L], Op{Z.p(), nullptr, zs, 0, np}, false,
           Op{Z.p(), nullptr, zs, 0, np}, true, G[1].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
      gemm(st, pp, kKindGram, dl(LP.Zc), np, rcA[L], np, FB, true,
           Op{Ad->W.p(), nullptr, A->W_stride, 0, np}, false, Z.p(), zcs, np, 0, 0, 1, 0);
      gemm(st, pp, kKindGram, dl(LP.G2c), np, np, rcA[L], Op{Z.p(), nullptr, zcs, 0, np}, false,
           Op{Z.p(), nullptr, zcs, 0, np}, true, Gc[1].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
    }
    {
      // case 3/4: the old bases V^A_i V^A_i^T (Gr3L) and W^B_k W^B_k^T (case3-ch)
      gemm(st, pp, kKindGram, dl(LP.G3), np, np, rrA[L], Op{Ad->V.p(), nullptr, A->V_stride, 0, np},
           false, Op{Ad->V.p(), nullptr, A->V_stride, 0, np}, true, G[2].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
      gemm(st, pp, kKindGram, dl(LP.G3c), np, np, rcB[L], Op{Bd->W.p(), nullptr, B->W_stride, 0, np},
           false, Op{Bd->W.p(), nullptr, B->W_stride, 0, np}, true, Gc[2].p(), nn2, np, 0, 0, 1, 0, kConjB | kLowerOnly);
    }
    eig_level(L, np, G, Gc, Ur_L, Uc_L, rank_r[L], rank_c[L], leaf_sizes.as<int>(), nullptr,
              leaf_sizes.as<int>(), nullptr, 1, np);
  }
  c = read_ranks(L);
  cpad[L] = c;
  {
    narrow(Ur_L, Urf[L]);
    narrow(Uc_L, Ucf[L]);
    const Op VC{bas(Urf[L], Ur_L), nullptr, nn2, 0, np}, WC{bas(Ucf[L], Uc_L), nullptr, nn2, 0, np};
    const Op FA{Ad->F.p(), nullptr, nn2, 0, np}, FB{Bd->F.p(), nullptr, nn2, 0, np};
    // projections (leafproj)
    PA_L = Buf(ctx, (size_t)nleaf * c * rrA[L] * eb, bulk, cplx);
    PB_L = Buf(ctx, (size_t)nleaf * rcB[L] * c * eb, bulk, cplx);
    gemm(st, pp, kKindOther, dl(LP.PA), c, rrA[L], np, VC, true,
         Op{Ad->V.p(), nullptr, A->V_stride, 0, np}, false, PA_L.p(), (long long)c * rrA[L], c, 0, 0, 1, 0, kConjA);
    gemm(st, pp, kKindOther, dl(LP.PB), rcB[L], c, np, Op{Bd->W.p(), nullptr, B->W_stride, 0, np},
         true, WC, false, PB_L.p(), (long long)rcB[L] * c, rcB[L], 0, 0, 1, 0, kConjB);
    // leaf-coordinate left / right operands of every leaf block
    const long long las = (long long)c * np;
    Buf LA(ctx, (size_t)nnL * las * eb, bulk, cplx), RB(ctx, (size_t)nnL * las * eb, bulk, cplx);
    {
      Buf PS(ctx, (size_t)nnL * c * rcA[L] * eb, bulk, cplx);
      Buf SP(ctx, (size_t)nnL * rrB[L] * c * eb, bulk, cplx);
      gemm(st, pp, kKindOther, dl(LP.LA_F), c, np, np, VC, true, FA, false, LA.p(), las, c, 0, 0, 1, 0, kConjA);
      gemm(st, pp, kKindOther, dl(LP.PS), c, rcA[L], rrA[L],
           Op{PA_L.p(), nullptr, (long long)c * rrA[L], 0, c}, false,
           Op{Ad->S[L].p(), nullptr, (long long)rrA[L] * rcA[L], 0, rrA[L]}, false, PS.p(),
           (long long)c * rcA[L], c, 0, 0, 1, 0);
      gemm(st, pp, kKindOther, dl(LP.LA_R), c, np, rcA[L],
           Op{PS.p(), nullptr, (long long)c * rcA[L], 0, c}, false,
           Op{Ad->W.p(), nullptr, A->W_stride, 0, np}, true, LA.p(), las, c, 0, 0, 1, 0);
      gemm(st, pp, kKindOther, dl(LP.RB_F), np, c, np, FB, false, WC, false, RB.p(), las, np, 0, 0, 1, 0, kConjB);
      gemm(st, pp, kKindOther, dl(LP.SP), rrB[L], c, rcB[L],
           Op{Bd->S[L].p(), nullptr, (long long)rrB[L] * rcB[L], 0, rrB[L]}, false,
           Op{PB_L.p(), nullptr, (long long)rcB[L] * c, 0, rcB[L]}, false, SP.p(),
           (long long)rrB[L] * c, rrB[L], 0, 0, 1, 0);
      gemm(st, pp, kKindOther, dl(LP.RB_R), np, c, rrB[L], Op{Bd->V.p(), nullptr, B->V_stride, 0, np},
           false, Op{SP.p(), nullptr, (long long)rrB[L] * c, 0, rrB[L]}, false, RB.p(), las, np, 0,
           0, 1, 0);
    }
    // collected leaf blocks for the level above (Fcollect; 2x2 grouped)
    if (L >= 1) {
      const int ntile = s.lev[L - 1].n_nl;
      Ahat_L = Buf(ctx, (size_t)ntile * 4 * c * rrB[L] * eb, bulk, cplx);
      Bhat_L = Buf(ctx, (size_t)ntile * 4 * rcA[L] * c * eb, bulk, cplx);
      gemm(st, pp, kKindOther, dl(LP.Ahat), c, rrB[L], np, Op{LA.p(), nullptr, las, 0, c}, false,
           Op{Bd->V.p(), nullptr, B->V_stride, 0, np}, false, Ahat_L.p(), 4LL * c * rrB[L], 2 * c,
           c, (long long)rrB[L] * 2 * c, 1, 0);
      gemm(st, pp, kKindOther, dl(LP.Bhat), rcA[L], c, np, Op{Ad->W.p(), nullptr, A->W_stride, 0, np},
           true, Op{RB.p(), nullptr, las, 0, np}, false, Bhat_L.p(), 4LL * rcA[L] * c, 2 * rcA[L],
           rcA[L], (long long)c * 2 * rcA[L], 1, 0);
    }
    // products into admissible and blue targets (leafcoup_simple)
    C->S[L] = Buf(ctx, (size_t)nnL * c * c * eb, bulk, cplx);
    later.push_back([=, out = C->S[L].p()] { zero(ax, out, (long long)nnL * c * c); });
    const int nbt = std::max(1, LP.n_blue_tiles);
    Acc_L = Buf(ctx, (size_t)nbt * 4 * c * c * eb, bulk, cplx);
    zero(st, Acc_L.p(), (long long)nbt * 4 * c * c);
    gemm(st, pp, kKindTriple, dl(LP.adm_B), c, c, np, Op{LA.p(), nullptr, las, 0, c}, false,
         Op{RB.p(), nullptr, las, 0, np}, false, Acc_L.p(), 4LL * c * c, 2 * c, c,
         (long long)c * 2 * c, 1, 1);
    later.push_back([=, &dl, &LP, la = LA.p(), rb = RB.p(), out = C->S[L].p()] {
      gemm(ax, pax, kKindTriple, dl(LP.adm_R), c, c, np, Op{la, nullptr, las, 0, c}, false,
           Op{rb, nullptr, las, 0, np}, false, out, (long long)c * c, c, 0, 0, 1, 1);
    });
    held.push_back(std::move(LA));
    held.push_back(std::move(RB));
  }
  // dense targets: exact leaf products with admissible factors densified
  FC = Buf(ctx, (size_t)nnL * nn2 * eb, bulk, cplx);
  later.push_back([=, &dl, &LP, &held, &rrA, &rcA, &rrB, &rcB, fc = FC.p()] {
    zero(ax, fc, nnL * nn2);
    held.emplace_back(ctx, (size_t)nnL * nn2 * eb, bulk, cplx);
    void* DA = held.back().p();
    held.emplace_back(ctx, (size_t)nnL * nn2 * eb, bulk, cplx);
    void* DB = held.back().p();
    held.emplace_back(ctx, (size_t)nnL * np * std::max(rcA[L], rcB[L]) * eb, bulk, cplx);
    void* T = held.back().p();
    gemm(ax, pax, kKindOther, dl(LP.densA1), np, rcA[L], rrA[L],
         Op{Ad->V.p(), nullptr, A->V_stride, 0, np}, false,
         Op{Ad->S[L].p(), nullptr, (long long)rrA[L] * rcA[L], 0, rrA[L]}, false, T,
         (long long)np * rcA[L], np, 0, 0, 1, 0);
    gemm(ax, pax, kKindOther, dl(LP.densA2), np, np, rcA[L],
         Op{T, nullptr, (long long)np * rcA[L], 0, np}, false,
         Op{Ad->W.p(), nullptr, A->W_stride, 0, np}, true, DA, nn2, np, 0, 0, 1, 0);
    gemm(ax, pax, kKindOther, dl(LP.densB1), np, rcB[L], rrB[L],
         Op{Bd->V.p(), nullptr, B->V_stride, 0, np}, false,
         Op{Bd->S[L].p(), nullptr, (long long)rrB[L] * rcB[L], 0, rrB[L]}, false, T,
         (long long)np * rcB[L], np, 0, 0, 1, 0);
    gemm(ax, pax, kKindOther, dl(LP.densB2), np, np, rcB[L],
         Op{T, nullptr, (long long)np * rcB[L], 0, np}, false,
         Op{Bd->W.p(), nullptr, B->W_stride, 0, np}, true, DB, nn2, np, 0, 0, 1, 0);
    gemm(ax, pax, kKindTriple, dl(LP.dense), np, np, np, Op{Ad->F.p(), DA, nn2, nn2, np}, false,
         Op{Bd->F.p(), DB, nn2, nn2, np}, false, fc, nn2, np, 0, 0, 1, 1);
  });

  // ========================================================= non-leaf levels
  std::vector<Buf> Ur(L + 1), Uc(L + 1), SNL(L + 1);
  Ur[L] = std::move(Ur_L);
  Uc[L] = std::move(Uc_L);
  Buf PA_ch = std::move(PA_L), PB_ch = std::move(PB_L);
  Buf Ahat_ch = std::move(Ahat_L), Bhat_ch = std::move(Bhat_L), Acc_ch = std::move(Acc_L);
  const AuxWait ax_wait_nl{ax, &ax_armed};
  for (int l = L - 1; l >= lmin; --l) {
    const int ch = l + 1;
    const int cc = cpad[ch];
    const int K = 2 * cc;
    const long long K2 = (long long)K * K;
    const LevelPlan& Q = P.lev[l];
    const int ncl = 1 << l;
    const int nn = s.lev[l].size();
    const Op AccT{Acc_ch.p(), nullptr, 4LL * cc * cc, 0, K};
    Buf G[3], Gc[3];
    for (int k = 0; k < 3; ++k) {
      G[k] = Buf(ctx, (size_t)ncl * K2 * gb, false, cplx);
      Gc[k] = Buf(ctx, (size_t)ncl * K2 * gb, false, cplx);
    }
    // case 1: merged children couplings M_IK (nonleafA; case1-ch-nl)
    if (fixed) {
      for (Buf* g : {&G[0], &G[1], &Gc[0], &Gc[1]}) zero(st, g->p(), (long long)ncl * K2);
    } else {
      gemm(st, pp, kKindGram, dl(Q.G1), K, K, K, AccT, false, AccT, true, G[0].p(), K2, K, 0, 0, 1, 0, kConjB | kLowerOnly);
      gemm(st, pp, kKindGram, dl(Q.G1c), K, K, K, AccT, true, AccT, false, Gc[0].p(), K2, K, 0, 0, 1, 0, kConjB | kLowerOnly);
    }
    // case 2: (NL^A)_coll T^B_J (case2-ch-nl) and its column mirror
    const long long ys = (long long)K * rrB[l], ycs = (long long)rcA[l] * K;
    Buf Y(ctx, (size_t)std::max(1, nn) * ys * gb, false, cplx);
    Buf Yc(ctx, (size_t)std::max(1, nn) * ycs * gb, false, cplx);
    gemm(st, pp, kKindGram, dl(Q.Y), K, rrB[l], 2 * rrB[ch],
         Op{Ahat_ch.p(), nullptr, 4LL * cc * rrB[ch], 0, K}, false,
         Op{Bd->Tr[l].p(), nullptr, B->Tr_stride[l], 0, 2 * rrB[ch]}, false, Y.p(), ys, K, 0, 0, 1, 0);
    if (!fixed)
      gemm(st, pp, kKindGram, dl(Q.G2), K, K, rrB[l], Op{Y.p(), nullptr, ys, 0, K}, false,
           Op{Y.p(), nullptr, ys, 0, K}, true, G[1].p(), K2, K, 0, 0, 1, 0, kConjB | kLowerOnly);
    gemm(st, pp, kKindGram, dl(Q.Yc), rcA[l], K, 2 * rcA[ch],
         Op{Ad->Tc[l].p(), nullptr, A->Tc_stride[l], 0, 2 * rcA[ch]}, true,
         Op{Bhat_ch.p(), nullptr, 4LL * rcA[ch] * cc, 0, 2 * rcA[ch]}, false, Yc.p(), ycs, rcA[l],
         0, 0, 1, 0);
    if (!fixed)
      gemm(st, pp, kKindGram, dl(Q.G2c), K, K, rcA[l], Op{Yc.p(), nullptr, ycs, 0, rcA[l]}, true,
           Op{Yc.p(), nullptr, ycs, 0, rcA[l]}, false, Gc[1].p(), K2, K, 0, 0, 1, 0, kConjB | kLowerOnly);
    // cases 3/4: old bases projected on the children's new bases (case3-ch-nl)
    const long long ds = (long long)K * rrA[l], qs = (long long)K * rcB[l];
    Buf Dm(ctx, (size_t)ncl * ds * gb, false, cplx), Qm(ctx, (size_t)ncl * qs * gb, false, cplx);
    gemm(st, pp, kKindGram, dl(Q.D), cc, rrA[l], rrA[ch],
         Op{PA_ch.p(), nullptr, (long long)cc * rrA[ch], 0, cc}, false,
         Op{Ad->Tr[l].p(), nullptr, A->Tr_stride[l], 0, 2 * rrA[ch], rrA[ch], 0}, false, Dm.p(), ds,
         K, cc, 0, 1, 0);
    gemm(st, pp, kKindGram, dl(Q.G3), K, K, rrA[l], Op{Dm.p(), nullptr, ds, 0, K}, false,
         Op{Dm.p(), nullptr, ds, 0, K}, true, G[2].p(), K2, K, 0, 0, 1, 0, kConjB | kLowerOnly);
    gemm(st, pp, kKindGram, dl(Q.Q), cc, rcB[l], rcB[ch],
         Op{PB_ch.p(), nullptr, (long long)rcB[ch] * cc, 0, rcB[ch]}, true,
         Op{Bd->Tc[l].p(), nullptr, B->Tc_stride[l], 0, 2 * rcB[ch], rcB[ch], 0}, false, Qm.p(), qs,
         K, cc, 0, 1, 0);
    gemm(st, pp, kKindGram, dl(Q.G3c), K, K, rcB[l], Op{Qm.p(), nullptr, qs, 0, K}, false,
         Op{Qm.p(), nullptr, qs, 0, K}, true, Gc[2].p(), K2, K, 0, 0, 1, 0, kConjB | kLowerOnly);
    // new transfer matrices (the deferred products start here when the
    // level's eigen-decompositions leave most compute units idle)
    if ((1 << l) <= kFewClusters) flush();
    eig_level(l, K, G, Gc, Ur[l], Uc[l], rank_r[l], rank_c[l], rank_r[ch].as<int>(),
              rank_r[ch].as<int>() + 1, rank_c[ch].as<int>(), rank_c[ch].as<int>() + 1, 2, cc);
    for (int k = 0; k < 3; ++k) {
      G[k].reset();
      Gc[k].reset();
    }
    const int cl = read_ranks(l);
    cpad[l] = cl;
    narrow(Ur[l], Urf[l]);
    narrow(Uc[l], Ucf[l]);
    const Op TCr{bas(Urf[l], Ur[l]), nullptr, K2, 0, K}, TCc{bas(Ucf[l], Uc[l]), nullptr, K2, 0, K};
    // projections (nonleafproj)
    Buf PA_l(ctx, (size_t)ncl * cl * rrA[l] * eb, bulk, cplx);
    Buf PB_l(ctx, (size_t)ncl * rcB[l] * cl * eb, bulk, cplx);
    gemm(st, pp, kKindOther, dl(Q.PA), cl, rrA[l], K, TCr, true, Op{Dm.p(), nullptr, ds, 0, K},
         false, PA_l.p(), (long long)cl * rrA[l], cl, 0, 0, 1, 0, kConjA);
    gemm(st, pp, kKindOther, dl(Q.PB), rcB[l], cl, K, Op{Qm.p(), nullptr, qs, 0, K}, true, TCc,
         false, PB_l.p(), (long long)rcB[l] * cl, rcB[l], 0, 0, 1, 0, kConjB);
    // collected blocks of this level (NLcollect; admissible ones projected)
    const int ntile = l >= 1 ? s.lev[l - 1].n_nl : 1;
    Buf Ahat_l(ctx, (size_t)std::max(1, ntile) * 4 * cl * rrB[l] * eb, bulk, cplx);
    Buf Bhat_l(ctx, (size_t)std::max(1, ntile) * 4 * rcA[l] * cl * eb, bulk, cplx);
    const long long pas_s = (long long)cl * rcA[l], sbp_s = (long long)rrB[l] * cl;
    Buf PAS(ctx, (size_t)std::max(1, nn) * pas_s * eb, bulk, cplx);
    Buf SBP(ctx, (size_t)std::max(1, nn) * sbp_s * eb, bulk, cplx);
    const long long at_s = 4LL * cl * rrB[l], bt_s = 4LL * rcA[l] * cl;
    gemm(st, pp, kKindOther, dl(Q.AhatNL), cl, rrB[l], K, TCr, true, Op{Y.p(), nullptr, ys, 0, K},
         false, Ahat_l.p(), at_s, 2 * cl, cl, (long long)rrB[l] * 2 * cl, 1, 0, kConjA);
    gemm(st, pp, kKindOther, dl(Q.PAS), cl, rcA[l], rrA[l],
         Op{PA_l.p(), nullptr, (long long)cl * rrA[l], 0, cl}, false,
         Op{Ad->S[l].p(), nullptr, (long long)rrA[l] * rcA[l], 0, rrA[l]}, false, PAS.p(), pas_s,
         cl, 0, 0, 1, 0);
    gemm(st, pp, kKindOther, dl(Q.AhatR), cl, rrB[l], rcA[l], Op{PAS.p(), nullptr, pas_s, 0, cl},
         false, Op{Pi[l].p(), nullptr, (long long)rcA[l] * rrB[l], 0, rcA[l]}, false, Ahat_l.p(),
         at_s, 2 * cl, cl, (long long)rrB[l] * 2 * cl, 1, 0);
    gemm(st, pp, kKindOther, dl(Q.BhatNL), rcA[l], cl, K, Op{Yc.p(), nullptr, ycs, 0, rcA[l]},
         false, TCc, false, Bhat_l.p(), bt_s, 2 * rcA[l], rcA[l], (long long)cl * 2 * rcA[l], 1, 0, kConjB);
    gemm(st, pp, kKindOther, dl(Q.SBP), rrB[l], cl, rcB[l],
         Op{Bd->S[l].p(), nullptr, (long long)rrB[l] * rcB[l], 0, rrB[l]}, false,
         Op{PB_l.p(), nullptr, (long long)rcB[l] * cl, 0, rcB[l]}, false, SBP.p(), sbp_s, rrB[l],
         0, 0, 1, 0);
    gemm(st, pp, kKindOther, dl(Q.BhatR), rcA[l], cl, rrB[l],
         Op{Pi[l].p(), nullptr, (long long)rcA[l] * rrB[l], 0, rcA[l]}, false,
         Op{SBP.p(), nullptr, sbp_s, 0, rrB[l]}, false, Bhat_l.p(), bt_s, 2 * rcA[l], rcA[l],
         (long long)cl * 2 * rcA[l], 1, 0);
    // targets of this level
    C->S[l] = Buf(ctx, (size_t)std::max(1, nn) * cl * cl * eb, bulk, cplx);
    SNL[l] = Buf(ctx, (size_t)std::max(1, nn) * cl * cl * eb, bulk, cplx);
    // both written only by deferred products: cleared on the helper stream
    later.push_back([=, a = C->S[l].p(), b = SNL[l].p(), n = (long long)std::max(1, nn) * cl * cl] {
      zero(ax, a, n);
      zero(ax, b, n);
    });
    const int nbt = std::max(1, Q.n_blue_tiles);
    Buf Acc_l(ctx, (size_t)nbt * 4 * cl * cl * eb, bulk, cplx);
    zero(st, Acc_l.p(), (long long)nbt * 4 * cl * cl);
    const long long cs = (long long)cl * cl, acs = 4LL * cl * cl;
    // case 1: T^C_I^T M_IK T^C_K (nonleafcoup_simple, first case)
    {
      Buf X1(ctx, (size_t)std::max(1, Q.n_case1) * cl * K * eb, bulk, cplx);
      gemm(st, pp, kKindTarget, dl(Q.c1X), cl, K, K, TCr, true, AccT, false, X1.p(),
           (long long)cl * K, cl, 0, 0, 1, 0, kConjA);
      const Op X1o{X1.p(), nullptr, (long long)cl * K, 0, cl};
      gemm(st, pp, kKindTarget, dl(Q.c1_B), cl, cl, K, X1o, false, TCc, false, Acc_l.p(), acs,
           2 * cl, cl, (long long)cl * 2 * cl, 1, 1, kConjB);
      later.push_back([=, &dl, d = &Q.c1_R, out = C->S[l].p()] {
        gemm(ax, pax, kKindTarget, dl(*d), cl, cl, K, X1o, false, TCc, false, out, cs, cl, 0, 0, 1,
             1, kConjB);
      });
      held.push_back(std::move(X1));
    }
    // cases 2-4 (nonleafcoup_simple), re-associated: for an admissible B
    // factor sum_J Ahat_IJ (S^B_JK P^B_K) = (sum_J Ahat_IJ S^B_JK) P^B_K, and
    // for an admissible A factor sum_J (P^A_I S^A_IJ) Bhat_JK =
    // P^A_I (sum_J S^A_IJ Bhat_JK): the per-triple product shrinks to
    // k_C x k x k and the projection is applied once per target
    const Op AhatT{Ahat_l.p(), nullptr, at_s, 0, 2 * cl, cl, (long long)rrB[l] * 2 * cl};
    const Op BhatT{Bhat_l.p(), nullptr, bt_s, 0, 2 * rcA[l], rcA[l], (long long)cl * 2 * rcA[l]};
    const Op SBo{Bd->S[l].p(), nullptr, (long long)rrB[l] * rcB[l], 0, rrB[l]};
    const Op SAo{Ad->S[l].p(), nullptr, (long long)rrA[l] * rcA[l], 0, rrA[l]};
    const Op PBo{PB_l.p(), nullptr, (long long)rcB[l] * cl, 0, rcB[l]};
    const Op PAo{PA_l.p(), nullptr, (long long)cl * rrA[l], 0, cl};
    struct Tgt {
      void* p;
      long long stride;
      int ld;
      long long sr, sc;
    };
    const Tgt tR{C->S[l].p(), cs, cl, 0, 0}, tB{Acc_l.p(), acs, 2 * cl, cl, (long long)cl * 2 * cl},
        tNL{SNL[l].p(), cs, cl, 0, 0};
    // stage 1: W_nl = Ahat S^B and W_r = S^A Bhat of one target class
    // (temporaries into `keep`); stage 2: the projections into the targets
    struct Cases24 {
      h2_ctx ctx;
      bool bulk, cplx;
      size_t eb;
      int cl, rcB, rrA, rrB, rcA;
      Op AhatT, BhatT, SBo, SAo, PBo, PAo;
      void *PA, *PB;
      long long wns, wrs;
      void run(hipStream_t s, Profiler* pp, const DevList& dn, const DevList& dr,
               const DevList& fnl, const DevList& fr, const DevList& fboth, const Tgt& t,
               std::vector<Buf>& keep) const {
        void *Wn = nullptr, *Wr = nullptr;
        if (dn.nout) {
          keep.emplace_back(ctx, (size_t)dn.nout * wns * eb, bulk, cplx);
          Wn = keep.back().p();
          gemm(s, pp, kKindTriple, dn, cl, rcB, rrB, AhatT, false, SBo, false, Wn, wns, cl, 0, 0,
               1, 0);
        }
        if (dr.nout) {
          keep.emplace_back(ctx, (size_t)dr.nout * wrs * eb, bulk, cplx);
          Wr = keep.back().p();
          gemm(s, pp, kKindTriple, dr, rrA, cl, rcA, SAo, false, BhatT, false, Wr, wrs, rrA, 0, 0,
               1, 0);
        }
        if (rcB == rrA && Wn && Wr) {
          // one pass over the targets: [W_nl | P^A_I] x [P^B_K ; W_r]
          gemm(s, pp, kKindTarget, fboth, cl, cl, rcB, Op{Wn, PA, wns, (long long)cl * rrA, cl},
               false, Op{PB, Wr, (long long)rcB * cl, wrs, rcB}, false, t.p, t.stride, t.ld, t.sr,
               t.sc, 1, 1);
          return;
        }
        if (Wn)
          gemm(s, pp, kKindTarget, fnl, cl, cl, rcB, Op{Wn, nullptr, wns, 0, cl}, false, PBo, false,
               t.p, t.stride, t.ld, t.sr, t.sc, 1, 1);
        if (Wr)
          gemm(s, pp, kKindTarget, fr, cl, cl, rrA, PAo, false, Op{Wr, nullptr, wrs, 0, rrA}, false,
               t.p, t.stride, t.ld, t.sr, t.sc, 1, 1);
      }
    };
    const Cases24 c24{ctx, bulk, cplx, eb, cl, rcB[l], rrA[l], rrB[l], rcA[l], AhatT, BhatT, SBo,
                      SAo, PBo, PAo, PA_l.p(), PB_l.p(),
                      (long long)cl * rcB[l], (long long)rrA[l] * cl};
    {
      std::vector<Buf> keep;  // main-stream temporaries, freed in stream order
      c24.run(st, pp, dl(Q.w_nl_B), dl(Q.w_r_B), dl(Q.f_nl_B), dl(Q.f_r_B), dl(Q.f_B), tB, keep);
    }
    // admissible targets (final couplings of C) and non-leaf targets (read
    // by the top-down split only): deferred
    for (int r = 1; r >= 0; --r) {
      const Tgt t = r ? tR : tNL;
      const DevList *dn = &dl(r ? Q.w_nl_R : Q.w_nl_NL), *dr = &dl(r ? Q.w_r_R : Q.w_r_NL),
                    *fnl = &dl(r ? Q.f_nl_R : Q.f_nl_NL), *fr = &dl(r ? Q.f_r_R : Q.f_r_NL),
                    *fb = &dl(r ? Q.f_R : Q.f_NL);
      later.push_back([=, &held] { c24.run(ax, pax, *dn, *dr, *fnl, *fr, *fb, t, held); });
    }
    // this level's operands of the deferred products stay alive until the join
    held.push_back(std::move(PA_ch));
    held.push_back(std::move(PB_ch));
    held.push_back(std::move(Ahat_ch));
    held.push_back(std::move(Bhat_ch));
    PA_ch = std::move(PA_l);
    PB_ch = std::move(PB_l);
    Ahat_ch = std::move(Ahat_l);
    Bhat_ch = std::move(Bhat_l);
    Acc_ch = std::move(Acc_l);
  }

  // join: the split reads the deferred products' targets
  flush();
  if (ax_armed) {
    H2_HIP(hipEventRecord(ctx->join_ev[0], ax));
    H2_HIP(hipStreamWaitEvent(st, ctx->join_ev[0], 0));
    ax_armed = false;
  }
  held.clear();  // later users of these blocks are ordered after the join
  prof.recs.insert(prof.recs.end(), prof_ax.recs.begin(), prof_ax.recs.end());
  prof_ax.recs.clear();

  // ===================================================== top-down split
  for (int l = lmin; l < L; ++l) {
    const int ch = l + 1;
    const int cl = cpad[l], cc = cpad[ch];
    const int K = 2 * cc;
    const SplitPlan& SP = P.split[l];
    const int nn = s.lev[l].size();
    if (SP.X.nout() == 0) continue;
    const long long xs = (long long)K * cl;
    Buf XS(ctx, (size_t)nn * xs * eb, bulk, cplx);
    gemm(st, pp, kKindOther, dl(SP.X), K, cl, cl, Op{bas(Urf[l], Ur[l]), nullptr, (long long)K * K, 0, K},
         false, Op{SNL[l].p(), nullptr, (long long)cl * cl, 0, cl}, false, XS.p(), xs, K, 0, 0, 1, 0);
    const Op XSo{XS.p(), nullptr, xs, 0, K, cc, 0};
    const Op TCc{bas(Ucf[l], Uc[l]), nullptr, (long long)K * K, 0, K, cc, 0};
    gemm(st, pp, kKindOther, dl(SP.toR), cc, cc, cl, XSo, false, TCc, true, C->S[ch].p(),
         (long long)cc * cc, cc, 0, 0, 1, 1);
    if (ch < L)
      gemm(st, pp, kKindOther, dl(SP.toNL), cc, cc, cl, XSo, false, TCc, true, SNL[ch].p(),
           (long long)cc * cc, cc, 0, 0, 1, 1);
    if (ch == L && SP.toF.nout() > 0) {
      Buf YF(ctx, (size_t)nnL * cc * cc * eb, bulk, cplx);
      Buf ZF(ctx, (size_t)nnL * np * cc * eb, bulk, cplx);
      gemm(st, pp, kKindOther, dl(SP.toF), cc, cc, cl, XSo, false, TCc, true, YF.p(),
           (long long)cc * cc, cc, 0, 0, 1, 0);
      gemm(st, pp, kKindOther, dl(SP.F1), np, cc, cc, Op{bas(Urf[L], Ur[L]), nullptr, nn2, 0, np}, false,
           Op{YF.p(), nullptr, (long long)cc * cc, 0, cc}, false, ZF.p(), (long long)np * cc, np,
           0, 0, 1, 0);
      gemm(st, pp, kKindOther, dl(SP.F2), np, np, cc, Op{ZF.p(), nullptr, (long long)np * cc, 0, np},
           false, Op{bas(Ucf[L], Uc[L]), nullptr, nn2, 0, np}, true, FC.p(), nn2, np, 0, 0, 1, 1);
    }
  }
  if (bulk) {
    // C is stored in FP64 like every matrix: widen the bulk-computed couplings
    // and dense blocks
    auto widen = [&](Buf& b) {
      const long long n = (long long)(b.bytes() / sizeof(float));
      if (n <= 0) return;
      Buf d(ctx, (size_t)n * sizeof(double));
      H2_HIP(h2k::launch_f2d(b.as<float>(), d.as<double>(), n, st));
      b = std::move(d);
    };
    for (int l = lmin; l <= L; ++l) widen(C->S[l]);
    widen(FC);
  }
  // the status flags were last read with the ranks of level l_min; nothing
  // after that level writes them
  H2_HIP(hipEventRecord(ev.b, st));
  if (prof.on) H2_HIP(hipStreamSynchronize(st));
  C->ev_begin = ev.a;
  C->ev_end = ev.b;
  C->timing_pending = true;
  ev.a = ev.b = nullptr;

  // ---------------------------------------------------------- assemble C
  for (int l = lmin; l <= L; ++l) {
    C->rr[l] = cpad[l];
    C->rc[l] = cpad[l];
  }
  C->cplx = cplx;
  C->V = std::move(Ur[L]);
  C->W = std::move(Uc[L]);
  C->V_stride = nn2;
  C->W_stride = nn2;
  for (int l = lmin; l < L; ++l) {
    C->Tr[l] = std::move(Ur[l]);
    C->Tc[l] = std::move(Uc[l]);
    C->Tr_stride[l] = 4LL * cpad[l + 1] * cpad[l + 1];
    C->Tc_stride[l] = C->Tr_stride[l];
  }
  C->F = std::move(FC);
  // stats
  h2_stats_t& S = C->stats;
  S.L = L;
  S.lmin = lmin;
  for (int l = 0; l <= L && l < H2_MAX_LEVELS; ++l) {
    long long mr = 0, mc = 0;
    double sr = 0, sc = 0;
    for (int c2 = 0; c2 < (1 << l); ++c2) {
      mr = std::max<long long>(mr, C->krow[cidx(l, c2)]);
      mc = std::max<long long>(mc, C->kcol[cidx(l, c2)]);
      sr += C->krow[cidx(l, c2)];
      sc += C->kcol[cidx(l, c2)];
    }
    S.rank_max_r[l] = mr;
    S.rank_max_c[l] = mc;
    S.rank_mean_r[l] = sr / (1 << l);
    S.rank_mean_c[l] = sc / (1 << l);
  }
  S.mmp_ms = 0.0;  // filled from the events by finish()
  S.symbolic_ms = sym_ms;
  S.n_triples = P.n_triples;
  S.sparsity_constant = s.sparsity_constant();
  C->flop_ranks = std::make_unique<FlopRanks>(
      FlopRanks{A->krow, A->kcol, B->krow, B->kcol, C->krow, C->kcol});
  C->flops_pending = true;
  S.bytes_device = (int64_t)ctx->peak_live;
  if (prof.on) {
    double pms[kKindCount], pfl[kKindCount];
    long long pl[kKindCount];
    prof.collect(pms, pl, pfl);
    S.contraction_ms = pms[kKindTriple];
    S.contraction_launches = pl[kKindTriple];
    S.contraction_flops = pfl[kKindTriple];
    S.eig_ms = pms[kKindEig] + pms[kKindEigVal] + pms[kKindEigVec];
    S.eig_launches = pl[kKindEig] + pl[kKindEigVal] + pl[kKindEigVec];
    S.eig_tri_ms = pms[kKindEig];
    S.eig_val_ms = pms[kKindEigVal];
    S.eig_vec_ms = pms[kKindEigVec];
    S.gram_ms = pms[kKindGram];
    S.gram_launches = pl[kKindGram];
    S.gram_flops = pfl[kKindGram];
    S.other_ms = pms[kKindOther];
    S.other_launches = pl[kKindOther];
    S.other_flops = pfl[kKindOther];
    S.target_ms = pms[kKindTarget];
    S.target_launches = pl[kKindTarget];
  }
  build_matvec_plan(ctx, C.get());
  *C_out = C.release();
  return H2_OK;
}

}  // namespace h2
