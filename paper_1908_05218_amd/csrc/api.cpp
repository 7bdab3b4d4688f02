// C-ABI of the h2mmp library: contexts, device memory pool, loading and
// exporting H^2 matrices, the exact H^2 mat-vec and dense expansion.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <exception>
#include <memory>
#include <thread>

#include "internal.h"

namespace h2 {

static thread_local std::string g_last_error;

h2_status set_error(h2_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

static hipEvent_t take_event(std::vector<hipEvent_t>* pool) {
  hipEvent_t e = nullptr;
  if (pool && !pool->empty()) {
    e = pool->back();
    pool->pop_back();
  } else {
    hipEventCreate(&e);
  }
  return e;
}

void Profiler::begin(int kind, double flops, hipEvent_t* out_a) {
  (void)kind;
  (void)flops;
  if (!on) return;
  *out_a = take_event(pool);
  hipEventRecord(*out_a, stream);
}

void Profiler::end(hipEvent_t a, int kind, double flops) {
  if (!on) return;
  hipEvent_t b = take_event(pool);
  hipEventRecord(b, stream);
  recs.push_back({a, b, kind, flops});
}

void Profiler::collect(double* ms, long long* launches, double* flops) {
  for (int k = 0; k < kKindCount; ++k) {
    ms[k] = 0;
    launches[k] = 0;
    flops[k] = 0;
  }
  for (auto& r : recs) {
    float t = 0;
    hipEventElapsedTime(&t, r.a, r.b);
    ms[r.kind] += t;
    launches[r.kind] += 1;
    flops[r.kind] += r.flops;
    if (pool) {
      pool->push_back(r.a);
      pool->push_back(r.b);
    } else {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
  }
  recs.clear();
}

thread_local h2_ctx g_active_ctx = nullptr;
thread_local bool g_bulk_f32 = false;

void scan_limits(const TaskList& t, DevList& d) {
  for (int v : t.a) d.max_a[(v >> 2) & 1] = std::max(d.max_a[(v >> 2) & 1], v >> 3);
  for (int v : t.b) d.max_b[(v >> 2) & 1] = std::max(d.max_b[(v >> 2) & 1], v >> 3);
  for (int v : t.out) d.max_out = std::max(d.max_out, v >> 3);
}

// Every block a launch can touch must lie inside the allocation its base
// pointer starts: checked on the host before the launch.
static void check_extent(const void* base, long long stride, int maxtile, long long sub_r,
                         long long sub_c, long long rows, long long cols, long long ld, size_t elt,
                         const char* what) {
  if (maxtile < 0) return;
  if (!base) throw Error(H2_ERR_INTERNAL, std::string(what) + ": null operand");
  if (ld < rows) throw Error(H2_ERR_INTERNAL, std::string(what) + ": leading dimension too small");
  if (!g_active_ctx) return;
  auto it = g_active_ctx->live.find(const_cast<void*>(base));
  if (it == g_active_ctx->live.end()) {
    it = g_active_ctx->ext.find(const_cast<void*>(base));
    if (it == g_active_ctx->ext.end())
      throw Error(H2_ERR_INTERNAL, std::string(what) + ": operand is not a live allocation");
  }
  const long long need = (long long)maxtile * stride + sub_r + sub_c + (rows - 1) + (cols - 1) * ld + 1;
  // a complex allocation is checked against its real plane (the imaginary
  // plane has the same layout one plane further)
  const long long pl = g_active_ctx->plane(base);
  if (pl > 0 && need > pl)
    throw Error(H2_ERR_INTERNAL, std::string(what) + ": block extent beyond its plane");
  if ((size_t)need * elt > it->second)
    throw Error(H2_ERR_INTERNAL, std::string(what) + ": block extent beyond its allocation (" +
                                     std::to_string(need * elt) + " > " +
                                     std::to_string(it->second) + " bytes)");
}

static size_t elt_of(const void* p) { return g_active_ctx ? g_active_ctx->elt(p) : 8; }

static h2k::Opnd to_opnd(const Op& o) {
  h2k::Opnd r;
  r.base[0] = o.base0;
  r.base[1] = o.base1 ? o.base1 : o.base0;
  r.stride[0] = o.stride0;
  r.stride[1] = o.base1 ? o.stride1 : o.stride0;
  r.ld = o.ld;
  r.sub_r = o.sub_r;
  r.sub_c = o.sub_c;
  r.f32 = elt_of(o.base0) == 4;
  if (o.base1 && elt_of(o.base1) != elt_of(o.base0))
    throw Error(H2_ERR_INTERNAL, "operand bases of different element types");
  return r;
}

template <typename T>
static void launch_gemm(hipStream_t s, Profiler* prof, int kind, const DevList& tl, int m, int n,
                        int k, const Op& A, bool tA, const Op& B, bool tB, void* C,
                        long long cstride, int ldc, long long csub_r, long long csub_c,
                        double alpha, double beta, bool lower = false) {
  h2k::BgemmArgs<T> a{};
  a.m = m;
  a.n = n;
  a.k = k;
  a.nout = tl.nout;
  a.transA = tA;
  a.transB = tB;
  a.A = to_opnd(A);
  a.B = to_opnd(B);
  a.C = C;
  a.c_f32 = elt_of(C) == 4;
  a.cstride = cstride;
  a.ldc = ldc;
  a.csub_r = csub_r;
  a.csub_c = csub_c;
  a.out_idx = tl.out;
  a.seg = tl.seg;
  a.a_idx = tl.a;
  a.b_idx = tl.b;
  a.alpha = (T)alpha;
  a.beta = (T)beta;
  a.symbol = kind == kKindTriple ? 1 : kind == kKindTarget ? 2 : kind == kKindGram ? 3 : 0;
  a.lower = lower ? 1 : 0;
  // the Gram sums share the tile table's keys with the other plain batches
  const std::string key = tile_key((int)sizeof(T), a.A.f32, a.B.f32, a.symbol == 3 ? 0 : a.symbol,
                                   tA, tB, m, n, k, tl.nout, (long long)tl.ntask);
  a.tile = tile_for(key);
  hipEvent_t ev = nullptr;
  // a symmetric output computed on and below its diagonal: n (n + 1) / 2 entries
  const double fl = 2.0 * (lower ? 0.5 * m * (n + 1.0) : (double)m * n) * k * tl.ntask;
  if (prof) prof->begin(kind, fl, &ev);
  if (tile_logging()) {
    hipEvent_t t0, t1;
    H2_HIP(hipEventCreate(&t0));
    H2_HIP(hipEventCreate(&t1));
    H2_HIP(hipEventRecord(t0, s));
    H2_HIP(h2k::launch_bgemm<T>(a, s));
    H2_HIP(hipEventRecord(t1, s));
    H2_HIP(hipEventSynchronize(t1));
    float ms = 0;
    hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    tile_log(key, a.tile, ms);
  } else {
    H2_HIP(h2k::launch_bgemm<T>(a, s));
  }
  if (prof) prof->end(ev, kind, fl);
}

// operand with its base pointers moved to the imaginary planes
static Op imag_of(const Op& o) {
  Op r = o;
  const long long p0 = g_active_ctx->plane(o.base0);
  r.base0 = (const double*)o.base0 + p0;
  if (o.base1) r.base1 = (const double*)o.base1 + g_active_ctx->plane(o.base1);
  return r;
}

static bool is_cplx(const void* p) { return g_active_ctx && p && g_active_ctx->plane(p) > 0; }

void gemm(hipStream_t s, Profiler* prof, int kind, const DevList& tl, int m, int n, int k,
          const Op& A, bool tA, const Op& B, bool tB, void* C, long long cstride, int ldc,
          long long csub_r, long long csub_c, double alpha, double beta, int conj) {
  if (tl.nout == 0) return;
  if (k % 16 != 0 || m <= 0 || n <= 0) throw Error(H2_ERR_INTERNAL, "gemm shape");
  {
    const long long ar = tA ? k : m, ac = tA ? m : k, br = tB ? n : k, bc = tB ? k : n;
    const void* a1 = A.base1 ? A.base1 : A.base0;
    const void* b1 = B.base1 ? B.base1 : B.base0;
    check_extent(A.base0, A.stride0, tl.max_a[0], A.sub_r, A.sub_c, ar, ac, A.ld, elt_of(A.base0),
                 "gemm A");
    check_extent(a1, A.base1 ? A.stride1 : A.stride0, tl.max_a[1], A.sub_r, A.sub_c, ar, ac, A.ld,
                 elt_of(a1), "gemm A(sel)");
    check_extent(B.base0, B.stride0, tl.max_b[0], B.sub_r, B.sub_c, br, bc, B.ld, elt_of(B.base0),
                 "gemm B");
    check_extent(b1, B.base1 ? B.stride1 : B.stride0, tl.max_b[1], B.sub_r, B.sub_c, br, bc, B.ld,
                 elt_of(b1), "gemm B(sel)");
    check_extent(C, cstride, tl.max_out, csub_r, csub_c, m, n, ldc, elt_of(C), "gemm C");
  }
  if (is_cplx(C)) {
    // (Ar + i sa Ai)(Br + i sb Bi): real part Ar Br - sa sb Ai Bi, imaginary
    // part sb Ar Bi + sa Ai Br; beta applies once per plane
    const bool ok = is_cplx(A.base0) && is_cplx(B.base0) && (!A.base1 || is_cplx(A.base1)) &&
                    (!B.base1 || is_cplx(B.base1));
    if (!ok) throw Error(H2_ERR_INTERNAL, "complex product with a real operand");
    const double sa = (conj & kConjA) ? -1.0 : 1.0, sb = (conj & kConjB) ? -1.0 : 1.0;
    const Op Ai = imag_of(A), Bi = imag_of(B);
    double* Cr = (double*)C;
    double* Ci = Cr + g_active_ctx->plane(C);
    auto run = [&](const Op& x, const Op& y, double* c, double al, double be) {
      launch_gemm<double>(s, prof, kind, tl, m, n, k, x, tA, y, tB, c, cstride, ldc, csub_r, csub_c,
                          al, be);
    };
    run(A, B, Cr, alpha, beta);
    run(Ai, Bi, Cr, -alpha * sa * sb, 1.0);
    run(A, Bi, Ci, alpha * sb, beta);
    run(Ai, B, Ci, alpha * sa, 1.0);
    return;
  }
  const bool lower = (conj & kLowerOnly) && m == n;
  if (g_bulk_f32 && kind != kKindGram)
    launch_gemm<float>(s, prof, kind, tl, m, n, k, A, tA, B, tB, C, cstride, ldc, csub_r, csub_c,
                       alpha, beta, lower);
  else
    launch_gemm<double>(s, prof, kind, tl, m, n, k, A, tA, B, tB, C, cstride, ldc, csub_r, csub_c,
                        alpha, beta, lower);
}

static void launch_segsum(hipStream_t s, const DevList& tl, int m, int n, const Op& A, void* C,
                          long long cstride, int ldc, long long csub_r, long long csub_c,
                          double beta) {
  h2k::SegsumArgs<double> a{};
  a.m = m;
  a.n = n;
  a.nout = tl.nout;
  a.A = to_opnd(A);
  a.C = (double*)C;
  a.cstride = cstride;
  a.ldc = ldc;
  a.csub_r = csub_r;
  a.csub_c = csub_c;
  a.out_idx = tl.out;
  a.seg = tl.seg;
  a.a_idx = tl.a;
  a.beta = beta;
  H2_HIP(h2k::launch_segsum<double>(a, s));
}

void segsum(hipStream_t s, const DevList& tl, int m, int n, const Op& A, void* C,
            long long cstride, int ldc, long long csub_r, long long csub_c, double beta) {
  if (tl.nout == 0) return;
  if (elt_of(A.base0) != 8 || elt_of(C) != 8) throw Error(H2_ERR_INTERNAL, "segsum: FP64 only");
  check_extent(A.base0, A.stride0, tl.max_a[0], A.sub_r, A.sub_c, m, n, A.ld, 8, "segsum A");
  check_extent(C, cstride, tl.max_out, csub_r, csub_c, m, n, ldc, 8, "segsum C");
  if (is_cplx(C) != is_cplx(A.base0)) throw Error(H2_ERR_INTERNAL, "segsum: mixed complex and real");
  launch_segsum(s, tl, m, n, A, C, cstride, ldc, csub_r, csub_c, beta);
  if (is_cplx(C))
    launch_segsum(s, tl, m, n, imag_of(A), (double*)C + g_active_ctx->plane(C), cstride, ldc,
                  csub_r, csub_c, beta);
}

void zero(hipStream_t s, void* p, long long n) {
  if (n > 0) H2_HIP(hipMemsetAsync(p, 0, (size_t)n * elt_of(p) * (is_cplx(p) ? 2 : 1), s));
}

const h2_mat_s& f32_shadow(h2_ctx ctx, h2_mat M, hipStream_t s) {
  if (M->f32) return *M->f32;
  auto S = std::make_unique<h2_mat_s>();
  auto cv = [&](const Buf& src) {
    Buf dst;
    const long long n = (long long)(src.bytes() / sizeof(double));
    if (n > 0) {
      dst = Buf(ctx, (size_t)n * sizeof(float), true);
      H2_HIP(h2k::launch_d2f(src.as<double>(), dst.as<float>(), n, s));
    }
    return dst;
  };
  S->ctx = ctx;
  S->shape = M->shape;
  S->rr = M->rr;
  S->rc = M->rc;
  S->V = cv(M->V);
  S->W = cv(M->W);
  S->V_stride = M->V_stride;
  S->W_stride = M->W_stride;
  for (const Buf& b : M->Tr) S->Tr.push_back(cv(b));
  for (const Buf& b : M->Tc) S->Tc.push_back(cv(b));
  S->Tr_stride = M->Tr_stride;
  S->Tc_stride = M->Tc_stride;
  for (const Buf& b : M->S) S->S.push_back(cv(b));
  S->F = cv(M->F);
  M->f32 = std::move(S);
  return *M->f32;
}

std::unique_ptr<DevPlan> upload_plan(h2_ctx ctx, const Plan& p) {
  std::vector<const TaskList*> all;
  auto addl = [&](const TaskList& t) { all.push_back(&t); };
  const LeafPlan& L = p.leaf;
  for (const TaskList* t :
       {&L.H, &L.X1, &L.G1, &L.G2, &L.G3, &L.Hc, &L.X1c, &L.G1c, &L.G2c, &L.G3c, &L.Z, &L.Zc,
        &L.gB, &L.hA, &L.PA, &L.PB, &L.LA_F, &L.PS, &L.LA_R, &L.RB_F, &L.SP, &L.RB_R, &L.Ahat,
        &L.Bhat, &L.adm_R, &L.adm_B, &L.dense, &L.densA1, &L.densA2, &L.densB1, &L.densB2})
    addl(*t);
  for (const LevelPlan& Q : p.lev)
    for (const TaskList* t :
         {&Q.G1, &Q.G1c, &Q.Y, &Q.G2, &Q.Yc, &Q.G2c, &Q.D, &Q.G3, &Q.Q, &Q.G3c, &Q.PA, &Q.PB,
          &Q.AhatNL, &Q.PAS, &Q.AhatR, &Q.BhatNL, &Q.SBP, &Q.BhatR, &Q.c1X, &Q.c1_R, &Q.c1_B,
          &Q.w_nl_R, &Q.w_nl_B, &Q.w_nl_NL, &Q.f_nl_R, &Q.f_nl_B, &Q.f_nl_NL, &Q.w_r_R,
          &Q.w_r_B, &Q.w_r_NL, &Q.f_r_R, &Q.f_r_B, &Q.f_r_NL, &Q.f_R, &Q.f_B, &Q.f_NL})
      addl(*t);
  for (const SplitPlan& S : p.split)
    for (const TaskList* t : {&S.X, &S.toR, &S.toNL, &S.toF, &S.F1, &S.F2}) addl(*t);
  addl(p.pi.leaf);
  for (const TaskList& t : p.pi.X) addl(t);
  for (const TaskList& t : p.pi.S) addl(t);
  size_t total = 0;
  for (const TaskList* t : all) total += t->out.size() + t->seg.size() + t->a.size() + t->b.size();
  std::vector<int> host(total + 1);
  auto dp = std::make_unique<DevPlan>();
  dp->mem = Buf(ctx, (total + 1) * sizeof(int));
  int* base = dp->mem.as<int>();
  size_t off = 0;
  for (const TaskList* t : all) {
    DevList d;
    d.nout = t->nout();
    d.ntask = t->ntask();
    auto put = [&](const std::vector<int>& v) -> const int* {
      std::copy(v.begin(), v.end(), host.begin() + off);
      const int* r = base + off;
      off += v.size();
      return r;
    };
    d.out = put(t->out);
    d.seg = put(t->seg);
    d.a = put(t->a);
    d.b = put(t->b);
    scan_limits(*t, d);
    dp->lists[t] = d;
  }
  H2_HIP(hipMemcpy(base, host.data(), total * sizeof(int), hipMemcpyHostToDevice));
  return dp;
}

static inline long long cidx(int l, int c) { return (1LL << l) - 1 + c; }

// ------------------------------------------------------------------ mat-vec
// Task lists of the exact H^2 mat-vec of M, built once per matrix: forward
// transform up the column tree, couplings per level, backward transform down
// the row tree, dense near field.  The host copy stays with the plan so that
// the upload needs no host wait.
void build_matvec_plan(h2_ctx ctx, h2_mat M) {
  if (M->shape->mv) {
    M->mv = M->shape->mv;
    return;
  }
  const Structure& s = M->st();
  const int L = s.L, nleaf = 1 << L, lo = s.lmin;
  auto mp = std::make_unique<MatvecPlan>();
  std::vector<TaskList> lists;
  // forward, leaves: xh_L(c) = W_c^T x_c
  {
    TaskList t;
    for (int c = 0; c < nleaf; ++c) {
      t.add_task(enc(c), enc(c));
      t.close(enc(c));
    }
    lists.push_back(std::move(t));
  }
  // forward, level l < L: xh_l(J) = sum over the two children E_j^T xh_{l+1}(j)
  for (int l = L - 1; l >= lo; --l) {
    TaskList t;
    for (int J = 0; J < (1 << l); ++J) {
      for (int a = 0; a < 2; ++a) t.add_task(enc(J, a), enc(2 * J + a));
      t.close(enc(J));
    }
    lists.push_back(std::move(t));
  }
  // couplings, level l: yh_l(I) = sum over admissible (I, J) of S_IJ xh_l(J)
  for (int l = lo; l <= L; ++l) {
    const LevelNodes& ln = s.lev[l];
    TaskList t;
    std::vector<std::vector<int>> byrow(1 << l);
    for (int q = 0; q < ln.size(); ++q)
      if (ln.type[q] == kR) byrow[ln.row[q]].push_back(q);
    for (int I = 0; I < (1 << l); ++I) {
      if (byrow[I].empty()) continue;
      for (int q : byrow[I]) t.add_task(enc(q), enc(ln.col[q]));
      t.close(enc(I));
    }
    lists.push_back(std::move(t));
  }
  // backward, level l < L: yh_{l+1}(c) += E_c yh_l(parent)
  for (int l = lo; l < L; ++l) {
    TaskList t;
    for (int c = 0; c < (2 << l); ++c) {
      t.add_task(enc(c >> 1, c & 1), enc(c >> 1));
      t.close(enc(c));
    }
    lists.push_back(std::move(t));
  }
  // leaves: y_c = V_c yh_L(c)
  {
    TaskList t;
    for (int c = 0; c < nleaf; ++c) {
      t.add_task(enc(c), enc(c));
      t.close(enc(c));
    }
    lists.push_back(std::move(t));
  }
  // dense near field: y_I += sum over dense (I, J) of F_IJ x_J
  {
    const LevelNodes& lf = s.lev[L];
    TaskList t;
    std::vector<std::vector<int>> byrow(nleaf);
    for (int q = 0; q < lf.size(); ++q)
      if (lf.type[q] == kF) byrow[lf.row[q]].push_back(q);
    for (int I = 0; I < nleaf; ++I) {
      if (byrow[I].empty()) continue;
      for (int q : byrow[I]) t.add_task(enc(q), enc(lf.col[q]));
      t.close(enc(I));
    }
    lists.push_back(std::move(t));
  }
  size_t total = 0;
  for (const TaskList& t : lists) total += t.out.size() + t.seg.size() + t.a.size() + t.b.size();
  mp->host.resize(total + 1);
  mp->mem = Buf(ctx, (total + 1) * sizeof(int));
  int* base = mp->mem.as<int>();
  size_t off = 0;
  for (const TaskList& t : lists) {
    DevList d;
    d.nout = t.nout();
    d.ntask = t.ntask();
    auto put = [&](const std::vector<int>& v) -> const int* {
      std::copy(v.begin(), v.end(), mp->host.begin() + off);
      const int* r = base + off;
      off += v.size();
      return r;
    };
    d.out = put(t.out);
    d.seg = put(t.seg);
    d.a = put(t.a);
    d.b = put(t.b);
    scan_limits(t, d);
    mp->lists.push_back(d);
  }
  H2_HIP(hipMemcpyAsync(base, mp->host.data(), total * sizeof(int), hipMemcpyHostToDevice,
                        ctx->stream));
  M->shape->mv = std::move(mp);
  M->mv = M->shape->mv;
}

// Device bytes of the mat-vec temporaries of M for nrhs right-hand sides
// (each part rounded to 256 bytes).
size_t matvec_scratch_bytes(const h2_mat_s* M, int64_t nrhs) {
  const Structure& s = M->st();
  const int L = s.L;
  const size_t nc = M->cplx ? 2 : 1;
  auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t b = 2 * r256((size_t)(1 << L) * s.npad * nrhs * nc * sizeof(double));
  for (int l = s.lmin; l <= L; ++l)
    b += r256((size_t)(1 << l) * M->rc[l] * nrhs * nc * sizeof(double)) +
         r256((size_t)(1 << l) * M->rr[l] * nrhs * nc * sizeof(double));
  return b;
}

// Exact H^2 mat-vec (the reference solution of equation `error`) on stream
// st.  scratch (nullable): a device region of scratch_bytes for the
// temporaries, checked against their size before any launch; without one
// they come from the context's pool.
void matvec_impl(h2_ctx ctx, h2_mat M, const double* x_dev, double* y_dev, int64_t nrhs,
                 hipStream_t st, void* scratch, size_t scratch_bytes) {
  ActiveCtx active(ctx);
  const Structure& s = M->st();
  Shape& sh = *M->shape;
  if (!M->mv) build_matvec_plan(ctx, M);
  const std::vector<DevList>& ml = M->mv->lists;
  const int L = s.L, np = s.npad, nleaf = 1 << L;
  const int lo = s.lmin;  // no admissible block above lmin
  const long long nt = (long long)nleaf * np;
  const int R = (int)nrhs;
  // complex: x and y planar (n x nrhs real parts, then the imaginary parts),
  // gathered and scattered as 2 nrhs real columns
  const int nc = M->cplx ? 2 : 1;
  const bool cx = M->cplx;
  // temporaries: pool buffers, or consecutive parts of the caller's region
  // registered with the context for the launches' extent checks
  std::vector<Buf> owned;
  std::vector<ExtRegion> regions;
  char* cursor = (char*)scratch;
  if (scratch && matvec_scratch_bytes(M, nrhs) > scratch_bytes)
    throw Error(H2_ERR_UNSUPPORTED,
                "the mat-vec temporaries (" + std::to_string(matvec_scratch_bytes(M, nrhs)) +
                    " bytes) exceed the scratch region of " + std::to_string(scratch_bytes) +
                    " bytes");
  regions.reserve(2 * (L + 2));
  auto take = [&](size_t bytes) -> double* {
    if (!scratch) {
      owned.emplace_back(ctx, bytes, false, cx);
      return owned.back().d();
    }
    double* p = (double*)cursor;
    cursor += (bytes + 255) & ~(size_t)255;
    regions.emplace_back(ctx, p, bytes, cx);
    return p;
  };
  owned.reserve(2 * (L + 2));
  double* xt = take(nt * R * nc * sizeof(double));
  double* yt = take(nt * R * nc * sizeof(double));
  H2_HIP(h2k::launch_gather_rows(x_dev, xt, sh.d_perm.as<long long>(),
                                 sh.d_leaf_off.as<long long>(), nleaf, np, s.n, R * nc, st));
  std::vector<double*> xh(L + 1, nullptr), yh(L + 1, nullptr);
  for (int l = lo; l <= L; ++l) {
    xh[l] = take((size_t)(1 << l) * M->rc[l] * R * nc * sizeof(double));
    yh[l] = take((size_t)(1 << l) * M->rr[l] * R * nc * sizeof(double));
    // a fill kernel, not a memset (the call may be captured in a graph)
    H2_HIP(h2k::launch_fill(yh[l], 0.0, (long long)(1 << l) * M->rr[l] * R * nc, st));
  }
  const long long ldx = nt;
  // independent branches on the helper streams (when the context has them):
  // the near field y_t = F x_t right after the gather, and each level's
  // couplings as soon as the forward sweep has produced that level; the
  // caller's stream joins them before the backward sweep and the leaf
  // expansion.  Events order the branches, so the call stays one stream
  // program (a graph with parallel branches when captured); the temporaries
  // return to the pool after the join, in the caller's stream order.
  const bool fork = ctx->aux[0] != nullptr;
  std::vector<int> used(h2_ctx_s::kAux, 0);
  // a call that fails between a fork and its join waits for the branches
  // before its temporaries go back to the pool
  struct Joined {
    h2_ctx c;
    const std::vector<int>& used;
    bool done = false;
    ~Joined() {
      if (done) return;
      for (int i = 0; i < h2_ctx_s::kAux; ++i)
        if (used[i]) (void)hipStreamSynchronize(c->aux[i]);
    }
  } joined{ctx, used};
  auto branch = [&](int i) -> hipStream_t {
    if (!fork) return st;
    H2_HIP(hipEventRecord(ctx->fork_ev, st));
    H2_HIP(hipStreamWaitEvent(ctx->aux[i], ctx->fork_ev, 0));
    used[i] = 1;
    return ctx->aux[i];
  };
  // task lists of the plan: forward (L - lo + 1), couplings (L - lo + 1),
  // backward (L - lo), leaves (1), near field (1)
  const size_t li_fwd = 0, li_cpl = li_fwd + (size_t)(L - lo + 1);
  const size_t li_bwd = li_cpl + (size_t)(L - lo + 1), li_leaf = li_bwd + (size_t)(L - lo);
  const size_t li_near = li_leaf + 1;
  {
    // the near field into y_t (zeroed by a fill kernel: a captured call
    // records no memset)
    const hipStream_t sd = branch(0);
    H2_HIP(h2k::launch_fill(yt, 0.0, nt * R * nc, sd));
    Op A{M->F.d(), nullptr, (long long)np * np, 0, np, 0, 0};
    Op B{xt, nullptr, np, 0, (int)ldx, 0, 0};
    gemm(sd, nullptr, 0, ml[li_near], np, R, np, A, false, B, false, yt, np, (int)ldx, 0, 0, 1.0,
         1.0);
  }
  auto couplings = [&](int l) {
    const DevList& d = ml[li_cpl + (size_t)(l - lo)];
    if (d.nout == 0) return;
    const hipStream_t sc = branch(1 + (l % (h2_ctx_s::kAux - 1)));
    Op A{M->S[l].d(), nullptr, (long long)M->rr[l] * M->rc[l], 0, M->rr[l], 0, 0};
    Op B{xh[l], nullptr, (long long)M->rc[l] * R, 0, M->rc[l], 0, 0};
    gemm(sc, nullptr, 0, d, M->rr[l], R, M->rc[l], A, false, B, false, yh[l],
         (long long)M->rr[l] * R, M->rr[l], 0, 0, 1.0, 1.0);
  };
  // forward, each level's couplings forked once its coefficients exist
  {
    Op A{M->W.d(), nullptr, M->W_stride, 0, np, 0, 0};
    Op B{xt, nullptr, np, 0, (int)ldx, 0, 0};
    gemm(st, nullptr, 0, ml[li_fwd], M->rc[L], R, np, A, true, B, false, xh[L],
         (long long)M->rc[L] * R, M->rc[L], 0, 0, 1.0, 0.0);
    couplings(L);
  }
  for (int l = L - 1; l >= lo; --l) {
    Op A{M->Tc[l].d(), nullptr, M->Tc_stride[l], 0, 2 * M->rc[l + 1], M->rc[l + 1], 0};
    Op B{xh[l + 1], nullptr, (long long)M->rc[l + 1] * R, 0, M->rc[l + 1], 0, 0};
    gemm(st, nullptr, 0, ml[li_fwd + (size_t)(L - l)], M->rc[l], R, M->rc[l + 1], A, true, B,
         false, xh[l], (long long)M->rc[l] * R, M->rc[l], 0, 0, 1.0, 0.0);
    couplings(l);
  }
  size_t li = li_bwd;
  // join the couplings before the backward sweep
  for (int i = 1; i < h2_ctx_s::kAux; ++i)
    if (used[i]) {
      H2_HIP(hipEventRecord(ctx->join_ev[i], ctx->aux[i]));
      H2_HIP(hipStreamWaitEvent(st, ctx->join_ev[i], 0));
    }
  // backward
  for (int l = lo; l < L; ++l) {
    Op A{M->Tr[l].d(), nullptr, M->Tr_stride[l], 0, 2 * M->rr[l + 1], M->rr[l + 1], 0};
    Op B{yh[l], nullptr, (long long)M->rr[l] * R, 0, M->rr[l], 0, 0};
    gemm(st, nullptr, 0, ml[li++], M->rr[l + 1], R, M->rr[l], A, false, B, false, yh[l + 1],
         (long long)M->rr[l + 1] * R, M->rr[l + 1], 0, 0, 1.0, 1.0);
  }
  // the near field must be complete before the leaf expansion adds to y_t
  if (used[0]) {
    H2_HIP(hipEventRecord(ctx->join_ev[0], ctx->aux[0]));
    H2_HIP(hipStreamWaitEvent(st, ctx->join_ev[0], 0));
  }
  joined.done = true;
  {
    Op A{M->V.d(), nullptr, M->V_stride, 0, np, 0, 0};
    Op B{yh[L], nullptr, (long long)M->rr[L] * R, 0, M->rr[L], 0, 0};
    gemm(st, nullptr, 0, ml[li++], np, R, M->rr[L], A, false, B, false, yt, np, (int)ldx, 0, 0,
         1.0, 1.0);
  }
  H2_HIP(h2k::launch_scatter_rows(yt, y_dev, sh.d_perm.as<long long>(),
                                  sh.d_leaf_off.as<long long>(), nleaf, np, s.n, R * nc, st));
}

}  // namespace h2

// ------------------------------------------------------------------ context
// Allocation sizes are rounded to classes: whole pages up to 1 MiB, above
// that eight classes per power of two (at most 12.5% rounding), so that the
// per-level temporaries of one product, and products of nearby sizes, reuse
// each other's cached blocks.
static size_t size_class(size_t b) {
  b = (b + 4095) & ~(size_t)4095;
  if (b <= ((size_t)1 << 20)) return b;
  const int e = 63 - __builtin_clzll((unsigned long long)b);
  const size_t step = (size_t)1 << (e - 3);
  return (b + step - 1) & ~(step - 1);
}

void* h2_ctx_s::alloc(size_t bytes, bool is_f32, bool is_cplx) {
  void* p = alloc_raw(bytes, is_f32);
  if (is_cplx) planes[p] = (long long)(bytes / 16);
  return p;
}

void* h2_ctx_s::alloc_raw(size_t bytes, bool is_f32) {
  if (n_alloc++ == fail_alloc)
    throw h2::Error(H2_ERR_OOM, "allocation " + std::to_string(fail_alloc) +
                                    " refused (H2_FAIL_ALLOC)");
  bytes = size_class(bytes);
  // best fit among the cached blocks, wasting at most a quarter
  auto it = pool.lower_bound(bytes);
  if (it != pool.end() && it->first <= bytes + bytes / 4) {
    void* p = it->second;
    const size_t got = it->first;
    pool.erase(it);
    pooled -= got;
    live[p] = got;
    live_bytes += got;
    peak_live = std::max(peak_live, live_bytes);
    if (is_f32) f32.insert(p);
    return p;
  }
  if (budget && used + bytes > budget) {
    // release cached blocks first
    for (auto& kv : pool) {
      hipFree(kv.second);
      used -= kv.first;
    }
    pool.clear();
    pooled = 0;
    if (used + bytes > budget)
      throw h2::Error(H2_ERR_OOM, "device memory budget exceeded (" + std::to_string(used + bytes) +
                                      " > " + std::to_string(budget) + " bytes)");
  }
  void* p = nullptr;
  if (has_hook) {
    // the supplier pools on its own: hand out its block directly
    p = hook.alloc(hook.user, bytes, device, stream);
    if (!p) throw h2::Error(H2_ERR_OOM, "the context's allocator has no " + std::to_string(bytes) +
                                            " bytes");
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    // the failed call leaves its error as the thread's last error, which the
    // next launch check would report: clear it before the retry
    (void)hipGetLastError();
    for (auto& kv : pool) {
      hipFree(kv.second);
      used -= kv.first;
    }
    pool.clear();
    pooled = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw h2::Error(H2_ERR_OOM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
  }
  used += bytes;
  live[p] = bytes;
  live_bytes += bytes;
  peak_live = std::max(peak_live, live_bytes);
  if (is_f32) f32.insert(p);
  return p;
}

void h2_ctx_s::trim(size_t keep) {
  if (pooled <= keep) return;
  if (stream) hipStreamSynchronize(stream);
  while (pooled > keep && !pool.empty()) {
    auto it = std::prev(pool.end());
    hipFree(it->second);
    used -= it->first;
    pooled -= it->first;
    pool.erase(it);
  }
}

void h2_ctx_s::end_call(size_t start) {
  const size_t base = std::min(start, live_bytes);
  trim(2 * (peak_live > base ? peak_live - base : 0));
}

void h2_ctx_s::release(void* p) {
  auto it = live.find(p);
  if (it == live.end()) return;
  if (has_hook) {
    // stream-ordered supplier: it may reuse the block for later work on this
    // context's stream only
    hook.free(hook.user, p, it->second, device, stream);
    used -= it->second;
  } else {
    pool.emplace(it->second, p);
    pooled += it->second;
  }
  live_bytes -= it->second;
  live.erase(it);
  f32.erase(p);
  planes.erase(p);
}

h2_ctx_s::~h2_ctx_s() {
  if (stream) hipStreamSynchronize(stream);
  for (auto& kv : pool) hipFree(kv.second);
  for (auto& kv : live) {
    if (has_hook)
      hook.free(hook.user, kv.first, kv.second, device, stream);
    else
      hipFree(kv.first);
  }
  for (int i = 0; i < kAux; ++i) {
    if (aux[i]) {
      hipStreamSynchronize(aux[i]);
      hipStreamDestroy(aux[i]);
    }
    if (join_ev[i]) hipEventDestroy(join_ev[i]);
  }
  if (fork_ev) hipEventDestroy(fork_ev);
  if (rb_ev) hipEventDestroy(rb_ev);
  for (hipEvent_t e : prof_events) hipEventDestroy(e);
  if (rb_host) hipHostFree(rb_host);
  if (stream) hipStreamDestroy(stream);
}

int* h2_ctx_s::readback(size_t n) {
  if (!rb_ev) H2_HIP(hipEventCreateWithFlags(&rb_ev, hipEventDisableTiming));
  if (n > rb_n) {
    if (rb_host) {
      // a call that failed between posting and reading may leave copies in flight
      H2_HIP(hipEventSynchronize(rb_ev));
      H2_HIP(hipHostFree(rb_host));
      rb_host = nullptr;
      rb_n = 0;
    }
    const size_t cap = std::max<size_t>(n, 4096);
    H2_HIP(hipHostMalloc((void**)&rb_host, cap * sizeof(int), hipHostMallocDefault));
    rb_n = cap;
  }
  return rb_host;
}

void h2_mat_s::finish() {
  if (ev_end) {
    if (hipEventSynchronize(ev_end) != hipSuccess)
      throw h2::Error(H2_ERR_DEVICE, "a launch of the product failed");
  }
  if (timing_pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev_begin, ev_end) == hipSuccess) stats.mmp_ms = ms;
    (void)hipGetLastError();
    timing_pending = false;
  }
}

h2_mat_s::~h2_mat_s() {
  // the context's stream may still run the launches that write M: the pool
  // (or supplier) reuses its blocks only for later work on that stream
  if (ev_begin) hipEventDestroy(ev_begin);
  if (ev_end) hipEventDestroy(ev_end);
}

extern "C" {

const char* h2_last_error(void) { return h2::g_last_error.c_str(); }
int h2_version(void) { return 1; }

h2_status h2_ctx_create(int device, size_t hbm_budget, const h2_allocator* alloc, h2_ctx* out) {
  if (!out) return h2::set_error(H2_ERR_ARG, "out is null");
  if (alloc && (!alloc->alloc || !alloc->free))
    return h2::set_error(H2_ERR_ARG, "an allocator needs both alloc and free");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return h2::set_error(H2_ERR_DEVICE, "no HIP device " + std::to_string(device));
  }
  if (hipSetDevice(device) != hipSuccess) return h2::set_error(H2_ERR_DEVICE, "hipSetDevice failed");
  auto* c = new h2_ctx_s();
  c->device = device;
  c->budget = hbm_budget;
  if (const char* f = std::getenv("H2_FAIL_ALLOC")) c->fail_alloc = std::atoll(f);
  if (alloc) {
    c->hook = *alloc;
    c->has_hook = true;
  }
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return h2::set_error(H2_ERR_DEVICE, "hipStreamCreate failed");
  }
  // the mat-vec's helper streams (default priority) and events
  bool aux_ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < h2_ctx_s::kAux && aux_ok; ++i)
    aux_ok = hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!aux_ok) {
    delete c;
    return h2::set_error(H2_ERR_DEVICE, "creating the mat-vec's helper streams failed");
  }
  // the allocation-free mat-vec's scratch array of this device
  if (h2::noalloc_setup(device) != H2_OK) {
    delete c;
    return H2_ERR_DEVICE;  // message set by noalloc_setup
  }
  *out = c;
  return H2_OK;
}

void h2_ctx_destroy(h2_ctx ctx) {
  if (!ctx) return;
  h2::stop_server(ctx);
  delete ctx;
}

h2_status h2_set_profiling(h2_ctx ctx, int on) {
  if (!ctx) return h2::set_error(H2_ERR_ARG, "null context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->profiling = on != 0;
  return H2_OK;
}

}  // extern "C"

namespace h2 {

// Upload of a host matrix.  device_blocks: the couplings and dense blocks are
// left zero on the device for the caller to fill (S, F and their offsets are
// not read).
// f(begin, end) over [0, n) split across host threads (one range when n is
// small); the first exception of any range is rethrown
template <typename F>
static void parallel_ranges(long long n, F&& f) {
  const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
  const long long nt = n < 256 ? 1 : std::min<long long>(std::min(16u, hc), n / 128);
  if (nt <= 1) {
    f(0LL, n);
    return;
  }
  std::exception_ptr ep;
  std::mutex emu;
  std::vector<std::thread> th;
  for (long long t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        f(n * t / nt, n * (t + 1) / nt);
      } catch (...) {
        std::lock_guard<std::mutex> g(emu);
        if (!ep) ep = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  if (ep) std::rethrow_exception(ep);
}

h2_status load_impl(h2_ctx ctx, const h2_host_matrix* m, bool device_blocks, h2_mat* out) {
  if (!ctx || !m || !out) return set_error(H2_ERR_ARG, "null argument");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ActiveCtx active(ctx);
  try {
    hipSetDevice(ctx->device);
    auto shape = std::make_shared<Shape>();
    std::string err = build_structure(shape->s, m->n, m->L, m->leaf_off, m->perm, m->node_off,
                                      m->node_row, m->node_col, m->node_type);
    if (!err.empty()) return set_error(H2_ERR_ARG, err);
    const Structure& s = shape->s;
    const int L = s.L, np = s.npad, nleaf = 1 << L;
    if (!m->krow || !m->kcol || !m->V || !m->W || !m->V_off || !m->W_off || !m->Er_off ||
        !m->Ec_off || (!device_blocks && (!m->S_off || !m->F_off)))
      return set_error(H2_ERR_ARG, "null matrix array");
    const long long ncl = (2LL << L) - 1;
    auto M = std::make_unique<h2_mat_s>();
    M->ctx = ctx;
    M->shape = shape;
    M->cplx = m->is_complex != 0;
    // complex input: interleaved (real, imaginary) pairs; on the device two
    // planes [real | imaginary] per buffer
    const int nc = M->cplx ? 2 : 1;
    auto upload_n = [&](const double* h, size_t count) {
      Buf b(ctx, count * sizeof(double), false, M->cplx);
      if (count) H2_HIP(hipMemcpy(b.d(), h, count * sizeof(double), hipMemcpyHostToDevice));
      return b;
    };
    auto upload = [&](const std::vector<double>& h) { return upload_n(h.data(), h.size()); };
    M->krow.assign(m->krow, m->krow + ncl);
    M->kcol.assign(m->kcol, m->kcol + ncl);
    M->rr.assign(L + 1, 16);
    M->rc.assign(L + 1, 16);
    for (int l = 0; l <= L; ++l)
      for (int c = 0; c < (1 << l); ++c) {
        const int64_t kr = M->krow[cidx(l, c)], kc = M->kcol[cidx(l, c)];
        if (kr < 0 || kc < 0 || kr > 4096 || kc > 4096) return set_error(H2_ERR_ARG, "bad rank");
        M->rr[l] = std::max(M->rr[l], pad16(kr));
        M->rc[l] = std::max(M->rc[l], pad16(kc));
      }
    // element count checks
    auto need = [&](const int64_t* off, long long i, long long len, const char* what) {
      if (off[i + 1] - off[i] != len)
        throw Error(H2_ERR_ARG, std::string("size mismatch in ") + what + " entry " + std::to_string(i));
    };
    // leaf bases
    auto upload_leaf = [&](const double* src, const int64_t* off, const std::vector<int64_t>& kk,
                           int rpad, Buf& dst, long long& stride, const char* what) {
      stride = (long long)np * rpad;
      const size_t pl = (size_t)stride * nleaf;
      std::vector<double> h(pl * nc, 0.0);
      for (int c = 0; c < nleaf; ++c) {
        const int nr = s.leaf_size[c];
        const int k = (int)kk[cidx(L, c)];
        need(off, c, (long long)nr * k, what);
        for (int j = 0; j < k; ++j)
          for (int i = 0; i < nr; ++i)
            for (int part = 0; part < nc; ++part) {
              const double v = src[(off[c] + i + (size_t)j * nr) * nc + part];
              if (!std::isfinite(v)) throw Error(H2_ERR_NUMERIC, std::string("non-finite entry in ") + what);
              h[part * pl + (size_t)c * stride + i + (size_t)j * np] = v;
            }
      }
      dst = upload(h);
    };
    upload_leaf(m->V, m->V_off, M->krow, M->rr[L], M->V, M->V_stride, "V");
    upload_leaf(m->W, m->W_off, M->kcol, M->rc[L], M->W, M->W_stride, "W");
    auto upload_tr = [&](const double* src, const int64_t* off, const std::vector<int64_t>& kk,
                         const std::vector<int>& rp, std::vector<Buf>& dst,
                         std::vector<long long>& stride, const char* what) {
      dst.clear();
      dst.resize(L);
      stride.assign(L, 0);
      for (int l = 0; l < L; ++l) {
        const int ld = 2 * rp[l + 1];
        stride[l] = (long long)ld * rp[l];
        const size_t pl = (size_t)stride[l] * (1 << l);
        std::vector<double> h(pl * nc, 0.0);
        for (int I = 0; I < (1 << l); ++I)
          for (int a = 0; a < 2; ++a) {
            const int c = 2 * I + a;
            const long long fi = cidx(l + 1, c);
            const int kc_ = (int)kk[fi], kp = (int)kk[cidx(l, I)];
            need(off, fi, (long long)kc_ * kp, what);
            if (kc_ * kp && !src) throw Error(H2_ERR_ARG, "null transfer array");
            for (int j = 0; j < kp; ++j)
              for (int i = 0; i < kc_; ++i)
                for (int part = 0; part < nc; ++part) {
                  const double v = src[(off[fi] + i + (size_t)j * kc_) * nc + part];
                  if (!std::isfinite(v)) throw Error(H2_ERR_NUMERIC, std::string("non-finite entry in ") + what);
                  h[part * pl + (size_t)I * stride[l] + a * rp[l + 1] + i + (size_t)j * ld] = v;
                }
          }
        dst[l] = upload(h);
      }
    };
    upload_tr(m->Er, m->Er_off, M->krow, M->rr, M->Tr, M->Tr_stride, "Er");
    upload_tr(m->Ec, m->Ec_off, M->kcol, M->rc, M->Tc, M->Tc_stride, "Ec");
    M->S.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
      const LevelNodes& ln = s.lev[l];
      const long long bs = (long long)M->rr[l] * M->rc[l];
      const size_t pl = (size_t)bs * std::max(1, ln.size());
      if (device_blocks) {
        M->S[l] = Buf(ctx, pl * nc * sizeof(double), false, M->cplx);
        zero(ctx->stream, M->S[l].p(), (long long)pl);
        continue;
      }
      // each node's slot (zero padding included) is written by one thread
      std::unique_ptr<double[]> h(new double[pl * nc]);
      if (ln.size() == 0) std::fill(h.get(), h.get() + pl * nc, 0.0);
      parallel_ranges(ln.size(), [&](long long q0, long long q1) {
        for (long long q = q0; q < q1; ++q) {
          for (int part = 0; part < nc; ++part)
            std::fill(h.get() + part * pl + (size_t)q * bs, h.get() + part * pl + (size_t)(q + 1) * bs,
                      0.0);
          const long long g = s.node_base[l] + q;
          if (ln.type[q] != kR) {
            need(m->S_off, g, 0, "S");
            continue;
          }
          const int kr = (int)M->krow[cidx(l, ln.row[q])], kc = (int)M->kcol[cidx(l, ln.col[q])];
          need(m->S_off, g, (long long)kr * kc, "S");
          for (int j = 0; j < kc; ++j)
            for (int i = 0; i < kr; ++i)
              for (int part = 0; part < nc; ++part) {
                const double v = m->S[(m->S_off[g] + i + (size_t)j * kr) * nc + part];
                if (!std::isfinite(v)) throw Error(H2_ERR_NUMERIC, "non-finite coupling entry");
                h[part * pl + (size_t)q * bs + i + (size_t)j * M->rr[l]] = v;
              }
        }
      });
      M->S[l] = upload_n(h.get(), pl * nc);
    }
    if (device_blocks) {
      const long long nb = (long long)np * np * s.lev[L].size();
      M->F = Buf(ctx, (size_t)nb * nc * sizeof(double), false, M->cplx);
      zero(ctx->stream, M->F.p(), nb);
    } else {
      const LevelNodes& ln = s.lev[L];
      const long long bs = (long long)np * np;
      const size_t pl = (size_t)bs * ln.size();
      std::unique_ptr<double[]> h(new double[pl * nc]);
      parallel_ranges(ln.size(), [&](long long q0, long long q1) {
        for (long long q = q0; q < q1; ++q) {
          for (int part = 0; part < nc; ++part)
            std::fill(h.get() + part * pl + (size_t)q * bs, h.get() + part * pl + (size_t)(q + 1) * bs,
                      0.0);
          const long long g = s.node_base[L] + q;
          if (ln.type[q] != kF) {
            need(m->F_off, g, 0, "F");
            continue;
          }
          const int ni = s.leaf_size[ln.row[q]], nj = s.leaf_size[ln.col[q]];
          need(m->F_off, g, (long long)ni * nj, "F");
          if (!m->F) throw Error(H2_ERR_ARG, "null F");
          for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i)
              for (int part = 0; part < nc; ++part) {
                const double v = m->F[(m->F_off[g] + i + (size_t)j * ni) * nc + part];
                if (!std::isfinite(v)) throw Error(H2_ERR_NUMERIC, "non-finite dense entry");
                h[part * pl + (size_t)q * bs + i + (size_t)j * np] = v;
              }
        }
      });
      M->F = upload_n(h.get(), pl * nc);
    }
    shape->d_perm = Buf(ctx, s.n * sizeof(long long));
    shape->d_leaf_off = Buf(ctx, (nleaf + 1) * sizeof(long long));
    H2_HIP(hipMemcpy(shape->d_perm.as<long long>(), s.perm.data(), s.n * sizeof(long long),
                     hipMemcpyHostToDevice));
    H2_HIP(hipMemcpy(shape->d_leaf_off.as<long long>(), s.leaf_off.data(),
                     (nleaf + 1) * sizeof(long long), hipMemcpyHostToDevice));
    M->stats.L = L;
    M->stats.lmin = s.lmin;
    M->stats.sparsity_constant = s.sparsity_constant();
    build_matvec_plan(ctx, M.get());
    *out = M.release();
    return H2_OK;
  } catch (const Error& e) {
    return set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}

}  // namespace h2

extern "C" {

h2_status h2_load(h2_ctx ctx, const h2_host_matrix* m, h2_mat* out) {
  return h2::load_impl(ctx, m, false, out);
}

// Orders the context's stream after the work queued on the caller's stream
// so far (no-op for a null stream or the context's own).
static void fence_in(h2_ctx ctx, hipStream_t caller) {
  if (!caller || caller == ctx->stream) return;
  hipEvent_t ev;
  H2_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  H2_HIP(hipEventRecord(ev, caller));
  const hipError_t e = hipStreamWaitEvent(ctx->stream, ev, 0);
  hipEventDestroy(ev);
  H2_HIP(e);
}

// Orders later work on the caller's stream after the context's stream, or,
// for a null caller stream, waits for the context's stream.
static void fence_out(h2_ctx ctx, hipStream_t caller) {
  if (!caller) {
    H2_HIP(hipStreamSynchronize(ctx->stream));
    return;
  }
  if (caller == ctx->stream) return;
  hipEvent_t ev;
  H2_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  H2_HIP(hipEventRecord(ev, ctx->stream));
  const hipError_t e = hipStreamWaitEvent(caller, ev, 0);
  hipEventDestroy(ev);
  H2_HIP(e);
}

h2_status h2_mmp(h2_ctx ctx, h2_mat A, h2_mat B, double eps, int trunc_mode, int precision,
                 hipStream_t stream, h2_mat* C_out) {
  using namespace h2;
  if (!ctx || !A || !B || !C_out) return set_error(H2_ERR_ARG, "null argument");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return set_error(H2_ERR_ARG, "eps must be finite and >= 0");
  if (trunc_mode < 0 || trunc_mode > 3) return set_error(H2_ERR_ARG, "bad truncation mode");
  if (precision < 0 || precision > 1) return set_error(H2_ERR_ARG, "bad precision");
  if (A->shape != B->shape && !A->st().same_as(B->st()))
    return set_error(H2_ERR_STRUCTURE, "A and B differ in tree or block partition");
  {
    h2_ctx ha = home_of(ctx, A), hb = home_of(ctx, B);
    if (!ha || ha != hb)
      return set_error(H2_ERR_ARG, "A and B must both belong to ctx (or to one served result)");
    ctx = ha;
  }
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ActiveCtx active(ctx);
  const size_t start = ctx->live_bytes;
  ctx->mark();
  h2_status r;
  try {
    hipSetDevice(ctx->device);
    fence_in(ctx, stream);
    r = mmp_impl(ctx, A, B, eps, trunc_mode, precision, C_out);
    if (r == H2_OK) {
      try {
        fence_out(ctx, stream);
        if (!stream) (*C_out)->finish();
      } catch (...) {
        h2_free(*C_out);
        *C_out = nullptr;
        throw;
      }
    }
  } catch (const Error& e) {
    (void)hipGetLastError();
    r = set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    r = set_error(H2_ERR_INTERNAL, e.what());
  }
  ctx->end_call(start);
  return r;
}

h2_status h2_sync(h2_mat M) {
  using namespace h2;
  if (!M) return set_error(H2_ERR_ARG, "null matrix");
  std::unique_lock<std::recursive_mutex> lk;
  if (M->ctx) lk = std::unique_lock<std::recursive_mutex>(M->ctx->mu);
  try {
    if (M->ctx) hipSetDevice(M->ctx->device);
    M->finish();
    if (M->ctx) H2_HIP(hipStreamSynchronize(M->ctx->stream));
    return H2_OK;
  } catch (const Error& e) {
    (void)hipGetLastError();
    return set_error(e.code, e.msg);
  }
}

h2_status h2_matvec(h2_ctx ctx, h2_mat M, const double* x, double* y, int64_t nrhs,
                    int x_on_device, hipStream_t stream) {
  using namespace h2;
  if (!ctx || !M || !x || !y || nrhs < 1) return set_error(H2_ERR_ARG, "bad argument");
  ctx = home_of(ctx, M);
  if (!ctx) return set_error(H2_ERR_ARG, "M belongs to another context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ActiveCtx active(ctx);
  try {
    hipSetDevice(ctx->device);
    const long long n = M->st().n;
    const long long len = n * nrhs * (M->cplx ? 2 : 1);
    if (x_on_device) {
      fence_in(ctx, stream);
      matvec_impl(ctx, M, x, y, nrhs, ctx->stream);
      fence_out(ctx, stream);
    } else {
      Buf xd(ctx, len * sizeof(double)), yd(ctx, len * sizeof(double));
      fence_in(ctx, stream);
      H2_HIP(hipMemcpyAsync(xd.d(), x, len * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      matvec_impl(ctx, M, xd.d(), yd.d(), nrhs, ctx->stream);
      H2_HIP(hipMemcpyAsync(y, yd.d(), len * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      H2_HIP(hipStreamSynchronize(ctx->stream));
    }
    return H2_OK;
  } catch (const Error& e) {
    return set_error(e.code, e.msg);
  }
}

h2_status h2_to_dense(h2_ctx ctx, h2_mat M, double* out, int64_t ld) {
  using namespace h2;
  if (!ctx || !M || !out) return set_error(H2_ERR_ARG, "null argument");
  const long long n = M->st().n;
  if (ld < n) return set_error(H2_ERR_ARG, "ld < n");
  if (n > 16384) return set_error(H2_ERR_UNSUPPORTED, "to_dense is limited to n <= 16384");
  ctx = home_of(ctx, M);
  if (!ctx) return set_error(H2_ERR_ARG, "M belongs to another context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ActiveCtx active(ctx);
  try {
    hipSetDevice(ctx->device);
    // complex: the identity's imaginary plane is zero; out holds interleaved pairs
    const int nc = M->cplx ? 2 : 1;
    const size_t nn = (size_t)n * n;
    std::vector<double> eye(nn * nc, 0.0);
    for (long long i = 0; i < n; ++i) eye[(size_t)i * n + i] = 1.0;
    Buf xd(ctx, nn * nc * sizeof(double)), yd(ctx, nn * nc * sizeof(double));
    H2_HIP(hipMemcpyAsync(xd.d(), eye.data(), nn * nc * sizeof(double), hipMemcpyHostToDevice,
                          ctx->stream));
    matvec_impl(ctx, M, xd.d(), yd.d(), n, ctx->stream);
    H2_HIP(hipMemcpyAsync(eye.data(), yd.d(), nn * nc * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    H2_HIP(hipStreamSynchronize(ctx->stream));
    for (long long j = 0; j < n; ++j)
      for (long long i = 0; i < n; ++i)
        for (int part = 0; part < nc; ++part)
          out[(j * ld + i) * nc + part] = eye[part * nn + (size_t)j * n + i];
    return H2_OK;
  } catch (const Error& e) {
    return set_error(e.code, e.msg);
  }
}

h2_status h2_export_size(h2_mat M, h2_export_sizes* sz) {
  using namespace h2;
  if (!M || !sz) return set_error(H2_ERR_ARG, "null argument");
  const Structure& s = M->st();
  const int L = s.L;
  memset(sz, 0, sizeof(*sz));
  sz->n = s.n;
  sz->L = L;
  sz->nnodes = s.node_base[L + 1];
  sz->is_complex = M->cplx ? 1 : 0;
  for (int c = 0; c < (1 << L); ++c) {
    sz->len_V += (int64_t)s.leaf_size[c] * M->krow[cidx(L, c)];
    sz->len_W += (int64_t)s.leaf_size[c] * M->kcol[cidx(L, c)];
  }
  for (int l = 1; l <= L; ++l)
    for (int c = 0; c < (1 << l); ++c) {
      sz->len_Er += M->krow[cidx(l, c)] * M->krow[cidx(l - 1, c >> 1)];
      sz->len_Ec += M->kcol[cidx(l, c)] * M->kcol[cidx(l - 1, c >> 1)];
    }
  for (int l = 0; l <= L; ++l) {
    const LevelNodes& ln = s.lev[l];
    for (int q = 0; q < ln.size(); ++q) {
      if (ln.type[q] == kR) sz->len_S += M->krow[cidx(l, ln.row[q])] * M->kcol[cidx(l, ln.col[q])];
      if (ln.type[q] == kF) sz->len_F += (int64_t)s.leaf_size[ln.row[q]] * s.leaf_size[ln.col[q]];
    }
  }
  return H2_OK;
}

h2_status h2_export(h2_mat M, const h2_export_buffers* o) {
  if (M && M->ctx) M->ctx->mu.lock();
  struct Unlock {
    h2_mat m;
    ~Unlock() {
      if (m && m->ctx) m->ctx->mu.unlock();
    }
  } unlock_{M};
  using namespace h2;
  if (!M || !o) return set_error(H2_ERR_ARG, "null argument");
  try {
    hipSetDevice(M->ctx->device);
    H2_HIP(hipStreamSynchronize(M->ctx->stream));
    const Structure& s = M->st();
    const int L = s.L, np = s.npad, nleaf = 1 << L;
    const long long ncl = (2LL << L) - 1;
    memcpy(o->leaf_off, s.leaf_off.data(), (nleaf + 1) * sizeof(int64_t));
    memcpy(o->perm, s.perm.data(), s.n * sizeof(int64_t));
    for (int l = 0; l <= L + 1; ++l) o->node_off[l] = s.node_base[l];
    for (int l = 0; l <= L; ++l)
      for (int q = 0; q < s.lev[l].size(); ++q) {
        const long long g = s.node_base[l] + q;
        o->node_row[g] = s.lev[l].row[q];
        o->node_col[g] = s.lev[l].col[q];
        o->node_type[g] = s.lev[l].type[q];
      }
    memcpy(o->krow, M->krow.data(), ncl * sizeof(int64_t));
    memcpy(o->kcol, M->kcol.data(), ncl * sizeof(int64_t));
    // complex matrices: device planes [real | imaginary] out as interleaved
    // pairs; offsets count complex elements
    const int nc = M->cplx ? 2 : 1;
    size_t pl = 0;  // plane length of the buffer fetched last
    auto fetch = [&](const Buf& b) {
      std::vector<double> h(b.bytes() / sizeof(double));
      pl = h.size() / nc;
      if (!h.empty())
        H2_HIP(hipMemcpy(h.data(), b.d(), h.size() * sizeof(double), hipMemcpyDeviceToHost));
      return h;
    };
    auto put = [&](double* dst, int64_t& p, const std::vector<double>& h, size_t idx) {
      for (int part = 0; part < nc; ++part) dst[p * nc + part] = h[part * pl + idx];
      ++p;
    };
    auto leaf = [&](const Buf& b, long long stride, const std::vector<int64_t>& kk, double* dst,
                    int64_t* off) {
      std::vector<double> h = fetch(b);
      int64_t p = 0;
      for (int c = 0; c < nleaf; ++c) {
        off[c] = p;
        const int nr = s.leaf_size[c], k = (int)kk[cidx(L, c)];
        for (int j = 0; j < k; ++j)
          for (int i = 0; i < nr; ++i) put(dst, p, h, (size_t)c * stride + i + (size_t)j * np);
      }
      off[nleaf] = p;
    };
    leaf(M->V, M->V_stride, M->krow, o->V, o->V_off);
    leaf(M->W, M->W_stride, M->kcol, o->W, o->W_off);
    auto trans = [&](const std::vector<Buf>& T, const std::vector<long long>& stride,
                     const std::vector<int>& rp, const std::vector<int64_t>& kk, double* dst,
                     int64_t* off) {
      int64_t p = 0;
      off[0] = 0;
      for (int l = 0; l < L; ++l) {
        const bool live = T[l].bytes() > 0;
        std::vector<double> h = live ? fetch(T[l]) : std::vector<double>();
        const int ld = 2 * rp[l + 1];
        for (int c = 0; c < (2 << l); ++c) {
          const long long fi = cidx(l + 1, c);
          off[fi] = p;
          const int kc_ = (int)kk[fi], kp = (int)kk[cidx(l, c >> 1)];
          for (int j = 0; j < kp; ++j)
            for (int i = 0; i < kc_; ++i)
              put(dst, p, h, (size_t)(c >> 1) * stride[l] + (c & 1) * rp[l + 1] + i + (size_t)j * ld);
        }
      }
      off[ncl] = p;
    };
    trans(M->Tr, M->Tr_stride, M->rr, M->krow, o->Er, o->Er_off);
    trans(M->Tc, M->Tc_stride, M->rc, M->kcol, o->Ec, o->Ec_off);
    int64_t ps = 0, pf = 0;
    for (int l = 0; l <= L; ++l) {
      const LevelNodes& ln = s.lev[l];
      std::vector<double> hs = M->S[l].bytes() ? fetch(M->S[l]) : std::vector<double>();
      const size_t pls = pl;
      const long long bs = (long long)M->rr[l] * M->rc[l];
      for (int q = 0; q < ln.size(); ++q) {
        const long long g = s.node_base[l] + q;
        o->S_off[g] = ps;
        if (ln.type[q] == kR) {
          const int kr = (int)M->krow[cidx(l, ln.row[q])], kc = (int)M->kcol[cidx(l, ln.col[q])];
          pl = pls;
          for (int j = 0; j < kc; ++j)
            for (int i = 0; i < kr; ++i) put(o->S, ps, hs, (size_t)q * bs + i + (size_t)j * M->rr[l]);
        }
      }
    }
    o->S_off[s.node_base[L + 1]] = ps;
    {
      const LevelNodes& ln = s.lev[L];
      std::vector<double> hf = fetch(M->F);
      for (int l = 0; l < L; ++l)
        for (int q = 0; q < s.lev[l].size(); ++q) o->F_off[s.node_base[l] + q] = 0;
      for (int q = 0; q < ln.size(); ++q) {
        const long long g = s.node_base[L] + q;
        o->F_off[g] = pf;
        if (ln.type[q] == kF) {
          const int ni = s.leaf_size[ln.row[q]], nj = s.leaf_size[ln.col[q]];
          for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i) put(o->F, pf, hf, (size_t)q * np * np + i + (size_t)j * np);
        }
      }
      o->F_off[s.node_base[L + 1]] = pf;
    }
    return H2_OK;
  } catch (const Error& e) {
    return set_error(e.code, e.msg);
  }
}

h2_status h2_stats(h2_mat M, h2_stats_t* out) {
  if (!M || !out) return h2::set_error(H2_ERR_ARG, "null argument");
  std::unique_lock<std::recursive_mutex> lk;
  if (M->ctx) lk = std::unique_lock<std::recursive_mutex>(M->ctx->mu);
  try {
    if (M->ctx) hipSetDevice(M->ctx->device);
    M->finish();
  } catch (const h2::Error& e) {
    (void)hipGetLastError();
    return h2::set_error(e.code, e.msg);
  }
  if (M->flops_pending && M->flop_ranks) {
    // a complex block product is four real ones
    const double m4 = M->cplx ? 4.0 : 1.0;
    const h2::FlopCounts fc = h2::flop_counts(M->st(), *M->flop_ranks);
    M->stats.flops_triple = fc.triple * m4;
    M->stats.flops_target = fc.target * m4;
    M->stats.flops_gram = fc.gram * m4;
    M->stats.eig_flops = fc.eig * (M->cplx ? 8.0 : 1.0);  // real embedding of twice the size
    M->stats.eig_tri_flops = fc.eig_tri * (M->cplx ? 8.0 : 1.0);
    M->stats.eig_vec_flops = fc.eig_vec * (M->cplx ? 8.0 : 1.0);
    M->stats.flops = M->stats.flops_triple + M->stats.flops_target + M->stats.flops_gram +
                     M->stats.eig_flops;
    M->flops_pending = false;
    M->flop_ranks.reset();
  }
  *out = M->stats;
  return H2_OK;
}

void h2_free(h2_mat M) {
  if (!M) return;
  h2_ctx c = M->ctx;
  if (c) {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    delete M;
  } else {
    delete M;
  }
}

h2_status h2_plan_info(const h2_host_matrix* m, int64_t max_levels, int64_t* triples,
                       int64_t* blue, int64_t* merged, int64_t* lmin) {
  using namespace h2;
  if (!m || !triples || !blue || !merged || !lmin) return set_error(H2_ERR_ARG, "null argument");
  try {
    Structure s;
    std::string err = build_structure(s, m->n, m->L, m->leaf_off, m->perm, m->node_off,
                                      m->node_row, m->node_col, m->node_type);
    if (!err.empty()) return set_error(H2_ERR_ARG, err);
    if (max_levels <= s.L) return set_error(H2_ERR_ARG, "max_levels <= L");
    Plan p;
    err = build_plan(s, p);
    if (!err.empty()) return set_error(H2_ERR_INTERNAL, err);
    for (int l = 0; l <= s.L; ++l) {
      triples[l] = p.triples_per_level[l];
      blue[l] = p.n_blue[l];
      merged[l] = p.n_case1[l];
    }
    *lmin = s.lmin;
    return H2_OK;
  } catch (const std::exception& e) {
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}

}  // extern "C"
