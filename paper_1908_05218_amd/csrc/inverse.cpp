// Approximate inverse by repeated H^2 matrix-matrix products (the use of the
// product for inverse-based fast solvers, Section I): Newton-Schulz
// iteration X_{j+1} = X_j (2 I - A X_j), started at X_1 = 2 alpha I -
// alpha^2 A.  The shift 2 I - Y keeps Y's partition and bases (the identity
// lives in the dense diagonal leaf blocks), so every step is two products
// and one scale-and-shift.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.h"

namespace h2 {

namespace {

// device copy of a buffer with the same element type and planes
Buf copy_buf(h2_ctx ctx, const Buf& src, hipStream_t st) {
  if (!src.bytes()) return Buf();
  const bool f32 = ctx->elt(src.p()) == 4, cplx = ctx->plane(src.p()) > 0;
  Buf dst(ctx, src.bytes(), f32, cplx);
  H2_HIP(hipMemcpyAsync(dst.p(), src.p(), src.bytes(), hipMemcpyDeviceToDevice, st));
  return dst;
}

// a M + b I as a new matrix of M's context, partition and bases
h2_mat scale_shift_impl(h2_ctx ctx, h2_mat M, double a, double b) {
  ActiveCtx active(ctx);
  hipStream_t st = ctx->stream;
  const Structure& s = M->st();
  auto X = std::make_unique<h2_mat_s>();
  X->ctx = ctx;
  X->shape = M->shape;
  X->product = M->product;
  X->rr = M->rr;
  X->rc = M->rc;
  X->krow = M->krow;
  X->kcol = M->kcol;
  X->cplx = M->cplx;
  X->V = copy_buf(ctx, M->V, st);
  X->W = copy_buf(ctx, M->W, st);
  X->V_stride = M->V_stride;
  X->W_stride = M->W_stride;
  for (const Buf& t : M->Tr) X->Tr.push_back(copy_buf(ctx, t, st));
  for (const Buf& t : M->Tc) X->Tc.push_back(copy_buf(ctx, t, st));
  X->Tr_stride = M->Tr_stride;
  X->Tc_stride = M->Tc_stride;
  const int nc = M->cplx ? 2 : 1;  // both planes scale by the real a
  for (const Buf& t : M->S) {
    X->S.push_back(copy_buf(ctx, t, st));
    const Buf& d = X->S.back();
    if (d.bytes())
      H2_HIP(h2k::launch_scale(d.d(), a, (long long)(d.bytes() / sizeof(double)), st));
  }
  X->F = copy_buf(ctx, M->F, st);
  if (X->F.bytes())
    H2_HIP(h2k::launch_scale(X->F.d(), a, (long long)(X->F.bytes() / sizeof(double)), st));
  (void)nc;
  // b I on the diagonal dense blocks (real plane), the leaf's own rows only
  const LevelNodes& lf = s.lev[s.L];
  std::vector<int> host;
  for (int q = 0; q < lf.size(); ++q)
    if (lf.type[q] == kF && lf.row[q] == lf.col[q]) host.push_back(q);
  const int nd = (int)host.size();
  if (nd > 0 && b != 0.0) {
    for (int t = 0; t < nd; ++t) host.push_back(s.leaf_size[lf.row[host[t]]]);
    Buf lists(ctx, host.size() * sizeof(int));
    H2_HIP(hipMemcpyAsync(lists.as<int>(), host.data(), host.size() * sizeof(int),
                          hipMemcpyHostToDevice, st));
    H2_HIP(h2k::launch_shift_diag(X->F.d(), lists.as<int>(), lists.as<int>() + nd, nd, s.npad, b,
                                  st));
    // the host list must outlive the copy
    H2_HIP(hipStreamSynchronize(st));
  }
  build_matvec_plan(ctx, X.get());
  H2_HIP(hipStreamSynchronize(st));
  return X.release();
}

}  // namespace

}  // namespace h2

extern "C" {

h2_status h2_scale_shift(h2_ctx ctx, h2_mat M, double a, double b, h2_mat* out) {
  using namespace h2;
  if (!ctx || !M || !out) return set_error(H2_ERR_ARG, "null argument");
  if (!std::isfinite(a) || !std::isfinite(b)) return set_error(H2_ERR_ARG, "a and b must be finite");
  ctx = home_of(ctx, M);
  if (!ctx) return set_error(H2_ERR_ARG, "M belongs to another context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  try {
    hipSetDevice(ctx->device);
    M->finish();
    *out = scale_shift_impl(ctx, M, a, b);
    return H2_OK;
  } catch (const Error& e) {
    (void)hipGetLastError();
    return set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}

h2_status h2_newton_schulz(h2_ctx ctx, h2_mat A, double alpha, int steps, double eps,
                           int trunc_mode, int precision, h2_mat* X_out) {
  using namespace h2;
  if (!ctx || !A || !X_out) return set_error(H2_ERR_ARG, "null argument");
  if (steps < 1) return set_error(H2_ERR_ARG, "steps must be >= 1");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return set_error(H2_ERR_ARG, "alpha must be > 0");
  h2_mat X = nullptr;
  h2_status r = h2_scale_shift(ctx, A, -alpha * alpha, 2.0 * alpha, &X);
  for (int j = 1; j < steps && r == H2_OK; ++j) {
    h2_mat Y = nullptr, W = nullptr, Xn = nullptr;
    r = h2_mmp(ctx, A, X, eps, trunc_mode, precision, nullptr, &Y);
    if (r == H2_OK) r = h2_scale_shift(ctx, Y, -1.0, 2.0, &W);
    h2_free(Y);
    if (r == H2_OK) r = h2_mmp(ctx, X, W, eps, trunc_mode, precision, nullptr, &Xn);
    h2_free(W);
    h2_free(X);
    X = Xn;
  }
  if (r != H2_OK) {
    h2_free(X);
    return r;
  }
  *X_out = X;
  return H2_OK;
}

}  // extern "C"
