// h2_build: an H^2 matrix of a kernel over a point set (Section II of Ma &
// Jiao: binary cluster tree, strong admissibility, nested cluster bases with
// transfer matrices, coupling matrices of admissible blocks, dense leaf
// blocks).  The bases come from tensor Chebyshev interpolation, the standard
// construction for such kernel matrices (the paper cites its construction
// without describing it):
//   * tree: every cluster of a level is split while ceil(n / 2^l) exceeds the
//     leaf size (all leaves at one depth), at the median along the longest
//     axis of its tight bounding box (ties to the lower axis), after a stable
//     sort by that coordinate and then by original index; the first child gets
//     floor(n/2) points;
//   * blocks: (t, s) is admissible when the gap between the tight boxes is
//     positive and max(diam t, diam s) <= eta * dist(t, s); other blocks are
//     dense at the leaf level and split into four children above it;
//   * bases: first-kind Chebyshev nodes of order p per axis on each cluster's
//     tight box (degenerate extents padded to 1e-9 times the root diameter,
//     or to 1e-9 when every point coincides);
//     the leaf basis is the tensor Lagrange basis at the cluster's points, the
//     transfer of a child the parent's Lagrange basis at the child's nodes,
//     and column bases equal row bases (symmetric kernel);
//   * couplings: the kernel at the two clusters' node sets; dense blocks: the
//     kernel at the points, with the configured value where r = 0.
// Tree, block tree and bases are built on the host; couplings and dense
// blocks are evaluated on the device directly into the padded layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace h2 {

h2_status load_impl(h2_ctx ctx, const h2_host_matrix* m, bool device_blocks, h2_mat* out);

namespace {

struct Box {
  std::array<double, 3> lo, hi;
};

struct Tree {
  int L = 0;
  std::vector<int64_t> perm, leaf_off;
  std::vector<std::vector<Box>> box;  // per level, per cluster (tight)
  int64_t start(int l, int c) const { return leaf_off[(size_t)c << (L - l)]; }
  int64_t stop(int l, int c) const { return leaf_off[(size_t)(c + 1) << (L - l)]; }
};

Tree make_tree(const double* xyz, int64_t n, int64_t leaf) {
  Tree t;
  int depth = 0;
  while ((n + (1LL << depth) - 1) >> depth > leaf) ++depth;
  t.L = depth;
  t.perm.resize(n);
  std::iota(t.perm.begin(), t.perm.end(), 0);
  std::vector<std::pair<int64_t, int64_t>> ranges{{0, n}};
  for (int d = 0; d < depth; ++d) {
    std::vector<std::pair<int64_t, int64_t>> nxt;
    for (auto [s, e] : ranges) {
      double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int64_t p = s; p < e; ++p)
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], xyz[3 * t.perm[p] + a]);
          hi[a] = std::max(hi[a], xyz[3 * t.perm[p] + a]);
        }
      int axis = 0;
      for (int a = 1; a < 3; ++a)
        if (hi[a] - lo[a] > hi[axis] - lo[axis]) axis = a;
      std::sort(t.perm.begin() + s, t.perm.begin() + e, [&](int64_t x, int64_t y) {
        const double cx = xyz[3 * x + axis], cy = xyz[3 * y + axis];
        return cx < cy || (cx == cy && x < y);
      });
      const int64_t m = s + (e - s) / 2;
      nxt.push_back({s, m});
      nxt.push_back({m, e});
    }
    ranges = std::move(nxt);
  }
  for (auto& r : ranges) t.leaf_off.push_back(r.first);
  t.leaf_off.push_back(n);
  t.box.resize(depth + 1);
  for (int l = 0; l <= depth; ++l) {
    t.box[l].resize((size_t)1 << l);
    for (int c = 0; c < (1 << l); ++c) {
      Box& b = t.box[l][c];
      b.lo = {INFINITY, INFINITY, INFINITY};
      b.hi = {-INFINITY, -INFINITY, -INFINITY};
      for (int64_t p = t.start(l, c); p < t.stop(l, c); ++p)
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = std::min(b.lo[a], xyz[3 * t.perm[p] + a]);
          b.hi[a] = std::max(b.hi[a], xyz[3 * t.perm[p] + a]);
        }
    }
  }
  return t;
}

double norm3(double x, double y, double z) { return std::sqrt(x * x + y * y + z * z); }
double diam(const Box& b) { return norm3(b.hi[0] - b.lo[0], b.hi[1] - b.lo[1], b.hi[2] - b.lo[2]); }
double dist(const Box& t, const Box& s) {
  double g[3];
  for (int a = 0; a < 3; ++a) g[a] = std::max(0.0, std::max(s.lo[a] - t.hi[a], t.lo[a] - s.hi[a]));
  return norm3(g[0], g[1], g[2]);
}

struct Blocks {
  std::vector<int64_t> node_off{0};
  std::vector<int32_t> row, col, type;
};

Blocks make_blocks(const Tree& t, double eta) {
  Blocks b;
  std::vector<std::pair<int, int>> cand{{0, 0}};
  for (int l = 0; l <= t.L; ++l) {
    std::sort(cand.begin(), cand.end());
    std::vector<std::pair<int, int>> nxt;
    for (auto [r, c] : cand) {
      const double d = dist(t.box[l][r], t.box[l][c]);
      const bool adm = d > 0.0 && std::max(diam(t.box[l][r]), diam(t.box[l][c])) <= eta * d;
      int typ;
      if (adm) {
        typ = kR;
      } else if (l == t.L) {
        typ = kF;
      } else {
        typ = kNL;
        for (int a = 0; a < 2; ++a)
          for (int e = 0; e < 2; ++e) nxt.push_back({2 * r + a, 2 * c + e});
      }
      b.row.push_back(r);
      b.col.push_back(c);
      b.type.push_back(typ);
    }
    b.node_off.push_back((int64_t)b.row.size());
    cand = std::move(nxt);
  }
  return b;
}

// Chebyshev node axes of a box: axes[a][m] = c_a + h_a cos((2m+1) pi / (2p))
std::array<std::vector<double>, 3> cheb_axes(const Box& b, int p, double pad) {
  std::array<std::vector<double>, 3> ax;
  for (int a = 0; a < 3; ++a) {
    const double c = 0.5 * (b.lo[a] + b.hi[a]);
    const double h = std::max(0.5 * (b.hi[a] - b.lo[a]), 0.5 * pad);
    ax[a].resize(p);
    for (int m = 0; m < p; ++m) ax[a][m] = c + h * std::cos((2.0 * m + 1.0) * M_PI / (2.0 * p));
  }
  return ax;
}

// 1-D Lagrange basis l_m(x) over the nodes xi
void lagrange_1d(const std::vector<double>& xi, double x, double* out) {
  const int p = (int)xi.size();
  for (int m = 0; m < p; ++m) {
    double v = 1.0;
    for (int q = 0; q < p; ++q)
      if (q != m) v *= (x - xi[q]) / (xi[m] - xi[q]);
    out[m] = v;
  }
}

// tensor Lagrange basis at one point; column (m0 p + m1) p + m2
void lagrange_3d(const std::array<std::vector<double>, 3>& ax, const double* x, double* out) {
  const int p = (int)ax[0].size();
  std::vector<double> l0(p), l1(p), l2(p);
  lagrange_1d(ax[0], x[0], l0.data());
  lagrange_1d(ax[1], x[1], l1.data());
  lagrange_1d(ax[2], x[2], l2.data());
  for (int a = 0; a < p; ++a)
    for (int b = 0; b < p; ++b)
      for (int c = 0; c < p; ++c) out[(a * p + b) * p + c] = l0[a] * l1[b] * l2[c];
}

}  // namespace

h2_status build_impl(h2_ctx ctx, const double* xyz, int64_t n, const h2_kernel* kernel,
                     const h2_build_opts* opts, h2_mat share, h2_mat* out) {
  if (!ctx || !xyz || !kernel || !opts || !out) return set_error(H2_ERR_ARG, "null argument");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ActiveCtx active(ctx);
  if (n < 1 || opts->leaf_size < 1 || !(opts->eta > 0.0) || opts->cheb_order < 1 ||
      opts->cheb_order > 6)
    return set_error(H2_ERR_ARG, "need n >= 1, leaf_size >= 1, eta > 0, 1 <= cheb_order <= 6");
  if (opts->recompress_eps != 0.0 &&
      !(std::isfinite(opts->recompress_eps) && opts->recompress_eps >= H2_RECOMPRESS_EPS_MIN))
    return set_error(H2_ERR_ARG, "recompress_eps must be 0 (off) or finite and >= 1e-8");
  if (kernel->kind != H2_KERNEL_LAPLACE && kernel->kind != H2_KERNEL_HELMHOLTZ)
    return set_error(H2_ERR_UNSUPPORTED, "unsupported kernel");
  const bool helm = kernel->kind == H2_KERNEL_HELMHOLTZ;
  if (!std::isfinite(kernel->self_value) ||
      (helm && (!std::isfinite(kernel->self_value_imag) || !std::isfinite(kernel->wavenumber))))
    return set_error(H2_ERR_ARG, "non-finite self value or wavenumber");
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return set_error(H2_ERR_ARG, "non-finite coordinate");
  if (share && share->st().n != n) return set_error(H2_ERR_ARG, "share_tree_with has another size");
  if (share && share->ctx != ctx)
    return set_error(H2_ERR_ARG, "share_tree_with belongs to another context");
  const int p = opts->cheb_order, p3 = p * p * p;
  const Tree t = make_tree(xyz, n, opts->leaf_size);
  const Blocks bl = make_blocks(t, opts->eta);
  const int L = t.L, nleaf = 1 << L;
  const double rd = diam(t.box[0][0]);
  const double pad = 1e-9 * (rd > 0.0 ? rd : 1.0);  // coinciding points: absolute pad
  std::vector<std::vector<std::array<std::vector<double>, 3>>> ax(L + 1);
  for (int l = 0; l <= L; ++l)
    for (int c = 0; c < (1 << l); ++c) ax[l].push_back(cheb_axes(t.box[l][c], p, pad));
  // leaf bases (n_c x p^3, column-major per leaf)
  std::vector<double> V;
  std::vector<int64_t> V_off{0};
  std::vector<double> row(p3);
  for (int c = 0; c < nleaf; ++c) {
    const int64_t s = t.leaf_off[c], e = t.leaf_off[c + 1], nc = e - s;
    const size_t base = V.size();
    V.resize(base + (size_t)nc * p3);
    for (int64_t i = 0; i < nc; ++i) {
      lagrange_3d(ax[L][c], xyz + 3 * t.perm[s + i], row.data());
      for (int m = 0; m < p3; ++m) V[base + i + (size_t)m * nc] = row[m];
    }
    V_off.push_back((int64_t)V.size());
  }
  // transfers: child c of level l, p^3 x p^3, the parent's Lagrange basis at
  // the child's nodes (node (a p + b) p + c at (ax0[a], ax1[b], ax2[c]))
  std::vector<double> E;
  std::vector<int64_t> E_off{0, 0};  // the root has none
  for (int l = 1; l <= L; ++l)
    for (int c = 0; c < (1 << l); ++c) {
      const auto& ch = ax[l][c];
      const size_t base = E.size();
      E.resize(base + (size_t)p3 * p3);
      for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b)
          for (int cc = 0; cc < p; ++cc) {
            const double x[3] = {ch[0][a], ch[1][b], ch[2][cc]};
            const int i = (a * p + b) * p + cc;
            lagrange_3d(ax[l - 1][c / 2], x, row.data());
            for (int m = 0; m < p3; ++m) E[base + i + (size_t)m * p3] = row[m];
          }
      E_off.push_back((int64_t)E.size());
    }
  const int64_t ncl = (2LL << L) - 1;
  std::vector<int64_t> k(ncl, p3);
  if (helm) {
    // complex matrix with real bases: interleave zero imaginary parts
    auto widen = [](std::vector<double>& v) {
      std::vector<double> w(2 * v.size(), 0.0);
      for (size_t i = 0; i < v.size(); ++i) w[2 * i] = v[i];
      v.swap(w);
    };
    widen(V);
    widen(E);
  }
  h2_host_matrix hm{};
  hm.n = n;
  hm.L = L;
  hm.is_complex = helm ? 1 : 0;
  hm.leaf_off = t.leaf_off.data();
  hm.perm = t.perm.data();
  hm.node_off = bl.node_off.data();
  hm.node_row = bl.row.data();
  hm.node_col = bl.col.data();
  hm.node_type = bl.type.data();
  hm.krow = k.data();
  hm.kcol = k.data();
  hm.V = hm.W = V.data();
  hm.V_off = hm.W_off = V_off.data();
  hm.Er = hm.Ec = E.data();
  hm.Er_off = hm.Ec_off = E_off.data();
  h2_mat M = nullptr;
  h2_status st = load_impl(ctx, &hm, true, &M);
  if (st != H2_OK) return st;
  try {
    hipSetDevice(ctx->device);
    if (share) {
      if (!share->st().same_as(M->st())) {
        h2_free(M);
        return set_error(H2_ERR_ARG, "share_tree_with has another structure");
      }
      M->shape = share->shape;
    }
    const Structure& s = M->st();
    hipStream_t strm = ctx->stream;
    // points in tree order
    std::vector<double> pts((size_t)3 * n);
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) pts[3 * i + a] = xyz[3 * t.perm[i] + a];
    Buf dpts(ctx, pts.size() * sizeof(double));
    H2_HIP(hipMemcpyAsync(dpts.d(), pts.data(), pts.size() * sizeof(double), hipMemcpyHostToDevice,
                          strm));
    Buf doff(ctx, (nleaf + 1) * sizeof(long long));
    H2_HIP(hipMemcpyAsync(doff.as<long long>(), t.leaf_off.data(), (nleaf + 1) * sizeof(long long),
                          hipMemcpyHostToDevice, strm));
    for (int l = 0; l <= L; ++l) {
      const LevelNodes& ln = s.lev[l];
      const int nn = ln.size();
      if (nn == 0) continue;
      std::vector<int> nodes((size_t)3 * nn);
      for (int q = 0; q < nn; ++q) {
        nodes[q] = ln.row[q];
        nodes[nn + q] = ln.col[q];
        nodes[2 * nn + q] = ln.type[q];
      }
      std::vector<double> axes((size_t)(1 << l) * 3 * p);
      for (int c = 0; c < (1 << l); ++c)
        for (int a = 0; a < 3; ++a)
          for (int m = 0; m < p; ++m) axes[((size_t)c * 3 + a) * p + m] = ax[l][c][a][m];
      Buf dn(ctx, nodes.size() * sizeof(int)), da(ctx, axes.size() * sizeof(double));
      H2_HIP(hipMemcpyAsync(dn.as<int>(), nodes.data(), nodes.size() * sizeof(int),
                            hipMemcpyHostToDevice, strm));
      H2_HIP(hipMemcpyAsync(da.d(), axes.data(), axes.size() * sizeof(double),
                            hipMemcpyHostToDevice, strm));
      h2k::BuildCouplingArgs ca{};
      ca.axes = da.d();
      ca.rows = dn.as<int>();
      ca.cols = dn.as<int>() + nn;
      ca.types = dn.as<int>() + 2 * nn;
      ca.nnodes = nn;
      ca.p = p;
      ca.rr = M->rr[l];
      ca.rc = M->rc[l];
      ca.self_value = kernel->self_value;
      ca.S = M->S[l].d();
      ca.helmholtz = helm ? 1 : 0;
      ca.kappa = helm ? kernel->wavenumber : 0.0;
      ca.self_imag = helm ? kernel->self_value_imag : 0.0;
      ca.plane = ctx->plane(M->S[l].p());
      H2_HIP(h2k::launch_build_coupling(ca, strm));
      if (l == L) {
        h2k::BuildDenseArgs fa{};
        fa.pts = dpts.d();
        fa.leaf_off = doff.as<long long>();
        fa.rows = ca.rows;
        fa.cols = ca.cols;
        fa.types = ca.types;
        fa.nnodes = nn;
        fa.npad = s.npad;
        fa.self_value = kernel->self_value;
        fa.F = M->F.d();
        fa.helmholtz = ca.helmholtz;
        fa.kappa = ca.kappa;
        fa.self_imag = ca.self_imag;
        fa.plane = ctx->plane(M->F.p());
        H2_HIP(h2k::launch_build_dense(fa, strm));
      }
      // the staging buffers return to the pool only after the launches ran
      H2_HIP(hipStreamSynchronize(strm));
    }
    if (opts->recompress_eps > 0.0) {
      h2_mat R = recompress_impl(ctx, M, opts->recompress_eps);
      h2_free(M);
      M = R;
    }
    *out = M;
    return H2_OK;
  } catch (const Error& e) {
    (void)hipGetLastError();
    h2_free(M);
    return set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    h2_free(M);
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}

}  // namespace h2

extern "C" h2_status h2_build(h2_ctx ctx, const double* xyz, int64_t n, const h2_kernel* kernel,
                              const h2_build_opts* opts, h2_mat share_tree_with, h2_mat* out) {
  if (!ctx) return h2::set_error(H2_ERR_ARG, "null argument");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  const size_t start = ctx->live_bytes;
  ctx->mark();
  const h2_status r = h2::build_impl(ctx, xyz, n, kernel, opts, share_tree_with, out);
  // the pool keeps at most twice the call's peak temporaries (the
  // recompression's are large)
  ctx->end_call(start);
  return r;
}
