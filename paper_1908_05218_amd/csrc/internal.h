// Internal types of the h2mmp library (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "h2mmp.h"
#include "kernels.h"
#include "structure.h"

namespace h2 {

h2_status set_error(h2_status s, const std::string& msg);

#define H2_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::h2::Error(H2_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Error {
  h2_status code;
  std::string msg;
  Error(h2_status c, std::string m) : code(c), msg(std::move(m)) {}
};

// ACCURACY-mode truncation factor: eigenvalues of a normalised Gram sum above
// (kTheta eps / n_t)^2 lambda_1 are kept, n_t = levels whose bases are
// truncated; fixed once on small members of each input family (the largest
// value of {1, 1/2, 1/4} whose error stays at or below eps/2 there)
constexpr double kTheta = 1.0;
// fixed-basis mode: relative eigenvalue floor of an old basis' numerical rank
constexpr double kFixedTau = 1e-12;

inline int pad16(long long x) { return (int)(x <= 16 ? 16 : ((x + 15) / 16) * 16); }

}  // namespace h2

namespace h2 {
struct Server;
// actual ranks (flat cluster index 2^l - 1 + c) of A, B and C
struct FlopRanks {
  std::vector<int64_t> ar, ac, br, bc, cr, cc;
};
struct FlopCounts {
  double triple = 0, target = 0, gram = 0, eig = 0;
  // parts of the eigensolver's work: (4/3) d^3 Householder reduction and
  // 6 d^2 k for the k kept eigenvectors (inverse iteration, Gram-Schmidt,
  // back-transformation), per Gram matrix
  double eig_tri = 0, eig_vec = 0;
};
}

struct h2_ctx_s {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;        // bytes held from the device (live + pooled)
  size_t pooled = 0;      // of which cached in the pool
  size_t live_bytes = 0;  // of which held by live allocations
  size_t peak_live = 0;   // high-water mark of live_bytes since the last mark()
  // serialises every entry point of the context (and its serving worker)
  std::recursive_mutex mu;
  h2::Server* server = nullptr;  // serving loop, started by the first h2_submit
  int serve_slots = 2;            // concurrent requests of the serving loop
  // a serving slot's context: the context whose h2_submit created it (its
  // results are used through the parent)
  h2_ctx_s* parent = nullptr;
  hipStream_t stream = nullptr;
  // helper streams and events of the mat-vec's independent branches (the
  // near field and the couplings of each level), forked from and joined
  // back into the caller's stream; created with the context (none: the
  // branches run in order on the caller's stream)
  static constexpr int kAux = 3;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kAux] = {};
  // pinned host memory for the ranks and flags a product reads back per
  // level, and the event that marks their arrival (created on first use)
  int* rb_host = nullptr;
  size_t rb_n = 0;
  hipEvent_t rb_ev = nullptr;
  int* readback(size_t n);  // at least n ints
  std::vector<hipEvent_t> prof_events;  // timing events of the per-class split, reused
  bool profiling = false;
  // external supplier of device memory (h2_ctx_create); without one the
  // context calls hipMalloc and pools freed blocks
  h2_allocator hook{};
  bool has_hook = false;
  // failure injection for tests of the error paths: the allocation with
  // this index (counted from the context's creation) raises H2_ERR_OOM once;
  // set from the environment variable H2_FAIL_ALLOC at creation, -1: never
  long long fail_alloc = -1;
  long long n_alloc = 0;
  std::multimap<size_t, void*> pool;
  std::unordered_map<void*, size_t> live;
  // device regions a call uses that the context did not allocate (the
  // allocation-free mat-vec's scratch parts), for the launches' extent checks
  std::unordered_map<void*, size_t> ext;
  std::unordered_set<void*> f32;  // live allocations that hold float elements
  // live complex allocations: [real plane | imaginary plane] of doubles, the
  // value is the plane's length in elements
  std::unordered_map<void*, long long> planes;
  void* alloc(size_t bytes, bool is_f32 = false, bool is_cplx = false);
  void* alloc_raw(size_t bytes, bool is_f32);
  // imaginary-plane offset (elements) of the complex allocation starting at p, else 0
  long long plane(const void* p) const {
    auto it = planes.find(const_cast<void*>(p));
    return it == planes.end() ? 0 : it->second;
  }
  // element size of the live allocation starting at p (4 or 8)
  size_t elt(const void* p) const { return f32.count(const_cast<void*>(p)) ? 4 : 8; }
  void release(void* p);
  // start a call's high-water mark of live bytes
  void mark() { peak_live = live_bytes; }
  // return cached blocks to the device, largest first, until at most keep
  // bytes stay cached
  void trim(size_t keep);
  // end of a call that started at live bytes `start`: keep in the pool at
  // most twice the call's peak temporaries (so a repeated call of the same
  // shape finds its blocks), never more than the budget allows
  void end_call(size_t start);
  ~h2_ctx_s();
};

namespace h2 {

// Device buffer owned by a context's pool.
class Buf {
 public:
  Buf() = default;
  // is_cplx: bytes / 16 complex elements stored as two planes of doubles
  Buf(h2_ctx c, size_t bytes, bool is_f32 = false, bool is_cplx = false) : ctx_(c), bytes_(bytes) {
    p_ = bytes ? c->alloc(bytes, is_f32, is_cplx) : nullptr;
  }
  ~Buf() { reset(); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept { *this = std::move(o); }
  Buf& operator=(Buf&& o) noexcept {
    if (this != &o) {
      reset();
      ctx_ = o.ctx_;
      p_ = o.p_;
      bytes_ = o.bytes_;
      o.p_ = nullptr;
      o.bytes_ = 0;
    }
    return *this;
  }
  void reset() {
    if (p_ && ctx_) ctx_->release(p_);
    p_ = nullptr;
    bytes_ = 0;
  }
  template <typename T>
  T* as() const { return (T*)p_; }
  double* d() const { return (double*)p_; }
  void* p() const { return p_; }
  size_t bytes() const { return bytes_; }

 private:
  h2_ctx ctx_ = nullptr;
  void* p_ = nullptr;
  size_t bytes_ = 0;
};

struct DevList {
  int nout = 0;
  int ntask = 0;
  // largest tile index referenced per operand and selector (-1: none)
  int max_a[2] = {-1, -1};
  int max_b[2] = {-1, -1};
  int max_out = -1;
  const int* out = nullptr;
  const int* seg = nullptr;
  const int* a = nullptr;
  const int* b = nullptr;
};

// All task lists of a plan uploaded to one device buffer.
struct DevPlan {
  Buf mem;
  std::unordered_map<const TaskList*, DevList> lists;
  const DevList& get(const TaskList& t) const { return lists.at(&t); }
};

// Registers a caller-owned device region with a context for the duration of
// a call (extent checks; complex regions also as two planes).
struct ExtRegion {
  h2_ctx c = nullptr;
  void* p = nullptr;
  ExtRegion(h2_ctx ctx, void* ptr, size_t bytes, bool cplx) : c(ctx), p(ptr) {
    c->ext[p] = bytes;
    if (cplx) c->planes[p] = (long long)(bytes / 16);
  }
  ExtRegion(ExtRegion&& o) noexcept : c(o.c), p(o.p) { o.c = nullptr; }
  ExtRegion(const ExtRegion&) = delete;
  ExtRegion& operator=(const ExtRegion&) = delete;
  ExtRegion& operator=(ExtRegion&&) = delete;
  ~ExtRegion() {
    if (c) {
      c->ext.erase(p);
      c->planes.erase(p);
    }
  }
};

// Task lists of M's exact mat-vec (uploaded once; the host copy is kept so
// the upload needs no wait).
struct MatvecPlan {
  Buf mem;
  std::vector<int> host;
  std::vector<DevList> lists;
};

struct Shape {
  Structure s;
  std::unique_ptr<Plan> plan;
  std::unique_ptr<DevPlan> dplan;
  // the exact mat-vec's task lists (they depend on the structure only),
  // shared by the matrices of this structure
  std::shared_ptr<MatvecPlan> mv;
  Buf d_perm, d_leaf_off;
};

}  // namespace h2

struct h2_mat_s {
  h2_ctx ctx = nullptr;
  std::shared_ptr<h2::Shape> shape;
  bool product = false;            // produced by h2_mmp (levels above lmin carry no basis)
  std::vector<int> rr, rc;         // padded ranks per level
  std::vector<int64_t> krow, kcol; // actual ranks, flat cluster index 2^l-1+c
  h2::Buf V, W;                    // leaf bases
  long long V_stride = 0, W_stride = 0;
  std::vector<h2::Buf> Tr, Tc;     // stacked transfers per parent cluster, level l < L
  std::vector<long long> Tr_stride, Tc_stride;
  std::vector<h2::Buf> S;          // per level, flat by node, rr[l] x rc[l]
  h2::Buf F;                       // leaf level, flat by node, npad x npad
  h2_stats_t stats{};
  bool cplx = false;  // complex128 data (every block buffer holds two planes)
  // ranks a product's algorithmic flop count needs (counted on the first
  // h2_stats call)
  std::unique_ptr<h2::FlopRanks> flop_ranks;
  bool flops_pending = false;
  // float copy of V, W, Tr, Tc, S and F for FP32-bulk products (made on the
  // first such product, kept with the matrix)
  std::unique_ptr<h2_mat_s> f32;
  // events around the numeric phase of the product that made M (on the
  // context's stream); mmp_ms is read from them once they have completed
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  bool timing_pending = false;
  // task lists of the exact mat-vec (built when M is made)
  std::shared_ptr<h2::MatvecPlan> mv;
  const h2::Structure& st() const { return shape->s; }
  // wait for the launches of the call that produced M; fills mmp_ms
  void finish();
  ~h2_mat_s();
};

namespace h2 {

FlopCounts flop_counts(const Structure& s, const FlopRanks& r);

// Operand description for the batched GEMM helpers.
struct Op {
  const void* base0 = nullptr;  // element type from the allocation (ctx->elt)
  const void* base1 = nullptr;
  long long stride0 = 0, stride1 = 0;
  int ld = 0;
  long long sub_r = 0, sub_c = 0;
};

// kernel classes of a product: projections, collects, split and cluster-basis
// products (other); one contraction per evaluated block product (triple);
// Gram sums; eigen-decompositions; products that apply the projections once
// per target (target)
enum KernelKind {
  kKindOther = 0,
  kKindTriple = 1,
  kKindGram = 2,
  kKindEig = 3,  // the tridiagonalisation kernels
  kKindTarget = 4,
  kKindEigVal = 5,
  kKindEigVec = 6,
  kKindCount = 7
};

struct Profiler {
  bool on = false;
  hipStream_t stream = nullptr;
  // timing events to reuse (the context's), else created and destroyed per launch
  std::vector<hipEvent_t>* pool = nullptr;
  struct Rec {
    hipEvent_t a, b;
    int kind;
    double flops;
  };
  std::vector<Rec> recs;
  void begin(int kind, double flops, hipEvent_t* out_a);
  void end(hipEvent_t a, int kind, double flops);
  void collect(double* ms, long long* launches, double* flops);
};

// Batched segmented product.  The arithmetic is FP32 for the bulk kinds
// (kKindOther, kKindTriple) while g_bulk_f32 is set, FP64 otherwise (always for
// kKindGram); operands and C may be float or double allocations.  When C is a
// complex allocation, A and B must be complex too: the product runs as four
// real products over the planes; conj bit 0 / bit 1 conjugates A / B (after
// the transposition flags, so tA with bit 0 is A^H).
constexpr int kConjA = 1, kConjB = 2;
// flag: C is symmetric and only its part on and below the diagonal is read
// (real data only; a complex product computes every tile)
constexpr int kLowerOnly = 4;
void gemm(hipStream_t s, Profiler* prof, int kind, const DevList& tl, int m, int n, int k,
          const Op& A, bool tA, const Op& B, bool tB, void* C, long long cstride, int ldc,
          long long csub_r, long long csub_c, double alpha, double beta, int conj = 0);
// segmented sums (both planes of complex allocations)
void segsum(hipStream_t s, const DevList& tl, int m, int n, const Op& A, void* C,
            long long cstride, int ldc, long long csub_r, long long csub_c, double beta);
// n elements (both planes of a complex allocation)
void zero(hipStream_t s, void* p, long long n);
// float copy of M's data for FP32-bulk products (cached in M->f32)
const h2_mat_s& f32_shadow(h2_ctx ctx, h2_mat M, hipStream_t s);

std::unique_ptr<DevPlan> upload_plan(h2_ctx ctx, const Plan& p);
void scan_limits(const TaskList& t, DevList& d);
// context whose allocations bound-check the launches of the current call
extern thread_local h2_ctx g_active_ctx;
// installs the context of an entry point for the duration of the call and
// restores the previous one (so no thread keeps a pointer to a context that
// may be destroyed later)
struct ActiveCtx {
  h2_ctx prev;
  explicit ActiveCtx(h2_ctx c) : prev(g_active_ctx) { g_active_ctx = c; }
  ~ActiveCtx() { g_active_ctx = prev; }
  ActiveCtx(const ActiveCtx&) = delete;
  ActiveCtx& operator=(const ActiveCtx&) = delete;
};
// FP32-bulk arithmetic for the bulk GEMM kinds during the current product
extern thread_local bool g_bulk_f32;
struct BulkScope {
  explicit BulkScope(bool on) { g_bulk_f32 = on; }
  ~BulkScope() { g_bulk_f32 = false; }
};

h2_status mmp_impl(h2_ctx ctx, h2_mat A, h2_mat B, double eps, int mode, int prec, h2_mat* C);
// Truncated eigen-decompositions of one level's row and column Gram sums,
// both sets in one launch per phase (complex Grams through their real
// embedding).  Gr / Gc: three components per side, each divided by its trace
// (an empty Buf is an absent component; the first must be present); k1/k2:
// live rows as in h2k::EigArgs; kmax_r / kmax_c (nullable, per cluster): at
// most that many vectors are kept.  Outputs U (D x D per cluster) and ranks.
struct EigLevel {
  h2_ctx ctx;
  hipStream_t st;
  Profiler* prof;
  int* status;  // device flags: [0] non-finite, [1] dimension over limit
  bool cplx;
  double tau;   // relative eigenvalue threshold
  bool exact;   // keep every eigenvector
  // pinned [rank_r (2^l) | rank_c (2^l) | status (4)] of the level, written
  // as soon as the ranks are fixed (before the eigenvectors), and the event
  // recorded after those copies
  int* host;
  hipEvent_t ready;
};
void eig_level(const EigLevel& e, int l, int D, const Buf* Gr, const Buf* Gc, Buf& Ur, Buf& Uc,
               Buf& rank_r, Buf& rank_c, const int* k1r, const int* k2r, const int* k1c,
               const int* k2c, int kstride, int half, const int* kmax_r = nullptr,
               const int* kmax_c = nullptr);
// waits for the level's read-back of eig_level; raises the eigensolver's
// flags; the pinned ranks: rows at [0, 2^l), columns at [2^l, 2^(l+1))
const int* wait_ranks(const EigLevel& e, int l);
// H^2 recompression of M at eps (new nested orthonormal bases, projected
// couplings, M's dense blocks), a new matrix of ctx
h2_mat recompress_impl(h2_ctx ctx, h2_mat M, double eps);
// measured tile choices of the batched GEMM (tiles.txt), tuning hooks
std::string tile_key(int tsize, int af32, int bf32, int triple, int tA, int tB, int m, int n, int k,
                     int nout, long long ntask);
int tile_for(const std::string& key);  // -1: shape heuristic
bool tile_logging();
void tile_log(const std::string& key, int tile, float ms);
// the context whose pool holds M: ctx itself or one of ctx's serving slots
// (nullptr when M belongs to neither)
inline h2_ctx home_of(h2_ctx ctx, const h2_mat_s* M) {
  if (!ctx || !M || !M->ctx) return nullptr;
  return (M->ctx == ctx || M->ctx->parent == ctx) ? M->ctx : nullptr;
}
// stop a context's serving worker (after its current request) and drop the
// requests still queued; no-op without one
void stop_server(h2_ctx ctx);
void matvec_impl(h2_ctx ctx, h2_mat M, const double* x_dev, double* y_dev, int64_t nrhs,
                 hipStream_t st, void* scratch = nullptr, size_t scratch_bytes = 0);
void build_matvec_plan(h2_ctx ctx, h2_mat M);
// locates the allocation-free mat-vec's scratch array on `device` (current)
// once per device; sets the error message on failure
h2_status noalloc_setup(int device);
size_t matvec_scratch_bytes(const h2_mat_s* M, int64_t nrhs);

}  // namespace h2
