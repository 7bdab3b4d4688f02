/*
 * h2mmp: accuracy-controlled, structure-preserving H^2 matrix-matrix product
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: M. Ma and D. Jiao, "Accuracy Controlled Structure-Preserving
 * H^2-Matrix-Matrix Product in Linear Complexity with Change of Cluster
 * Bases" (arXiv 1908.05218).  C = A B is computed level by level from the
 * leaves up (Sections III and IV): leaf dense-block products, coupling
 * products through the cluster-basis products, and for every cluster a new
 * basis of C found from normalised Gram sums truncated at eps, followed by a
 * top-down split of couplings attached to non-leaf blocks.
 *
 * Conventions for every entry point:
 *  - Functions return H2_OK or an error code; on error no output handle is
 *    written, nothing leaks, and h2_last_error() returns a message
 *    (thread-local, valid until the next call on the same thread).
 *  - Host pointers are read during the call only; the library copies what it
 *    keeps.  Device pointers are arguments only where a name says "_dev".
 *  - Matrices are column-major, real FP64 or complex128.  Complex data at
 *    the boundary: interleaved (real, imaginary) pairs in h2_load, h2_export
 *    and h2_to_dense; planar vectors (all real parts, then all imaginary
 *    parts) in h2_matvec.
 *  - Device work runs on the context's own HIP stream (default priority).
 *    h2_mmp and h2_matvec also take a caller stream: with a non-null stream
 *    the call's work is ordered after the work queued on that stream before
 *    the call, work queued on it after the call is ordered after the call's
 *    work, and the call may return before its last kernels finish (h2_sync
 *    waits for them).  With a null stream, and for every other entry point,
 *    the call returns after its work has finished.
 */
#ifndef H2MMP_H
#define H2MMP_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_OK = 0,
  H2_ERR_ARG = 1,         /* invalid argument (null pointer, negative size, bad mode) */
  H2_ERR_DEVICE = 2,      /* HIP runtime failure or no usable device */
  H2_ERR_OOM = 3,         /* device allocation failed or over the context's budget */
  H2_ERR_STRUCTURE = 4,   /* A and B do not share tree and block partition */
  H2_ERR_NUMERIC = 5,     /* non-finite input or result */
  H2_ERR_UNSUPPORTED = 6, /* a size or feature the library does not handle */
  H2_ERR_INTERNAL = 7,
  H2_ERR_BUSY = 8         /* a served request is not finished yet */
} h2_status;

typedef struct h2_ctx_s* h2_ctx;
typedef struct h2_mat_s* h2_mat;

/* Truncation rule for the eigenvalues lambda_1 >= lambda_2 ... of a cluster's
 * summed normalised Gram matrix (Section III-C "singular vectors whose
 * normalized singular values are greater than eps_trunc"):
 *  ACCURACY: keep lambda_m > (eps / n_t)^2 lambda_1, n_t = L - l_min + 1 the
 *            number of levels whose bases are truncated (normalised singular
 *            values of the stacked contributions above eps / n_t: the
 *            budget eps split evenly over the levels, whose truncation
 *            errors add up in C; aims at ||C-AB||_F <= eps ||AB||_F)
 *  PAPER:    keep lambda_m > eps lambda_1 (the Gram's own singular values)
 *  EXACT:    keep every eigenvector (no truncation; eps ignored)
 *  FIXED:    the fixed-basis ("formatted") product the paper compares
 *            against (Section I; Table IV): C keeps A's row bases and B's
 *            column bases, orthonormalised (eigenvalues of the old basis'
 *            Gram component alone above 1e-12 lambda_1); no contribution
 *            changes a basis, so the error of C is not controlled (eps
 *            ignored). */
typedef enum {
  H2_TRUNC_ACCURACY = 0,
  H2_TRUNC_PAPER = 1,
  H2_TRUNC_EXACT = 2,
  H2_TRUNC_FIXED = 3
} h2_trunc_mode;

/* Arithmetic of the bulk products.  FP64: everything in double.
 * FP32_BULK: block products in float on the matrix cores, Gram sums,
 * eigen-decompositions and bases in double. */
typedef enum { H2_PREC_FP64 = 0, H2_PREC_FP32_BULK = 1 } h2_precision;

/* Device memory supplier of a context (e.g. a framework's caching
 * allocator).  alloc returns `bytes` of device memory on `device` for work on
 * `stream` (the context's stream), or NULL when it has none; free returns a
 * block from alloc.  free may be called while work already queued on
 * `stream` still reads the block: the allocator must not hand the block to
 * work on another stream before that work has finished (a stream-ordered
 * caching allocator does this).  Both may be called from the library's
 * serving threads.  `user` is passed back unchanged. */
typedef struct {
  void* (*alloc)(void* user, size_t bytes, int device, hipStream_t stream);
  void (*free)(void* user, void* ptr, size_t bytes, int device, hipStream_t stream);
  void* user;
} h2_allocator;

/* Create a context on HIP device `device`.  hbm_budget (bytes) bounds the
 * device memory the context may hold; 0 means no bound.  alloc (nullable,
 * copied): the supplier of every device allocation of the context and of its
 * serving slots; without one the context takes memory with hipMalloc and
 * keeps freed blocks in a pool of its own.  For tests of the error paths,
 * the environment variable H2_FAIL_ALLOC=n (read here) makes the context's
 * allocation number n (counted from 0 over its lifetime) fail once with
 * H2_ERR_OOM.  Errors: H2_ERR_DEVICE (no such device), H2_ERR_ARG
 * (out == NULL, or an allocator without alloc or free). */
h2_status h2_ctx_create(int device, size_t hbm_budget, const h2_allocator* alloc, h2_ctx* out);
void h2_ctx_destroy(h2_ctx ctx);

/* Host description of an H^2 matrix in the flat interchange layout
 * (Section II: nested cluster bases V_t = diag(V_t1, V_t2)[E_t1; E_t2],
 * coupling matrices of admissible blocks, dense leaf blocks):
 *   n points, tree depth L (levels 0..L, 2^l clusters at level l);
 *   leaf_off[2^L+1]: leaf c covers tree positions [leaf_off[c], leaf_off[c+1]);
 *   perm[n]: original index of the point at tree position p;
 *   node_off[L+2], node_row/col/type[]: block-tree nodes level by level,
 *     type 0 = admissible, 1 = dense leaf, 2 = non-leaf;
 *   krow/kcol[2^(L+1)-1]: rank of cluster (l,c) at index 2^l-1+c;
 *   V/W: leaf bases (#leaf x rank), offsets V_off/W_off[2^L+1] in elements;
 *   Er/Ec: transfer of cluster (l,c), l >= 1 (k(l,c) x k(l-1,c/2)), at the
 *     flat cluster index, offsets Er_off/Ec_off[2^(L+1)];
 *   S: coupling of every admissible node, offsets S_off[nnodes+1];
 *   F: dense block of every dense node, offsets F_off[nnodes+1].
 * Entries not used by a node have zero length. */
typedef struct {
  int64_t n, L, is_complex;
  const int64_t* leaf_off;
  const int64_t* perm;
  const int64_t* node_off;
  const int32_t* node_row;
  const int32_t* node_col;
  const int32_t* node_type;
  const int64_t* krow;
  const int64_t* kcol;
  const double *V, *W, *Er, *Ec, *S, *F;
  const int64_t *V_off, *W_off, *Er_off, *Ec_off, *S_off, *F_off;
} h2_host_matrix;

/* Upload an H^2 matrix to the device (padded per-level layout, FP64; with
 * is_complex != 0 the arrays V ... F hold interleaved complex pairs, counts
 * and offsets in complex elements).  Errors: H2_ERR_ARG (inconsistent
 * offsets, sizes or types), H2_ERR_NUMERIC (a non-finite entry),
 * H2_ERR_OOM. */
h2_status h2_load(h2_ctx ctx, const h2_host_matrix* m, h2_mat* out);

/* Kernel of h2_build: H2_KERNEL_LAPLACE is 1/(4 pi r) (real), with
 * self_value where r = 0 (coincident points; e.g. the mean of 1/(4 pi r) over
 * a panel).  H2_KERNEL_HELMHOLTZ is exp(-j kappa r)/(4 pi r) with kappa =
 * wavenumber (complex128 matrix; the scattering kernel of Section VI), with
 * self_value + j self_value_imag where r = 0. */
typedef enum { H2_KERNEL_LAPLACE = 0, H2_KERNEL_HELMHOLTZ = 1 } h2_kernel_kind;
typedef struct {
  int32_t kind;
  double self_value;
  double wavenumber;      /* Helmholtz only */
  double self_value_imag; /* Helmholtz only */
} h2_kernel;

/* Construction options of h2_build.  leaf_size: leaves hold at most this many
 * points (all leaves at one depth); eta: strong admissibility
 * max(diam t, diam s) <= eta dist(t, s) on tight bounding boxes (Section II);
 * cheb_order p: nested tensor Chebyshev interpolation of order p per axis,
 * rank p^3 at every cluster; recompress_eps: 0 = off, else the built matrix
 * is recompressed at this accuracy as by h2_recompress (>= 1e-8). */
typedef struct {
  int64_t leaf_size;
  double eta;
  int32_t cheb_order;
  double recompress_eps;
} h2_build_opts;

/* Build the H^2 matrix (Section II: binary cluster tree by median bisection
 * along the longest axis of each cluster's tight box, block tree by the
 * admissibility rule, nested bases with transfer matrices, couplings of the
 * admissible blocks, dense leaf blocks) of `kernel` over the n points xyz
 * (host, n x 3 row-major, original order; copied).  Tree, block tree, leaf
 * bases and transfers are built on the host; couplings and dense blocks are
 * evaluated on the device.  The result matches h2_load of the same matrix
 * assembled on the host.  share_tree_with (nullable): a matrix of the same
 * points and options whose structure object is then shared.  Synchronous.
 * Errors: H2_ERR_ARG (null pointer, n < 1, leaf_size < 1, eta <= 0,
 * cheb_order outside 1..6, non-finite input, recompress_eps neither 0 nor a
 * finite value >= 1e-8, share_tree_with of another size or structure),
 * H2_ERR_UNSUPPORTED (another kernel), H2_ERR_OOM, H2_ERR_DEVICE. */
h2_status h2_build(h2_ctx ctx, const double* xyz, int64_t n, const h2_kernel* kernel,
                   const h2_build_opts* opts, h2_mat share_tree_with, h2_mat* out);

/* Smallest accuracy h2_recompress accepts: a Gram matrix's eigenvalues are
 * the squared singular values of a cluster's far field, so FP64 resolves
 * singular values down to about 1e-8 of the largest. */
#define H2_RECOMPRESS_EPS_MIN 1e-8

/* Recompression of M (input construction; the paper cites its construction
 * of the inputs without describing it, Section VI): new orthonormal nested
 * bases of the smallest ranks that keep every cluster's whole far field (the
 * admissible blocks of the cluster and of its ancestors, restricted to its
 * rows; for the column side its columns) to relative accuracy eps, and the
 * couplings projected onto them; partition and dense blocks are M's.  Steps
 * on the device: basis Grams B_t = X_t^T X_t^* bottom-up; far-field weights
 * K_t = sum S_ts B_s S_ts^H + E_t K_parent E_t^H top-down; at the leaves the
 * dominant eigenvectors of V_t K_t V_t^H, above them of Z_t K_t Z_t^H with
 * Z_t the old basis written in the children's new bases; couplings
 * S'_ts = P^row_t S_ts (P^col_s)^T with P_t = (new basis)^H (old basis).
 * Eigenvalues above (eps / n_t)^2 lambda_1 are kept (n_t = L - l_min + 1,
 * the product's ACCURACY rule), at most the old rank and at least one; levels
 * above l_min carry no basis, as in a product.  FP64 (complex128 for complex
 * M).  *out is a new matrix of ctx (h2_free); M is unchanged.  Synchronous.
 * Errors: H2_ERR_ARG (null pointer, eps not finite or below
 * H2_RECOMPRESS_EPS_MIN, M of another context), H2_ERR_UNSUPPORTED (a Gram
 * matrix beyond the eigensolver's dimension limit), H2_ERR_NUMERIC
 * (non-finite data), H2_ERR_OOM, H2_ERR_DEVICE. */
h2_status h2_recompress(h2_ctx ctx, h2_mat M, double eps, h2_mat* out);

/* Serving: a request loop of the context with continuous batching.  A
 * request names a point set and a kernel (built as by h2_build) and a
 * product C = A A at eps.  The loop runs up to `slots` requests at once
 * (h2_serve_slots, default 2), each on a slot context of its own (same
 * device, own stream and memory pool), so that the device work of one request
 * overlaps the host-side steps of another.  Requests start in submission
 * order: the first queued request starts once a slot is free and its
 * device-memory estimate fits the context's hbm_budget next to the bytes of
 * the results still held and the estimates of the requests running.  The
 * estimate is kappa N^1.5 (cheb_order / 3)^3 bytes plus 64 MiB, kappa per
 * precision starting at 9000 (FP64) and 7000 (FP32-bulk) and raised to the
 * largest value a finished request has shown; with no budget, requests only
 * wait for a slot.  A request that runs out of device memory while another
 * runs is queued again once, first in line, to run alone.  Results do not
 * depend on what runs beside them (every kernel is deterministic).  A and C of
 * a finished request stay resident until h2_release; they can be passed to
 * h2_matvec, h2_to_dense, h2_export and h2_stats with the submitting context,
 * to h2_mmp together with other matrices of the same request (not with
 * matrices of the context itself), and must not be freed with h2_free.  A
 * product of served matrices belongs to the request's slot: free it with
 * h2_free before h2_ctx_destroy, like every matrix of the context.
 * h2_ctx_destroy stops the loop after the requests it is running and drops
 * the queued ones. */
typedef struct {
  const double* xyz;  /* host, n x 3 row-major, original order; copied */
  int64_t n;
  h2_kernel kernel;
  h2_build_opts opts;
  double eps;
  int32_t trunc_mode; /* h2_trunc_mode */
  int32_t precision;  /* h2_precision */
} h2_request;

typedef struct {
  h2_status status;   /* outcome of the request (H2_OK or the error of its build/product) */
  h2_mat A, C;        /* owned by the context until h2_release; NULL on error */
  double queue_ms;    /* submission to admission */
  double build_ms;    /* h2_build of A */
  double mmp_ms;      /* h2_mmp of C = A A (host wall time, synchronised) */
  double total_ms;    /* submission to completion */
  char message[160];  /* error text when status != H2_OK */
  int64_t bytes;      /* device bytes held by A and C until h2_release */
} h2_result;

/* Number of concurrent requests of the serving loop (1..8), before the first
 * h2_submit.  Errors: H2_ERR_ARG (out of range), H2_ERR_BUSY (the loop has
 * started). */
h2_status h2_serve_slots(h2_ctx ctx, int slots);
/* Queue a request; *ticket identifies it.  Errors: H2_ERR_ARG (null
 * pointer, invalid sizes, options or eps), H2_ERR_OOM (its estimate exceeds
 * the context's whole budget). */
h2_status h2_submit(h2_ctx ctx, const h2_request* req, uint64_t* ticket);
/* H2_OK when the request has finished (whatever its own status), H2_ERR_BUSY
 * while it is queued or running, H2_ERR_ARG for an unknown ticket. */
h2_status h2_poll(h2_ctx ctx, uint64_t ticket);
/* Block until the request has finished and fill *out.  Errors: H2_ERR_ARG
 * (unknown ticket or null out). */
h2_status h2_wait(h2_ctx ctx, uint64_t ticket, h2_result* out);
/* Free A and C of a finished request and forget its ticket.  Errors:
 * H2_ERR_ARG (unknown ticket), H2_ERR_BUSY (not finished). */
h2_status h2_release(h2_ctx ctx, uint64_t ticket);

/* C = A B (Sections III and IV).  A and B must have been loaded with the
 * same tree (leaf_off, perm) and block partition; C shares them (the
 * product keeps A's partition).  eps >= 0; eps == 0 selects EXACT.  A and
 * B both real or both complex (complex: FP64 only).  The Gram dimension of
 * a cluster (twice the children's padded rank) is at most 1024 (512 for
 * complex data, whose Hermitian Grams are solved through their real
 * embedding).
 * stream: see the conventions above.  The call blocks the host once per
 * level to read back the kept ranks (they size the next level's launches);
 * the launches after the last level (the top-down split, the conversion of
 * FP32-bulk results) may still run when it returns.  The products whose
 * targets only the top-down split reads run on one of the context's helper
 * streams, forked from the call's stream and joined back into it by events
 * before the split, so the conventions above hold for the whole call.
 * Errors: H2_ERR_STRUCTURE, H2_ERR_ARG (eps < 0, bad mode/precision),
 * H2_ERR_UNSUPPORTED (a cluster whose Gram dimension exceeds the on-chip
 * eigensolver limit, reported in the message), H2_ERR_OOM, H2_ERR_NUMERIC. */
h2_status h2_mmp(h2_ctx ctx, h2_mat A, h2_mat B, double eps, int trunc_mode, int precision,
                 hipStream_t stream, h2_mat* C_out);

/* Wait until every launch of the call that produced M (h2_mmp or
 * h2_matvec into M's context) has finished.  Errors: H2_ERR_ARG (null),
 * H2_ERR_DEVICE (a failed launch). */
h2_status h2_sync(h2_mat M);

/* a M + b I as a new matrix (a, b real): M's partition and bases, couplings
 * and dense blocks scaled by a, b added to the diagonal of the dense diagonal
 * leaf blocks (the identity of the partition lives there).  Errors:
 * H2_ERR_ARG (null pointers, non-finite a or b, M of another context),
 * H2_ERR_OOM. */
h2_status h2_scale_shift(h2_ctx ctx, h2_mat M, double a, double b, h2_mat* out);

/* Approximate inverse by repeated products (the use Section I names for the
 * product: inverse-based fast solvers): Newton-Schulz iteration
 * X_{j+1} = X_j (2 I - A X_j) from X_1 = 2 alpha I - alpha^2 A, `steps`
 * iterates (steps - 1 rounds of two h2_mmp at eps, trunc_mode and precision,
 * and one h2_scale_shift).  For A with eigenvalues in (0, 1/alpha] (e.g.
 * symmetric positive definite, alpha <= 1/lambda_max) the residual I - A X_j
 * squares every step until the truncation limits it.  X has A's partition.
 * Synchronous.  Errors: H2_ERR_ARG (steps < 1, alpha <= 0), and those of
 * h2_mmp. */
h2_status h2_newton_schulz(h2_ctx ctx, h2_mat A, double alpha, int steps, double eps,
                           int trunc_mode, int precision, h2_mat* X_out);

/* y = M x for nrhs right-hand sides, x and y n x nrhs column-major in the
 * original point order, host memory (x_on_device = 0) or device memory
 * (x_on_device = 1, both pointers device); complex M: x and y hold the
 * n x nrhs real parts followed by the n x nrhs imaginary parts (2 n nrhs
 * doubles).  Exact H^2 mat-vec: forward
 * transform up the column tree, couplings, backward transform down the row
 * tree, dense near field (the reference solution of equation `error`).
 * stream: see the conventions above (host vectors: the call always returns
 * with y filled). */
h2_status h2_matvec(h2_ctx ctx, h2_mat M, const double* x, double* y, int64_t nrhs,
                    int x_on_device, hipStream_t stream);

/* Allocation-free variant of h2_matvec with device vectors, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation).  y = M x as h2_matvec computes it (the
 * same kernels in the same order: identical results).  x_dev, y_dev: device
 * memory, n x nrhs column-major (complex M: planar, as in h2_matvec).  The
 * temporaries live in a library-wide device array of H2_MATVEC_SCRATCH_BYTES
 * per device, located when the first context on that device is created and
 * held until the process ends; they take 2 npad 2^L + sum over the levels
 * l_min..L of 2^l (rr_l + rc_l) doubles per right-hand side (twice for
 * complex M; npad, rr, rc the padded leaf size and ranks), each part rounded
 * to 256 bytes.  The work is launched on `stream` (null: the context's
 * stream) with no host wait, no event and no memset; M must be complete
 * (h2_sync after an h2_mmp on a caller stream).  Every call on one device
 * shares the array and it keeps the last call's contents: calls that overlap
 * on one GPU (other contexts or streams) race and must be serialised by the
 * caller.  Errors: H2_ERR_ARG (null pointers, nrhs < 1, M of another
 * context), H2_ERR_UNSUPPORTED (temporaries beyond the array; nothing is
 * launched). */
#define H2_MATVEC_SCRATCH_BYTES ((size_t)64 << 20)
h2_status h2_matvec_noalloc(h2_ctx ctx, h2_mat M, const double* x_dev, double* y_dev,
                            int64_t nrhs, hipStream_t stream);

/* Dense M (original order) into host memory `out` (column-major, ld >= n;
 * complex M: interleaved pairs, ld in complex elements).  Only for
 * n <= 16384 (H2_ERR_UNSUPPORTED above). */
h2_status h2_to_dense(h2_ctx ctx, h2_mat M, double* out, int64_t ld);

/* Sizes of M in the flat layout, for h2_export. */
typedef struct {
  int64_t n, L, nnodes;
  int64_t len_V, len_W, len_Er, len_Ec, len_S, len_F;
  int64_t is_complex; /* lengths count complex elements (two doubles each) */
} h2_export_sizes;
h2_status h2_export_size(h2_mat M, h2_export_sizes* sz);

/* Copy M to host in the flat layout (ranks stripped of padding).  Every
 * pointer must hold the number of elements h2_export_size reports:
 * leaf_off[2^L+1], perm[n], node_off[L+2], node_row/col/type[nnodes],
 * krow/kcol[2^(L+1)-1], V_off/W_off[2^L+1], Er_off/Ec_off[2^(L+1)],
 * S_off/F_off[nnodes+1], V[len_V] ... F[len_F]. */
typedef struct {
  int64_t *leaf_off, *perm, *node_off;
  int32_t *node_row, *node_col, *node_type;
  int64_t *krow, *kcol;
  double *V, *W, *Er, *Ec, *S, *F;
  int64_t *V_off, *W_off, *Er_off, *Ec_off, *S_off, *F_off;
} h2_export_buffers;
h2_status h2_export(h2_mat M, const h2_export_buffers* out);

/* File interchange in the flat layout above: a NumPy .npz archive (zip of
 * stored, uncompressed .npy members; numpy.load reads it, numpy.savez writes
 * what h2_load_file reads) with members n, L, is_complex (int64 scalars),
 * leaf_off, perm, node_off, krow, kcol and the *_off arrays (int64),
 * node_row, node_col, node_type (int32), and V, W, Er, Ec, S, F (float64, or
 * complex128 when is_complex).  Archives and members are limited to 4 GiB
 * (no zip64).
 * h2_save: writes M (the h2_export data) to `path`, replacing the file.
 *   Errors: H2_ERR_ARG (cannot write), H2_ERR_UNSUPPORTED (over 4 GiB).
 * h2_load_file: reads `path` and uploads it as h2_load does; members other
 *   than those listed are ignored.  Errors: H2_ERR_ARG (not an archive, a
 *   missing member, a wrong element type, sizes that do not match n and L,
 *   offsets that run past their arrays, a checksum mismatch), H2_ERR_UNSUPPORTED
 *   (compressed or zip64 members), and those of h2_load. */
h2_status h2_save(h2_mat M, const char* path);
h2_status h2_load_file(h2_ctx ctx, const char* path, h2_mat* out);

/* Statistics of the last h2_mmp that produced M (zeros for loaded
 * matrices).  rank_max/rank_mean per level for the row (r) and column (c)
 * bases; algorithmic work at the actual ranks (Sections III-IV), counted on
 * the first h2_stats call for M by a host pass over every evaluated block
 * product: flops_triple = one contraction per evaluated block product
 * (2 n^3 for a dense target, 2 r1 r2 r3 in rank form otherwise),
 * flops_target = the per-target products that apply the projections,
 * flops_gram = 2 d^2 per column contributed to a Gram sum of dimension d,
 * eig_flops = 9 d^3 per Gram matrix, flops = their sum (complex: four real
 * products per complex one, eight for the eigen-decompositions of the real
 * embedding); device time of the numeric phase in ms (waits for the product
 * to finish); per kernel class (with h2_set_profiling on) summed device ms,
 * launches and executed (padded) flops. */
#define H2_MAX_LEVELS 40
typedef struct {
  int64_t L, lmin;
  int64_t rank_max_r[H2_MAX_LEVELS], rank_max_c[H2_MAX_LEVELS];
  double rank_mean_r[H2_MAX_LEVELS], rank_mean_c[H2_MAX_LEVELS];
  double flops;
  double mmp_ms;
  double symbolic_ms;
  int64_t n_triples;
  int64_t sparsity_constant;
  /* the per-triple contraction kernels (k_bgemm_triple) */
  double contraction_ms;
  int64_t contraction_launches;
  double contraction_flops;
  double eig_ms;
  /* peak device bytes held by live allocations of the context during the
   * product (operands, the product and its temporaries; blocks cached by
   * the context's pool are not counted) */
  int64_t bytes_device;
  /* Gram-sum products, and the remaining batched products other than the
   * per-target ones (projections, collects, split, cluster-basis products) */
  double gram_ms, other_ms;
  int64_t eig_launches, gram_launches, other_launches;
  double gram_flops, other_flops;
  double eig_flops;
  double flops_triple, flops_target, flops_gram;
  /* the per-target products (k_bgemm_target): summed device ms and launches */
  double target_ms;
  int64_t target_launches;
  /* the eigensolver's three kernels (eig_ms is their sum): tridiagonalisation,
   * eigenvalues and kept count, eigenvectors */
  double eig_tri_ms, eig_val_ms, eig_vec_ms;
  /* algorithmic work of two of them: (4/3) d^3 per reduction, 6 d^2 k per
   * set of k kept eigenvectors (not part of flops, whose eigensolver term is
   * the 9 d^3 of eig_flops) */
  double eig_tri_flops, eig_vec_flops;
} h2_stats_t;
h2_status h2_stats(h2_mat M, h2_stats_t* out);

/* Symbolic phase of C = A A' for the structure in m (block tree only; no
 * device work, callable without a GPU).  Fills per level l (0..L): the
 * number of evaluated block products ("triples": an A node (I,J) and a B node
 * (J,K) of level l, not both non-leaf; Sections III-IV), of temporary
 * couplings of targets that lie inside an upper-level admissible block
 * ("blue" blocks of Fig. 3(c)) and of merged targets (equation nonleafA).
 * Arrays have max_levels entries; *lmin receives the lowest level with an
 * admissible block.  Errors: H2_ERR_ARG (invalid structure, max_levels <= L). */
h2_status h2_plan_info(const h2_host_matrix* m, int64_t max_levels, int64_t* triples,
                       int64_t* blue, int64_t* merged, int64_t* lmin);

/* Enable (1) or disable (0) per-kernel event timing inside h2_mmp. */
h2_status h2_set_profiling(h2_ctx ctx, int on);

void h2_free(h2_mat M);
const char* h2_last_error(void);
int h2_version(void);

#ifdef __cplusplus
}
#endif
#endif /* H2MMP_H */
