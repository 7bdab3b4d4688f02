// Internal launch interface of the HIP kernels (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace h2k {

// A batch of equally shaped column-major blocks.  Block index v encodes
// (tile << 3) | (sel << 2) | (col_half << 1) | row_half; the block starts at
// base[sel] + tile*stride[sel] + row_half*sub_r + col_half*sub_c.
struct Opnd {
  const void* base[2];
  long long stride[2];
  int ld;
  long long sub_r;
  long long sub_c;
  int f32;  // elements are float (else double); both bases share the type
};

// T is the arithmetic type (FP64 or FP32 MFMA) and the type of C (c_f32 must
// match); each operand may be stored in either precision.
template <typename T>
struct BgemmArgs {
  int m, n, k, nout, tiles_m, tiles_n;
  int transA, transB;
  Opnd A, B;
  void* C;
  int c_f32;
  long long cstride;
  int ldc;
  long long csub_r, csub_c;
  const int* out_idx;  // [nout], encoded like operand indices (sel ignored)
  const int* seg;      // [nout+1] task ranges
  const int* a_idx;    // [ntask]
  const int* b_idx;    // [ntask]
  T alpha, beta;
  int symbol;  // kernel symbol for traces: 0 k_bgemm, 1 k_bgemm_triple (per-triple
               // contractions), 2 k_bgemm_target (per-target products),
               // 3 k_bgemm_gram (Gram sums, FP64 only)
  int tile;    // workgroup tile (kTile* id), -1: chosen from the output shape
  // symmetric outputs read only on and below the diagonal: compute only the
  // tiles there (m == n and a square tile; otherwise ignored)
  int lower;
};

// Workgroup tiles of the batched GEMM (rows x columns of C per workgroup)
// (kTile32x32ws: the wave-split 32 x 32 tile, each wave a quarter of the
// segment's tasks)
enum {
  kTile32x32 = 0, kTile96x32 = 1, kTile32x96 = 2, kTile96x96 = 3,
  kTile32x64 = 4, kTile64x32 = 5, kTile64x64 = 6, kTile32x32ws = 7, kTileCount = 8
};

template <typename T>
struct SegsumArgs {
  int m, n, nout;
  Opnd A;
  T* C;
  long long cstride;
  int ldc;
  long long csub_r, csub_c;
  const int* out_idx;
  const int* seg;
  const int* a_idx;
  T beta;
};

struct GramNormArgs {
  const double* G[3];  // G[1], G[2] may be null (absent components)
  long long stride;
  int D;
  double* out;
  int* status;
};

// Batched truncated eigen-decomposition of symmetric positive semi-definite
// Gram matrices (FP64).  Cluster c: the D x D matrix at G + c*gstride (ld D)
// restricted to rows/columns [0,k1[c]) and [half, half+k2[c]) (the children's
// live coordinates); output orthonormal eigenvectors (descending) in
// U + c*ustride (D x D, ld D) scattered back to the padded rows, zero columns
// beyond the kept rank, rank[c] = kept count.
struct EigArgs {
  const double* G;
  long long gstride;
  int D;
  double* U;
  long long ustride;
  int* rank;
  const int* k1;   // k1[c*kstride]: live rows of the first child (or of the leaf)
  const int* k2;   // k2[c*kstride]: live rows of the second child (null: none)
  int kstride;
  int half;
  double* scratch;  // per cluster eig_scratch_doubles(D) doubles
  long long sstride;
  double tau;
  int exact;
  const int* kmax;  // nullable: kmax[c] caps the kept count of cluster c (at least 1 kept)
  int* status;  // [0] non-finite, [1] dimension over limit
};

// Complex Hermitian Gram matrices through the real eigensolver.  A Hermitian
// H = X + iY has the same eigenvalues as the real symmetric [[X, -Y], [Y, X]],
// each twice; an eigenvector [a; b] of the embedding gives the complex
// eigenvector a + ib, and the two copies of an eigenvalue give the same
// complex direction (up to a phase).
//  embed: H = sum_m G_m / Re tr(G_m) (Hermitian part) of cluster c, rows and
//    columns restricted to [0,k1) and [half, half+k2) and compacted to n live
//    rows, into E (2D x 2D): [0,n) real block, [D, D+n) imaginary block;
//    nlive[c] = n;
//  extract: the kept real eigenvectors (column m of Ue, rank_e[c] of them)
//    mapped to a + ib and orthonormalised in order by complex Gram-Schmidt
//    (twice); a vector left with less than half its norm repeats an accepted
//    direction and is dropped.  The accepted vectors go to U (D x D, planes
//    [real | imaginary] at +uplane, padded rows), rank[c] = their count.
struct CEigArgs {
  const double* G[3];  // complex Gram components (cluster stride D*D, planes at +gplane; G[1], G[2] may be null)
  long long gplane;
  int D, half;
  const int* k1;
  const int* k2;  // null: none
  int kstride;
  double* E;      // 2D x 2D per cluster
  int* nlive;
  const double* Ue;  // 2D x 2D per cluster: real eigenvectors of E
  const int* rank_e;
  double* U;
  long long uplane;
  int* rank;
  const int* kmax;  // nullable: kmax[c] caps the accepted count (at least 1)
  int* status;
};
hipError_t launch_ceig_embed(const CEigArgs& a, const CEigArgs& b, int nclusters, hipStream_t s);
hipError_t launch_ceig_extract(const CEigArgs& a, const CEigArgs& b, int nclusters, hipStream_t s);

constexpr int kEigNmax = 1024;  // largest Gram dimension
constexpr int kEigLdsN = 195;  // largest dimension whose packed triangle stays in LDS
constexpr int kEigRegN = 256;  // largest dimension the register-resident reduction holds
// scratch per cluster (doubles) the eigensolver needs for padded dimension D
inline long long eig_scratch_doubles(int D) { return 7LL * D * D + 4LL * D + 8; }

template <typename T>
hipError_t launch_bgemm(const BgemmArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_segsum(const SegsumArgs<T>& a, hipStream_t s);
hipError_t launch_gram_norm(const GramNormArgs& a, int nclusters, hipStream_t s);
// two problem sets (row and column bases of one level) in one launch per
// phase: tridiagonalisation, eigenvalues and kept count, eigenvectors (the
// phases in order, any subset per call)
constexpr int kEigPhaseTri = 1, kEigPhaseVal = 2, kEigPhaseVec = 4, kEigPhaseAll = 7;
hipError_t launch_eig(const EigArgs& a, const EigArgs& b, int nclusters, hipStream_t s,
                      int phases = kEigPhaseAll);
// Kernel entries of h2_build (1/(4 pi r), self_value at r = 0).  Coupling
// matrices of one level: node q (rows[q], cols[q], types[q]; type 0 =
// admissible) gets the kernel at the row and column clusters' p^3 tensor
// Chebyshev nodes (axes: per cluster 3 x p node coordinates) at
// S + q*rr*rc (ld rr).  Dense leaf blocks (type 1): the kernel at the points
// (pts: tree order, 3 per point) of the two leaves at F + q*npad^2 (ld npad).
struct BuildCouplingArgs {
  const double* axes;
  const int *rows, *cols, *types;
  int nnodes, p, rr, rc;
  double self_value;
  double* S;
  int helmholtz;      // exp(-j kappa r)/(4 pi r) into two planes, else 1/(4 pi r)
  double kappa, self_imag;
  long long plane;    // imaginary-plane offset of S (Helmholtz)
};
struct BuildDenseArgs {
  const double* pts;
  const long long* leaf_off;
  const int *rows, *cols, *types;
  int nnodes, npad;
  double self_value;
  double* F;
  int helmholtz;
  double kappa, self_imag;
  long long plane;    // imaginary-plane offset of F (Helmholtz)
};
hipError_t launch_build_coupling(const BuildCouplingArgs& a, hipStream_t s);
hipError_t launch_build_dense(const BuildDenseArgs& a, hipStream_t s);

hipError_t launch_fill(double* p, double v, long long n, hipStream_t s);
hipError_t launch_scale(double* p, double a, long long n, hipStream_t s);
// F[node[t] npad^2 + r (npad + 1)] += b for r < size[t], t < nblocks
hipError_t launch_shift_diag(double* F, const int* node, const int* size, int nblocks, int npad,
                             double b, hipStream_t s);
hipError_t launch_fill_f(float* p, float v, long long n, hipStream_t s);
hipError_t launch_d2f(const double* in, float* out, long long n, hipStream_t s);
hipError_t launch_f2d(const float* in, double* out, long long n, hipStream_t s);
hipError_t launch_gather_rows(const double* x, double* out, const long long* perm,
                              const long long* leaf_off, int nleaf, int npad, long long n,
                              int nrhs, hipStream_t s);
hipError_t launch_scatter_rows(const double* in, double* y, const long long* perm,
                               const long long* leaf_off, int nleaf, int npad, long long n,
                               int nrhs, hipStream_t s);

}  // namespace h2k
