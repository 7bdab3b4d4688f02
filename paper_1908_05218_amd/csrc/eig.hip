// Batched truncated eigen-decomposition of the summed normalised Gram
// matrices that fix each new cluster basis of C (Sections III-C and IV-C of
// Ma & Jiao).  The Gram matrix is symmetric positive semi-definite, so the
// left singular vectors the method keeps are its leading eigenvectors; the
// kept count follows from the truncation threshold tau * lambda_1.
//
// One workgroup per cluster (NT = 64..512 lanes chosen from the padded
// dimension D <= 1024; each lane holds SL = 1, 2, 4, 8 or 16 rows of a column,
// as many as D needs, so one wave covers a whole column), FP64 throughout:
//   1. gather the live rows/columns (the children's actual ranks; only the
//      Gram's lower triangle is read);
//   2. Householder reduction to tridiagonal form.  Up to D = 256 the matrix
//      stays in registers (kernel k_eig_tri_reg: block lower triangle spread
//      over the waves by columns, transposed terms of the symmetric product
//      summed by a lane-swap butterfly, three barriers per step).  Above, a
//      packed lower triangle in LDS (n <= kEigLdsN) or in the cluster's
//      scratch: the symmetric product split over waves, the rank-2 update
//      by lanes over rows of one column at a time.  Finished reflectors go to
//      the cluster's scratch;
//   3. lambda_1 by multisection of Sturm counts, the kept count k by one
//      Sturm count at the threshold, then the k leading eigenvalues by
//      grouped multisection (G lanes and two interleaved Sturm sequences per
//      eigenvalue, G chosen for the fewest waves per SIMD x iterations);
//   4. eigenvectors of the tridiagonal matrix by two steps of inverse
//      iteration per lane (Gaussian elimination with partial pivoting fused
//      with the forward sweep of the right-hand side); eigenvalues closer than
//      1e-12 ||T|| are handled as clusters (fresh start, orthogonalisation
//      against the earlier members between solves);
//   5. block Gram-Schmidt with one re-orthogonalisation over all kept
//      vectors, in descending eigenvalue order.  Up to D = 256 each wave
//      holds one vector of a block in registers and projects it out of the
//      earlier blocks eight vectors at a time, then the waves orthonormalise
//      inside the block in turn; above, blocks of 8 projected by the
//      workgroup and orthonormalised inside by one wave;
//   6. back-transformation by the reflectors, one wave per eight (four, two
//      for the largest dimensions) vectors held in registers, and scatter to
//      the padded row layout.
// Wave reductions use DPP row operations, lane-half swaps and lane reads,
// not LDS permutes.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace h2k {
namespace {

constexpr int kLdsBytes = 163840;  // LDS per workgroup on gfx950
constexpr int kVB = 4;             // vectors per wave in the back-transformation
constexpr int kRed = 8;            // reduction slots in LDS: one per wave, up to 512 lanes

// index of the calling wave in its workgroup, as a wave-uniform (scalar) value
// so that per-wave index arithmetic runs on the scalar unit
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave; every lane gets the same value.  Every lane
// of the wave must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror: each row of 16 lanes now holds its sum
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Maximum (MAX) or minimum over aligned groups of G in {1, 2, 4, 8} lanes.
template <bool MAX>
__device__ __forceinline__ double group_red(double v, int G) {
  if (G >= 2) v = MAX ? fmax(v, dpp<0xB1>(v)) : fmin(v, dpp<0xB1>(v));
  if (G >= 4) v = MAX ? fmax(v, dpp<0x4E>(v)) : fmin(v, dpp<0x4E>(v));
  if (G >= 8) v = MAX ? fmax(v, dpp<0x141>(v)) : fmin(v, dpp<0x141>(v));
  return v;
}

// exchange of 64-bit values between lane halves (xor 32) or between odd and
// even rows of 16 lanes (xor 16): afterwards x holds the first operand's
// lower part and the second operand's lower part, y the two upper parts
__device__ __forceinline__ void swap_halves32(double& x, double& y) {
  const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
  const unsigned long long yb = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap_rows16(double& x, double& y) {
  const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
  const unsigned long long yb = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// Sums over the 64 lanes of t[0..7]; every lane receives all eight in
// out[] (wave-uniform).  Halving exchanges (lane-half swaps for xor 32 and
// xor 16, a quad permute for xor 1) leave each lane one of the eight values,
// the rest of its lanes are summed by quad permute and row rotates, and the
// eight sums are read from one lane each.  Every lane of the wave must be
// active.
__device__ __forceinline__ void wave_sum8(const double* t, double* out) {
  double t1[4], t2[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double x = t[2 * k], y = t[2 * k + 1];
    swap_halves32(x, y);
    t1[k] = x + y;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double x = t1[2 * k], y = t1[2 * k + 1];
    swap_rows16(x, y);
    t2[k] = x + y;
  }
  // lane l now holds partial sums of values 4k + 2 b4 + b5 (b_k: bit k of l)
  const bool b0 = threadIdx.x & 1;
  const double keep = b0 ? t2[1] : t2[0], give = b0 ? t2[0] : t2[1];
  double v = keep + dpp<0xB1>(give);  // value 4 b0 + 2 b4 + b5
  v += dpp<0x4E>(v);                  // quad_perm [2,3,0,1]
  v += dpp<0x128>(v);                 // row_ror:8
  v += dpp<0x124>(v);                 // row_ror:4
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q] = read_lane(v, ((q >> 2) & 1) | (((q >> 1) & 1) << 4) | ((q & 1) << 5));
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// start of column j of a packed lower triangle of order n
__device__ __forceinline__ int cs(int j, int n) { return j * n - (j * (j - 1)) / 2; }

// 1/q from the hardware reciprocal refined by two Newton steps (to about one
// ulp): the Sturm recurrence below only needs its result to a few ulps, the
// count being exact for a matrix perturbed at that level
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return fma(r, fma(-q, r, 1.0), r);
}

// number of eigenvalues below xa and below xb (Sturm counts, two sequences
// interleaved)
__device__ __forceinline__ void sturm2(const double* d, const double* e2, int n, double xa,
                                       double xb, double pivmin, int& ca, int& cb) {
  double qa = d[0] - xa, qb = d[0] - xb;
  int na = qa < 0.0, nb = qb < 0.0;
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
    if (fabs(qa) < pivmin) qa = -pivmin;
    if (fabs(qb) < pivmin) qb = -pivmin;
    qa = (di - xa) - ei * recip(qa);
    qb = (di - xb) - ei * recip(qb);
    na += qa < 0.0;
    nb += qb < 0.0;
  }
  ca = na;
  cb = nb;
}

__device__ __forceinline__ int sturm1(const double* d, const double* e2, int n, double x,
                                      double pivmin) {
  double q = d[0] - x;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d[i] - x) - e2[i - 1] * recip(q);
    cnt += q < 0.0;
  }
  return cnt;
}

__device__ __forceinline__ double start_vec(int r, int m) {
  return cos(0.7548776662 * r + 0.5698402909 * m) + 0.1;
}

// Per-lane solve (T - lm I) x = b for the tridiagonal T = (dd, ee): Gaussian
// elimination with partial pivoting, the factor and the right-hand side swept
// together; the factor rows (reciprocal pivot, two superdiagonals) and the
// swept right-hand side are kept interleaved by m in F[0..3] (stride fs) for
// the backward sweep.  b is the start vector of seed `seed` (fresh) or zm
// itself; x overwrites zm and is normalised.  Near-singular pivots are
// clamped to +-tiny (one hardware reciprocal refined by Newton steps serves
// both the multiplier and the stored reciprocal pivot); a growing solution is
// rescaled before it can overflow.
__device__ __forceinline__ void invit_solve(const double* dd, const double* ee, int n, double lm, double tiny,
                            double* F0, double* F1, double* F2, double* F3, int fs, int m,
                            double* zm, bool fresh, int seed) {
  // Global loads and stores share one in-order completion counter, so a load
  // issued after a store waits for that store too.  Every sweep below works
  // in batches of C steps and issues the next batch's loads before the
  // current batch's stores.
  constexpr int C = 4;
  double di = dd[0] - lm;
  double ui = n > 1 ? ee[0] : 0.0;
  double bi = fresh ? start_vec(0, seed) : zm[0];
  double rb[C], rn[C];  // right-hand side entries of this batch and the next
  if (!fresh) {
#pragma unroll
    for (int t = 0; t < C; ++t) rb[t] = zm[1 + t < n ? 1 + t : n - 1];
  }
  for (int i0 = 0; i0 < n - 1; i0 += C) {
    if (!fresh) {
#pragma unroll
      for (int t = 0; t < C; ++t) {
        const int r = i0 + C + 1 + t;
        rn[t] = zm[r < n ? r : n - 1];
      }
    }
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const int i = i0 + t;
      if (i < n - 1) {
        const double li = ee[i];
        const double dn = dd[i + 1] - lm;
        const double un = i < n - 2 ? ee[i + 1] : 0.0;
        const double bn = fresh ? start_vec(i + 1, seed) : rb[t];
        double rp, u1, u2, y;  // rp: reciprocal of the pivot
        if (fabs(di) >= fabs(li)) {
          if (fabs(di) < tiny) di = di < 0.0 ? -tiny : tiny;
          rp = recip(di);
          u1 = ui;
          u2 = 0.0;
          y = bi;
          const double f = li * rp;
          di = dn - f * ui;
          ui = un;
          bi = bn - f * bi;
        } else {
          const double lp = fabs(li) < tiny ? (li < 0.0 ? -tiny : tiny) : li;
          rp = recip(lp);
          u1 = dn;
          u2 = un;
          y = bn;
          const double f = di * rp;
          di = ui - f * dn;
          ui = -f * un;
          bi = bi - f * bn;
        }
        const long long o = (long long)i * fs + m;
        F0[o] = rp;
        F1[o] = u1;
        F2[o] = u2;
        F3[o] = y;
      }
    }
    if (!fresh) {
#pragma unroll
      for (int t = 0; t < C; ++t) rb[t] = rn[t];
    }
  }
  if (fabs(di) < tiny) di = di < 0.0 ? -tiny : tiny;
  double x1 = bi / di, x2 = 0.0;
  zm[n - 1] = x1;
  double amax = fabs(x1);
  // backward sweep: factor rows of the next batch fetched before this
  // batch's solution entries are stored
  double r0[C], r1[C], r2[C], r3[C], q0[C], q1[C], q2[C], q3[C];
#pragma unroll
  for (int t = 0; t < C; ++t) {
    const int ii = n - 2 - t;
    const long long o = (long long)(ii < 0 ? 0 : ii) * fs + m;
    r0[t] = F0[o];
    r1[t] = F1[o];
    r2[t] = F2[o];
    r3[t] = F3[o];
  }
  for (int i = n - 2; i >= 0; i -= C) {
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const int ii = i - C - t;
      const long long o = (long long)(ii < 0 ? 0 : ii) * fs + m;
      q0[t] = F0[o];
      q1[t] = F1[o];
      q2[t] = F2[o];
      q3[t] = F3[o];
    }
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const int ii = i - t;
      if (ii >= 0) {
        const double xi = (r3[t] - r1[t] * x1 - r2[t] * x2) * r0[t];
        x2 = x1;
        x1 = xi;
        zm[ii] = xi;
        amax = fmax(amax, fabs(xi));
        if (fabs(xi) > 1e150) {
          for (int r = ii; r < n; ++r) zm[r] *= 1e-150;
          for (int r = 0; r < ii; ++r) F3[(long long)r * fs + m] *= 1e-150;
          for (int u = t + 1; u < C; ++u) r3[u] *= 1e-150;
#pragma unroll
          for (int u = 0; u < C; ++u) q3[u] *= 1e-150;
          x1 *= 1e-150;
          x2 *= 1e-150;
          amax *= 1e-150;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < C; ++t) {
      r0[t] = q0[t];
      r1[t] = q1[t];
      r2[t] = q2[t];
      r3[t] = q3[t];
    }
  }
  if (!(amax > 0.0) || !(amax < 1e308)) return;
  double s = 0.0;
  for (int r = 0; r < n; ++r) {
    const double v = zm[r] / amax;
    s += v * v;
  }
  const double inv = 1.0 / (amax * sqrt(s));
  // scale in batches, the next batch loaded before this batch is stored
  double v[C], w[C];
#pragma unroll
  for (int t = 0; t < C; ++t) v[t] = zm[t < n ? t : n - 1];
  for (int r0b = 0; r0b < n; r0b += C) {
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const int r = r0b + C + t;
      w[t] = zm[r < n ? r : n - 1];
    }
#pragma unroll
    for (int t = 0; t < C; ++t)
      if (r0b + t < n) zm[r0b + t] = v[t] * inv;
#pragma unroll
    for (int t = 0; t < C; ++t) v[t] = w[t];
  }
}

// Z[:, m] -= sum_{q0 <= q < m} (Z[:,q] . Z[:,m]) Z[:,q], twice (classical
// Gram-Schmidt with one re-orthogonalisation), then normalise.  Z is
// column-major with leading dimension ldz.  Whole workgroup.
template <int NT>
__device__ void cgs2(double* Z, int ldz, int n, int m, int q0, double* dots, double* red) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  double* zm = Z + (long long)m * ldz;
  for (int pass = 0; pass < 2 && m > q0; ++pass) {
    for (int q = q0 + wave; q < m; q += NW) {
      const double* zq = Z + (long long)q * ldz;
      double s = 0.0;
      for (int r = lane; r < n; r += 64) s += zq[r] * zm[r];
      s = wave_sum(s);
      if (lane == 0) dots[q] = s;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += NT) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int q = q0;
      for (; q + 3 < m; q += 4) {
        s0 += dots[q] * Z[(long long)q * ldz + r];
        s1 += dots[q + 1] * Z[(long long)(q + 1) * ldz + r];
        s2 += dots[q + 2] * Z[(long long)(q + 2) * ldz + r];
        s3 += dots[q + 3] * Z[(long long)(q + 3) * ldz + r];
      }
      for (; q < m; ++q) s0 += dots[q] * Z[(long long)q * ldz + r];
      zm[r] -= (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
  }
  double part = 0.0;
  for (int r = threadIdx.x; r < n; r += NT) part += zm[r] * zm[r];
  const double nrm2 = block_sum<NT>(part, red);
  const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  for (int r = threadIdx.x; r < n; r += NT) zm[r] *= inv;
  __syncthreads();
}

// Orthonormalises vectors m0 .. m0+b-1 (b <= 8) of Z among themselves, in
// order, by the calling wave (every lane active): each vector twice against
// the block's earlier members; a vector that loses more than half its norm
// there is re-orthogonalised twice against every earlier vector; then it is
// normalised.
template <int SL>
__device__ void orth_block(double* Z, int ldz, int n, int m0, int b) {
  const int lane = threadIdx.x & 63;
  for (int j = 0; j < b; ++j) {
    double* zj = Z + (long long)(m0 + j) * ldz;
    double z[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int r = lane + 64 * s;
      z[s] = r < n ? zj[r] : 0.0;
    }
    double t0 = 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) t0 += z[s] * z[s];
    const double nb2 = wave_sum(t0);
    for (int pass = 0; pass < 2 && j > 0; ++pass) {
      double t8[8], d[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        double t = 0.0;
        if (jj < j) {
          const double* zq = Z + (long long)(m0 + jj) * ldz;
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const int r = lane + 64 * s;
            if (r < n) t += zq[r] * z[s];
          }
        }
        t8[jj] = t;
      }
      wave_sum8(t8, d);
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        if (jj < j) {
          const double* zq = Z + (long long)(m0 + jj) * ldz;
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const int r = lane + 64 * s;
            if (r < n) z[s] -= d[jj] * zq[r];
          }
        }
      }
    }
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) t += z[s] * z[s];
    double nrm2 = wave_sum(t);
    if (nrm2 < 0.25 * nb2) {
      // the vector was nearly dependent on the block's earlier members:
      // what is left is rounding noise that still leans on the earlier
      // blocks, so it is re-orthogonalised against every earlier vector,
      // twice, before it is normalised
      for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < m0 + j; ++q) {
          const double* zq = Z + (long long)q * ldz;
          double u = 0.0;
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const int r = lane + 64 * s;
            if (r < n) u += zq[r] * z[s];
          }
          const double dq = wave_sum(u);
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const int r = lane + 64 * s;
            if (r < n) z[s] -= dq * zq[r];
          }
        }
      t = 0.0;
#pragma unroll
      for (int s = 0; s < SL; ++s) t += z[s] * z[s];
      nrm2 = wave_sum(t);
    }
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int r = lane + 64 * s;
      if (r < n) zj[r] = z[s] * inv;
    }
  }
}

// Block classical Gram-Schmidt with re-orthogonalisation over the k kept
// vectors (columns of Z, leading dimension ldz), in blocks of at most 8 (the
// path for dimensions above 256 and for workgroups of fewer than four waves):
// two passes project a block on all earlier vectors (whole workgroup), then
// wave 0 orthonormalises inside the block (each vector twice against the
// block's earlier members; a vector that loses more than half its norm there
// is re-orthogonalised twice against every earlier vector; then normalised).  Dc: cap doubles of LDS for the
// projection coefficients.
template <int NT, int SL>
__device__ void bcgs2(double* Z, int ldz, int n, int k, double* Dc, int cap) {
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  for (int m0 = 0; m0 < k;) {
    int b = k - m0 < 8 ? k - m0 : 8;
    if (m0 > 0 && b * m0 > cap) b = cap / m0 > 0 ? cap / m0 : 1;
    for (int pass = 0; pass < 2 && m0 > 0; ++pass) {
      for (int e = tid; e < m0 * b; e += NT) {
        const int q = e % m0, j = e / m0;
        const double* zq = Z + (long long)q * ldz;
        const double* zj = Z + (long long)(m0 + j) * ldz;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int r = 0;
        for (; r + 3 < n; r += 4) {
          s0 += zq[r] * zj[r];
          s1 += zq[r + 1] * zj[r + 1];
          s2 += zq[r + 2] * zj[r + 2];
          s3 += zq[r + 3] * zj[r + 3];
        }
        for (; r < n; ++r) s0 += zq[r] * zj[r];
        Dc[j * m0 + q] = (s0 + s1) + (s2 + s3);
      }
      __syncthreads();
      for (int e = tid; e < n * b; e += NT) {
        const int r = e % n, j = e / n;
        const double* dj = Dc + j * m0;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int q = 0;
        for (; q + 3 < m0; q += 4) {
          s0 += dj[q] * Z[(long long)q * ldz + r];
          s1 += dj[q + 1] * Z[(long long)(q + 1) * ldz + r];
          s2 += dj[q + 2] * Z[(long long)(q + 2) * ldz + r];
          s3 += dj[q + 3] * Z[(long long)(q + 3) * ldz + r];
        }
        for (; q < m0; ++q) s0 += dj[q] * Z[(long long)q * ldz + r];
        Z[(long long)(m0 + j) * ldz + r] -= (s0 + s1) + (s2 + s3);
      }
      __syncthreads();
    }
    if (wave == 0) orth_block<SL>(Z, ldz, n, m0, b);
    __syncthreads();
    m0 += b;
  }
}

// Block Gram-Schmidt with re-orthogonalisation for dimensions up to 256
// (four row slots), in blocks of NW vectors; wave j holds vector m0 + j in
// registers throughout.  It first projects the vector out of all earlier
// blocks, twice, eight vectors at a time (one batched wave sum per eight dot
// products, the projection subtracted at once).  Inside the block the waves
// then take turns: at step t wave t normalises its vector (after
// re-orthogonalising it twice against every earlier vector if it kept less
// than half its norm) and stores it, and each later wave projects it out,
// twice.
template <int NT, int SL>
__device__ void bcgs2_waves(double* Z, int ldz, int n, int k) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = wave_id();
  for (int m0 = 0; m0 < k; m0 += NW) {
    const int b = k - m0 < NW ? k - m0 : NW;
    const bool mine = wave < b;
    double* zj = Z + (long long)(m0 + (mine ? wave : 0)) * ldz;
    double z[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int r = lane + 64 * s;
      z[s] = (mine && r < n) ? zj[r] : 0.0;
    }
    if (mine && m0 > 0) {
      // groups of eight earlier vectors, the next group loaded while this
      // one is applied (the loads' latency, not the arithmetic, sets the pace)
      double zq[8][SL], zn[8][SL];
      for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int qq = 0; qq < 8; ++qq) {
          const double* col = Z + (long long)(qq < m0 ? qq : 0) * ldz;
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const int r = lane + 64 * s;
            zq[qq][s] = (qq < m0 && r < n) ? col[r] : 0.0;
          }
        }
        for (int q0 = 0; q0 < m0; q0 += 8) {
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            const int q = q0 + 8 + qq;
            const double* col = Z + (long long)(q < m0 ? q : 0) * ldz;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
              const int r = lane + 64 * s;
              zn[qq][s] = (q < m0 && r < n) ? col[r] : 0.0;
            }
          }
          double t[8], d[8];
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            t[qq] = 0.0;
#pragma unroll
            for (int s = 0; s < SL; ++s) t[qq] += zq[qq][s] * z[s];
          }
          wave_sum8(t, d);
#pragma unroll
          for (int qq = 0; qq < 8; ++qq)
#pragma unroll
            for (int s = 0; s < SL; ++s) z[s] -= d[qq] * zq[qq][s];
#pragma unroll
          for (int qq = 0; qq < 8; ++qq)
#pragma unroll
            for (int s = 0; s < SL; ++s) zq[qq][s] = zn[qq][s];
        }
      }
    }
    double nb2 = 0.0;
    if (mine) {
      double t0 = 0.0;
#pragma unroll
      for (int s = 0; s < SL; ++s) t0 += z[s] * z[s];
      nb2 = wave_sum(t0);
    }
    for (int t = 0; t < b; ++t) {
      if (wave == t) {
        double t1 = 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s) t1 += z[s] * z[s];
        double nrm2 = wave_sum(t1);
        if (nrm2 < 0.25 * nb2) {
          // nearly dependent on the block's earlier members: what is left is
          // rounding noise that still leans on earlier vectors
          for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < m0 + t; ++q) {
              const double* zq = Z + (long long)q * ldz;
              double u = 0.0;
#pragma unroll
              for (int s = 0; s < SL; ++s) {
                const int r = lane + 64 * s;
                if (r < n) u += zq[r] * z[s];
              }
              const double dq = wave_sum(u);
#pragma unroll
              for (int s = 0; s < SL; ++s) {
                const int r = lane + 64 * s;
                if (r < n) z[s] -= dq * zq[r];
              }
            }
          t1 = 0.0;
#pragma unroll
          for (int s = 0; s < SL; ++s) t1 += z[s] * z[s];
          nrm2 = wave_sum(t1);
        }
        const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const int r = lane + 64 * s;
          z[s] *= inv;
          if (r < n) zj[r] = z[s];
        }
      }
      __syncthreads();
      if (mine && wave > t) {
        const double* qt = Z + (long long)(m0 + t) * ldz;
        double qv[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const int r = lane + 64 * s;
          qv[s] = r < n ? qt[r] : 0.0;
        }
        for (int pass = 0; pass < 2; ++pass) {
          double u = 0.0;
#pragma unroll
          for (int s = 0; s < SL; ++s) u += qv[s] * z[s];
          const double dq = wave_sum(u);
#pragma unroll
          for (int s = 0; s < SL; ++s) z[s] -= dq * qv[s];
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace

// LDS layout (doubles): [0, zr) packed triangle, later the eigenvectors |
// dd[dv] | ee[dv] | vv[dv] (reflector, later the eigenvalues) | pv[dv]
// (squared off-diagonal, later Gram-Schmidt coefficients) | ybuf[NT] |
// red[8].  Cluster scratch (doubles, sstride >= 7 D^2): [0, D^2) packed
// reflectors (or the whole packed matrix when it is not in LDS) | 4 D^2
// factor rows | (D|1) D eigenvectors when they are not in LDS.
// Phases 1-2 for one cluster: gather and Householder tridiagonalisation.
// PL: the packed triangle P lives in LDS (the caller passes the LDS base, so
// every access compiles to an LDS instruction), else P is the scratch copy Pg.
template <int NT, int SL, bool PL>
__device__ __forceinline__ void gather_tridiag(const EigArgs& p, const double* Gc, int n, int k1,
                                               int half, int D, double* P, double* Pg,
                                               double* dd, double* ee, double* vv,
                                               double* ybuf, double* trash, int stop) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  // 1. gather the live block, packed lower triangle
  int bad = 0;
  for (int j = wave; j < n; j += NW) {
    const int oj = j < k1 ? j : half + (j - k1);
    const int cj = cs(j, n) - j;
    for (int i = j + lane; i < n; i += 64) {
      const int oi = i < k1 ? i : half + (i - k1);
      const double v = Gc[oi + (long long)oj * D];
      if (!(v == v) || v - v != 0.0) bad = 1;
      P[cj + i] = v;
    }
  }
  if (bad) p.status[0] = 1;
  __syncthreads();

  // 2. Householder tridiagonalisation (lower); reflector u_i (unit norm,
  // H_i = I - 2 u_i u_i^T) kept in column i of Pg.  With stop < n - 2 only
  // the first `stop` steps run and the trailing block stays in P
  for (int i = 0; i + 2 < n && i < stop; ++i) {
    const int m = n - i - 1;
    const int ci = cs(i, n);
    double xr[SL], ur[SL];
    double part = 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int r = i + 1 + lane + 64 * s;
      xr[s] = r < n ? P[ci + r - i] : 0.0;
      part += xr[s] * xr[s];
    }
    const double xx = wave_sum(part);
    const double x0 = P[ci + 1];
    const double nx = sqrt(xx);
    if (!(nx > 0.0)) {  // column already reduced: H_i = I
      if (wave == 0) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const int r = i + 1 + lane + 64 * s;
          if (r < n) Pg[ci + r - i] = 0.0;
        }
        if (lane == 0) {
          dd[i] = P[ci];
          ee[i] = 0.0;
        }
      }
      __syncthreads();
      continue;
    }
    const double alpha = -copysign(nx, x0);
    const double v0 = x0 - alpha;
    const double vn = sqrt(xx - x0 * x0 + v0 * v0);
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int r = i + 1 + lane + 64 * s;
      ur[s] = r < n ? (r == i + 1 ? v0 : xr[s]) / vn : 0.0;
    }
    if (wave == 0) {
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int r = i + 1 + lane + 64 * s;
        if (r < n) vv[r] = ur[s];
      }
      if (lane == 0) {
        dd[i] = P[ci];
        ee[i] = alpha;
      }
    }
    __syncthreads();
    // p = 2 A22 u: row r by T waves, each over a contiguous range of columns
    // (more 64-row slots than waves: T = 1 and the waves loop over slots)
    const int nslot = (m + 63) >> 6;
    const int T = nslot >= NW ? 1 : NW / nslot;
    for (int unit = wave; unit < nslot * T; unit += NW) {
      const int slot = unit % nslot, t = unit / nslot;
      {
        const int r = i + 1 + slot * 64 + lane;
        const int c_lo = i + 1 + (m * t) / T, c_hi = i + 1 + (m * (t + 1)) / T;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (r < n) {
          int cc = c_lo;
          int addr = cc <= r ? cs(cc, n) + r - cc : cs(r, n) + cc - r;
          for (; cc + 3 < c_hi; cc += 4) {
            const int a0 = addr;
            const int a1 = a0 + (cc < r ? n - cc - 1 : 1);
            const int a2 = a1 + (cc + 1 < r ? n - cc - 2 : 1);
            const int a3 = a2 + (cc + 2 < r ? n - cc - 3 : 1);
            addr = a3 + (cc + 3 < r ? n - cc - 4 : 1);
            s0 += P[a0] * vv[cc];
            s1 += P[a1] * vv[cc + 1];
            s2 += P[a2] * vv[cc + 2];
            s3 += P[a3] * vv[cc + 3];
          }
          for (; cc < c_hi; ++cc) {
            s0 += P[addr] * vv[cc];
            addr += cc < r ? n - cc - 1 : 1;
          }
        }
        ybuf[(t * nslot + slot) * 64 + lane] = (s0 + s1) + (s2 + s3);
      }
    }
    if (PL && wave == NW - 1) {
      // the finished reflector to the cluster's scratch
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int r = i + 1 + lane + 64 * s;
        if (r < n) Pg[ci + r - i] = ur[s];
      }
    }
    __syncthreads();
    if (!PL && wave == 0) {
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int r = i + 1 + lane + 64 * s;
        if (r < n) Pg[ci + r - i] = ur[s];
      }
    }
    // K = u . p and w = p - K u, by every wave
    const int ts = nslot * 64;
    double pr[SL], wr[SL];
    part = 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int r = i + 1 + lane + 64 * s;
      double q = 0.0;
      if (r < n)
        for (int t = 0; t < T; ++t) q += ybuf[t * ts + (r - i - 1)];
      pr[s] = 2.0 * q;
      part += ur[s] * pr[s];
    }
    const double K = wave_sum(part);
#pragma unroll
    for (int s = 0; s < SL; ++s) wr[s] = pr[s] - K * ur[s];
    // A22 -= u w^T + w u^T on the lower triangle: waves over columns
    // (cc = i+1+wave+NW*j), lanes over rows.  Lane j first forms u and w of
    // the wave's column j; the loop takes them back by lane reads and keeps
    // four columns' loads in flight
    {
      // columns per inner step (fewer with more row slots: registers)
      constexpr int GC = SL > 8 ? 1 : 4;
      const int J = (m - wave + NW - 1) / NW;
      for (int jb = 0; jb < J; jb += 64) {  // 64 of the wave's columns at a time
        const int JB = J - jb < 64 ? J - jb : 64;
        double ucol = 0.0, wcol = 0.0;
        if (lane < JB) {
          const int cc = i + 1 + wave + NW * (jb + lane);
          double q = 0.0;
          for (int t = 0; t < T; ++t) q += ybuf[t * ts + (cc - i - 1)];
          ucol = vv[cc];
          wcol = 2.0 * q - K * ucol;
        }
        // branch-free: lanes outside the triangle load and store a trash slot
        for (int j = 0; j < JB; j += GC) {
          double pc[GC][SL], uc[GC], wc[GC];
          double* ptr[GC][SL];
#pragma unroll
          for (int g = 0; g < GC; ++g) {
            const int cg = j + g < JB ? i + 1 + wave + NW * (jb + j + g) : n;
            uc[g] = read_lane(ucol, j + g);
            wc[g] = read_lane(wcol, j + g);
            const int base = cs(cg < n ? cg : 0, n) - cg;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
              const int r = i + 1 + lane + 64 * s;
              ptr[g][s] = (r >= cg && r < n) ? P + (base + r) : trash;
              pc[g][s] = *ptr[g][s];
            }
          }
#pragma unroll
          for (int g = 0; g < GC; ++g)
#pragma unroll
            for (int s = 0; s < SL; ++s) *ptr[g][s] = pc[g][s] - (ur[s] * wc[g] + wr[s] * uc[g]);
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && stop >= n - 2) {
    if (n >= 2) {
      dd[n - 2] = P[cs(n - 2, n)];
      dd[n - 1] = P[cs(n - 1, n)];
      ee[n - 2] = P[cs(n - 2, n) + 1];
    } else {
      dd[0] = P[0];
    }
  }
  __syncthreads();
}

// Phases 4-6 for one cluster: eigenvectors of the tridiagonal matrix by
// inverse iteration (with cluster handling), block Gram-Schmidt, and the
// back-transformation into the padded rows of Uc.  Z (column-major, leading
// dimension ldz) is the LDS base or the cluster's scratch; the caller makes
// the choice at the call site so that each inlined copy addresses one
// memory kind directly.
template <int NT, int SL>
__device__ __forceinline__ void eigvecs(double* Z, int ldz, const EigArgs& p, int n, int k, int D,
                                        long long DD, double* S, const double* Pg,
                                        const double* dd, const double* ee, const double* lam,
                                        double bnd, double* pv, double* red, int dv, int k1,
                                        int half, double* Uc) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  // 4. inverse iteration, lane m owns vector m
  double* F0 = S + DD;
  double* F1 = S + 2 * DD;
  double* F2 = S + 3 * DD;
  double* F3 = S + 4 * DD;
  // pivot floor, kept in the normal range so that reciprocals stay finite
  const double tiny = 1e-16 * fmax(bnd, 1e-270);
  for (int m = tid; m < k; m += NT) {
    double* zm = Z + (long long)m * ldz;
    invit_solve(dd, ee, n, lam[m], tiny, F0, F1, F2, F3, D, m, zm, true, m);
    invit_solve(dd, ee, n, lam[m], tiny, F0, F1, F2, F3, D, m, zm, false, 0);
  }
  __syncthreads();

  // eigenvalues closer than delta form a cluster: independent inverse
  // iterations cannot separate them, so each further member restarts from a
  // fresh vector and alternates orthogonalisation against the earlier
  // members with solves
  double* dots = pv;
  const double delta = 1e-12 * bnd;
  int c0 = 0;
  for (int m = 1; m < k; ++m) {
    if (lam[m - 1] - lam[m] > delta) {
      c0 = m;
      continue;
    }
    double* zm = Z + (long long)m * ldz;
    for (int r = tid; r < n; r += NT) zm[r] = start_vec(r, m + 7919);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      cgs2<NT>(Z, ldz, n, m, c0, dots, red);
      if (tid == 0) invit_solve(dd, ee, n, lam[m], tiny, F0, F1, F2, F3, D, m, zm, false, 0);
      __syncthreads();
    }
    cgs2<NT>(Z, ldz, n, m, c0, dots, red);
  }

  // 5. Gram-Schmidt with re-orthogonalisation over all kept vectors, in
  // blocks (coefficients in the contiguous pv | ybuf region of LDS)
  if constexpr (SL <= 5 && NW >= 4)
    bcgs2_waves<NT, SL>(Z, ldz, n, k);
  else
    bcgs2<NT, SL>(Z, ldz, n, k, pv, dv + NT);

  // 6. back-transformation: z <- H_0 ... H_{n-3} z, VB vectors per wave
  // (eight with four row slots: their dot products share one batched wave sum)
  constexpr int VB = SL > 8 ? 2 : SL > 5 ? kVB : 8;
  for (int b0 = wave * VB; b0 < k; b0 += NW * VB) {
    double z[VB][SL];
#pragma unroll
    for (int v = 0; v < VB; ++v)
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int r = lane + 64 * s;
        z[v][s] = (b0 + v < k && r < n) ? Z[(long long)(b0 + v) * ldz + r] : 0.0;
      }
    // reflectors in groups of RG, the next group fetched while this one is
    // applied (the loads' latency is several reflectors' arithmetic)
    constexpr int RG = SL > 8 ? 1 : 2;
    double ug[RG][SL], un[RG][SL];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int ii = n - 3 - g;
      const int cn = ii >= 0 ? cs(ii, n) : 0;
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int r = lane + 64 * s;
        ug[g][s] = (ii >= 0 && r > ii && r < n) ? Pg[cn + r - ii] : 0.0;
      }
    }
    for (int i0 = n - 3; i0 >= 0; i0 -= RG) {
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const int ii = i0 - RG - g;
        const int cn = ii >= 0 ? cs(ii, n) : 0;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const int r = lane + 64 * s;
          un[g][s] = (ii >= 0 && r > ii && r < n) ? Pg[cn + r - ii] : 0.0;
        }
      }
#pragma unroll
      for (int g = 0; g < RG; ++g) {
      const int i = i0 - g;
      if (i < 0) break;
      double u[SL];
#pragma unroll
      for (int s = 0; s < SL; ++s) u[s] = ug[g][s];
      double d[VB];
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        double t = 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s) t += u[s] * z[v][s];
        d[v] = t;
      }
      if constexpr (VB == 8) {
        double t8[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) t8[v] = d[v];
        wave_sum8(t8, d);
#pragma unroll
        for (int v = 0; v < 8; ++v) d[v] *= 2.0;
      } else {
#pragma unroll
        for (int v = 0; v < VB; ++v) d[v] = 2.0 * wave_sum(d[v]);
      }
#pragma unroll
      for (int v = 0; v < VB; ++v)
#pragma unroll
        for (int s = 0; s < SL; ++s) z[v][s] -= d[v] * u[s];
      }
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int s = 0; s < SL; ++s) ug[g][s] = un[g][s];
    }
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      const int m = b0 + v;
      if (m < k) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const int r = lane + 64 * s;
          if (r < n) {
            const int orow = r < k1 ? r : half + (r - k1);
            Uc[orow + (long long)m * D] = z[v][s];
          }
        }
      }
    }
  }
}

// Per-cluster scratch (doubles, eig_scratch_doubles(D)): [0, D^2) packed
// reflectors (the whole packed matrix when it is not in LDS) | [D^2, 5D^2)
// factor rows of the inverse iteration | [5D^2, 6D^2 + D) eigenvectors when
// they are not in LDS | d[D], e[D], lambda[D] and the kept count, handed from
// one kernel to the next.
struct ClusterView {
  int c, D, half, k1, k2, n;
  bool ok;
  double* S;
  double* tri;  // d | e | lambda | k
};

__device__ __forceinline__ ClusterView cluster_view(const EigArgs& p) {
  ClusterView v;
  v.c = blockIdx.x;
  v.D = p.D;
  v.half = p.half;
  v.k1 = p.k1[(long long)v.c * p.kstride];
  v.k2 = p.k2 ? p.k2[(long long)v.c * p.kstride] : 0;
  v.n = v.k1 + v.k2;
  v.ok = !(v.n > kEigNmax || v.n <= 0 || v.k1 < 0 || v.k2 < 0 || v.k1 > v.half ||
           v.k2 > v.D - v.half);
  v.S = p.scratch + (long long)v.c * p.sstride;
  v.tri = v.S + 6LL * v.D * v.D + v.D;
  return v;
}

// length of the symmetric product's partial sums: one per lane and 64-row
// slot, at least NT
__host__ __device__ __forceinline__ int partials_len(int dv, int nt) {
  const int r = (dv + 63) & ~63;
  return r > nt ? r : nt;
}

// Kernel 1: gather and tridiagonalise; zero the output columns.  LDS: packed
// triangle [zr] | d[dv] | e[dv] | v[dv] | p-partials[partials_len] | red[8].
// split: reduce only the leading n - kEigRegN columns (none when n <= kEigRegN)
// and leave the trailing block, packed in the cluster's scratch, to
// k_eig_tri_reg
template <int NT, int SL>
__global__ __launch_bounds__(NT) void k_eig_tri(EigArgs p0, EigArgs p1, int zr, int dv, int split) {
  extern __shared__ double sm[];
  const EigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const ClusterView v = cluster_view(p);
  const int tid = threadIdx.x;
  double* Uc = p.U + (long long)v.c * p.ustride;
  for (long long e = tid; e < (long long)v.D * v.D; e += NT) Uc[e] = 0.0;
  if (!v.ok || v.D > dv) {
    if (tid == 0) {
      p.rank[v.c] = 0;
      if (v.n != 0) p.status[1] = 1;
    }
    return;
  }
  const int n = v.n;
  const int np = n * (n + 1) / 2;
  const int stop = split ? (n > kEigRegN ? n - kEigRegN : 0) : n;
  if (stop == 0) return;
  double* dd = sm + zr;
  double* ee = dd + dv;
  double* vv = ee + dv;
  double* ybuf = vv + dv;
  const int yb = partials_len(dv, NT);
  const double* Gc = p.G + (long long)v.c * p.gstride;
  // trash slot of the update: the unused reduction slots in LDS, or the unused
  // factor area of the scratch when the triangle is not in LDS
  if (!split && n <= kEigLdsN && np <= zr)
    gather_tridiag<NT, SL, true>(p, Gc, n, v.k1, v.half, v.D, sm, v.S, dd, ee, vv, ybuf, ybuf + yb,
                                 stop);
  else
    gather_tridiag<NT, SL, false>(p, Gc, n, v.k1, v.half, v.D, v.S, v.S, dd, ee, vv, ybuf,
                              v.S + (long long)v.D * v.D, stop);
  // with a split, d and e of the finished columns only
  const int ndone = stop < n ? stop : n;
  for (int j = tid; j < ndone; j += NT) {
    v.tri[j] = dd[j];
    v.tri[v.D + j] = j < n - 1 ? ee[j] : 0.0;
  }
}

// ---------------------------------------------------------------------
// Kernel 1 for dimensions up to 32 NW (NW waves, NW in {1, 2, 4, 8}): the
// matrix stays in registers for the whole reduction.  Wave w holds columns
// c = w + NW j (j < 32); lane l holds rows l + 64 s of each column for the
// 64-row blocks s from the column's own block c / 64 on (the symmetric block
// lower triangle, diagonal blocks stored in full).  Per Householder step:
//   * the pivot column (written to LDS by its owner during the previous
//     update) gives the reflector u in every wave's registers;
//   * p = 2 A u: every stored entry contributes lane-locally to its row
//     (A[r,c] u[c]); the entries of the strictly lower blocks also stand for
//     their transposes, whose contributions A[r,c] u[r] to row c are one dot
//     product per column, summed across lanes for 16 columns at once by a
//     halving butterfly (each exchange halves the values a lane carries);
//     the waves' partial vectors meet in LDS;
//   * A -= u w^T + w u^T in registers, w = p - (u.p) u, rows of the finished
//     part left untouched (u = w = 0 there).
// Three workgroup barriers per step; LDS holds only vectors.

// columns per wave; 64-row block of local column j
constexpr int kRegCols = 32;
template <int NW>
__device__ constexpr int diag_slot(int j) { return (NW * j) >> 6; }

// t[q] (q < 16) summed over all 64 lanes: lane l returns the sum for column
// q = 8 b1 + 4 b0 + 2 b4 + b5 (b_k: bit k of l).  Each halving exchange
// leaves a lane one of every two values, summed with its partner's: xor 32
// and xor 16 by lane-half swaps, xor 1 and xor 2 by quad permutes; the four
// lanes left with the same column (bits 2 and 3) are summed by row rotates.
__device__ __forceinline__ double butterfly16(const double* t, int lane) {
  double t1[8], t2[4], t3[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    double x = t[2 * k], y = t[2 * k + 1];
    swap_halves32(x, y);
    t1[k] = x + y;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double x = t1[2 * k], y = t1[2 * k + 1];
    swap_rows16(x, y);
    t2[k] = x + y;
  }
  const bool b0 = lane & 1, b1 = lane & 2;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double keep = b0 ? t2[2 * k + 1] : t2[2 * k], give = b0 ? t2[2 * k] : t2[2 * k + 1];
    t3[k] = keep + dpp<0xB1>(give);  // quad_perm [1,0,3,2]
  }
  const double keep = b1 ? t3[1] : t3[0], give = b1 ? t3[0] : t3[1];
  double v = keep + dpp<0x4E>(give);  // quad_perm [2,3,0,1]
  v += dpp<0x128>(v);                 // row_ror:8
  v += dpp<0x124>(v);                 // row_ror:4
  return v;
}

// RS: 64-row slots per lane (NW / 2 for four and eight waves, fewer when the
// dimension allows: three for D <= 192 with eight waves).  split: a cluster
// with n > kEigRegN had its leading n - kEigRegN columns reduced by k_eig_tri;
// this kernel loads the trailing block from the packed matrix in the
// cluster's scratch and finishes the reduction (global step i0 + i)
template <int NW, int RS>
__global__ __launch_bounds__(NW * 64) void k_eig_tri_reg(EigArgs p0, EigArgs p1, int dv, int split) {
  constexpr int NT = NW * 64, J = kRegCols, RM = 64 * RS;
  // a group of 16 columns has cross-block (transposed) terms when its first
  // column's block is not the last one
  constexpr int NG = RS > 1 ? (diag_slot<NW>(16) < RS - 1 ? 2 : 1) : 0;
  __shared__ double pc[2][RM];      // pivot column, by step parity
  __shared__ double ypart[NW][RM];  // per-wave partials of the row-wise terms
  __shared__ double tsum[RM];       // transposed terms, by column
  __shared__ double yfull[RM];      // p = 2 A u
  __shared__ double dd[RM], ee[RM], last[RM];
  const EigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const ClusterView v = cluster_view(p);
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  double* Uc = p.U + (long long)v.c * p.ustride;
  for (long long e = tid; e < (long long)v.D * v.D; e += NT) Uc[e] = 0.0;
  const int ng = v.n;  // the cluster's dimension; this kernel reduces [i0, ng)
  const int i0 = (split && ng > kEigRegN) ? ng - kEigRegN : 0;
  if (!v.ok || v.D > dv || ng - i0 > NW * J || ng - i0 > RM) {
    if (tid == 0) {
      p.rank[v.c] = 0;
      if (v.n != 0) p.status[1] = 1;
    }
    return;
  }
  const int n = ng - i0;
  double* Pg = v.S;
  const double* Gc = p.G + (long long)v.c * p.gstride;

  // gather the live block (rows and columns [0,k1) and [half, half+k2));
  // only the Gram's lower triangle is read (entries above the diagonal of
  // the diagonal blocks from their mirror images).  After a split: the
  // trailing block from the packed lower triangle (column c at cs(c, ng))
  double a[J][RS];
  int bad = 0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = w + NW * j;
    const int oc = c < v.k1 ? c : v.half + (c - v.k1);
#pragma unroll
    for (int s = diag_slot<NW>(j); s < RS; ++s) {
      const int r = lane + 64 * s;
      double x = 0.0;
      if (c < n && r < n) {
        if (i0 > 0) {
          const int gr = i0 + r, gc = i0 + c;
          x = gr >= gc ? Pg[cs(gc, ng) + gr - gc] : Pg[cs(gr, ng) + gc - gr];
        } else {
          const int orow = r < v.k1 ? r : v.half + (r - v.k1);
          x = r >= c ? Gc[orow + (long long)oc * v.D] : Gc[oc + (long long)orow * v.D];
          if (!(x == x) || x - x != 0.0) bad = 1;
        }
      }
      a[j][s] = x;
    }
  }
  if (bad) p.status[0] = 1;
  if (w == 0) {
#pragma unroll
    for (int s = 0; s < RS; ++s) pc[0][lane + 64 * s] = a[0][s];
  }
  __syncthreads();

  for (int i = 0; i + 2 < n; ++i) {
    // this wave's active columns i < c < n are local j in [jlo, jhi).  Work
    // is skipped by blocks of 8 columns: an inactive column has u[c] = w[c] = 0
    // and contributes nothing, and whole blocks schedule better than single
    // columns.  The opaque copy of the wave index keeps per-column quantities
    // from being precomputed for all columns outside the loop
    int wl = w;
    asm volatile("" : "+s"(wl));
    const int jlo = (i + 1 - wl + NW - 1) / NW, jhi = (n - wl + NW - 1) / NW;
    const double* col = pc[i & 1];
    double* next = pc[(i + 1) & 1];
    double u[RS];
    double part = 0.0;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      u[s] = (r > i && r < n) ? col[r] : 0.0;
      part += u[s] * u[s];
    }
    const double xx = wave_sum(part);
    const double x0 = col[i + 1];
    const double diag = col[i];
    const double nx = sqrt(xx);
    // packed column of the global step i0 + i (rows r > i lie at ci + r - i)
    const long long ci = cs(i0 + i, ng);
    if (!(nx > 0.0)) {  // column already reduced: H_i = I, A unchanged
      if (w == 0) {
#pragma unroll
        for (int s = 0; s < RS; ++s) {
          const int r = lane + 64 * s;
          if (r > i && r < n) Pg[ci + r - i] = 0.0;
        }
        if (lane == 0) {
          dd[i] = diag;
          ee[i] = 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (wl + NW * j == i + 1) {
#pragma unroll
          for (int s = diag_slot<NW>(j); s < RS; ++s) next[lane + 64 * s] = a[j][s];
        }
      }
      __syncthreads();
      continue;
    }
    const double alpha = -copysign(nx, x0);
    const double v0 = x0 - alpha;
    const double rvn = 1.0 / sqrt(xx - x0 * x0 + v0 * v0);
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      u[s] = (r == i + 1 ? v0 : u[s]) * rvn;
    }
    if (w == 0) {
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = lane + 64 * s;
        if (r > i && r < n) Pg[ci + r - i] = u[s];
      }
      if (lane == 0) {
        dd[i] = diag;
        ee[i] = alpha;
      }
    }

    // p = 2 A u
    double y[RS];
#pragma unroll
    for (int s = 0; s < RS; ++s) y[s] = 0.0;
#pragma unroll
    for (int g = 0; g < J / 16; ++g) {
      double t[16];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jb = 16 * g + 8 * h;
        if (jb + 8 > jlo && jb < jhi) {
#pragma unroll
          for (int q = 8 * h; q < 8 * h + 8; ++q) {
            const int j = 16 * g + q;
            const int sd = diag_slot<NW>(j);
            t[q] = 0.0;
            if (sd >= RS) continue;  // a column past the last row slot (folded away)
            const double uc = read_lane(u[sd], (wl + NW * j) & 63);
#pragma unroll
            for (int s = sd; s < RS; ++s) y[s] += a[j][s] * uc;
#pragma unroll
            for (int s = sd + 1; s < RS; ++s) t[q] += a[j][s] * u[s];
          }
        } else {
#pragma unroll
          for (int q = 8 * h; q < 8 * h + 8; ++q) t[q] = 0.0;
        }
      }
      // a group without active columns leaves its (stale) partials: they
      // only reach rows outside (i, n), where w is cleared below
      if (g < NG && jlo < 16 * g + 16 && jhi > 16 * g) {
        const int q = ((lane >> 1) & 1) * 8 + (lane & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 5) & 1);
        const double sum = butterfly16(t, lane);
        if ((lane & 12) == 0) tsum[wl + NW * (16 * g + q)] = sum;
      }
    }
#pragma unroll
    for (int s = 0; s < RS; ++s) ypart[w][lane + 64 * s] = y[s];
    __syncthreads();
    if (lane < 32 && 32 * w + lane < RM) {
      const int r = 32 * w + lane;
      double acc = 0.0;
      // rows of the last block receive no transposed terms
      if (NG > 0 && r < 64 * (RS - 1)) acc = tsum[r];
#pragma unroll
      for (int x = 0; x < NW; ++x) acc += ypart[x][r];
      yfull[r] = 2.0 * acc;
    }
    __syncthreads();
    double wv[RS];
    part = 0.0;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      wv[s] = (r > i && r < n) ? yfull[r] : 0.0;
      part += u[s] * wv[s];
    }
    const double K = wave_sum(part);
#pragma unroll
    for (int s = 0; s < RS; ++s) wv[s] -= K * u[s];

    // A -= u w^T + w u^T on the stored blocks; the owner of column i+1 hands
    // it on as the next pivot
#pragma unroll
    for (int jb = 0; jb < J; jb += 8) {
      if (jb + 8 > jlo && jb < jhi) {
#pragma unroll
        for (int j = jb; j < jb + 8; ++j) {
          const int sd = diag_slot<NW>(j);
          if (sd >= RS) continue;  // a column past the last row slot (folded away)
          const int lc = (wl + NW * j) & 63;
          const double uc = read_lane(u[sd], lc), wc = read_lane(wv[sd], lc);
#pragma unroll
          for (int s = sd; s < RS; ++s) a[j][s] -= u[s] * wc + wv[s] * uc;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (wl + NW * j == i + 1) {
#pragma unroll
        for (int s = diag_slot<NW>(j); s < RS; ++s) next[lane + 64 * s] = a[j][s];
      }
    }
    __syncthreads();
  }
  // the trailing 2x2 (or 1x1) block
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (w + NW * j == n - 1) {
#pragma unroll
      for (int s = diag_slot<NW>(j); s < RS; ++s) last[lane + 64 * s] = a[j][s];
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = pc[(n - 2) & 1][n - 2];
      ee[n - 2] = pc[(n - 2) & 1][n - 1];
    }
    dd[n - 1] = last[n - 1];
  }
  __syncthreads();
  for (int j = tid; j < n; j += NT) {
    v.tri[i0 + j] = dd[j];
    v.tri[v.D + i0 + j] = j < n - 1 ? ee[j] : 0.0;
  }
}

// Gershgorin bound of the tridiagonal matrix (d, e)
__device__ __forceinline__ void gershgorin(const double* dd, const double* ee, int n, double& gl,
                                           double& gu) {
  gl = 1e300;
  gu = -1e300;
  for (int j = 0; j < n; ++j) {
    const double rad = (j > 0 ? fabs(ee[j - 1]) : 0.0) + (j < n - 1 ? fabs(ee[j]) : 0.0);
    gl = fmin(gl, dd[j] - rad);
    gu = fmax(gu, dd[j] + rad);
  }
}

// Kernel 2: eigenvalues and the kept count.  LDS: d | e | e^2 | lambda (dv
// each) | red[8].
template <int NT>
__global__ __launch_bounds__(NT) void k_eig_val(EigArgs p0, EigArgs p1, int dv) {
  constexpr int NW = NT / 64;
  extern __shared__ double sm[];
  const EigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const ClusterView v = cluster_view(p);
  if (!v.ok || v.D > dv) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int n = v.n;
  double* dd = sm;
  double* ee = dd + dv;
  double* e2 = ee + dv;
  double* lam = e2 + dv;
  double* red = lam + dv;
  for (int j = tid; j < n; j += NT) {
    dd[j] = v.tri[j];
    ee[j] = v.tri[v.D + j];
    e2[j] = ee[j] * ee[j];
  }
  __syncthreads();
  double gl, gu;
  gershgorin(dd, ee, n, gl, gu);
  const double bnd = fmax(fabs(gl), fabs(gu));
  const double tol = 4e-16 * bnd + 1e-300;
  gl -= tol;
  gu += tol;
  const double pivmin = 1e-290;
  int k;
  double lo0 = gl, hi0 = gu;
  if (p.exact) {
    k = n;
  } else {
    // lambda_1 by multisection over the first NP lanes (at most two waves:
    // the Sturm counts are issue-bound, so one wave per SIMD and a few more
    // iterations beat more points per iteration)
    constexpr int NP = NT < 128 ? NT : 128;
    double lo = gl, hi = gu;
    for (int it = 0; it < 64 && hi - lo > tol; ++it) {
      const double h = hi - lo;
      int below = 0;
      if (tid < NP) {
        const double x = lo + h * (double)(tid + 1) / (double)(NP + 1);
        below = sturm1(dd, e2, n, x, pivmin) < n;
      }
      const int wc = __popcll(__ballot(below));
      __syncthreads();
      if (lane == 0) red[wave] = (double)wc;
      __syncthreads();
      int cnt = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) cnt += (int)red[w];
      const double nlo = cnt > 0 ? lo + h * (double)cnt / (double)(NP + 1) : lo;
      const double nhi = cnt < NP ? lo + h * (double)(cnt + 1) / (double)(NP + 1) : hi;
      lo = nlo;
      hi = nhi;
    }
    const double l1 = 0.5 * (lo + hi);
    hi0 = hi;
    if (!(l1 > 0.0)) {
      k = 1;
    } else {
      const double thr = p.tau * l1;
      k = n - sturm1(dd, e2, n, thr, pivmin);
      k = k < 1 ? 1 : (k > n ? n : k);
      lo0 = fmin(thr, lo) - tol;
    }
  }
  if (p.kmax) {
    const int m = p.kmax[v.c];
    k = k < m ? k : (m < 1 ? 1 : m);
  }
  // the k leading eigenvalues by grouped multisection: G lanes per
  // eigenvalue, two points each.  The Sturm counts are issue-bound, so G
  // minimises (waves per SIMD) x (iterations) rather than the iterations
  {
    const double span = hi0 - lo0;
    const double bits = span > tol ? log2(span / tol) : 0.0;
    int G = 1;
    double best = 1e300;
    for (int g = 1; g <= 8; g *= 2) {
      if (g > 1 && g * k > NT) break;
      const int waves = (g * k + 63) / 64;
      const int per_simd = (waves + 3) / 4;
      const double cost = (double)per_simd * ceil(bits / log2((double)(2 * g + 1)));
      if (cost < best) {
        best = cost;
        G = g;
      }
    }
    const int Q = 2 * G;
    int R = span > tol ? (int)ceil(bits / log2((double)(Q + 1))) : 0;
    R = R > 200 ? 200 : R;
    const int jl = tid % G;
    for (int g = tid / G; g < k; g += NT / G) {
      const int jt = n - 1 - g;
      double lo = lo0, hi = hi0;
      for (int it = 0; it < R; ++it) {
        const double h = (hi - lo) / (double)(Q + 1);
        const double xa = lo + h * (double)(2 * jl + 1);
        const double xb = lo + h * (double)(2 * jl + 2);
        int ca, cb;
        sturm2(dd, e2, n, xa, xb, pivmin, ca, cb);
        double nlo = lo, nhi = hi;
        if (ca <= jt) nlo = xa;
        if (cb <= jt) nlo = xb;
        if (cb > jt) nhi = xb;
        if (ca > jt) nhi = xa;
        lo = group_red<true>(nlo, G);
        hi = group_red<false>(nhi, G);
      }
      if (jl == 0) v.tri[2 * v.D + g] = 0.5 * (lo + hi);
    }
  }
  if (tid == 0) {
    v.tri[3 * v.D] = (double)k;
    p.rank[v.c] = k;
  }
}

// Kernel 3: eigenvectors, orthogonalisation and back-transformation.  LDS:
// eigenvectors [zr] (ZL only) | d | e | lambda (dv each) | coefficients
// [dv + NT] | red[8].
// ZL: this launch handles the clusters whose eigenvectors fit the LDS region
// (the other launch those that do not), so that each kernel holds one copy of
// the phases
template <int NT, int SL, bool ZL>
__global__ __launch_bounds__(NT) void k_eig_vec(EigArgs p0, EigArgs p1, int zr, int dv) {
  extern __shared__ double sm[];
  const EigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const ClusterView v = cluster_view(p);
  if (!v.ok || v.D > dv) return;
  const int tid = threadIdx.x;
  const int n = v.n;
  double* dd = sm + (ZL ? zr : 0);
  double* ee = dd + dv;
  double* lam = ee + dv;
  double* pv = lam + dv;
  double* red = pv + dv + NT;
  const int k = (int)v.tri[3 * v.D];
  if (((long long)(n | 1) * k <= zr) != ZL) return;
  for (int j = tid; j < n; j += NT) {
    dd[j] = v.tri[j];
    ee[j] = v.tri[v.D + j];
    lam[j] = j < k ? v.tri[2 * v.D + j] : 0.0;
  }
  __syncthreads();
  double gl, gu;
  gershgorin(dd, ee, n, gl, gu);
  const double bnd = fmax(fabs(gl), fabs(gu));
  const long long DD = (long long)v.D * v.D;
  double* Uc = p.U + (long long)v.c * p.ustride;
  const int ldz = n | 1;
  if (ZL)
    eigvecs<NT, SL>(sm, ldz, p, n, k, v.D, DD, v.S, v.S, dd, ee, lam, bnd, pv, red, dv, v.k1, v.half,
                Uc);
  else
    eigvecs<NT, SL>(v.S + 5 * DD, ldz, p, n, k, v.D, DD, v.S, v.S, dd, ee, lam, bnd, pv, red, dv, v.k1,
                v.half, Uc);
}

namespace {

int eig_threads(int D) { return D <= 32 ? 64 : D <= 64 ? 128 : D <= 128 ? 256 : 512; }

// LDS regions (doubles) of the packed triangle (kernel 1) and of the
// eigenvectors (kernel 3) for a launch of padded dimension D
int tri_zr(int D, int nt) {
  const int cap = kLdsBytes / 8 - 3 * D - partials_len(D, nt) - kRed;
  if (D > kEigLdsN) return cap;
  const int zr = D * (D + 1) / 2;
  return zr < cap ? zr : cap;
}
int vec_zr(int D, int nt) {
  // dimensions in (64, 128] come in launches of many clusters: the
  // eigenvectors go to scratch so that several workgroups share a CU (one
  // would fill its LDS)
  if (D > 64 && D <= 128) return 0;
  const int cap = kLdsBytes / 8 - 4 * D - nt - kRed;
  const long long zfull = (long long)(D | 1) * D;
  return zfull < cap ? (int)zfull : cap;
}

template <int NT, int SL>
hipError_t launch_nt(const EigArgs& a, const EigArgs& b, int nclusters, int D, hipStream_t s,
                     int phases) {
  static bool attr_set = false;
  if (!attr_set) {
    // kernels with dynamic LDS (the register-resident tridiagonalisation has
    // only static LDS and keeps the default)
    const void* tri = nullptr;
    if constexpr (SL > 4) tri = (const void*)k_eig_tri<NT, SL>;  // the others use static LDS only
    for (const void* f : {tri, (const void*)k_eig_val<NT>, (const void*)k_eig_vec<NT, SL, true>,
                          (const void*)k_eig_vec<NT, SL, false>}) {
      if (!f) continue;
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
  const dim3 grid(nclusters, 2);
  const int zt = tri_zr(D, NT), zv = vec_zr(D, NT);
  if (!(phases & kEigPhaseTri)) {
  } else if constexpr (SL <= 4) {  // dimensions up to 4 x 64: the triangle in registers
    constexpr int NW = NT / 64, RS = NW >= 4 ? NW / 2 : 1;
    bool done = false;
    if constexpr (NW == 8) {
      if (D <= 192) {
        hipLaunchKernelGGL((k_eig_tri_reg<8, 3>), grid, dim3(NT), 0, s, a, b, D, 0);
        done = true;
      }
    }
    if (!done) hipLaunchKernelGGL((k_eig_tri_reg<NW, RS>), grid, dim3(NT), 0, s, a, b, D, 0);
  } else {
    // the leading n - kEigRegN columns with the matrix in the cluster's
    // scratch, the trailing kEigRegN with the matrix in registers
    hipLaunchKernelGGL((k_eig_tri<NT, SL>), grid, dim3(NT),
                       sizeof(double) * ((size_t)zt + 3 * D + partials_len(D, NT) + kRed), s, a, b,
                       zt, D, 1);
    hipLaunchKernelGGL((k_eig_tri_reg<8, 4>), grid, dim3(512), 0, s, a, b, D, 1);
  }
  if (phases & kEigPhaseVal)
    hipLaunchKernelGGL(k_eig_val<NT>, grid, dim3(NT), sizeof(double) * (4 * (size_t)D + kRed), s,
                       a, b, D);
  if (phases & kEigPhaseVec) {
    const size_t lv = sizeof(double) * ((size_t)zv + 4 * D + NT + kRed);
    hipLaunchKernelGGL((k_eig_vec<NT, SL, true>), grid, dim3(NT), lv, s, a, b, zv, D);
    hipLaunchKernelGGL((k_eig_vec<NT, SL, false>), grid, dim3(NT),
                       sizeof(double) * (4 * D + NT + kRed), s, a, b, zv, D);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eig(const EigArgs& a, const EigArgs& b, int nclusters, hipStream_t s,
                      int phases) {
  if (nclusters <= 0) return hipSuccess;
  const int D = a.D > b.D ? a.D : b.D;
  if (D > kEigNmax || D < 1) return hipErrorInvalidValue;
  if (a.sstride < eig_scratch_doubles(a.D) || b.sstride < eig_scratch_doubles(b.D))
    return hipErrorInvalidValue;
  // SL row slots per lane: a wave holds a column of up to 64 SL rows
  if (D > 512) return launch_nt<512, 16>(a, b, nclusters, D, s, phases);
  if (D > 320) return launch_nt<512, 8>(a, b, nclusters, D, s, phases);
  if (D > 256) return launch_nt<512, 5>(a, b, nclusters, D, s, phases);
  switch (eig_threads(D)) {
    // row slots per lane: as many as the dimension needs (fewer registers
    // and no padding work in the eigenvector phases)
    case 64: return launch_nt<64, 1>(a, b, nclusters, D, s, phases);
    case 128: return launch_nt<128, 1>(a, b, nclusters, D, s, phases);
    case 256: return launch_nt<256, 2>(a, b, nclusters, D, s, phases);
    default: return launch_nt<512, 4>(a, b, nclusters, D, s, phases);
  }
}

// ------------------------------------------------ complex Hermitian Grams
namespace {

__device__ __forceinline__ int live_row(int r, int k1, int half) {
  return r < k1 ? r : half + (r - k1);
}

__global__ __launch_bounds__(256) void k_ceig_embed(CEigArgs p0, CEigArgs p1) {
  const CEigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const int c = blockIdx.x, D = p.D, D2 = 2 * D, tid = threadIdx.x;
  __shared__ double red[8];
  const int k1 = p.k1[(long long)c * p.kstride];
  const int k2 = p.k2 ? p.k2[(long long)c * p.kstride] : 0;
  const int n = k1 + k2;
  const long long gs = (long long)c * D * D;
  double w[3];
  for (int m = 0; m < 3; ++m) {
    double t = 0.0;
    if (p.G[m])
      for (int i = tid; i < D; i += 256) t += p.G[m][gs + i + (long long)i * D];
    t = block_sum<256>(t, red);
    w[m] = t > 0.0 ? 1.0 / t : 0.0;
  }
  double* E = p.E + (long long)c * D2 * D2;
  for (long long e = tid; e < (long long)D2 * D2; e += 256) E[e] = 0.0;
  __syncthreads();
  int bad = 0;
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, q = e / n;
    const long long a = gs + live_row(r, k1, p.half) + (long long)live_row(q, k1, p.half) * D;
    const long long b = gs + live_row(q, k1, p.half) + (long long)live_row(r, k1, p.half) * D;
    double xr = 0.0, xi = 0.0;
    for (int m = 0; m < 3; ++m) {
      const double* g = p.G[m];
      if (!g) continue;
      xr += w[m] * 0.5 * (g[a] + g[b]);
      xi += w[m] * 0.5 * (g[p.gplane + a] - g[p.gplane + b]);
    }
    if (!(xr == xr) || xr - xr != 0.0 || !(xi == xi) || xi - xi != 0.0) bad = 1;
    E[r + (long long)q * D2] = xr;
    E[(D + r) + (long long)(D + q) * D2] = xr;
    E[(D + r) + (long long)q * D2] = xi;
    E[r + (long long)(D + q) * D2] = -xi;
  }
  if (bad) p.status[0] = 1;
  if (tid == 0) p.nlive[c] = n;
}

__global__ __launch_bounds__(256) void k_ceig_extract(CEigArgs p0, CEigArgs p1) {
  constexpr int NT = 256, NW = NT / 64;
  const CEigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const int c = blockIdx.x, D = p.D, D2 = 2 * D, tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_id();
  __shared__ double zr[512], zi[512], cr[512], ci[512], red[8];
  const int k1 = p.k1[(long long)c * p.kstride];
  const int k2 = p.k2 ? p.k2[(long long)c * p.kstride] : 0;
  const int n = k1 + k2;
  const int ke = p.rank_e[c];
  const double* Ue = p.Ue + (long long)c * D2 * D2;
  double* Ur = p.U + (long long)c * D * D;
  double* Ui = Ur + p.uplane;
  for (long long e = tid; e < (long long)D * D; e += NT) {
    Ur[e] = 0.0;
    Ui[e] = 0.0;
  }
  __syncthreads();
  int acc = 0;
  const int cap = p.kmax ? (p.kmax[c] < 1 ? 1 : (p.kmax[c] < n ? p.kmax[c] : n)) : n;
  for (int m = 0; m < ke && acc < cap; ++m) {
    for (int r = tid; r < n; r += NT) {
      zr[r] = Ue[r + (long long)m * D2];
      zi[r] = Ue[D + r + (long long)m * D2];
    }
    __syncthreads();
    for (int pass = 0; pass < 2 && acc > 0; ++pass) {
      // coefficients <u_j, z> = sum conj(u_j) z
      for (int j = wave; j < acc; j += NW) {
        double sr = 0.0, si = 0.0;
        for (int r = lane; r < n; r += 64) {
          const long long o = live_row(r, k1, p.half) + (long long)j * D;
          const double ur = Ur[o], ui = Ui[o];
          sr += ur * zr[r] + ui * zi[r];
          si += ur * zi[r] - ui * zr[r];
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) {
          cr[j] = sr;
          ci[j] = si;
        }
      }
      __syncthreads();
      for (int r = tid; r < n; r += NT) {
        const int pr = live_row(r, k1, p.half);
        double dr = 0.0, di = 0.0;
        for (int j = 0; j < acc; ++j) {
          const double ur = Ur[pr + (long long)j * D], ui = Ui[pr + (long long)j * D];
          dr += cr[j] * ur - ci[j] * ui;
          di += cr[j] * ui + ci[j] * ur;
        }
        zr[r] -= dr;
        zi[r] -= di;
      }
      __syncthreads();
    }
    double t = 0.0;
    for (int r = tid; r < n; r += NT) t += zr[r] * zr[r] + zi[r] * zi[r];
    const double nrm2 = block_sum<NT>(t, red);
    if (nrm2 > 0.5) {
      const double inv = 1.0 / sqrt(nrm2);
      for (int r = tid; r < n; r += NT) {
        const long long o = live_row(r, k1, p.half) + (long long)acc * D;
        Ur[o] = zr[r] * inv;
        Ui[o] = zi[r] * inv;
      }
      ++acc;
    }
    __syncthreads();
  }
  if (tid == 0) p.rank[c] = acc;
}

}  // namespace

hipError_t launch_ceig_embed(const CEigArgs& a, const CEigArgs& b, int nclusters, hipStream_t s) {
  if (nclusters <= 0) return hipSuccess;
  if (2 * (a.D > b.D ? a.D : b.D) > kEigNmax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ceig_embed, dim3(nclusters, 2), dim3(256), 0, s, a, b);
  return hipGetLastError();
}

hipError_t launch_ceig_extract(const CEigArgs& a, const CEigArgs& b, int nclusters,
                               hipStream_t s) {
  if (nclusters <= 0) return hipSuccess;
  if (a.D > 512 || b.D > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ceig_extract, dim3(nclusters, 2), dim3(256), 0, s, a, b);
  return hipGetLastError();
}

}  // namespace h2k
