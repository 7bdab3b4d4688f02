// Batched truncated eigen-decomposition of the summed normalised Gram
// matrices that fix each new cluster basis of C (Section III-C and IV-C of
// Ma & Jiao: "perform an SVD on G and keep the singular vectors whose
// normalised singular values exceed eps"; G is Hermitian positive
// semi-definite, so its SVD is its eigen-decomposition).
//
// One workgroup per cluster, FP64 throughout:
//   1. gather the live rows/columns (the children's actual ranks) into a
//      packed lower triangle, in LDS for n <= 192 (148 KiB), else in the
//      cluster's L2-resident scratch (n <= 256);
//   2. Householder reduction to tridiagonal form in place, reflectors kept in
//      the packed columns;
//   3. all eigenvalues by Sturm-sequence bisection, one thread per eigenvalue;
//   4. kept count from the threshold tau * lambda_1;
//   5. eigenvectors of the tridiagonal matrix by two steps of inverse
//      iteration (Gaussian elimination with partial pivoting), one thread per
//      kept vector, then two passes of modified Gram-Schmidt in descending
//      eigenvalue order;
//   6. back-transformation by the reflectors, one wave per vector, and scatter
//      to the padded row layout.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace h2k {

constexpr int kEigThreads = 512;
constexpr int kEigWaves = kEigThreads / 64;

__device__ __forceinline__ int pidx(int i, int j, int n) {  // i >= j
  return j * n - (j * (j - 1)) / 2 + (i - j);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < kEigWaves; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ int sturm_count(const double* dd, const double* e2, int n, double x,
                                           double pivmin) {
  double q = dd[0] - x;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = dd[i] - x - e2[i - 1] / q;
    cnt += q < 0.0;
  }
  return cnt;
}


__device__ __forceinline__ double start_vec(int r, int m) {
  return cos(0.7548776662 * r + 0.5698402909 * m) + 0.1;
}

// Gaussian elimination with partial pivoting of (T - lambda I), T tridiagonal
// (diagonal dd, off-diagonal ee); factors of vector m interleaved by m.  The
// running row is carried in registers, so the loop only stores.
__device__ void tri_factor(const double* dd, const double* ee, int n, double lm, double tiny,
                           double* sd, double* sl, double* su, double* su2, double* spv, int D,
                           int m) {
  double di = dd[0] - lm;
  double ui = n > 1 ? ee[0] : 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double li = ee[i];
    const double dn = dd[i + 1] - lm;
    const double un = i < n - 2 ? ee[i + 1] : 0.0;
    if (fabs(di) >= fabs(li)) {
      if (fabs(di) < tiny) di = di < 0.0 ? -tiny : tiny;
      const double fact = li / di;
      sd[i * D + m] = di;
      sl[i * D + m] = fact;
      su[i * D + m] = ui;
      su2[i * D + m] = 0.0;
      spv[i * D + m] = 0.0;
      di = dn - fact * ui;
      ui = un;
    } else {
      const double fact = di / li;
      sd[i * D + m] = li;
      sl[i * D + m] = fact;
      su[i * D + m] = dn;
      su2[i * D + m] = un;
      spv[i * D + m] = 1.0;
      di = ui - fact * dn;
      ui = -fact * un;
    }
  }
  if (fabs(di) < tiny) di = di < 0.0 ? -tiny : tiny;
  sd[(n - 1) * D + m] = di;
}

// Z[:, m] <- (T - lambda_m I)^{-1} Z[:, m] with the stored factors; the
// running entries are carried in registers.  Near-singular shifts make the
// solution grow: the whole system is rescaled before it can overflow.
__device__ void tri_solve(int n, const double* sd, const double* sl, const double* su,
                          const double* su2, const double* spv, int D, int m, double* Z) {
  double zi = Z[m];
  for (int i = 0; i < n - 1; ++i) {
    const double f = sl[i * D + m];
    const double zn = Z[(i + 1) * D + m];
    if (spv[i * D + m] == 0.0) {
      Z[i * D + m] = zi;
      zi = zn - f * zi;
    } else {
      Z[i * D + m] = zn;
      zi = zi - f * zn;
    }
  }
  double x2 = 0.0;  // x_{i+2}
  double x1 = zi / sd[(n - 1) * D + m];
  Z[(n - 1) * D + m] = x1;
  for (int i = n - 2; i >= 0; --i) {
    const double xi = (Z[i * D + m] - su[i * D + m] * x1 - (i < n - 2 ? su2[i * D + m] * x2 : 0.0)) /
                      sd[i * D + m];
    x2 = x1;
    x1 = xi;
    Z[i * D + m] = xi;
    if (fabs(xi) > 1e150) {
      for (int r = 0; r < n; ++r) Z[r * D + m] *= 1e-150;
      x1 *= 1e-150;
      x2 *= 1e-150;
    }
  }
}

// Scale-safe normalisation of column m by one thread.
__device__ void normalize_serial(double* Z, int D, int n, int m) {
  double amax = 0.0;
  for (int r = 0; r < n; ++r) amax = fmax(amax, fabs(Z[r * D + m]));
  if (!(amax > 0.0) || !(amax < 1e308)) return;
  double s = 0.0;
  for (int r = 0; r < n; ++r) {
    const double v = Z[r * D + m] / amax;
    s += v * v;
  }
  const double inv = 1.0 / (amax * sqrt(s));
  for (int r = 0; r < n; ++r) Z[r * D + m] *= inv;
}

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < kEigWaves; ++w) s = fmax(s, red[w]);
  return s;
}

// Scale-safe normalisation of column m by the whole workgroup.
__device__ void normalize_col(double* Z, int D, int n, int m, double* red) {
  double amax = 0.0;
  for (int r = threadIdx.x; r < n; r += kEigThreads) amax = fmax(amax, fabs(Z[r * D + m]));
  amax = block_max(amax, red);
  double part = 0.0;
  if (amax > 0.0 && amax < 1e308)
    for (int r = threadIdx.x; r < n; r += kEigThreads) {
      const double v = Z[r * D + m] / amax;
      part += v * v;
    }
  const double nrm = block_sum(part, red);
  const double inv = nrm > 0.0 ? 1.0 / (amax * sqrt(nrm)) : 0.0;
  for (int r = threadIdx.x; r < n; r += kEigThreads) Z[r * D + m] *= inv;
  __syncthreads();
}

// Z[:, m] -= sum_{q0 <= q < m} (Z[:,q] . Z[:,m]) Z[:,q] twice (classical Gram-Schmidt
// with one re-orthogonalisation), then normalise (whole workgroup).
__device__ void mgs_step(double* Z, int D, int n, int m, int q0, double* dots, double* red,
                         int passes = 2) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int pass = 0; pass < passes && m > q0; ++pass) {
    for (int q = q0 + wave; q < m; q += kEigWaves) {
      double s = 0.0;
      for (int r = lane; r < n; r += 64) s += Z[r * D + q] * Z[r * D + m];
      s = wave_sum(s);
      if (lane == 0) dots[q] = s;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += kEigThreads) {
      double s = Z[r * D + m];
      for (int q = q0; q < m; ++q) s -= dots[q] * Z[r * D + q];
      Z[r * D + m] = s;
    }
    __syncthreads();
  }
  normalize_col(Z, D, n, m, red);
}

__global__ __launch_bounds__(kEigThreads) void k_eig(EigArgs p0, EigArgs p1) {
  extern __shared__ double sm[];
  const EigArgs& p = blockIdx.y == 0 ? p0 : p1;
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int D = p.D;
  const int k1 = p.k1[(long long)c * p.kstride];
  const int k2 = p.k2 ? p.k2[(long long)c * p.kstride] : 0;
  const int n = k1 + k2;
  double* Uc = p.U + (long long)c * p.ustride;
  for (long long e = tid; e < (long long)D * D; e += kEigThreads) Uc[e] = 0.0;
  if (n > kEigNmax || n <= 0) {
    if (tid == 0) {
      p.rank[c] = 0;
      if (n > kEigNmax) p.status[1] = 1;
    }
    return;
  }
  const int np = n * (n + 1) / 2;
  // packed triangle in LDS up to kEigLdsN, else in the cluster's scratch (L2)
  const bool lds_p = n <= kEigLdsN;
  double* S = p.scratch + (long long)c * p.sstride;
  double* P = lds_p ? sm : S + 6LL * D * D;
  double* dd = lds_p ? sm + np : sm;
  double* ee = dd + n;
  double* lam = ee + n;
  double* pv = lam + n;
  double* wv = pv + n;
  double* red = wv + n;
  const double* Gc = p.G + (long long)c * p.gstride;
  const int half = p.half;

  // 1. gather the live block, packed lower triangle
  int bad = 0;
  for (int j = wave; j < n; j += kEigWaves) {
    const int oj = j < k1 ? j : half + (j - k1);
    for (int i = j + lane; i < n; i += 64) {
      const int oi = i < k1 ? i : half + (i - k1);
      const double v = Gc[oi + (long long)oj * D];
      if (!(v == v) || v - v != 0.0) bad = 1;
      P[pidx(i, j, n)] = v;
    }
  }
  if (bad) p.status[0] = 1;
  __syncthreads();

  // 2. Householder tridiagonalisation (lower), reflector v_i in column i
  for (int i = 0; i < n - 2; ++i) {
    double part = 0;
    for (int r = i + 1 + tid; r < n; r += kEigThreads) {
      const double x = P[pidx(r, i, n)];
      part += x * x;
    }
    const double xx = block_sum(part, red);
    const double x0 = P[pidx(i + 1, i, n)];
    const double nx = sqrt(xx);
    double alpha = 0.0;
    double vn = 1.0;
    if (nx > 0.0) {
      alpha = -copysign(nx, x0);
      const double v0 = x0 - alpha;
      vn = sqrt(xx - x0 * x0 + v0 * v0);
    }
    __syncthreads();
    if (nx > 0.0) {
      for (int r = i + 1 + tid; r < n; r += kEigThreads) {
        const double x = (r == i + 1) ? (x0 - alpha) : P[pidx(r, i, n)];
        P[pidx(r, i, n)] = x / vn;
      }
    }
    if (tid == 0) {
      dd[i] = P[pidx(i, i, n)];
      ee[i] = alpha;
    }
    __syncthreads();
    if (nx > 0.0) {
      for (int r = i + 1 + tid; r < n; r += kEigThreads) {
        double s = 0.0;
        int cc = i + 1;
        for (; cc <= r; ++cc) s += P[pidx(r, cc, n)] * P[pidx(cc, i, n)];
        const int base = pidx(r, r, n);
        for (; cc < n; ++cc) s += P[base + (cc - r)] * P[pidx(cc, i, n)];
        pv[r] = 2.0 * s;
      }
      __syncthreads();
      double part2 = 0.0;
      for (int r = i + 1 + tid; r < n; r += kEigThreads) part2 += P[pidx(r, i, n)] * pv[r];
      const double K = block_sum(part2, red);
      for (int r = i + 1 + tid; r < n; r += kEigThreads) wv[r] = pv[r] - K * P[pidx(r, i, n)];
      __syncthreads();
      for (int cc = i + 1 + wave; cc < n; cc += kEigWaves) {
        const double vc = P[pidx(cc, i, n)];
        const double wc = wv[cc];
        const int base = pidx(cc, cc, n) - cc;
        for (int r = cc + lane; r < n; r += 64) {
          P[base + r] -= P[pidx(r, i, n)] * wc + wv[r] * vc;
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = P[pidx(n - 2, n - 2, n)];
      dd[n - 1] = P[pidx(n - 1, n - 1, n)];
      ee[n - 2] = P[pidx(n - 1, n - 2, n)];
    } else {
      dd[0] = P[0];
    }
  }
  __syncthreads();
  // e^2 for the Sturm counts (pv is free now)
  for (int i = tid; i < n - 1; i += kEigThreads) pv[i] = ee[i] * ee[i];
  __syncthreads();

  // 3. eigenvalues by bisection, lam[m] = m-th largest
  double gl = 1e300, gu = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < n - 1 ? fabs(ee[i]) : 0.0);
    gl = fmin(gl, dd[i] - r);
    gu = fmax(gu, dd[i] + r);
  }
  const double bnd = fmax(fabs(gl), fabs(gu));
  const double tol = 4e-16 * bnd + 1e-300;
  gl -= tol;
  gu += tol;
  const double pivmin = 1e-290;
  for (int m = tid; m < n; m += kEigThreads) {
    const int j = n - 1 - m;
    double lo = gl, hi = gu;
    for (int it = 0; it < 160 && hi - lo > tol; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (sturm_count(dd, pv, n, mid, pivmin) > j)
        hi = mid;
      else
        lo = mid;
    }
    lam[m] = 0.5 * (lo + hi);
  }
  __syncthreads();

  // 4. kept count
  int k;
  if (p.exact) {
    k = n;
  } else if (!(lam[0] > 0.0)) {
    k = 1;
  } else {
    const double thr = p.tau * lam[0];
    k = 0;
    for (int m = 0; m < n; ++m) k += lam[m] > thr;
    if (k < 1) k = 1;
  }

  // 5a. inverse iteration, thread m owns vector m; scratch interleaved by m
  double* sd = S;
  double* sl = S + (long long)D * D;
  double* su = S + 2LL * D * D;
  double* su2 = S + 3LL * D * D;
  double* Z = S + 4LL * D * D;    // Z[r*D + m]
  double* spv = S + 5LL * D * D;  // pivot flags of the factorisation of vector m
  const double tiny = 1e-16 * fmax(bnd, 1e-300);
  if (tid < k) {
    const int m = tid;
    tri_factor(dd, ee, n, lam[m], tiny, sd, sl, su, su2, spv, D, m);
    for (int r = 0; r < n; ++r) Z[r * D + m] = start_vec(r, m);
    for (int it = 0; it < 2; ++it) {
      tri_solve(n, sd, sl, su, su2, spv, D, m, Z);
      normalize_serial(Z, D, n, m);
    }
  }
  __syncthreads();

  // 5b. eigenvalues closer than delta form a cluster: independent inverse
  // iterations cannot separate them, so each further member restarts from a
  // fresh vector and alternates orthogonalisation against the earlier
  // members with solves (the cluster handling of classical inverse iteration)
  const double delta = 1e-12 * bnd;
  int c0 = 0;
  for (int m = 1; m < k; ++m) {
    if (lam[m - 1] - lam[m] > delta) {
      c0 = m;
      continue;
    }
    for (int r = tid; r < n; r += kEigThreads) Z[r * D + m] = start_vec(r, m + 7919);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      mgs_step(Z, D, n, m, c0, pv, red);
      if (tid == 0) tri_solve(n, sd, sl, su, su2, spv, D, m, Z);
      __syncthreads();
      normalize_col(Z, D, n, m, red);
    }
    mgs_step(Z, D, n, m, c0, pv, red);
  }

  // 5c. Gram-Schmidt with re-orthogonalisation over all kept vectors: a vector
  // left with almost no component outside the earlier ones needs the second
  // pass to come out orthogonal
  for (int m = 0; m < k; ++m) mgs_step(Z, D, n, m, 0, pv, red, 2);

  // 6. back-transformation, one wave per vector, scatter to padded rows
  for (int m = wave; m < k; m += kEigWaves) {
    double z[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = lane + 64 * s;
      z[s] = r < n ? Z[r * D + m] : 0.0;
    }
    for (int i = n - 3; i >= 0; --i) {
      double part = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = lane + 64 * s;
        if (r > i && r < n) part += P[pidx(r, i, n)] * z[s];
      }
      const double sum2 = 2.0 * wave_sum(part);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = lane + 64 * s;
        if (r > i && r < n) z[s] -= sum2 * P[pidx(r, i, n)];
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = lane + 64 * s;
      if (r < n) {
        const int orow = r < k1 ? r : half + (r - k1);
        Uc[orow + (long long)m * D] = z[s];
      }
    }
  }
  if (tid == 0) p.rank[c] = k;
}

static size_t eig_lds_bytes(int D) {
  const size_t nl = D < kEigLdsN ? D : kEigLdsN;
  const size_t nv = D < kEigNmax ? D : kEigNmax;
  return sizeof(double) * (nl * (nl + 1) / 2 + 5 * nv + kEigWaves);
}

hipError_t launch_eig(const EigArgs& a, const EigArgs& b, int nclusters, hipStream_t s) {
  if (nclusters <= 0) return hipSuccess;
  const size_t lds = eig_lds_bytes(a.D > b.D ? a.D : b.D);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_eig,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)eig_lds_bytes(kEigNmax));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_eig, dim3(nclusters, 2), dim3(kEigThreads), lds, s, a, b);
  return hipGetLastError();
}

}  // namespace h2k
