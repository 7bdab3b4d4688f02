// Device evaluation of the kernel entries of h2_build: coupling matrices of
// the admissible blocks (the kernel at the two clusters' tensor Chebyshev
// nodes) and dense leaf blocks (the kernel at the points), written straight
// into the padded per-level layout.  One thread per entry; r = |x - y| and
// 1/(4 pi r) are formed in the same order as the host construction, so the
// entries agree to the last bit.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace h2k {

__device__ __forceinline__ double laplace(double x0, double x1, double x2, double y0, double y1,
                                          double y2, double self_value) {
  const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
  const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  return r == 0.0 ? self_value : 1.0 / (4.0 * M_PI * r);
}

// exp(-j kappa r)/(4 pi r) = (cos(kappa r) - j sin(kappa r))/(4 pi r)
__device__ __forceinline__ void helmholtz(double x0, double x1, double x2, double y0, double y1,
                                          double y2, double kappa, double self_re, double self_im,
                                          double& re, double& im) {
  const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
  const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  if (r == 0.0) {
    re = self_re;
    im = self_im;
    return;
  }
  const double kr = kappa * r, den = 4.0 * M_PI * r;
  re = cos(kr) / den;
  im = -sin(kr) / den;
}

__global__ void k_build_coupling(BuildCouplingArgs a) {
  const int p = a.p, p3 = p * p * p;
  const long long per = (long long)p3 * p3;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per * a.nnodes) return;
  const int q = (int)(e / per);
  if (a.types[q] != 0) return;  // admissible blocks only
  const int ij = (int)(e - (long long)q * per);
  const int i = ij % p3, j = ij / p3;
  const double* at = a.axes + (long long)a.rows[q] * 3 * p;
  const double* as = a.axes + (long long)a.cols[q] * 3 * p;
  const long long o = (long long)q * a.rr * a.rc + i + (long long)j * a.rr;
  if (a.helmholtz) {
    double re, im;
    helmholtz(at[i / (p * p)], at[p + (i / p) % p], at[2 * p + i % p], as[j / (p * p)],
              as[p + (j / p) % p], as[2 * p + j % p], a.kappa, a.self_value, a.self_imag, re, im);
    a.S[o] = re;
    a.S[a.plane + o] = im;
    return;
  }
  a.S[o] = laplace(at[i / (p * p)], at[p + (i / p) % p], at[2 * p + i % p], as[j / (p * p)],
                   as[p + (j / p) % p], as[2 * p + j % p], a.self_value);
}

__global__ void k_build_dense(BuildDenseArgs a) {
  const long long per = (long long)a.npad * a.npad;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per * a.nnodes) return;
  const int q = (int)(e / per);
  if (a.types[q] != 1) return;  // dense leaf blocks only
  const int ij = (int)(e - (long long)q * per);
  const int i = ij % a.npad, j = ij / a.npad;
  const long long r0 = a.leaf_off[a.rows[q]], c0 = a.leaf_off[a.cols[q]];
  if (r0 + i >= a.leaf_off[a.rows[q] + 1] || c0 + j >= a.leaf_off[a.cols[q] + 1]) return;
  const double* x = a.pts + 3 * (r0 + i);
  const double* y = a.pts + 3 * (c0 + j);
  const long long o = (long long)q * per + i + (long long)j * a.npad;
  if (a.helmholtz) {
    double re, im;
    helmholtz(x[0], x[1], x[2], y[0], y[1], y[2], a.kappa, a.self_value, a.self_imag, re, im);
    a.F[o] = re;
    a.F[a.plane + o] = im;
    return;
  }
  a.F[o] = laplace(x[0], x[1], x[2], y[0], y[1], y[2], a.self_value);
}

hipError_t launch_build_coupling(const BuildCouplingArgs& a, hipStream_t s) {
  const long long p3 = (long long)a.p * a.p * a.p;
  const long long total = p3 * p3 * a.nnodes;
  if (total <= 0) return hipSuccess;
  if (p3 > a.rr || p3 > a.rc) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_build_coupling, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_build_dense(const BuildDenseArgs& a, hipStream_t s) {
  const long long total = (long long)a.npad * a.npad * a.nnodes;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_dense, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace h2k
