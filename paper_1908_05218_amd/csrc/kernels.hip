// Batched kernels of the H^2 matrix-matrix product for gfx950.
//
// Every per-level step of the product (Sections III and IV of Ma & Jiao) is a
// batch of small dense products of uniform shape within one launch: cluster
// basis products (equation nonleafproduct), Gram sums (Gr1L..case3-ch-nl),
// projections (leafproj, nonleafproj), collects (Fcollect, NLcollect),
// coupling products (leafcoup_simple, nonleafcoup_simple) and the top-down
// split.  They all run through one segmented batched GEMM:
//
//   C[out(o)] = alpha * sum_{t in seg(o)} op(A[a(t)]) op(B[b(t)]) + beta * C[out(o)]
//
// One workgroup owns one TM x TN tile (32..96 per side) of one output and
// loops over the tasks of that output's segment, so every output is reduced
// in registers in a fixed order (deterministic, no atomics).  Four wave64s
// hold 16x16 MFMA accumulators; operand tiles are staged through LDS so that
// transposed and plain operands load coalesced.  The arithmetic runs in FP64
// or FP32 MFMA (the output has that type); each operand is stored in float or
// double (template parameters) and converted when staged into LDS, so the
// bulk products of the FP32 mode and the FP64 Gram sums over FP32 factors
// share one kernel.
//
// Operand addressing: an index v encodes (tile << 3) | (sel << 2) | (ch << 1) | rh.
// The block lives at base[sel] + tile*stride[sel] + rh*sub_r + ch*sub_c, so a
// child block inside its parent's 2x2 tile (the "collected" non-leaf blocks
// of equations nonleafA and nonleafB) is addressed in place.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

#include "kernels.h"

namespace h2k {

__device__ __forceinline__ long long opnd_off(const Opnd& o, int v, int& sel) {
  sel = (v >> 2) & 1;
  return (long long)(v >> 3) * o.stride[sel] + ((v & 1) ? o.sub_r : 0LL) +
         ((v & 2) ? o.sub_c : 0LL);
}

// 64-bit exchange between odd and even rows of 16 lanes: afterwards x holds
// x's and y's values of the even rows (x's in the even rows, y's in the odd
// ones), y those of the odd rows (x's in the even rows, y's in the odd ones)
__device__ __forceinline__ void swap_rows16(double& x, double& y) {
  const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
  const unsigned long long yb = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

template <typename T>
struct Mfma;

// Output lane layout of the 16x16x4 MFMAs (verified on gfx950): column
// lane % 16; row (lane/16) + 4*v for the f64 form, 4*(lane/16) + v for f32.
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// One workgroup = 4 wave64 in a 2x2 grid computes a TM x TN output tile;
// each wave holds (TM/32) x (TN/32) 16x16 MFMA accumulators.  The segment's
// (task, k-chunk) steps are software-pipelined: the global loads of step s+1
// are issued into registers before the MFMAs of step s run from one LDS
// buffer, then stored into the other buffer (one barrier per step).  PF2
// (the Gram sums and the block products, measured faster there): two
// register sets, the loads of step s+2 issued before the MFMAs of step s and
// stored one step later.  Plain and transposed operands both load coalesced.
template <typename T, int TM, int TN, typename TA, typename TB, bool PF2>
__device__ __forceinline__ void bgemm_body(const BgemmArgs<T>& p) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int KC = 16;
  constexpr int SM = TM / 32;  // 16-row subtiles per wave
  constexpr int SN = TN / 32;
  constexpr int LA = (TM * KC) / 256;  // A elements per thread per step
  constexpr int LB = (TN * KC) / 256;
  const bool low = p.lower && TM == TN && p.tiles_m == p.tiles_n;
  const int ntile = low ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  const int o = blockIdx.x / ntile;
  const int tt = blockIdx.x - o * ntile;
  int tm, tn;
  if (low) {
    // tt enumerates the tiles on and below the diagonal row by row:
    // row r holds tiles r(r+1)/2 .. r(r+1)/2 + r
    int r = (int)((sqrtf(8.0f * (float)tt + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > tt) --r;
    while ((r + 1) * (r + 2) / 2 <= tt) ++r;
    tm = r;
    tn = tt - r * (r + 1) / 2;
  } else {
    tm = tt % p.tiles_m;
    tn = tt / p.tiles_m;
  }
  __shared__ T As[2][KC][TM + 1];
  __shared__ T Bs[2][KC][TN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave & 1) * (TM / 2);
  const int wc = (wave >> 1) * (TN / 2);
  v4 acc[SM][SN];
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int b = 0; b < SN; ++b) acc[a][b] = v4{0, 0, 0, 0};
  const int s0 = p.seg[o];
  const int nk = p.k / KC;
  const int nsteps = (p.seg[o + 1] - s0) * nk;
  const int row0 = tm * TM;
  const int col0 = tn * TN;
  const int lda = p.A.ld;
  const int ldb = p.B.ld;
  // per-thread element coordinates within a step's A and B tiles
  int ai[LA], aq[LA], bj[LB], bq[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int e = tid + r * 256;
    if (!p.transA) { ai[r] = e % TM; aq[r] = e / TM; } else { aq[r] = e % KC; ai[r] = e / KC; }
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int e = tid + r * 256;
    if (!p.transB) { bq[r] = e % KC; bj[r] = e / KC; } else { bj[r] = e % TN; bq[r] = e / TN; }
  }
  // prefetch registers hold the operands in their storage types TA/TB; the
  // conversion to T happens at the LDS store, after the step's MFMAs, so the
  // loads stay in flight across them
  TA ra[LA], ra2[LA];
  TB rb[LB], rb2[LB];
  auto load_into = [&](int st, TA (&xa)[LA], TB (&xb)[LB]) {
    const int t = s0 + st / nk;
    const int kk = (st % nk) * KC;
    int sa, sb;
    const long long oa = opnd_off(p.A, p.a_idx[t], sa);
    const long long ob = opnd_off(p.B, p.b_idx[t], sb);
    const TA* Ab = (const TA*)p.A.base[sa] + oa;
    const TB* Bb = (const TB*)p.B.base[sb] + ob;
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gi = row0 + ai[r];
      xa[r] = gi < p.m ? (p.transA ? Ab[(kk + aq[r]) + (long long)gi * lda]
                                   : Ab[gi + (long long)(kk + aq[r]) * lda])
                       : (TA)0;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gj = col0 + bj[r];
      xb[r] = gj < p.n ? (p.transB ? Bb[gj + (long long)(kk + bq[r]) * ldb]
                                   : Bb[(kk + bq[r]) + (long long)gj * ldb])
                       : (TB)0;
    }
  };
  auto store_from = [&](int buf, const TA (&xa)[LA], const TB (&xb)[LB]) {
#pragma unroll
    for (int r = 0; r < LA; ++r) As[buf][aq[r]][ai[r]] = (T)xa[r];
#pragma unroll
    for (int r = 0; r < LB; ++r) Bs[buf][bq[r]][bj[r]] = (T)xb[r];
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int q4 = 0; q4 < KC / 4; ++q4) {
      T av[SM], bv[SN];
#pragma unroll
      for (int a = 0; a < SM; ++a) av[a] = As[buf][q4 * 4 + (lane >> 4)][wr + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < SN; ++b) bv[b] = Bs[buf][q4 * 4 + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < SM; ++a)
#pragma unroll
        for (int b = 0; b < SN; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
    }
  };
  if constexpr (PF2) {
    // two steps in flight: the loads of step s + 2 are issued before the
    // MFMAs of step s and stored to LDS one step later
    if (nsteps > 0) {
      load_into(0, ra, rb);
      store_from(0, ra, rb);
      if (nsteps > 1) load_into(1, ra2, rb2);
      __syncthreads();
    }
    for (int st = 0; st < nsteps; st += 2) {
      if (st + 2 < nsteps) load_into(st + 2, ra, rb);
      compute(0);
      if (st + 1 < nsteps) store_from(1, ra2, rb2);
      __syncthreads();
      if (st + 1 >= nsteps) break;
      if (st + 3 < nsteps) load_into(st + 3, ra2, rb2);
      compute(1);
      if (st + 2 < nsteps) store_from(0, ra, rb);
      __syncthreads();
    }
  } else {
    if (nsteps > 0) {
      load_into(0, ra, rb);
      store_from(0, ra, rb);
      __syncthreads();
    }
    for (int st = 0; st < nsteps; ++st) {
      const int buf = st & 1;
      const bool more = st + 1 < nsteps;
      if (more) load_into(st + 1, ra, rb);
      compute(buf);
      if (more) store_from(buf ^ 1, ra, rb);
      __syncthreads();
    }
  }
  const int ov = p.out_idx[o];
  const long long coff = (long long)(ov >> 3) * p.cstride + ((ov & 1) ? p.csub_r : 0LL) +
                         ((ov & 2) ? p.csub_c : 0LL);
  T* Cb = (T*)p.C + coff;
  // FP32: a lane holds four consecutive rows of one column, written as one
  // 16-byte access where the output's rows and columns keep that alignment.
  // FP64: a lane holds rows r, r+4, r+8, r+12 (r = lane / 16); two swaps with
  // the neighbouring 16-lane group leave it two pairs of adjacent rows, each
  // written as one 16-byte access
  const bool vec4 = sizeof(T) == 4 && ((coff | p.ldc | row0) & 3) == 0 &&
                    (((uintptr_t)p.C) & 15) == 0;
  const bool vec2 = sizeof(T) == 8 && ((coff | p.ldc | row0) & 1) == 0 &&
                    (((uintptr_t)p.C) & 15) == 0;
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int b = 0; b < SN; ++b) {
      const int gj = col0 + wc + b * 16 + (lane & 15);
      if constexpr (sizeof(T) == 8) {
        if (vec2) {
          double x0 = acc[a][b][0], x1 = acc[a][b][1], x2 = acc[a][b][2], x3 = acc[a][b][3];
          swap_rows16(x0, x1);  // rows base, base + 1
          swap_rows16(x2, x3);  // rows base + 8, base + 9
          const int g = lane >> 4;
          const int gi = row0 + wr + a * 16 + (g & 1) * 4 + (g >> 1) * 2;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = gi + 8 * h;
            const double e0 = (double)p.alpha * (h ? x2 : x0), e1 = (double)p.alpha * (h ? x3 : x1);
            if (gj < p.n && r + 1 < p.m) {
              double2* c = (double2*)(Cb + r + (long long)gj * p.ldc);
              double2 val = make_double2(e0, e1);
              if (p.beta != (T)0) {
                const double2 old = *c;
                val.x += (double)p.beta * old.x;
                val.y += (double)p.beta * old.y;
              }
              *c = val;
            } else if (gj < p.n) {
              for (int q = 0; q < 2; ++q) {
                if (r + q < p.m) {
                  T* c = Cb + r + q + (long long)gj * p.ldc;
                  T val = q ? e1 : e0;
                  if (p.beta != (T)0) val += p.beta * (*c);
                  *c = val;
                }
              }
            }
          }
          continue;
        }
      }
      const int gi0 = row0 + wr + a * 16 + Mfma<T>::row(lane, 0);
      if (vec4 && gi0 + 3 < p.m && gj < p.n) {
        float4* c = (float4*)(Cb + gi0 + (long long)gj * p.ldc);
        float4 val = make_float4((float)(p.alpha * acc[a][b][0]), (float)(p.alpha * acc[a][b][1]),
                                 (float)(p.alpha * acc[a][b][2]), (float)(p.alpha * acc[a][b][3]));
        if (p.beta != (T)0) {
          const float4 old = *c;
          const float bt = (float)p.beta;
          val.x += bt * old.x;
          val.y += bt * old.y;
          val.z += bt * old.z;
          val.w += bt * old.w;
        }
        *c = val;
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + wr + a * 16 + Mfma<T>::row(lane, v);
        if (gi < p.m && gj < p.n) {
          T* c = Cb + gi + (long long)gj * p.ldc;
          T val = p.alpha * acc[a][b][v];
          if (p.beta != (T)0) val += p.beta * (*c);
          *c = val;
        }
      }
    }
}

// Entry points over the same body, one per kernel class so that traces and
// counters separate them: the block-product ("triple") batches of the
// coupling step, the per-target products, the Gram sums (FP64) and the rest
// (projections, collects, splits, basis products).
template <typename T, int TM, int TN, typename TA, typename TB>
__global__ __launch_bounds__(256) void k_bgemm(BgemmArgs<T> p) {
  bgemm_body<T, TM, TN, TA, TB, false>(p);
}

template <typename T, int TM, int TN, typename TA, typename TB>
__global__ __launch_bounds__(256) void k_bgemm_triple(BgemmArgs<T> p) {
  bgemm_body<T, TM, TN, TA, TB, true>(p);
}

template <typename T, int TM, int TN, typename TA, typename TB>
__global__ __launch_bounds__(256) void k_bgemm_target(BgemmArgs<T> p) {
  bgemm_body<T, TM, TN, TA, TB, false>(p);
}

template <typename T, int TM, int TN, typename TA, typename TB>
__global__ __launch_bounds__(256) void k_bgemm_gram(BgemmArgs<T> p) {
  bgemm_body<T, TM, TN, TA, TB, true>(p);
}

// Wave-split 32 x 32 tile for segments of many tasks: each wave takes every
// fourth task of the output's segment for the whole tile (four independent
// 16 x 16 accumulators), stages its operands in a wave-private LDS region (no
// workgroup barrier in the main loop, the next step's loads in flight during
// the MFMAs), and the four partial tiles are summed in wave order at the end
// (deterministic).
template <typename T, typename TA, typename TB, bool TRA, bool TRB>
__device__ __forceinline__ void bgemm_ws_body(const BgemmArgs<T>& p) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int TM = 32, KC = 16, LD = TM + 1;
  constexpr int LA = TM * KC / 64;  // elements per lane and step, A and B alike
  constexpr int WREG = 2 * KC * LD;  // a wave's staging region (A then B)
  __shared__ T sm[4 * WREG];    // also the reduction buffer (4 x 32 x 32)
  static_assert(4 * WREG >= 4 * TM * TM, "reduction buffer");
  const bool low = p.lower && p.tiles_m == p.tiles_n;
  const int ntile = low ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  const int o = blockIdx.x / ntile;
  const int tt = blockIdx.x - o * ntile;
  int tm, tn;
  if (low) {
    int r = (int)((sqrtf(8.0f * (float)tt + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > tt) --r;
    while ((r + 1) * (r + 2) / 2 <= tt) ++r;
    tm = r;
    tn = tt - r * (r + 1) / 2;
  } else {
    tm = tt % p.tiles_m;
    tn = tt / p.tiles_m;
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = tm * TM, col0 = tn * TM;
  const int lda = p.A.ld, ldb = p.B.ld;
  const int s0 = p.seg[o], ntask = p.seg[o + 1] - s0;
  const int nk = p.k / KC;
  const int mine = ntask > wave ? (ntask - wave + 3) / 4 : 0;
  const int nsteps = mine * nk;
  // element r of a lane's share of a step (e = lane + 64 r): plain
  // operands take row e % 32 of column e / 32, transposed ones column e % 16
  // of row e / 16, so the coordinates are affine in r
  const int l32 = lane & 31, h32 = lane >> 5, l16 = lane & 15, h16 = lane >> 4;
  constexpr bool ta = TRA, tb = TRB;
  auto ai = [&](int r) { return ta ? h16 + 4 * r : l32; };
  auto aq = [&](int r) { return ta ? l16 : h32 + 2 * r; };
  auto bj = [&](int r) { return tb ? l32 : h16 + 4 * r; };
  auto bq = [&](int r) { return tb ? h32 + 2 * r : l16; };
  TA ra[LA];
  TB rb[LA];
  auto load_step = [&](int st) {
    const int t = __builtin_amdgcn_readfirstlane(s0 + wave + 4 * (st / nk));
    const int kk = (st % nk) * KC;
    int sa, sb;
    const long long oa = opnd_off(p.A, p.a_idx[t], sa);
    const long long ob = opnd_off(p.B, p.b_idx[t], sb);
    const TA* Ab = (const TA*)p.A.base[sa] + oa;
    const TB* Bb = (const TB*)p.B.base[sb] + ob;
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gi = row0 + ai(r), ka = kk + aq(r);
      ra[r] = gi < p.m ? Ab[ta ? ka + gi * lda : gi + ka * lda] : (TA)0;
      const int gj = col0 + bj(r), kb = kk + bq(r);
      rb[r] = gj < p.n ? Bb[tb ? gj + kb * ldb : kb + gj * ldb] : (TB)0;
    }
  };
  T* Aw = sm + wave * WREG;
  T* Bw = Aw + KC * LD;
  v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};
  if (nsteps > 0) load_step(0);
  for (int st = 0; st < nsteps; ++st) {
    // the region is the wave's own: its LDS operations run in program order,
    // so the compiler barrier alone orders this step's stores after the
    // previous step's reads
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      Aw[aq(r) * LD + ai(r)] = (T)ra[r];
      Bw[bq(r) * LD + bj(r)] = (T)rb[r];
    }
    __builtin_amdgcn_wave_barrier();
    if (st + 1 < nsteps) load_step(st + 1);
#pragma unroll
    for (int q4 = 0; q4 < KC / 4; ++q4) {
      const int kq = (q4 * 4 + (lane >> 4)) * LD + (lane & 15);
      const T a0 = Aw[kq], a1 = Aw[kq + 16], b0 = Bw[kq], b1 = Bw[kq + 16];
      acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
    }
  }
  __syncthreads();
  // partial tiles, column-major 32 x 32 per wave
  T* red = sm;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = a * 16 + Mfma<T>::row(lane, v), c = b * 16 + (lane & 15);
        red[wave * TM * TM + r + c * TM] = acc[a][b][v];
      }
  __syncthreads();
  const int ov = p.out_idx[o];
  const long long coff = (long long)(ov >> 3) * p.cstride + ((ov & 1) ? p.csub_r : 0LL) +
                         ((ov & 2) ? p.csub_c : 0LL);
  T* Cb = (T*)p.C + coff;
#pragma unroll
  for (int i = 0; i < TM * TM / 256; ++i) {
    const int e = tid + 256 * i, r = e & (TM - 1), c = e / TM;
    const int gi = row0 + r, gj = col0 + c;
    if (gi < p.m && gj < p.n) {
      const T sum = ((red[e] + red[TM * TM + e]) + red[2 * TM * TM + e]) + red[3 * TM * TM + e];
      T* cp = Cb + gi + (long long)gj * p.ldc;
      T val = p.alpha * sum;
      if (p.beta != (T)0) val += p.beta * (*cp);
      *cp = val;
    }
  }
}

template <typename T, typename TA, typename TB, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_bgemm_ws(BgemmArgs<T> p) {
  bgemm_ws_body<T, TA, TB, TRA, TRB>(p);
}
template <typename T, typename TA, typename TB, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_bgemm_triple_ws(BgemmArgs<T> p) {
  bgemm_ws_body<T, TA, TB, TRA, TRB>(p);
}
template <typename T, typename TA, typename TB, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_bgemm_target_ws(BgemmArgs<T> p) {
  bgemm_ws_body<T, TA, TB, TRA, TRB>(p);
}
template <typename T, typename TA, typename TB, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_bgemm_gram_ws(BgemmArgs<T> p) {
  bgemm_ws_body<T, TA, TB, TRA, TRB>(p);
}

template <typename T>
__global__ __launch_bounds__(256) void k_segsum(SegsumArgs<T> p) {
  const int per = (p.m * p.n + 255) / 256;
  const int o = blockIdx.x / per;
  const int chunk = blockIdx.x - o * per;
  const int e = chunk * 256 + threadIdx.x;
  if (e >= p.m * p.n) return;
  const int i = e % p.m;
  const int j = e / p.m;
  T s = 0;
  for (int t = p.seg[o]; t < p.seg[o + 1]; ++t) {
    int sel;
    const long long off = opnd_off(p.A, p.a_idx[t], sel);
    s += ((const T*)p.A.base[sel])[off + i + (long long)j * p.A.ld];
  }
  const int v = p.out_idx[o];
  T* c = p.C + (long long)(v >> 3) * p.cstride + ((v & 1) ? p.csub_r : 0LL) +
         ((v & 2) ? p.csub_c : 0LL) + i + (long long)j * p.ldc;
  *c = (p.beta != (T)0) ? (*c) * p.beta + s : s;
}

// Normalised Gram sum of one cluster: sum over the non-empty components of
// G_c / trace(G_c) (each component divided by its trace).  The workgroups
// blockIdx.y of a cluster each take every gridDim.y-th group of four columns
// (one column per wave, the lanes down its rows: coalesced), after computing
// the cluster's traces themselves.
__global__ __launch_bounds__(256) void k_gram_norm(GramNormArgs p) {
  const int c = blockIdx.x;
  const int D = p.D;
  __shared__ double tr[3];
  __shared__ double red[256];
  for (int comp = 0; comp < 3; ++comp) {
    double s = 0;
    if (p.G[comp]) {
      const double* g = p.G[comp] + (long long)c * p.stride;
      for (int i = threadIdx.x; i < D; i += 256) s += g[i + (long long)i * D];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) tr[comp] = red[0];
    __syncthreads();
  }
  const double w0 = tr[0] > 0 ? 1.0 / tr[0] : 0.0;
  const double w1 = tr[1] > 0 ? 1.0 / tr[1] : 0.0;
  const double w2 = tr[2] > 0 ? 1.0 / tr[2] : 0.0;
  const long long base = (long long)c * p.stride;
  const double* g0 = p.G[0] + base;
  const double* g1 = p.G[1] ? p.G[1] + base : nullptr;
  const double* g2 = p.G[2] ? p.G[2] + base : nullptr;
  double* out = p.out + base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int bad = 0;
  // the sums are symmetric and read on and below the diagonal only (the
  // products may leave the part above it unwritten)
  for (int j = 4 * blockIdx.y + wave; j < D; j += 4 * gridDim.y) {
    const long long cj = (long long)j * D;
    for (int i = j + lane; i < D; i += 64) {
      double v = w0 * g0[cj + i];
      if (g1) v += w1 * g1[cj + i];
      if (g2) v += w2 * g2[cj + i];
      if (!(v == v) || v - v != 0.0) bad = 1;
      out[cj + i] = v;
    }
  }
  if (bad) p.status[0] = 1;
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* in, Tout* out, long long n) {
  // four elements per thread (16-byte float and 2 x 16-byte double accesses;
  // the pool's buffers are 256-byte aligned), a scalar tail for the rest
  const long long i = 4 * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
  if (i + 3 < n) {
    Tin v[4];
    if constexpr (sizeof(Tin) == 4) {
      const float4 f = *(const float4*)(in + i);
      v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else {
      const double2 a = *(const double2*)(in + i), b = *(const double2*)(in + i + 2);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    if constexpr (sizeof(Tout) == 4) {
      *(float4*)(out + i) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    } else {
      *(double2*)(out + i) = make_double2((double)v[0], (double)v[1]);
      *(double2*)(out + i + 2) = make_double2((double)v[2], (double)v[3]);
    }
  } else {
    for (long long j = i; j < n; ++j) out[j] = (Tout)in[j];
  }
}

__global__ void k_scale(double* p, double a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] *= a;
}

// F[node] += b I on the first size[t] diagonal entries of the dense diagonal
// leaf blocks listed in node[] (one workgroup per block)
__global__ void k_shift_diag(double* F, const int* node, const int* size, int npad, double b) {
  const int t = blockIdx.x;
  double* f = F + (long long)node[t] * npad * npad;
  for (int r = threadIdx.x; r < size[t]; r += blockDim.x) f[r + (long long)r * npad] += b;
}

__global__ void k_fill(double* p, double v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f(float* p, float v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// x (n x nrhs, original order, ld = n) -> padded tree order
// (leaf c, local row r) at out[(c*npad + r) + col*(nleaf*npad)].
__global__ void k_gather_rows(const double* x, double* out, const long long* perm,
                              const long long* leaf_off, int nleaf, int npad, long long n,
                              int nrhs) {
  const long long total = (long long)nleaf * npad;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total * nrhs) return;
  const long long col = e / total;
  const long long rr = e - col * total;
  const int c = (int)(rr / npad);
  const int r = (int)(rr - (long long)c * npad);
  const long long pos = leaf_off[c] + r;
  double v = 0;
  if (pos < leaf_off[c + 1]) v = x[perm[pos] + col * n];
  out[e] = v;
}

__global__ void k_scatter_rows(const double* in, double* y, const long long* perm,
                               const long long* leaf_off, int nleaf, int npad, long long n,
                               int nrhs) {
  const long long total = (long long)nleaf * npad;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total * nrhs) return;
  const long long col = e / total;
  const long long rr = e - col * total;
  const int c = (int)(rr / npad);
  const int r = (int)(rr - (long long)c * npad);
  const long long pos = leaf_off[c] + r;
  if (pos < leaf_off[c + 1]) y[perm[pos] + col * n] = in[e];
}

// ---------------------------------------------------------------- launches
static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

template <typename T, int TM, int TN>
static hipError_t launch_tile(BgemmArgs<T> a, hipStream_t s) {
  a.tiles_m = cdiv(a.m, TM);
  a.tiles_n = cdiv(a.n, TN);
  const bool low = a.lower && TM == TN && a.tiles_m == a.tiles_n;
  const long long per = low ? (long long)a.tiles_m * (a.tiles_m + 1) / 2
                            : (long long)a.tiles_m * a.tiles_n;
  const long long grid = (long long)a.nout * per;
  const dim3 g((unsigned)grid), b(256);
#define H2K_LAUNCH(K)                                                  \
  do {                                                                 \
    if (a.A.f32 && a.B.f32)                                            \
      hipLaunchKernelGGL((K<T, TM, TN, float, float>), g, b, 0, s, a);   \
    else if (a.A.f32)                                                  \
      hipLaunchKernelGGL((K<T, TM, TN, float, double>), g, b, 0, s, a);  \
    else if (a.B.f32)                                                  \
      hipLaunchKernelGGL((K<T, TM, TN, double, float>), g, b, 0, s, a);  \
    else                                                               \
      hipLaunchKernelGGL((K<T, TM, TN, double, double>), g, b, 0, s, a); \
  } while (0)
  if (a.symbol == 1)
    H2K_LAUNCH(k_bgemm_triple);
  else if (a.symbol == 2)
    H2K_LAUNCH(k_bgemm_target);
  else if constexpr (std::is_same<T, double>::value) {
    if (a.symbol == 3)
      H2K_LAUNCH(k_bgemm_gram);
    else
      H2K_LAUNCH(k_bgemm);
  } else
    H2K_LAUNCH(k_bgemm);
#undef H2K_LAUNCH
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_ws(BgemmArgs<T> a, hipStream_t s) {
  a.tiles_m = cdiv(a.m, 32);
  a.tiles_n = cdiv(a.n, 32);
  const bool low = a.lower && a.tiles_m == a.tiles_n;
  const long long per = low ? (long long)a.tiles_m * (a.tiles_m + 1) / 2
                            : (long long)a.tiles_m * a.tiles_n;
  const dim3 g((unsigned)((long long)a.nout * per)), b(256);
#define H2K_WS1(K, TRA, TRB)                                                           \
  do {                                                                                 \
    if (a.A.f32 && a.B.f32)                                                            \
      hipLaunchKernelGGL((K<T, float, float, TRA, TRB>), g, b, 0, s, a);               \
    else if (a.A.f32)                                                                  \
      hipLaunchKernelGGL((K<T, float, double, TRA, TRB>), g, b, 0, s, a);              \
    else if (a.B.f32)                                                                  \
      hipLaunchKernelGGL((K<T, double, float, TRA, TRB>), g, b, 0, s, a);              \
    else                                                                               \
      hipLaunchKernelGGL((K<T, double, double, TRA, TRB>), g, b, 0, s, a);             \
  } while (0)
#define H2K_WS(K)                     \
  do {                                \
    if (a.transA && a.transB)         \
      H2K_WS1(K, true, true);         \
    else if (a.transA)                \
      H2K_WS1(K, true, false);        \
    else if (a.transB)                \
      H2K_WS1(K, false, true);        \
    else                              \
      H2K_WS1(K, false, false);       \
  } while (0)
  if (a.symbol == 1)
    H2K_WS(k_bgemm_triple_ws);
  else if (a.symbol == 2)
    H2K_WS(k_bgemm_target_ws);
  else if constexpr (std::is_same<T, double>::value) {
    if (a.symbol == 3)
      H2K_WS(k_bgemm_gram_ws);
    else
      H2K_WS(k_bgemm_ws);
  } else
    H2K_WS(k_bgemm_ws);
#undef H2K_WS
#undef H2K_WS1
  return hipGetLastError();
}

// Workgroup tile: the whole output when it fits 96 x 96 (96 x 32, 32 x 96 and
// 96 x 96 shapes), otherwise 32 or 64 per side.
template <typename T>
hipError_t launch_bgemm(const BgemmArgs<T>& a, hipStream_t s) {
  if (a.nout <= 0) return hipSuccess;
  if (a.c_f32 != (sizeof(T) == sizeof(float))) return hipErrorInvalidValue;  // C has type T
  switch (a.tile) {  // a measured choice (every tile masks partial edges)
    case kTile32x32: return launch_tile<T, 32, 32>(a, s);
    case kTile32x32ws: return launch_ws<T>(a, s);
    case kTile96x32: return launch_tile<T, 96, 32>(a, s);
    case kTile32x96: return launch_tile<T, 32, 96>(a, s);
    case kTile96x96: return launch_tile<T, 96, 96>(a, s);
    case kTile32x64: return launch_tile<T, 32, 64>(a, s);
    case kTile64x32: return launch_tile<T, 64, 32>(a, s);
    case kTile64x64: return launch_tile<T, 64, 64>(a, s);
    default: break;
  }
  const int mx = a.m > a.n ? a.m : a.n;
  if (a.m <= 32 && a.n <= 32) return launch_tile<T, 32, 32>(a, s);
  if (a.m > 64 && a.m <= 96 && a.n <= 32) return launch_tile<T, 96, 32>(a, s);
  if (a.n > 64 && a.n <= 96 && a.m <= 32) return launch_tile<T, 32, 96>(a, s);
  if (mx > 64 && a.m <= 96 && a.n <= 96) return launch_tile<T, 96, 96>(a, s);
  if (a.m <= 32) return launch_tile<T, 32, 64>(a, s);
  if (a.n <= 32) return launch_tile<T, 64, 32>(a, s);
  return launch_tile<T, 64, 64>(a, s);
}

template <typename T>
hipError_t launch_segsum(const SegsumArgs<T>& a, hipStream_t s) {
  if (a.nout <= 0) return hipSuccess;
  const long long per = (a.m * (long long)a.n + 255) / 256;
  hipLaunchKernelGGL(k_segsum<T>, dim3((unsigned)(per * a.nout)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gram_norm(const GramNormArgs& a, int nclusters, hipStream_t s) {
  if (nclusters <= 0) return hipSuccess;
  // about 2048 workgroups in all, at most one per group of four columns
  const int groups = (a.D + 3) / 4;
  int per = (2048 + nclusters - 1) / nclusters;
  per = per < 1 ? 1 : (per > groups ? groups : per);
  hipLaunchKernelGGL(k_gram_norm, dim3(nclusters, per), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scale(double* p, double a, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(cdiv(n, 256)), dim3(256), 0, s, p, a, n);
  return hipGetLastError();
}

hipError_t launch_shift_diag(double* F, const int* node, const int* size, int nblocks, int npad,
                             double b, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift_diag, dim3(nblocks), dim3(64), 0, s, F, node, size, npad, b);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f(float* p, float v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_d2f(const double* in, float* out, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<double, float>), dim3(cdiv(n, 1024)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_f2d(const float* in, double* out, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(cdiv(n, 1024)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double* x, double* out, const long long* perm,
                              const long long* leaf_off, int nleaf, int npad, long long n,
                              int nrhs, hipStream_t s) {
  const long long tot = (long long)nleaf * npad * nrhs;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3(cdiv(tot, 256)), dim3(256), 0, s, x, out, perm,
                     leaf_off, nleaf, npad, n, nrhs);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const double* in, double* y, const long long* perm,
                               const long long* leaf_off, int nleaf, int npad, long long n,
                               int nrhs, hipStream_t s) {
  const long long tot = (long long)nleaf * npad * nrhs;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3(cdiv(tot, 256)), dim3(256), 0, s, in, y, perm,
                     leaf_off, nleaf, npad, n, nrhs);
  return hipGetLastError();
}

template hipError_t launch_bgemm<double>(const BgemmArgs<double>&, hipStream_t);
template hipError_t launch_bgemm<float>(const BgemmArgs<float>&, hipStream_t);
template hipError_t launch_segsum<double>(const SegsumArgs<double>&, hipStream_t);
template hipError_t launch_segsum<float>(const SegsumArgs<float>&, hipStream_t);

}  // namespace h2k
