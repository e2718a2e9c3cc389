// MI355X (gfx950) evaluation of one-electron nuclear-attraction integrals over contracted
// solid-harmonic Gaussian orbitals, behind the C ABI declared in include/shgo.h.
//
// Method (arXiv:2404.16245): Gaussian product (Eq. 5), shift of both solid harmonics to the
// product center P with the vector-coupling coefficients (Eqs. 7-8), product rule of solid
// harmonics (the supplement's Eq. 4), one-center Coulomb integral by Hobson's theorem and the
// Boys function (Eqs. 11-12, each r^{2k} Y^L_M term of the product rule giving
// Y^L_M(c-P) 2 pi k!/p^{k+1} sum_j T^j/j! F_{L+j}(T)), sum over nuclei, contraction.
//
// Device design (one process, one GPU):
//   a1  k_classify, k_scan_keys, k_scatter: per-shell normalisation (extra k_classify workgroups), shell-pair
//       enumeration, screening, counting sort by class (LA >= LB) and surviving primitive pairs,
//       the work-item list and each pair's output destination.
//   a2-a8  k_integrals: persistent, one workgroup of eight wavefronts per CU. A work item is a
//       block of tiles of 64 class-sorted shell pairs (one per lane); its (tile, group) tasks go
//       to the wavefronts, group g owning some half-families |M| of W. Work is done in the frame
//       whose z axis is A->B, where the shift of Eq. 7 keeps m (only Y^lambda_0 of a z-directed
//       vector survives). Per primitive pair and nucleus (nuclei read through the scalar cache):
//       C = c - P in the frame, Boys F_m, monic solid-harmonic recurrences, W(L,M,k) += Z G_{L,k} Q
//       in registers; then the product-rule and shift coefficients map W onto the block V' in the
//       item's LDS accumulator (atomic adds); after a barrier the blocks are rotated back with
//       D^T = Z(phi) J^T Z(theta) J by all wavefronts and written with coalesced stores.
//   P3  k_grad<LA,LB>: the adjoint of the above for dE/d(centers, nuclei) of E = sum D V.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <utility>
#include <string>
#include <vector>

#include "shgo.h"
#define SHGO_TILE 64  // shell pairs per tile: one per lane of a wavefront
#define SHGO_ACC_STRIDE (SHGO_TILE + 1)  // doubles between entries of a tile accumulator
#include "generated/shgo_classes.inc"
#include "generated/shgo_grad.inc"

namespace {

// ---------------------------------------------------------------------------------------------
// Constants and small types
// ---------------------------------------------------------------------------------------------
constexpr int kBoysOrders = 22;    // F_0..F_21 stored per grid point (mmax <= 14 with 8 Taylor terms)
constexpr int kBoysPoints = 1153;  // grid t_i = i/16, i = 0..1152
constexpr double kBoysTcut = 72.0; // below: table; above: asymptotic form (e^{-t} < 6e-32)
constexpr int kNumClasses = (SHGO_LMAX + 1) * (SHGO_LMAX + 2) / 2;  // (la, lb) with la >= lb
constexpr int kKeysPerClass = 256;
constexpr int kTile = SHGO_TILE;
constexpr int kNumKeys = kNumClasses * kKeysPerClass;
constexpr int kIntegralThreads = 512;  // one workgroup per CU: 8 wavefronts share a tile's accumulator
constexpr int kMaxTilesPerItem = 8;
constexpr int kAccStride = SHGO_ACC_STRIDE;
constexpr int kFrameDoubles = 4 * kTile;  // pair frames of one tile: cos/sin of theta and phi
// Dynamic LDS of a work item, in doubles: per tile an accumulator of NA*NB x kAccStride doubles and
// its frames. The kernel's static LDS (queue words, per-tile iteration counts) fits in the last
// 256 bytes of the CU's 160 KB.
constexpr int kLdsDoubles = (163840 - 256) / 8;
constexpr int kPrefetchMaxW = 32;      // groups up to this many W doubles prefetch the next nucleus

__host__ __device__ constexpr int class_id(int la, int lb) { return la * (la + 1) / 2 + lb; }

struct alignas(32) Nuc {
  double x, y, z, Z;
};
// Nuclei are read through the scalar data cache: the index is the same in every lane, and the
// constant address space lets the compiler use scalar loads.
typedef const __attribute__((address_space(4))) Nuc* NucPtr;


__device__ __forceinline__ NucPtr uniform_nuclei(const Nuc* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (NucPtr)(((uint64_t)hi << 32) | lo);
}

struct DevBasis {
  const double* center;    // [n][3]
  const int32_t* l;        // [n]
  const int32_t* nprim;    // [n]
  const int64_t* prim_off; // [n]
  const double* expo;      // [nprim total]
  const double* coef;      // [nprim total]
  double* w;               // [nprim total] normalised weights (written by k_classify)
  const int64_t* bf_off;   // [n] first basis function of each shell
  int32_t n_shells;
  int64_t nbf;
};

struct DevPairs {
  int64_t n_cand;          // candidate shell pairs
  int32_t full;            // 1: all a <= b of the basis; 0: explicit list
  const int32_t* pa;       // [n_cand] (explicit list)
  const int32_t* pb;
  const int64_t* blk_off;  // [n_cand] output offset of each block (explicit list)
  int32_t* key;            // [n_cand] sort key
  int32_t* s1;             // [n_cand] sorted: shell with the higher l
  int32_t* s2;             // [n_cand] sorted: the other shell
  int32_t* orig;           // [n_cand] sorted: candidate index
  int32_t* nsurv;          // [n_cand] sorted: surviving primitive pairs
  int32_t* key_count;      // [kNumKeys]
  int32_t* rank;           // [n_cand] position inside the key's bucket
  int32_t* key_off;        // [kNumKeys + 1]
  int64_t* dst0;           // [n_cand] sorted: output row offset of s1 (matrix) or block offset (list)
  int64_t* dst1;           // [n_cand] sorted: output offset of s2 (matrix) or 1 if the listed pair is (s2, s1)
  double screen;
};

// Schedule of the persistent integral kernel.
struct ClassMeta {
  float weight[kNumClasses];   // relative time of one primitive-pair iteration of a tile of the class
  int32_t tiles[kNumClasses];  // tiles per work item, 1..8, within the LDS of a workgroup
  int32_t groups[kNumClasses]; // wavefront groups of the class (fixed by the generated code)
};
constexpr int kCostBuckets = 128;  // work items are dispatched by cost bucket, 4 per octave
constexpr int kSliceIters = 8;     // primitive-pair iterations per task of a long tile

// ---------------------------------------------------------------------------------------------
// Exponential (device)
// ---------------------------------------------------------------------------------------------
// The polynomial constants of an exponential inside the integral kernel's loops would otherwise be
// kept in vector registers across the loop and, under the kernel's register pressure, spilled and
// reloaded on every iteration. These helpers take the constant as a scalar operand (one per
// instruction, the constant-bus limit), materialised in scalar registers.
__device__ __forceinline__ double fma_vvs(double a, double b, double c) {  // a * b + c, c scalar
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}
__device__ __forceinline__ double mul_vs(double a, double b) {  // a * b, b scalar
  double r;
  asm("v_mul_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}
__device__ __forceinline__ double add_vs(double a, double b) {  // a + b, b scalar
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}

// e^{-t} for t >= 0 (0 once it underflows): Cody-Waite reduction t = n ln 2 - r with the two-part
// ln 2 of fdlibm (n ln2_hi exact), |r| <= ln(2)/2, and the Taylor polynomial of e^r to degree 13
// (remainder below 5e-18 relative) by Horner's rule, then the exponent n.
__device__ __forceinline__ double exp_neg(double t) {
  const double x = -fmin(t, 746.0);
  const double n = rint(x * 1.4426950408889634074);  // log2(e)
  double r = fma(n, -6.93147180369123816490e-01, x);
  r = fma(n, -1.90821492927058770002e-10, r);
  double q = add_vs(mul_vs(r, 1.6059043836821614599e-10), 2.0876756987868098979e-09);  // 1/13!, 1/12!
  q = fma_vvs(q, r, 2.5052108385441718775e-08);  // 1/11!
  q = fma_vvs(q, r, 2.7557319223985890653e-07);  // 1/10!
  q = fma_vvs(q, r, 2.7557319223985890653e-06);  // 1/9!
  q = fma_vvs(q, r, 2.4801587301587301587e-05);  // 1/8!
  q = fma_vvs(q, r, 1.9841269841269841270e-04);  // 1/7!
  q = fma_vvs(q, r, 1.3888888888888888889e-03);  // 1/6!
  q = fma_vvs(q, r, 8.3333333333333333333e-03);  // 1/5!
  q = fma_vvs(q, r, 4.1666666666666666667e-02);  // 1/4!
  q = fma_vvs(q, r, 1.6666666666666666667e-01);  // 1/3!
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return ldexp(q, (int)n);
}

// ---------------------------------------------------------------------------------------------
// Boys function (device)
// ---------------------------------------------------------------------------------------------
// F_m(t) for m = 0..M. Below kBoysTcut: Taylor expansion of F_M about the nearest grid point,
//   F_M(t_i + d) = sum_{k<8} F_{M+k}(t_i) (-d)^k / k!,  |d| <= 1/32,
// then the stable downward recursion F_m = (2t F_{m+1} + e^{-t})/(2m+1).  Above: the asymptote
//   F_0 = sqrt(pi/t)/2 - e^{-t}/(2t) (1 - 1/(2t) + 3/(4t^2)) (the erfc term, tail < 1e-18),
// then the upward recursion F_{m+1} = ((2m+1) F_m - e^{-t})/(2t), stable for t > m.
template <int M>
__device__ __forceinline__ void boys(double t, double (&F)[M + 1], const double* __restrict__ tab) {
  const double e = exp_neg(t);
  if (t < kBoysTcut) {
    const int i = (int)(t * 16.0 + 0.5);
    const double d = -(t - 0.0625 * (double)i);
    const double* __restrict__ row = tab + i * kBoysOrders + M;
    double f = row[7];
    f = fma(f, d * (1.0 / 7.0), row[6]);
    f = fma(f, d * (1.0 / 6.0), row[5]);
    f = fma(f, d * (1.0 / 5.0), row[4]);
    f = fma(f, d * (1.0 / 4.0), row[3]);
    f = fma(f, d * (1.0 / 3.0), row[2]);
    f = fma(f, d * (1.0 / 2.0), row[1]);
    f = fma(f, d, row[0]);
    F[M] = f;
    const double t2 = 2.0 * t;
#pragma unroll
    for (int m = M - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (2 * m + 1));
  } else {
    // 1/sqrt(t) from the hardware estimate and two Newton steps (each doubles the bits)
    double rs = __builtin_amdgcn_rsq(t);
    rs = rs * fma(-0.5 * t * rs, rs, 1.5);
    rs = rs * fma(-0.5 * t * rs, rs, 1.5);
    const double it = rs * rs;
    const double f0 = 0.88622692545275801365 * rs;  // sqrt(pi)/2 / sqrt(t)
    const double corr = 0.5 * e * it * fma(it, fma(it, 0.75, -0.5), 1.0);
    F[0] = f0 - corr;
    const double h = 0.5 * it;
#pragma unroll
    for (int m = 0; m < M; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * h;
  }
}

// x^N by repeated squaring (depth log2 N).
template <int N>
__device__ __forceinline__ double pow_n(double x) {
  if constexpr (N == 0) {
    return 1.0;
  } else if constexpr (N == 1) {
    return x;
  } else {
    const double h = pow_n<N / 2>(x);
    return (N & 1) ? h * h * x : h * h;
  }
}
// Gamma(M + 1/2) / 2 = sqrt(pi) (2M-1)!! / 2^{M+1}
__host__ __device__ constexpr double half_gamma_half(int M) {
  double c = 0.88622692545275801365;
  for (int k = 1; k <= M; ++k) c *= (2.0 * k - 1.0) * 0.5;
  return c;
}

// The same evaluation for the integral kernel, with the Taylor row F_{M..M+7}(t_i) of the nearest
// grid point (clamped to the table) already loaded and e = exp(-t), and no divergent branch: F_M
// is the table's Taylor series below kBoysTcut and the leading asymptotic term
// Gamma(M+1/2) / (2 t^{M+1/2}) above it (the neglected part is below e^{-t}/t, 1e-17 relative for
// M <= 12 at t = 72), selected per lane; then the downward recursion, stable for every t.
template <int M>
__device__ __forceinline__ void boys_row(double t, double e, const double (&row)[8], double (&F)[M + 1]) {
  const int i = (int)(fmin(t, kBoysTcut) * 16.0 + 0.5);
  const double d = -(t - 0.0625 * (double)i);
  double f = row[7];
  f = fma(f, d * (1.0 / 7.0), row[6]);
  f = fma(f, d * (1.0 / 6.0), row[5]);
  f = fma(f, d * (1.0 / 5.0), row[4]);
  f = fma(f, d * (1.0 / 4.0), row[3]);
  f = fma(f, d * (1.0 / 3.0), row[2]);
  f = fma(f, d * (1.0 / 2.0), row[1]);
  f = fma(f, d, row[0]);
  // 1/sqrt(t) from the hardware estimate and two Newton steps (each doubles the bits)
  double rs = __builtin_amdgcn_rsq(t);
  rs = rs * fma(-0.5 * t * rs, rs, 1.5);
  rs = rs * fma(-0.5 * t * rs, rs, 1.5);
  const double fa = half_gamma_half(M) * rs * pow_n<M>(rs * rs);
  F[M] = t < kBoysTcut ? f : fa;
  const double t2 = 2.0 * t;
#pragma unroll
  for (int m = M - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (2 * m + 1));
}

template <int M>
__global__ void k_boys(int64_t n, const double* __restrict__ T, double* __restrict__ F,
                       const double* __restrict__ tab) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double f[M + 1];
  boys<M>(T[i], f, tab);
#pragma unroll
  for (int m = 0; m <= M; ++m) F[i * (M + 1) + m] = f[m];
}

// ---------------------------------------------------------------------------------------------
// a1: normalisation, enumeration, screening, class sort
// ---------------------------------------------------------------------------------------------
// Normalised weight of primitive k of a shell: w_k = d_k N_k / sqrt(sum_kk' d_k d_k' <phi_k|phi_k'>)
// with N(l,a)^2 = 2^l (2a)^{l+3/2}/((2l-1)!! pi^{3/2}) and, for normalised primitives,
// <phi_k|phi_k'> = n_k n_k' / (a_k + a_k')^{l+3/2}, n_k = (2 a_k)^{(l+3/2)/2}. The half-integer
// powers are products of integer powers and square roots.
__device__ __forceinline__ double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}
__device__ __forceinline__ double pow_half_q(double x, int l) {  // x^{(l+3/2)/2}
  const double s = sqrt(x);
  return ipow(x, l >> 1) * ((l & 1) ? s : 1.0) * sqrt(x * s);
}
__device__ __forceinline__ double pow_q(double y, int l) {  // y^{l+3/2}
  return ipow(y, l) * y * sqrt(y);
}
__device__ void prim_weights_of(const DevBasis& b, int s) {
  const int l = b.l[s], K = b.nprim[s];
  const int64_t o = b.prim_off[s];
  double dfac = 1.0;
  for (int i = 2 * l - 1; i > 1; i -= 2) dfac *= i;
  const double cn = sqrt(ldexp(1.0, l) / (dfac * 5.5683279968317078453));  // pi^{3/2}
  double ss = 0.0;
  for (int k = 0; k < K; ++k) {
    const double ak = b.expo[o + k], nk = pow_half_q(2.0 * ak, l), dk = b.coef[o + k];
    for (int j = 0; j < K; ++j) {
      const double aj = b.expo[o + j], nj = pow_half_q(2.0 * aj, l);
      ss += dk * b.coef[o + j] * nk * nj / pow_q(ak + aj, l);
    }
  }
  const double inv = 1.0 / sqrt(ss);
  for (int k = 0; k < K; ++k) b.w[o + k] = b.coef[o + k] * cn * pow_half_q(2.0 * b.expo[o + k], l) * inv;
}

// (a, b) with a <= b from the linear index of the upper triangle in row-major order.
__device__ __forceinline__ void tri_pair(int64_t i, int n, int& a, int& b) {
  const int64_t m = (int64_t)n * (n + 1) / 2;
  const int64_t j = m - 1 - i;
  int64_t r = (int64_t)((sqrt(8.0 * (double)j + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= j) ++r;
  while (r * (r + 1) / 2 > j) --r;
  a = n - 1 - (int)r;
  b = n - 1 - (int)(j - r * (r + 1) / 2);
}

__device__ __forceinline__ bool keep_prim(double a, double b, double R2, double screen) {
  if (!(screen > 0.0)) return true;
  return exp_neg(a * b / (a + b) * R2) > screen;
}

// Classification in workgroups of 1024 candidates: the key of each candidate, its rank among
// the workgroup's candidates with the same key (LDS atomics), and one global atomic per
// (workgroup, key) that reserves the workgroup's range inside the key's bucket. Workgroups from
// classify_blocks on compute the shells' normalised primitive weights instead (independent work,
// in the same launch).
constexpr int kClassifyThreads = 1024;
__global__ void __launch_bounds__(kClassifyThreads) k_classify(DevBasis bs, DevPairs pr, int classify_blocks) {
  if ((int)blockIdx.x >= classify_blocks) {
    const int s = ((int)blockIdx.x - classify_blocks) * blockDim.x + threadIdx.x;
    if (s < bs.n_shells) prim_weights_of(bs, s);
    return;
  }
  __shared__ int hist[kNumKeys];  // counts, then the workgroup's base in each key's bucket
  for (int b = threadIdx.x; b < kNumKeys; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1, rank = 0;
  if (i < pr.n_cand) {
    int a, b;
    if (pr.full) {
      tri_pair(i, bs.n_shells, a, b);
    } else {
      a = pr.pa[i];
      b = pr.pb[i];
    }
    const int la = bs.l[a], lb = bs.l[b];
    const int s1 = la >= lb ? a : b, s2 = la >= lb ? b : a;
    const int L1 = bs.l[s1], L2 = bs.l[s2];
    double R2 = 0.0;
    for (int x = 0; x < 3; ++x) {
      const double d = bs.center[3 * s2 + x] - bs.center[3 * s1 + x];
      R2 += d * d;
    }
    int ns = 0;
    const int64_t o1 = bs.prim_off[s1], o2 = bs.prim_off[s2];
    for (int p = 0; p < bs.nprim[s1]; ++p)
      for (int q = 0; q < bs.nprim[s2]; ++q) ns += keep_prim(bs.expo[o1 + p], bs.expo[o2 + q], R2, pr.screen);
    key = class_id(L1, L2) * kKeysPerClass + min(ns, kKeysPerClass - 1);
    rank = atomicAdd(&hist[key], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kNumKeys; b += blockDim.x)
    if (hist[b] > 0) hist[b] = atomicAdd(&pr.key_count[b], hist[b]);
  __syncthreads();
  if (i < pr.n_cand) {
    pr.key[i] = key;
    pr.rank[i] = hist[key] + rank;
  }
}

// Cost bucket of work item i (class c = the one whose items start at or below i): the class's
// weight times the primitive-pair iterations of the item's longest tile (the surviving-pair count
// of its last slot, keys being sorted within the class) times its tiles, over the wavefronts its
// tasks keep busy; four buckets per octave.
__device__ int item_bucket(int i, const int* ioff, const int* koff, const ClassMeta& meta, int& c, int& blk) {
  int lo_c = 0, hi_c = kNumClasses - 1;  // the last class whose items start at or below i
  while (lo_c < hi_c) {
    const int mid = (lo_c + hi_c + 1) >> 1;
    if (ioff[mid] <= i)
      lo_c = mid;
    else
      hi_c = mid - 1;
  }
  c = lo_c;
  blk = i - ioff[c];
  const int T = meta.tiles[c];
  const int start = koff[c * kKeysPerClass], end = koff[(c + 1) * kKeysPerClass];
  const int tiles = (end - start + kTile - 1) / kTile;
  const int nt = min(T, tiles - blk * T);
  const int last = min(start + (blk * T + nt) * kTile, end) - 1;
  int lo = 0, hi = kKeysPerClass - 1;  // largest key k of the class with koff <= last
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (koff[c * kKeysPerClass + mid] <= last)
      lo = mid;
    else
      hi = mid - 1;
  }
  // eight wavefronts share the item's (tile, slice, group) tasks
  const int m = max(lo, 1);
  const int tasks = nt * meta.groups[c] * max(1, (m + kSliceIters - 1) / kSliceIters);
  const float cost = meta.weight[c] * (float)m * (float)nt / (float)min(8, tasks);
  if (!(cost >= 1.0f)) return 0;
  return min(kCostBuckets - 1, (int)(4.0f * log2f(cost)));
}

// Inclusive prefix sum of v over the 1024 threads of the workgroup: each wavefront scans its 64
// values with shuffles, the first wavefront scans the 16 wavefront totals (wsum, LDS), two
// barriers in all. Every thread of the workgroup must call it.
__device__ __forceinline__ int scan_1024(int v, int* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(v, off);
    if (lane >= off) v += u;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  if (w == 0) {
    int x = lane < 16 ? wsum[lane] : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int u = __shfl_up(x, off);
      if (lane >= off) x += u;
    }
    if (lane < 16) wsum[lane] = x;
  }
  __syncthreads();
  return w > 0 ? v + wsum[w - 1] : v;
}

// Exclusive scan of key_count into key_off (one workgroup of 1024 threads), then the work-item
// list of the integral kernel: every class's blocks of tiles[c] tiles, sorted by decreasing cost
// bucket (a counting sort in LDS), so that the persistent kernel takes the longest items first.
// Also clears key_count for the next evaluation and resets the queue head.
__global__ void __launch_bounds__(1024) k_scan_keys(DevPairs pr, ClassMeta meta, int32_t* item_off, int32_t* items,
                                                    int32_t* queue) {
  static_assert(kCostBuckets == 128, "the bucket scan gives each lane of one wavefront two buckets");
  __shared__ int wsum[16];
  __shared__ int citems[kNumClasses];
  __shared__ int koff[kNumKeys + 1];
  __shared__ int ioff[kNumClasses + 1];  // first item of each class, in class-id order
  __shared__ int bcount[kCostBuckets];
  constexpr int per = (kNumKeys + 1023) / 1024;
  const int t = threadIdx.x;
  int loc[per];
  int s = 0;
  for (int j = 0; j < per; ++j) {
    const int k = t * per + j;
    loc[j] = k < kNumKeys ? pr.key_count[k] : 0;
    if (k < kNumKeys) pr.key_count[k] = 0;  // cleared for the next evaluation's k_classify
    s += loc[j];
  }
  if (t < kCostBuckets) bcount[t] = 0;
  const int incl = scan_1024(s, wsum);
  int run = incl - s;
  for (int j = 0; j < per; ++j) {
    const int k = t * per + j;
    if (k < kNumKeys) {
      pr.key_off[k] = run;
      koff[k] = run;
    }
    run += loc[j];
  }
  if (t == 1023) {
    pr.key_off[kNumKeys] = incl;
    koff[kNumKeys] = incl;
  }
  __syncthreads();
  if (t < kNumClasses) {  // items of class t
    const int tiles = (koff[(t + 1) * kKeysPerClass] - koff[t * kKeysPerClass] + kTile - 1) / kTile;
    citems[t] = (tiles + meta.tiles[t] - 1) / meta.tiles[t];
  }
  __syncthreads();
  if (t <= kNumClasses) {  // first item of class t (t = kNumClasses: the total)
    int off = 0;
    for (int c = 0; c < t; ++c) off += citems[c];
    ioff[t] = off;
    if (t == kNumClasses) {
      item_off[0] = off;
      queue[0] = 0;
    }
  }
  __syncthreads();
  const int total = ioff[kNumClasses];
  int c, blk;
  for (int i = t; i < total; i += 1024) atomicAdd(&bcount[item_bucket(i, ioff, koff, meta, c, blk)], 1);
  __syncthreads();
  // bucket starts, most expensive bucket first: rank r = kCostBuckets - 1 - bucket; lane t of the
  // first wavefront holds ranks 2t and 2t + 1 and scans their sums with shuffles
  if (t < 64) {
    const int b0 = kCostBuckets - 1 - 2 * t, b1 = b0 - 1;
    const int a0 = bcount[b0], a1 = bcount[b1];
    int x = a0 + a1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(x, off);
      if (t >= off) x += u;
    }
    const int start = x - a0 - a1;
    bcount[b0] = start;
    bcount[b1] = start + a0;
  }
  __syncthreads();
  for (int i = t; i < total; i += 1024) {
    const int b = item_bucket(i, ioff, koff, meta, c, blk);
    items[atomicAdd(&bcount[b], 1)] = (c << 24) | blk;
  }
}

__global__ void k_scatter(DevBasis bs, DevPairs pr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pr.n_cand) return;
  int a, b;
  if (pr.full) {
    tri_pair(i, bs.n_shells, a, b);
  } else {
    a = pr.pa[i];
    b = pr.pb[i];
  }
  const int key = pr.key[i];
  const int slot = pr.key_off[key] + pr.rank[i];
  const bool sw = bs.l[a] < bs.l[b];
  pr.s1[slot] = sw ? b : a;
  pr.s2[slot] = sw ? a : b;
  pr.orig[slot] = (int32_t)i;
  pr.nsurv[slot] = key % kKeysPerClass;
  if (pr.full) {
    pr.dst0[slot] = bs.bf_off[sw ? b : a];
    pr.dst1[slot] = bs.bf_off[sw ? a : b];
  } else {
    pr.dst0[slot] = pr.blk_off[i];
    pr.dst1[slot] = sw ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------------------------
// a2-a8: the persistent integral kernel
// ---------------------------------------------------------------------------------------------
// Work item = (class, block of up to T tiles of SHGO_TILE class-sorted shell pairs). Every
// workgroup (one per CU, eight wavefronts) pulls items from one queue (classes in decreasing cost
// per tile). Its wavefronts take the item's (tile, group of half-families) tasks from an LDS
// counter, run the group's primitive-pair and nucleus loops for the tile's pairs (one pair per
// lane) and add the group's part of each block V' into the item's accumulator in LDS. After a
// workgroup barrier each tile's blocks are rotated back to the laboratory frame and written.
// Nothing crosses a workgroup: no global atomics on partial sums and no device-scope fences.

__host__ __device__ constexpr int class_nab(int c) {
  int la = 0;
  while ((la + 1) * (la + 2) / 2 <= c) ++la;
  const int lb = c - la * (la + 1) / 2;
  return (2 * la + 1) * (2 * lb + 1);
}
__host__ __device__ constexpr int class_tile_doubles(int c) { return class_nab(c) * kAccStride + kFrameDoubles; }
__host__ __device__ constexpr int class_max_tiles(int c) {
  return kLdsDoubles / class_tile_doubles(c) < kMaxTilesPerItem ? kLdsDoubles / class_tile_doubles(c) : kMaxTilesPerItem;
}

struct WorkArgs {
  DevBasis bs;
  DevPairs pr;
  const Nuc* __restrict__ nuc;
  int32_t n_nuc;
  const double* __restrict__ boys_tab;
  int32_t* __restrict__ queue;     // [0]: next work item
  int32_t* __restrict__ item_off;  // [0]: number of work items
  int32_t* __restrict__ items;     // work items, longest first: class << 24 | tile block
  unsigned long long* __restrict__ item_ns;  // per-item durations (10 ns ticks) when tuning, else null
  ClassMeta meta;
};
// The work arguments live in device memory (one copy per plan) and are read through the scalar
// data cache: every lane of a wavefront reads the same fields.
typedef const __attribute__((address_space(4))) WorkArgs* WAP;

__device__ __forceinline__ WAP uniform_args(const WorkArgs* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (WAP)(((uint64_t)hi << 32) | lo);
}

// Per-lane shell-pair state.
struct PairState {
  int s1, s2;
  bool active;
  double A[3], B[3];
  double R, ct, st, cp, sp;  // |B-A| and the frame angles
  int64_t o1, o2;
  int K1, K2;
  int nsurv;
};

__device__ __forceinline__ void frame_of(PairState& ps) {
  const double rx = ps.B[0] - ps.A[0], ry = ps.B[1] - ps.A[1], rz = ps.B[2] - ps.A[2];
  const double rho2 = rx * rx + ry * ry;
  const double R = sqrt(rho2 + rz * rz);
  const double rho = sqrt(rho2);
  ps.R = R;
  if (R > 0.0) {
    ps.ct = rz / R;
    ps.st = rho / R;
  } else {
    ps.ct = 1.0;
    ps.st = 0.0;
  }
  if (rho > 0.0) {
    ps.cp = rx / rho;
    ps.sp = ry / rho;
  } else {
    ps.cp = 1.0;
    ps.sp = 0.0;
  }
}

// Advance (i, j) to the next primitive pair that survives screening; false when exhausted.
__device__ __forceinline__ bool next_prim(const PairState& ps, WAP wa, int& i, int& j) {
  const double R2 = ps.R * ps.R;
  while (true) {
    ++j;
    if (j >= ps.K2) {
      j = 0;
      ++i;
    }
    if (i >= ps.K1) return false;
    if (keep_prim(wa->bs.expo[ps.o1 + i], wa->bs.expo[ps.o2 + j], R2, wa->pr.screen)) return true;
  }
}

// Primitive-pair iterations [it_begin, it_end) of group G for the wavefront's 64 pairs: the pair's
// surviving primitive pairs in order, the first it_begin skipped.
template <int LA, int LB, int G>
__device__ __forceinline__ void run_group(const PairState& ps, WAP wa, int it_begin, int it_end, int c_begin, int c_end,
                                          double* __restrict__ Vp) {
  using Grp = GroupOf<LA, LB, G>;
  constexpr int LM = LA + LB;
  int pi = 0, pj = -1;
  if (ps.active)
    for (int it = 0; it < it_begin; ++it) (void)next_prim(ps, wa, pi, pj);
  for (int it = it_begin; it < it_end; ++it) {
    const bool have = ps.active && next_prim(ps, wa, pi, pj);
    if (have) {
      const double a = wa->bs.expo[ps.o1 + pi], b = wa->bs.expo[ps.o2 + pj];
      const double p = a + b, ip = 1.0 / p;
      const double Px = (a * ps.A[0] + b * ps.B[0]) * ip;
      const double Py = (a * ps.A[1] + b * ps.B[1]) * ip;
      const double Pz = (a * ps.A[2] + b * ps.B[2]) * ip;
      double W[Grp::NW];
#pragma unroll
      for (int q = 0; q < Grp::NW; ++q) W[q] = 0.0;
      // nucleus loop: geometry in the pair frame, Boys row from LDS, then the group's step
      double nx = 0.0, ny = 0.0, nz = 0.0, nr2 = 0.0, nt = 0.0, nZ = 0.0, nrow[8];
      const NucPtr nucs = uniform_nuclei(wa->nuc);
      const int c_lo = __builtin_amdgcn_readfirstlane(c_begin), n_nuc = __builtin_amdgcn_readfirstlane(c_end);
      auto geometry = [&](int c) {
        const double cx = nucs[c].x - Px, cy = nucs[c].y - Py, cz = nucs[c].z - Pz;
        const double u = fma(ps.cp, cx, ps.sp * cy);
        nx = fma(ps.ct, u, -ps.st * cz);
        ny = fma(-ps.sp, cx, ps.cp * cy);
        nz = fma(ps.st, u, ps.ct * cz);
        nr2 = fma(cx, cx, fma(cy, cy, cz * cz));
        nt = p * nr2;
        nZ = nucs[c].Z;
        const int i = (int)(fmin(nt, kBoysTcut) * 16.0 + 0.5);  // 0 .. kBoysPoints - 1
        const double* __restrict__ r = wa->boys_tab + i * kBoysOrders + LM;
#pragma unroll
        for (int k = 0; k < 8; ++k) nrow[k] = r[k];
      };
      auto nucleus = [&](double x, double y, double z, double r2, double t, double Zc, const double (&row)[8]) {
        const double e = exp_neg(t);
        double F[LM + 1];
        boys_row<LM>(t, e, row, F);
        double tj[LB + 1];
        tj[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LB; ++k) tj[k] = tj[k - 1] * t * (1.0 / k);
        Grp::step(W, x, y, z, r2, Zc, F, tj);
      };
      if constexpr (Grp::NW <= kPrefetchMaxW) {
        // small groups have registers to spare: the next nucleus is fetched one step ahead
        if (c_lo < n_nuc) geometry(c_lo);
        for (int c = c_lo; c < n_nuc; ++c) {
          const double x = nx, y = ny, z = nz, r2 = nr2, t = nt, Zc = nZ;
          double row[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) row[k] = nrow[k];
          if (c + 1 < n_nuc) geometry(c + 1);
          nucleus(x, y, z, r2, t, Zc, row);
        }
      } else {
        for (int c = c_lo; c < n_nuc; ++c) {
          geometry(c);
          nucleus(nx, ny, nz, nr2, nt, nZ, nrow);
        }
      }
      // prefactor -w_a w_b exp(-mu R^2) and 2 pi k!/p^{k+1}
      const double K = exp_neg(a * b * ip * ps.R * ps.R);
      const double pre = -wa->bs.w[ps.o1 + pi] * wa->bs.w[ps.o2 + pj] * K;
      double fk[LB + 1];
      fk[0] = pre * 6.283185307179586477 * ip;
#pragma unroll
      for (int k = 1; k <= LB; ++k) fk[k] = fk[k - 1] * (double)k * ip;
      Grp::scale(W, fk);
      double ta[LA + 1], tb[LB + 1];
      const double tav = b * ps.R * ip, tbv = -a * ps.R * ip;
      ta[0] = 1.0;
      tb[0] = 1.0;
#pragma unroll
      for (int k = 1; k <= LA; ++k) ta[k] = ta[k - 1] * tav;
#pragma unroll
      for (int k = 1; k <= LB; ++k) tb[k] = tb[k - 1] * tbv;
      Grp::couple(W, ta, tb, Vp);
    }
  }
}

template <int LA, int LB, int G>
__device__ __forceinline__ void dispatch_group(int g, const PairState& ps, WAP wa, int it0, int it1, int c0, int c1,
                                               double* Vp) {
  if constexpr (G < ClassInfo<LA, LB>::Q) {
    if (g == G) {
      run_group<LA, LB, G>(ps, wa, it0, it1, c0, c1, Vp);
      return;
    }
    dispatch_group<LA, LB, G + 1>(g, ps, wa, it0, it1, c0, c1, Vp);
  }
}

template <int L>
__device__ __forceinline__ void angles(double c1, double s1, double (&c)[L + 1], double (&s)[L + 1]) {
  c[0] = 1.0;
  s[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= L; ++m) {
    c[m] = c[m - 1] * c1 - s[m - 1] * s1;
    s[m] = s[m - 1] * c1 + c[m - 1] * s1;
  }
}

// Dynamic LDS of the integral kernel, for a work item of nt tiles:
//   accumulator [tile][NA*NB][kAccStride]  V' of each pair (lane-contiguous; one pad double per row
//               keeps a pair's strided reads free of bank conflicts)
//   frames      [tile][4][SHGO_TILE]       cos/sin of theta and phi of each pair
extern __shared__ double s_lds[];
__shared__ int s_tile_iters[kMaxTilesPerItem];  // primitive-pair iterations of each tile of the item

template <int LA, int LB>
__device__ __forceinline__ void load_pair(PairState& ps, WAP wa, int slot, int end) {
  ps.active = slot < end;
  const int sl = ps.active ? slot : end - 1;
  ps.s1 = wa->pr.s1[sl];
  ps.s2 = wa->pr.s2[sl];
  ps.nsurv = ps.active ? wa->pr.nsurv[sl] : 0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    ps.A[x] = wa->bs.center[3 * ps.s1 + x];
    ps.B[x] = wa->bs.center[3 * ps.s2 + x];
  }
  ps.o1 = wa->bs.prim_off[ps.s1];
  ps.o2 = wa->bs.prim_off[ps.s2];
  ps.K1 = wa->bs.nprim[ps.s1];
  ps.K2 = wa->bs.nprim[ps.s2];
  frame_of(ps);
}

// One work item of class (LA, LB): tile block b, run by the whole workgroup. Kept out of line
// so that every class is compiled and register-allocated on its own.
template <int LA, int LB>
__device__ __attribute__((noinline)) void process_block(int b, const WorkArgs* wa_ptr, double* __restrict__ out,
                                                        int* task_ctr, int* next_item) {
  const WAP wa = uniform_args(wa_ptr);
  constexpr int Q = ClassInfo<LA, LB>::Q;
  constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NAB = NA * NB;
  constexpr int cls = class_id(LA, LB);
  constexpr int kWaves = kIntegralThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int T = wa->meta.tiles[cls];
  const int start = wa->pr.key_off[cls * kKeysPerClass];
  const int end = wa->pr.key_off[(cls + 1) * kKeysPerClass];
  const int tiles = (end - start + kTile - 1) / kTile;
  const int t0 = b * T, nt = min(T, tiles - t0);
  double* const acc = s_lds;
  double* const frm = s_lds + nt * NAB * kAccStride;
  {
    double2* const a2 = (double2*)acc;
    const int n = nt * NAB * kAccStride;
    for (int i = threadIdx.x; i < n / 2; i += kIntegralThreads) a2[i] = make_double2(0.0, 0.0);
    if ((n & 1) && threadIdx.x == 0) acc[n - 1] = 0.0;
  }
  // primitive-pair iterations of each tile (the most over its pairs; keys saturate at 255 and then
  // every candidate primitive pair is visited, the screened ones skipped): wavefront w, tile w
  if (wave < nt) {
    const int slot = start + (t0 + wave) * kTile + lane;
    int it = 0;
    if (slot < end) {
      it = wa->pr.nsurv[slot];
      if (it >= kKeysPerClass - 1) it = wa->bs.nprim[wa->pr.s1[slot]] * wa->bs.nprim[wa->pr.s2[slot]];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) it = max(it, __shfl_xor(it, off));
    if (lane == 0) s_tile_iters[wave] = it;
  }
  __syncthreads();
  // tasks (tile, slice of at most kSliceIters primitive-pair iterations, group), tile-major, handed
  // to the wavefronts by an LDS counter
  // The first task of wavefront w is task w (groups are generated heaviest first, and the older
  // wavefronts of a SIMD issue first), the rest come from the counter, which starts at kWaves.
  const int n_nuc = wa->n_nuc;
  bool first = true;
  while (true) {
    int task = wave;
    if (!first) {
      if (lane == 0) task = atomicAdd(task_ctr, 1);
      task = __shfl(task, 0);
    }
    first = false;
    int u = task / Q;
    const int g = task - u * Q;
    int t = 0, m = 0;
    for (; t < nt; ++t) {
      m = s_tile_iters[t];
      const int slices = max(1, (m + kSliceIters - 1) / kSliceIters);
      if (u < slices) break;
      u -= slices;
    }
    if (t >= nt) break;
    PairState ps;
    load_pair<LA, LB>(ps, wa, start + (t0 + t) * kTile + lane, end);
    if (g == 0 && u == 0) {
      double* const f = frm + t * 4 * kTile + lane;
      f[0] = ps.ct;
      f[kTile] = ps.st;
      f[2 * kTile] = ps.cp;
      f[3 * kTile] = ps.sp;
    }
    const int it0 = u * kSliceIters;
    dispatch_group<LA, LB, 0>(g, ps, wa, it0, min(m, it0 + kSliceIters), 0, n_nuc, acc + t * NAB * kAccStride + lane);
  }
  __syncthreads();
  // the workgroup's next work item, fetched now so that the atomic's latency hides behind the
  // rotations and stored for the caller at the end (every thread has read the current one)
  int next = 0;
  if (threadIdx.x == 0) next = atomicAdd(wa->queue, 1);
  // Back to the laboratory frame, V = D_a^T V' D_b with D^T = Z(phi) J^T Z(theta) J: the rows of
  // every tile, then its columns, as (tile, row) and (tile, column) tasks over all wavefronts.
  for (int k = wave; k < nt * NA; k += kWaves) {
    const int t = k / NA, r = k - t * NA;
    const double* f = frm + t * 4 * kTile + lane;
    double cth[LA + 1], sth[LA + 1], cph[LA + 1], sph[LA + 1];
    angles<LA>(f[0], f[kTile], cth, sth);
    angles<LA>(f[2 * kTile], f[3 * kTile], cph, sph);
    double* V = acc + (t * NAB + r * NB) * kAccStride + lane;
    double v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) v[j] = V[j * kAccStride];
    Rot<LB>::apply(v, cth, sth, cph, sph);
#pragma unroll
    for (int j = 0; j < NB; ++j) V[j * kAccStride] = v[j];
  }
  __syncthreads();
  for (int k = wave; k < nt * NB; k += kWaves) {
    const int t = k / NB, col = k - t * NB;
    const double* f = frm + t * 4 * kTile + lane;
    double cth[LA + 1], sth[LA + 1], cph[LA + 1], sph[LA + 1];
    angles<LA>(f[0], f[kTile], cth, sth);
    angles<LA>(f[2 * kTile], f[3 * kTile], cph, sph);
    double* V = acc + (t * NAB + col) * kAccStride + lane;
    double v[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) v[i] = V[i * NB * kAccStride];
    Rot<LA>::apply(v, cth, sth, cph, sph);
#pragma unroll
    for (int i = 0; i < NA; ++i) V[i * NB * kAccStride] = v[i];
  }
  __syncthreads();
  // Output: consecutive threads take consecutive entries of one pair's block, so every store
  // instruction covers a few contiguous lines. The pairs' destinations from the pair build (dst0,
  // dst1) are first copied into the frames area, which the rotations no longer need.
  const int base = start + t0 * kTile;
  const int n_out = nt * kTile * NAB;
  int64_t* const dst = (int64_t*)frm;  // [tile * 64 + pair][2]
  for (int j = threadIdx.x; j < nt * kTile; j += kIntegralThreads) {
    const int slot = base + j;
    if (slot < end) {
      dst[2 * j] = wa->pr.dst0[slot];
      dst[2 * j + 1] = wa->pr.dst1[slot];
    }
  }
  __syncthreads();
  constexpr int kU = 4;
  if (wa->pr.full) {
    const int64_t n = wa->bs.nbf;
    // rows of the (s1, s2) block (entry e = i NB + col), then of the mirrored (s2, s1) block
    // (entry e = col NA + i)
    for (int pass = 0; pass < 2; ++pass) {
      for (int j0 = threadIdx.x; j0 < n_out; j0 += kU * kIntegralThreads) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int j = j0 + u * kIntegralThreads;
          const int tp = j / NAB, e = j - tp * NAB;  // tp = tile * 64 + pair
          const int slot = base + tp;
          if (j < n_out && slot < end) {
            const int64_t r0 = dst[2 * tp], c0 = dst[2 * tp + 1];
            int i, col;
            if (pass == 0) {
              i = e / NB;
              col = e - i * NB;
            } else {
              col = e / NA;
              i = e - col * NA;
            }
            const double v = acc[((tp >> 6) * NAB + i * NB + col) * kAccStride + (tp & 63)];
            if (r0 != c0 || i <= col) {
              if (pass == 0)
                out[(r0 + i) * n + c0 + col] = v;
              else
                out[(c0 + col) * n + r0 + i] = v;
            }
          }
        }
      }
    }
  } else {
    // pair blocks: (s1, s2) order, or transposed where the listed pair is (s2, s1)
    for (int j0 = threadIdx.x; j0 < n_out; j0 += kU * kIntegralThreads) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * kIntegralThreads;
        const int tp = j / NAB, e = j - tp * NAB;
        const int slot = base + tp;
        if (j < n_out && slot < end) {
          const int64_t bo = dst[2 * tp];
          const bool sw = dst[2 * tp + 1] != 0;
          int src = e;
          if (sw) {  // output entry e = col NA + i holds V(i, col)
            const int col = e / NA, i = e - col * NA;
            src = i * NB + col;
          }
          out[bo + e] = acc[((tp >> 6) * NAB + src) * kAccStride + (tp & 63)];
        }
      }
    }
  }
  if (threadIdx.x == 0) *next_item = next;
}

template <int LA, int LB>
__device__ __forceinline__ void dispatch_class(int c, int j, const WorkArgs* wa, double* out, int* task_ctr,
                                               int* next_item) {
  if constexpr (LA <= SHGO_LMAX) {
    if (c == class_id(LA, LB)) {
      process_block<LA, LB>(j, wa, out, task_ctr, next_item);
      return;
    }
    if constexpr (LB < LA)
      dispatch_class<LA, LB + 1>(c, j, wa, out, task_ctr, next_item);
    else
      dispatch_class<LA + 1, 0>(c, j, wa, out, task_ctr, next_item);
  }
}

// Every workgroup loops: take the next item, run it with its eight wavefronts; the loop ends
// once the queue is drained.
__global__ void __launch_bounds__(kIntegralThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_integrals(const WorkArgs* __restrict__ wa_ptr, double* __restrict__ out) {
  const WAP wa = uniform_args(wa_ptr);
  __shared__ int s_item, s_task;
  if (threadIdx.x == 0) s_item = atomicAdd(wa->queue, 1);
  const int total = wa->item_off[0];
  while (true) {
    if (threadIdx.x == 0) s_task = kIntegralThreads / 64;
    __syncthreads();
    const int q = s_item;
    if (q >= total) break;
    const int item = wa->items[q];
    unsigned long long* const tick = wa->item_ns;
    const unsigned long long t0 = tick ? wall_clock64() : 0ull;
    dispatch_class<0, 0>(item >> 24, item & 0xffffff, wa_ptr, out, &s_task, &s_item);
    if (tick && threadIdx.x == 0) tick[q] = wall_clock64() - t0;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Overlap matrix S (Eqs. 4-10): the shell pairs, pair frame, rotation back and output layout of V
// ---------------------------------------------------------------------------------------------
// In the pair frame (z along A -> B) the shifts of both harmonics to P run along z and keep m
// (Eqs. 7-8), and the one-center overlap of S^lam_m(u) with S^lam'_m'(u) under e^{-p u^2} vanishes
// unless lam = lam' and m = m' (Eq. 9: orthogonality of the harmonics; the coupling of Eq. 10 keeps
// only L = 0). With the scaled regular solid harmonics R_l^m = Y_l^m / sqrt((l+m)!(l-m)!), whose
// z-shift is R_l^m(u + t z) = sum_lam R_lam^m(u) t^(l-lam) / (l-lam)!, the frame block is diagonal:
//   S'(m, m) = sum over primitive pairs of w_a w_b e^{-mu R^2} sum_{lam=|m|}^{lb} A(la,lam,m) A(lb,lam,m)
//              t_a^(la-lam) t_b^(lb-lam) (4 pi / (2 lam + 1)) Gamma(lam + 3/2) / (2 p^(lam + 3/2)),
//   A(l, lam, m) = sqrt((l+m)! (l-m)! / ((lam+m)! (lam-m)!)) / (l-lam)!,  t_a = beta R / p,  t_b = -alpha R / p.
// Every primitive pair counts (no screening). One lane per class-sorted shell pair.
__host__ __device__ constexpr double fact_d(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

// Staged stores: the wavefront's 64 blocks (all of one class) leave through LDS a row at a time,
// consecutive lanes on consecutive entries, then a column at a time for the mirror.
constexpr int kOvlStage = 64 * (2 * SHGO_LMAX + 1);  // doubles per wavefront
__shared__ double s_ovl_stage[4][kOvlStage];
__shared__ int64_t s_ovl_d0[4][64], s_ovl_d1[4][64];

__device__ __forceinline__ void ovl_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// kStaged: every lane of the wavefront runs this class (inactive lanes, past the last pair, with
// active = false: no loads, no stores of their own) and the stores go through LDS; otherwise each
// active lane stores its own block.
template <int LA, int LB, bool kStaged>
__device__ __forceinline__ void overlap_pair(const DevBasis& bs, const DevPairs& pr, int slot, bool active,
                                             double* __restrict__ out) {
  constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1;
  PairState ps;
  const int s1 = active ? pr.s1[slot] : 0, s2 = active ? pr.s2[slot] : 0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    ps.A[x] = active ? bs.center[3 * s1 + x] : 0.0;
    ps.B[x] = active ? bs.center[3 * s2 + x] : 0.0;
  }
  frame_of(ps);
  const double R = ps.R;
  // A(la, lam, m) A(lb, lam, m) (4 pi / (2 lam + 1)) Gamma(lam + 3/2) / 2, for m <= lam <= lb
  double cf[LB + 1][LB + 1];
#pragma unroll
  for (int m = 0; m <= LB; ++m)
#pragma unroll
    for (int lam = 0; lam <= LB; ++lam) {
      if (lam < m) {
        cf[m][lam] = 0.0;
        continue;
      }
      const double den = fact_d(lam + m) * fact_d(lam - m);
      const double aa = sqrt(fact_d(LA + m) * fact_d(LA - m) / den) / fact_d(LA - lam);
      const double ab = sqrt(fact_d(LB + m) * fact_d(LB - m) / den) / fact_d(LB - lam);
      double dfac = 1.0;  // (2 lam + 1)!!
      for (int i = 2 * lam + 1; i > 1; i -= 2) dfac *= (double)i;
      const double gam = dfac * 1.7724538509055160273 / ldexp(1.0, lam + 1);  // Gamma(lam + 3/2)
      cf[m][lam] = aa * ab * (12.566370614359172954 / (2 * lam + 1)) * 0.5 * gam;
    }
  double sm[LB + 1];
#pragma unroll
  for (int m = 0; m <= LB; ++m) sm[m] = 0.0;
  const int64_t o1 = active ? bs.prim_off[s1] : 0, o2 = active ? bs.prim_off[s2] : 0;
  const int K1 = active ? bs.nprim[s1] : 0, K2 = active ? bs.nprim[s2] : 0;
  for (int i = 0; i < K1; ++i)
    for (int j = 0; j < K2; ++j) {
      const double a = bs.expo[o1 + i], b = bs.expo[o2 + j];
      const double p = a + b, ip = 1.0 / p, mu = a * b * ip;
      const double pre = bs.w[o1 + i] * bs.w[o2 + j] * exp_neg(mu * R * R) * ip * sqrt(ip);
      const double ta = b * R * ip, tb = -a * R * ip;
      double pa[LA + 1], pb[LB + 1], pl[LB + 1];
      pa[0] = 1.0;
      pb[0] = 1.0;
      pl[0] = 1.0;
#pragma unroll
      for (int k = 1; k <= LA; ++k) pa[k] = pa[k - 1] * ta;
#pragma unroll
      for (int k = 1; k <= LB; ++k) {
        pb[k] = pb[k - 1] * tb;
        pl[k] = pl[k - 1] * ip;
      }
#pragma unroll
      for (int m = 0; m <= LB; ++m) {
        double t = 0.0;
#pragma unroll
        for (int lam = m; lam <= LB; ++lam) t = fma(cf[m][lam] * pa[LA - lam], pb[LB - lam] * pl[lam], t);
        sm[m] = fma(pre, t, sm[m]);
      }
    }
  // the frame block (entry (ma + la, mb + lb)), then back to the laboratory frame as for V
  double V[NA * NB];
#pragma unroll
  for (int e = 0; e < NA * NB; ++e) V[e] = 0.0;
#pragma unroll
  for (int m = -LB; m <= LB; ++m) V[(m + LA) * NB + (m + LB)] = sm[m < 0 ? -m : m];
  double cth[LA + 1], sth[LA + 1], cph[LA + 1], sph[LA + 1];
  angles<LA>(ps.ct, ps.st, cth, sth);
  angles<LA>(ps.cp, ps.sp, cph, sph);
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    double v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) v[j] = V[r * NB + j];
    Rot<LB>::apply(v, cth, sth, cph, sph);
#pragma unroll
    for (int j = 0; j < NB; ++j) V[r * NB + j] = v[j];
  }
#pragma unroll
  for (int col = 0; col < NB; ++col) {
    double v[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) v[i] = V[i * NB + col];
    Rot<LA>::apply(v, cth, sth, cph, sph);
#pragma unroll
    for (int i = 0; i < NA; ++i) V[i * NB + col] = v[i];
  }
  const int64_t d0 = active ? pr.dst0[slot] : -1, d1 = active ? pr.dst1[slot] : 0;
  if constexpr (kStaged) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* const stg = s_ovl_stage[w];
    s_ovl_d0[w][lane] = d0;
    s_ovl_d1[w][lane] = d1;
    const int64_t n = bs.nbf;
    // rows i of every block: entry k = p NB + j is block p's (i, j)
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
      for (int j = 0; j < NB; ++j) stg[lane * NB + j] = V[i * NB + j];
      ovl_wave_sync();
      for (int k = lane; k < 64 * NB; k += 64) {
        const int q = k / NB, j = k - q * NB;
        const int64_t e0 = s_ovl_d0[w][q], e1 = s_ovl_d1[w][q];
        if (e0 < 0) continue;
        if (pr.full) {
          if (e0 != e1 || i <= j) out[(e0 + i) * n + e1 + j] = stg[k];
        } else if (e1 == 0) {
          out[e0 + i * NB + j] = stg[k];
        } else {
          out[e0 + j * NA + i] = stg[k];
        }
      }
      ovl_wave_sync();
    }
    if (pr.full) {
      // the mirror, column col of every block: entry k = p NA + i is block p's (i, col)
#pragma unroll
      for (int col = 0; col < NB; ++col) {
#pragma unroll
        for (int i = 0; i < NA; ++i) stg[lane * NA + i] = V[i * NB + col];
        ovl_wave_sync();
        for (int k = lane; k < 64 * NA; k += 64) {
          const int q = k / NA, i = k - q * NA;
          const int64_t e0 = s_ovl_d0[w][q], e1 = s_ovl_d1[w][q];
          if (e0 < 0) continue;
          if (e0 != e1 || i <= col) out[(e1 + col) * n + e0 + i] = stg[k];
        }
        ovl_wave_sync();
      }
    }
    return;
  }
  if (pr.full) {
    // the (s1, s2) block and its mirror; a shell with itself writes each entry once per orientation
    const int64_t n = bs.nbf;
    for (int i = 0; i < NA; ++i)
      for (int col = 0; col < NB; ++col)
        if (d0 != d1 || i <= col) {
          out[(d0 + i) * n + d1 + col] = V[i * NB + col];
          out[(d1 + col) * n + d0 + i] = V[i * NB + col];
        }
  } else {
    // the listed orientation: (s1, s2) row-major, or transposed where the listed pair is (s2, s1)
    for (int i = 0; i < NA; ++i)
      for (int col = 0; col < NB; ++col) {
        if (d1 == 0)
          out[d0 + i * NB + col] = V[i * NB + col];
        else
          out[d0 + col * NA + i] = V[i * NB + col];
      }
  }
}

template <int LA, int LB, bool kStaged>
__device__ __forceinline__ void overlap_dispatch(int c, const DevBasis& bs, const DevPairs& pr, int slot, bool active,
                                                 double* __restrict__ out) {
  if constexpr (LA <= SHGO_LMAX) {
    if (c == class_id(LA, LB)) {
      overlap_pair<LA, LB, kStaged>(bs, pr, slot, active, out);
      return;
    }
    if constexpr (LB < LA)
      overlap_dispatch<LA, LB + 1, kStaged>(c, bs, pr, slot, active, out);
    else
      overlap_dispatch<LA + 1, 0, kStaged>(c, bs, pr, slot, active, out);
  }
}

// One thread per class-sorted shell pair of the plan (slots from k_scatter; s1 has the higher l).
// A wavefront whose active lanes all hold one class (all but those at class boundaries) stores
// through LDS; the others store lane by lane.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_overlap(DevBasis bs, DevPairs pr, double* __restrict__ out) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = slot < pr.n_cand;
  const int c = active ? class_id(bs.l[pr.s1[slot]], bs.l[pr.s2[slot]]) : -1;
  const int c0 = __shfl(c, 0);  // lanes past the last pair come after the active ones
  if (c0 < 0) return;           // no active lane in this wavefront
  if (__all(!active || c == c0)) {
    overlap_dispatch<0, 0, true>(c0, bs, pr, (int)(active ? slot : 0), active, out);
  } else if (active) {
    overlap_dispatch<0, 0, false>(c, bs, pr, (int)slot, true, out);
  }
}

__global__ void k_fill_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------------------------
// P3: adjoint kernel for the gradient of E = sum_ij D_ij V_ij
// ---------------------------------------------------------------------------------------------
// One wavefront per shell pair of a class, its 64 lanes over the nuclei. In the pair frame (fixed
// at the current geometry) E = sum over primitive pairs and entries of Wbar(L,M,k) W(L,M,k), where
// W is the nucleus sum of the forward kernel and Wbar its adjoint: the coupling applied in
// reverse to the density block rotated into the frame, D' = D_a D~ D_b^T. Then
//   dE/dc     = Q^T grad_C f_c,  f_c = Z_c sum Wbar G_{L,k}(p|C|^2) Q_{L,M}(C)   (dG/dT = -T^k/k! F_{L+k+1})
//   dE/dP     = -sum_c grad_C f_c
//   dE/dR'    = sum W(L,M,k) WR(L,M,k): the shift (Eq. 7) differentiated off the z axis, i.e. the
//               coupling of classes (LA-1, LB) and (LA, LB-1) on the density block contracted with
//               the gradient matrices of the solid harmonics, plus -2 mu R Wbar along z from
//               exp(-mu R^2)
//   dE/dA     = (alpha/p) dE/dP - dE/dR',  dE/dB = (beta/p) dE/dP + dE/dR'
// Boys values are recomputed per nucleus (orders up to LA+LB+1), never stored.
struct GradArgs {
  DevBasis bs;
  DevPairs pr;
  const Nuc* __restrict__ nuc;
  int32_t n_nuc;
  const double* __restrict__ boys_tab;
  const double* __restrict__ D;  // nbf x nbf
  double* __restrict__ dnuc;     // [n_nuc][3]
  double* __restrict__ dcen;     // [n_shells][3]
  double* __restrict__ energy;   // [1]
};

constexpr int kGradThreads = 256;

template <int LA, int LB>
struct GradLds {  // per-wavefront LDS layout, in doubles
  static constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1;
  static constexpr int D0 = 0;
  static constexpr int DA = D0 + NA * NB;
  static constexpr int DB = DA + (LA >= 1 ? 3 * (NA - 2) * NB : 0);
  static constexpr int PW = DB + (LB >= 1 ? 3 * NA * (NB - 2) : 0);
  static constexpr int ADJ = (PW + LA + LB + 2 + 1) / 2 * 2;
  static constexpr int SIZE = (ADJ + 4 * GradClass<LA, LB>::NW + 1) / 2 * 2;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Waves per SIMD the gradient kernel of a class is register-allocated for: two up to l_a = 3
// (measured 30-40% faster there than one wave with 266-344 registers, despite a few spills),
// the compiler's own choice above.
template <int LA>
struct GradWaves {
  static constexpr int value = LA <= 3 ? 2 : 1;
};

template <int LA, int LB>
__global__ void __launch_bounds__(kGradThreads) __attribute__((amdgpu_waves_per_eu(GradWaves<LA>::value)))
k_grad(GradArgs ga) {
  extern __shared__ double sm[];
  using GC = GradClass<LA, LB>;
  using LY = GradLds<LA, LB>;
  constexpr int NA = LY::NA, NB = LY::NB, LM = LA + LB, NW = GC::NW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n_nuc = ga.n_nuc;
  double* ngrad = sm;
  double* wl = sm + (3 * n_nuc + 1) / 2 * 2 + wave * LY::SIZE;
  for (int i = threadIdx.x; i < 3 * n_nuc; i += blockDim.x) ngrad[i] = 0.0;
  __syncthreads();
  constexpr int cls = class_id(LA, LB);
  // pairs whose primitive pairs are all screened out (key 0 of the class, sorted first) add
  // nothing to E or its gradient: the loop starts after them
  const int start = ga.pr.key_off[cls * kKeysPerClass + 1];
  const int count = ga.pr.key_off[(cls + 1) * kKeysPerClass] - start;
  const int nwaves = gridDim.x * (kGradThreads / 64);
  const int64_t nbf = ga.bs.nbf;
  double e_lane = 0.0;
  for (int j = blockIdx.x * (kGradThreads / 64) + wave; j < count; j += nwaves) {
    // the class's pairs are sorted by surviving primitive pairs, ascending: take them from the
    // long end so that the last round of the grid-stride loop holds the shortest pairs
    const int slot = start + (count - 1 - j);
    const int s1 = ga.pr.s1[slot], s2 = ga.pr.s2[slot];
    PairState ps;
    ps.active = true;
    ps.s1 = s1;
    ps.s2 = s2;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      ps.A[x] = ga.bs.center[3 * s1 + x];
      ps.B[x] = ga.bs.center[3 * s2 + x];
    }
    frame_of(ps);
    const double R = ps.R;
    double cth[LA + 1], sth[LA + 1], cph[LA + 1], sph[LA + 1];
    angles<LA>(ps.ct, ps.st, cth, sth);
    angles<LA>(ps.cp, ps.sp, cph, sph);
    // density block D~ = D_ab + D_ba^T (a != b) and its rotation into the frame
    const int64_t r0 = ga.bs.bf_off[s1], c0 = ga.bs.bf_off[s2];
    for (int i = lane; i < NA * NB; i += 64) {
      const int r = i / NB, c = i - r * NB;
      double v = ga.D[(r0 + r) * nbf + c0 + c];
      if (s1 != s2) v += ga.D[(c0 + c) * nbf + r0 + r];
      wl[LY::D0 + i] = v;
    }
    wave_sync();
    if (lane < NA) {
      double v[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = wl[LY::D0 + lane * NB + c];
      RotInv<LB>::apply(v, cth, sth, cph, sph);
#pragma unroll
      for (int c = 0; c < NB; ++c) wl[LY::D0 + lane * NB + c] = v[c];
    }
    wave_sync();
    if (lane < NB) {
      double v[NA];
#pragma unroll
      for (int r = 0; r < NA; ++r) v[r] = wl[LY::D0 + r * NB + lane];
      RotInv<LA>::apply(v, cth, sth, cph, sph);
#pragma unroll
      for (int r = 0; r < NA; ++r) wl[LY::D0 + r * NB + lane] = v[r];
    }
    wave_sync();
    // gradient blocks: D'^{a,xi}(m', mb) = sum_ma g_xi(LA; ma, m') D'(ma, mb), and the b side
    if constexpr (LA >= 1) {
      const double* __restrict__ g = grad_matrix(LA);
      constexpr int n1 = (NA - 2) * NB;
      for (int i = lane; i < 3 * n1; i += 64) {
        const int xi = i / n1, rem = i - xi * n1, mp = rem / NB, mb = rem - mp * NB;
        double v = 0.0;
        for (int ma = 0; ma < NA; ++ma) v = fma(g[(xi * NA + ma) * (NA - 2) + mp], wl[LY::D0 + ma * NB + mb], v);
        wl[LY::DA + i] = v;
      }
    }
    if constexpr (LB >= 1) {
      const double* __restrict__ g = grad_matrix(LB);
      constexpr int n2 = NA * (NB - 2);
      for (int i = lane; i < 3 * n2; i += 64) {
        const int xi = i / n2, rem = i - xi * n2, ma = rem / (NB - 2), mp = rem - ma * (NB - 2);
        double v = 0.0;
        for (int mb = 0; mb < NB; ++mb) v = fma(g[(xi * NB + mb) * (NB - 2) + mp], wl[LY::D0 + ma * NB + mb], v);
        wl[LY::DB + i] = v;
      }
    }
    wave_sync();
    // frame rows in laboratory coordinates (lab -> frame: v' = Q v)
    const double qx[3] = {ps.ct * ps.cp, ps.ct * ps.sp, -ps.st};
    const double qy[3] = {-ps.sp, ps.cp, 0.0};
    const double qz[3] = {ps.st * ps.cp, ps.st * ps.sp, ps.ct};
    double accA[3] = {0.0, 0.0, 0.0}, accB[3] = {0.0, 0.0, 0.0};
    const int64_t o1 = ga.bs.prim_off[s1], o2 = ga.bs.prim_off[s2];
    const int K1 = ga.bs.nprim[s1], K2 = ga.bs.nprim[s2];
    for (int pi = 0; pi < K1; ++pi)
      for (int pj = 0; pj < K2; ++pj) {
        const double a = ga.bs.expo[o1 + pi], b = ga.bs.expo[o2 + pj];
        if (!keep_prim(a, b, R * R, ga.pr.screen)) continue;
        const double p = a + b, ip = 1.0 / p, mu = a * b * ip;
        const double P[3] = {(a * ps.A[0] + b * ps.B[0]) * ip, (a * ps.A[1] + b * ps.B[1]) * ip,
                             (a * ps.A[2] + b * ps.B[2]) * ip};
        const double K = exp_neg(mu * R * R);
        const double pre = -ga.bs.w[o1 + pi] * ga.bs.w[o2 + pj] * K;
        const double ta = b * R * ip, tb = -a * R * ip;
        if (lane <= LA) {
          double v = 1.0;
          for (int q = 0; q < lane; ++q) v *= ta;
          wl[LY::PW + lane] = v;
        } else if (lane <= LA + LB + 1) {
          double v = 1.0;
          for (int q = 0; q < lane - LA - 1; ++q) v *= tb;
          wl[LY::PW + lane] = v;
        }
        wave_sync();
        // adjoint quadruples (Wbar, WRx, WRy, WRz), lanes over the entries
        const int* __restrict__ off = GC::off();
        const GradTerm* __restrict__ terms = GC::terms();
        for (int e = lane; e < NW; e += 64) {
          double s0 = 0.0, sa[3] = {0.0, 0.0, 0.0}, sb[3] = {0.0, 0.0, 0.0};
          for (int t = off[e]; t < off[e + 1]; ++t) {
            const GradTerm T = terms[t];
            const double f = T.coef * wl[LY::PW + T.pa] * wl[LY::PW + LA + 1 + T.pb];
            if (T.kind == 0) {
              s0 = fma(f, wl[LY::D0 + T.src], s0);
            } else if (T.kind == 1) {
#pragma unroll
              for (int x = 0; x < 3; ++x) sa[x] = fma(f, wl[LY::DA + x * (NA - 2) * NB + T.src], sa[x]);
            } else {
#pragma unroll
              for (int x = 0; x < 3; ++x) sb[x] = fma(f, wl[LY::DB + x * NA * (NB - 2) + T.src], sb[x]);
            }
          }
          double sc = pre * 6.283185307179586477 * ip * GC::cl()[e];
          const int k = GC::kk()[e];
          for (int q = 1; q <= k; ++q) sc *= (double)q * ip;
          const double wb = sc * s0;
          double* w = wl + LY::ADJ + 4 * e;
          w[0] = wb;
          w[1] = sc * (b * ip * sa[0] - a * ip * sb[0]);
          w[2] = sc * (b * ip * sa[1] - a * ip * sb[1]);
          w[3] = sc * (b * ip * sa[2] - a * ip * sb[2]) - 2.0 * mu * R * wb;
        }
        wave_sync();
        // nucleus loop, lanes over the nuclei
        double gP[3] = {0.0, 0.0, 0.0}, eR[3] = {0.0, 0.0, 0.0};
        for (int c = lane; c < n_nuc; c += 64) {
          const Nuc n = ga.nuc[c];
          const double cx = n.x - P[0], cy = n.y - P[1], cz = n.z - P[2];
          const double x = qx[0] * cx + qx[1] * cy + qx[2] * cz;
          const double y = qy[0] * cx + qy[1] * cy;
          const double z = qz[0] * cx + qz[1] * cy + qz[2] * cz;
          const double r2 = fma(cx, cx, fma(cy, cy, cz * cz));
          const double T = p * r2;
          static_assert(LM + 1 + 7 < kBoysOrders, "the Taylor row must lie inside the table");
          // Boys F_0..F_{LM+1} without a divergent branch, as in the integral kernel: the Taylor
          // row of the nearest grid point (index clamped to the table), or the asymptote above
          // kBoysTcut, selected per lane
          double row[8];
          {
            const int i = (int)(fmin(T, kBoysTcut) * 16.0 + 0.5);  // 0 .. kBoysPoints - 1
            const double* __restrict__ r = ga.boys_tab + i * kBoysOrders + LM + 1;
#pragma unroll
            for (int k = 0; k < 8; ++k) row[k] = r[k];
          }
          double F[LM + 2];
          boys_row<LM + 1>(T, exp_neg(T), row, F);
          double tj[LB + 1];
          tj[0] = 1.0;
#pragma unroll
          for (int k = 1; k <= LB; ++k) tj[k] = tj[k - 1] * T * (1.0 / k);
          double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          GC::step(wl + LY::ADJ, x, y, z, r2, F, tj, acc);
          const double gx = n.Z * fma(2.0 * p * acc[3], x, acc[0]);
          const double gy = n.Z * fma(2.0 * p * acc[3], y, acc[1]);
          const double gz = n.Z * fma(2.0 * p * acc[3], z, acc[2]);
          gP[0] -= gx;
          gP[1] -= gy;
          gP[2] -= gz;
          eR[0] = fma(n.Z, acc[4], eR[0]);
          eR[1] = fma(n.Z, acc[5], eR[1]);
          eR[2] = fma(n.Z, acc[6], eR[2]);
          e_lane = fma(n.Z, acc[7], e_lane);
#pragma unroll
          for (int X = 0; X < 3; ++X) atomicAdd(&ngrad[3 * c + X], qx[X] * gx + qy[X] * gy + qz[X] * gz);
        }
#pragma unroll
        for (int X = 0; X < 3; ++X) {
          accA[X] += a * ip * gP[X] - eR[X];
          accB[X] += b * ip * gP[X] + eR[X];
        }
        wave_sync();
      }
    // pair totals, back to laboratory axes
    double fa[3], fb[3];
#pragma unroll
    for (int X = 0; X < 3; ++X) {
      fa[X] = wave_sum(accA[X]);
      fb[X] = wave_sum(accB[X]);
    }
    if (lane < 3) {
      const int X = lane;
      atomicAdd(&ga.dcen[3 * s1 + X], qx[X] * fa[0] + qy[X] * fa[1] + qz[X] * fa[2]);
      atomicAdd(&ga.dcen[3 * s2 + X], qx[X] * fb[0] + qy[X] * fb[1] + qz[X] * fb[2]);
    }
  }
  const double e_wave = wave_sum(e_lane);
  if (lane == 0 && e_wave != 0.0) atomicAdd(ga.energy, e_wave);
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * n_nuc; i += blockDim.x)
    if (ngrad[i] != 0.0) atomicAdd(&ga.dnuc[i], ngrad[i]);
}

template <int LA, int LB>
size_t grad_lds_bytes(int n_nuc) {
  return sizeof(double) * ((size_t)(3 * n_nuc + 1) / 2 * 2 + (size_t)(kGradThreads / 64) * GradLds<LA, LB>::SIZE);
}

// ---------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------
// Boys table F_m(i/16), m < kBoysOrders, by the convergent series in long double (positive terms).
std::vector<double> boys_table() {
  std::vector<double> tab((size_t)kBoysPoints * kBoysOrders);
  for (int i = 0; i < kBoysPoints; ++i) {
    const long double t = (long double)i / 16.0L;
    const long double et = expl(-t);
    for (int m = 0; m < kBoysOrders; ++m) {
      long double term = 1.0L / (2 * m + 1), sum = term;
      for (int k = 1; k < 4000; ++k) {
        term *= 2.0L * t / (2 * m + 2 * k + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
      }
      tab[(size_t)i * kBoysOrders + m] = (double)(et * sum);
    }
  }
  return tab;
}

// Relative cost of one tile of a class (orders the queue only): nucleus-step and coupling
// operation counts.
double class_cost(int la, int lb, int n_nuc) {
  const int lm = la + lb;
  double nw = 0.0;
  for (int k = 0; k <= lb; ++k) nw += (double)(lm - 2 * k + 1) * (lm - 2 * k + 1);
  return (double)n_nuc * (60.0 + 4.0 * (lm + 1) * (lm + 1) + 2.0 * nw) + 40.0 + 30.0 * nw;
}

// Class weights of the work-item order from the cost model, scaled so that the largest is 1024.
void model_weights(int n_nuc, float* w) {
  double mx = 0.0;
  for (int la = 0; la <= SHGO_LMAX; ++la)
    for (int lb = 0; lb <= la; ++lb) mx = std::max(mx, class_cost(la, lb, n_nuc));
  for (int la = 0; la <= SHGO_LMAX; ++la)
    for (int lb = 0; lb <= la; ++lb) w[class_id(la, lb)] = (float)(1024.0 * class_cost(la, lb, n_nuc) / mx);
}

}  // namespace

struct shgo_context {
  int device = 0;
  int n_cu = 0;
  int grid = 0;  // workgroups of the persistent kernel resident on the device at once
  double* boys_tab = nullptr;
  std::string err;
};

struct shgo_plan {
  shgo_context* ctx = nullptr;
  int full = 0;
  int32_t n_shells = 0, n_nuc = 0;
  int64_t nbf = 0, n_cand = 0, out_size = 0, integrals = 0;
  double screen = 0.0;
  int class_cand[kNumClasses] = {0};  // candidate pairs per class (bounds the sorted counts)
  int32_t def_tiles[kNumClasses] = {0};  // default tiles per work item of each class
  int32_t grad_occ[kNumClasses] = {0};    // resident workgroups per CU of each class's gradient kernel
  std::vector<void*> allocs;
  DevBasis bs{};
  DevPairs pr{};
  Nuc* nuc = nullptr;
  // persistent-kernel workspace
  ClassMeta meta{};
  int32_t* queue = nullptr;  // head of the persistent kernel's work queue
  int32_t* item_off = nullptr;  // [0]: number of work items
  int32_t* items = nullptr;     // work items, longest first (capacity: one tile per item)
  WorkArgs* d_wa = nullptr;  // the integral kernel's arguments, in device memory
  double* d_energy = nullptr;  // gradient: E when the caller does not ask for it
  // captured graph of one evaluation (shgo_execute_graph) and its output buffer
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* graph_out = nullptr;
  hipStream_t cap_stream = nullptr;
  // phase timing (off when slots == 0): events [slot][phase][start, end]
  int32_t slots = 0;
  int64_t exec_count = 0;
  std::vector<hipEvent_t> events;
};

namespace {

constexpr int kTuneCandidates = 5;

void drop_graph(shgo_plan* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->graph_out = nullptr;
}

shgo_status fail(shgo_context* ctx, shgo_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

template <class T>
hipError_t dalloc(shgo_plan* p, T** ptr, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count == 0 ? 8 : count * sizeof(T));
  if (e == hipSuccess) p->allocs.push_back(q);
  *ptr = (T*)q;
  return e;
}

shgo_status validate(shgo_context* ctx, const shgo_basis* b, const shgo_nuclei* n, double screen) {
  if (!b || !n) return fail(ctx, SHGO_ERR_INVALID_ARG, "null basis or nuclei");
  if (b->n_shells < 0 || n->n_nuclei < 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "negative count");
  if (b->n_shells > 0 && (!b->center || !b->l || !b->n_prim || !b->prim_offset || !b->exponent || !b->coef))
    return fail(ctx, SHGO_ERR_INVALID_ARG, "null basis array");
  if (n->n_nuclei > 0 && (!n->position || !n->charge)) return fail(ctx, SHGO_ERR_INVALID_ARG, "null nuclei array");
  if (!std::isfinite(screen) || screen < 0.0) return fail(ctx, SHGO_ERR_INVALID_ARG, "screen must be finite and >= 0");
  for (int s = 0; s < b->n_shells; ++s) {
    if (b->l[s] < 0 || b->l[s] > SHGO_LMAX) return fail(ctx, SHGO_ERR_UNSUPPORTED_L, "shell l out of range 0..6");
    if (b->n_prim[s] < 1 || b->prim_offset[s] < 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "shell with no primitives");
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(b->center[3 * s + x])) return fail(ctx, SHGO_ERR_NOT_FINITE, "non-finite shell center");
    for (int k = 0; k < b->n_prim[s]; ++k) {
      const double a = b->exponent[b->prim_offset[s] + k], d = b->coef[b->prim_offset[s] + k];
      if (!std::isfinite(a) || !std::isfinite(d)) return fail(ctx, SHGO_ERR_NOT_FINITE, "non-finite exponent or coefficient");
      if (!(a > 0.0)) return fail(ctx, SHGO_ERR_INVALID_ARG, "exponent must be > 0");
    }
  }
  for (int c = 0; c < n->n_nuclei; ++c) {
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(n->position[3 * c + x])) return fail(ctx, SHGO_ERR_NOT_FINITE, "non-finite nucleus position");
    if (!std::isfinite(n->charge[c])) return fail(ctx, SHGO_ERR_NOT_FINITE, "non-finite nuclear charge");
  }
  return SHGO_OK;
}

int64_t total_prims(const shgo_basis* b) {
  int64_t t = 0;
  for (int s = 0; s < b->n_shells; ++s) t = std::max<int64_t>(t, b->prim_offset[s] + b->n_prim[s]);
  return t;
}

// The integral kernel's arguments (device copy, read through the scalar cache). item_ns turns the
// per-item timing of the kernel on (tuning runs) or off (null).
hipError_t upload_args(shgo_plan* p, unsigned long long* item_ns) {
  const WorkArgs wa{p->bs, p->pr, p->nuc, p->n_nuc, p->ctx->boys_tab, p->queue, p->item_off, p->items, item_ns, p->meta};
  return hipMemcpy(p->d_wa, &wa, sizeof(WorkArgs), hipMemcpyHostToDevice);
}

// Work items of the queue for the plan's candidate counts (an upper bound of the device count).
int64_t max_items(const shgo_plan* p) {
  int64_t n = 0;
  for (int c = 0; c < kNumClasses; ++c)
    n += (((int64_t)p->class_cand[c] + kTile - 1) / kTile + p->meta.tiles[c] - 1) / p->meta.tiles[c];
  return n;
}

// Dynamic LDS the plan's schedule needs: the largest tiles x (accumulator + frames) over its
// classes.
size_t acc_bytes(const shgo_plan* p) {
  size_t m = sizeof(double);
  for (int c = 0; c < kNumClasses; ++c)
    if (p->class_cand[c] > 0) m = std::max(m, sizeof(double) * (size_t)p->meta.tiles[c] * class_tile_doubles(c));
  return m;
}

// Default tiles per work item of class c: enough (tile, slice, group) tasks for the eight
// wavefronts, within LDS. `slices` is the class's mean over its candidate pairs of
// ceil(K_a K_b / kSliceIters), capped at 8 (screening only lowers it).
int default_tiles(int c, double slices) {
  const double tasks_per_tile = kClassGroups[c] * std::max(1.0, slices);
  const int t = (int)std::ceil(8.0 / tasks_per_tile - 1e-9);
  return std::max(1, std::min(class_max_tiles(c), t));
}

// Mean primitive-pair slices per candidate pair of each class, before screening (the matrix
// plan's pairs a <= b counted from a histogram of shells by l and primitive count).
void mean_slices(const shgo_basis* b, int full, int64_t n_pairs, const int32_t* pa, const int32_t* pb,
                 double* mean) {
  double sum[kNumClasses] = {0}, cnt[kNumClasses] = {0};
  auto sl = [](int64_t ka, int64_t kb) { return (double)std::min<int64_t>(8, (ka * kb + kSliceIters - 1) / kSliceIters); };
  auto cls = [](int la, int lb) { return class_id(std::max(la, lb), std::min(la, lb)); };
  if (full) {
    constexpr int kK = 64;  // primitive counts above this have the capped slice count too
    std::vector<double> h((size_t)(SHGO_LMAX + 1) * (kK + 1), 0.0);
    for (int s = 0; s < b->n_shells; ++s) h[(size_t)b->l[s] * (kK + 1) + std::min(b->n_prim[s], kK)] += 1.0;
    for (int la = 0; la <= SHGO_LMAX; ++la)
      for (int lb = 0; lb <= la; ++lb)
        for (int ka = 1; ka <= kK; ++ka)
          for (int kb = 1; kb <= kK; ++kb) {
            const double na = h[(size_t)la * (kK + 1) + ka], nb = h[(size_t)lb * (kK + 1) + kb];
            if (na == 0.0 || nb == 0.0) continue;
            double n;
            if (la != lb)
              n = na * nb;
            else if (ka < kb)
              n = na * nb;
            else if (ka == kb)
              n = na * (na + 1.0) / 2.0;
            else
              continue;
            sum[cls(la, lb)] += n * sl(ka, kb);
            cnt[cls(la, lb)] += n;
          }
  } else {
    for (int64_t i = 0; i < n_pairs; ++i) {
      const int c = cls(b->l[pa[i]], b->l[pb[i]]);
      sum[c] += sl(b->n_prim[pa[i]], b->n_prim[pb[i]]);
      cnt[c] += 1.0;
    }
  }
  for (int c = 0; c < kNumClasses; ++c) mean[c] = cnt[c] > 0.0 ? sum[c] / cnt[c] : 1.0;
}

// The launches of one evaluation on `st`: pair build (a1), then the persistent integral kernel.
// With `timed`, HIP events bracket the two phases (never inside a graph capture).
void enqueue(shgo_plan* p, double* out, hipStream_t st, bool timed) {
  const int tb = 256;
  auto blocks = [&](int64_t n) { return (int)((n + tb - 1) / tb); };
  const int slot = timed && p->slots > 0 ? (int)(p->exec_count % p->slots) : -1;
  auto mark = [&](int phase, int edge) {
    if (slot >= 0) (void)hipEventRecord(p->events[((size_t)slot * SHGO_NUM_PHASES + phase) * 2 + edge], st);
  };
  mark(0, 0);
  // key_count is zero here: cleared at plan creation and by every k_scan_keys after reading it
  const int cb = (int)((p->n_cand + kClassifyThreads - 1) / kClassifyThreads);
  const int wb = (int)((p->n_shells + kClassifyThreads - 1) / kClassifyThreads);
  hipLaunchKernelGGL(k_classify, dim3(cb + wb), dim3(kClassifyThreads), 0, st, p->bs, p->pr, cb);
  hipLaunchKernelGGL(k_scan_keys, dim3(1), dim3(1024), 0, st, p->pr, p->meta, p->item_off, p->items, p->queue);
  hipLaunchKernelGGL(k_scatter, dim3(blocks(p->n_cand)), dim3(tb), 0, st, p->bs, p->pr);
  mark(0, 1);  // also the start of phase 1: three event records per timed execution
  hipLaunchKernelGGL(k_integrals, dim3(p->ctx->grid), dim3(kIntegralThreads), acc_bytes(p), st,
                     (const WorkArgs*)p->d_wa, out);
  mark(1, 1);
  if (slot >= 0) p->exec_count++;
}

shgo_status make_plan(shgo_context* ctx, const shgo_basis* b, const shgo_nuclei* n, int full, int64_t n_pairs,
                      const int32_t* pa, const int32_t* pb, double screen, shgo_plan** out) {
  if (!ctx || !out) return fail(ctx, SHGO_ERR_INVALID_ARG, "null context or output pointer");
  *out = nullptr;
  shgo_status st = validate(ctx, b, n, screen);
  if (st != SHGO_OK) return st;
  if (!full) {
    if (n_pairs < 0 || (n_pairs > 0 && (!pa || !pb))) return fail(ctx, SHGO_ERR_INVALID_ARG, "bad pair list");
    for (int64_t i = 0; i < n_pairs; ++i)
      if (pa[i] < 0 || pa[i] >= b->n_shells || pb[i] < 0 || pb[i] >= b->n_shells)
        return fail(ctx, SHGO_ERR_INVALID_ARG, "pair index out of range");
    if (n_pairs > (int64_t)INT32_MAX) return fail(ctx, SHGO_ERR_INVALID_ARG, "too many pairs");
  } else if ((int64_t)b->n_shells * (b->n_shells + 1) / 2 > (int64_t)INT32_MAX) {
    return fail(ctx, SHGO_ERR_INVALID_ARG, "too many shells");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  shgo_plan* p = new shgo_plan();
  p->ctx = ctx;
  p->full = full;
  p->n_shells = b->n_shells;
  p->n_nuc = n->n_nuclei;
  p->screen = screen;
  std::vector<int64_t> bf(b->n_shells);
  int64_t nbf = 0;
  for (int s = 0; s < b->n_shells; ++s) {
    bf[s] = nbf;
    nbf += 2 * b->l[s] + 1;
  }
  p->nbf = nbf;
  const int64_t np = total_prims(b);
  // candidates, grid bounds and output size
  std::vector<int64_t> blk;
  if (full) {
    p->n_cand = (int64_t)b->n_shells * (b->n_shells + 1) / 2;
    int64_t cnt[SHGO_LMAX + 1] = {0};
    for (int s = 0; s < b->n_shells; ++s) cnt[b->l[s]]++;
    for (int la = 0; la <= SHGO_LMAX; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        const int64_t c = la == lb ? cnt[la] * (cnt[la] + 1) / 2 : cnt[la] * cnt[lb];
        p->class_cand[class_id(la, lb)] = (int)c;
        p->integrals += c * (2 * la + 1) * (2 * lb + 1);
      }
    p->out_size = nbf * nbf;
  } else {
    p->n_cand = n_pairs;
    blk.resize(n_pairs);
    int64_t o = 0;
    for (int64_t i = 0; i < n_pairs; ++i) {
      const int la = b->l[pa[i]], lb = b->l[pb[i]];
      blk[i] = o;
      o += (int64_t)(2 * la + 1) * (2 * lb + 1);
      p->class_cand[class_id(std::max(la, lb), std::min(la, lb))]++;
    }
    p->out_size = o;
    p->integrals = o;
  }
  // a work item holds its tile block in 24 bits (class << 24 | block)
  for (int c = 0; c < kNumClasses; ++c)
    if (((int64_t)p->class_cand[c] + kTile - 1) / kTile >= ((int64_t)1 << 24)) {
      shgo_plan_destroy(p);
      return fail(ctx, SHGO_ERR_INVALID_ARG, "more than 2^30 shell pairs in one (la, lb) class");
    }
  // device copies and workspace
  hipError_t e = hipSuccess;
  double *center, *expo, *coef, *w;
  int32_t *l, *nprim;
  int64_t *poff, *bfo;
  e = e != hipSuccess ? e : dalloc(p, &center, 3 * (size_t)b->n_shells);
  e = e != hipSuccess ? e : dalloc(p, &l, (size_t)b->n_shells);
  e = e != hipSuccess ? e : dalloc(p, &nprim, (size_t)b->n_shells);
  e = e != hipSuccess ? e : dalloc(p, &poff, (size_t)b->n_shells);
  e = e != hipSuccess ? e : dalloc(p, &bfo, (size_t)b->n_shells);
  e = e != hipSuccess ? e : dalloc(p, &expo, (size_t)np);
  e = e != hipSuccess ? e : dalloc(p, &coef, (size_t)np);
  e = e != hipSuccess ? e : dalloc(p, &w, (size_t)np);
  e = e != hipSuccess ? e : dalloc(p, &p->nuc, (size_t)n->n_nuclei);
  DevPairs& pr = p->pr;
  pr.n_cand = p->n_cand;
  pr.full = full;
  pr.screen = screen;
  int32_t *dpa = nullptr, *dpb = nullptr;
  int64_t* dblk = nullptr;
  if (!full) {
    e = e != hipSuccess ? e : dalloc(p, &dpa, (size_t)n_pairs);
    e = e != hipSuccess ? e : dalloc(p, &dpb, (size_t)n_pairs);
    e = e != hipSuccess ? e : dalloc(p, &dblk, (size_t)n_pairs);
  }
  e = e != hipSuccess ? e : dalloc(p, &pr.key, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.s1, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.s2, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.orig, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.nsurv, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.key_count, (size_t)kNumKeys);
  e = e != hipSuccess ? e : dalloc(p, &pr.rank, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.key_off, (size_t)kNumKeys + 1);
  e = e != hipSuccess ? e : dalloc(p, &pr.dst0, (size_t)p->n_cand);
  e = e != hipSuccess ? e : dalloc(p, &pr.dst1, (size_t)p->n_cand);
  // persistent-kernel schedule: tiles per work item and the model weight of each class
  model_weights(n->n_nuclei, p->meta.weight);
  {
    double slices[kNumClasses];
    mean_slices(b, full, n_pairs, pa, pb, slices);
    for (int c = 0; c < kNumClasses; ++c) {
      p->def_tiles[c] = default_tiles(c, slices[c]);
      p->meta.tiles[c] = p->def_tiles[c];
      p->meta.groups[c] = kClassGroups[c];
    }
  }
  e = e != hipSuccess ? e : dalloc(p, &p->queue, 1);
  e = e != hipSuccess ? e : dalloc(p, &p->item_off, (size_t)kNumClasses + 1);
  {
    int64_t cap = 0;
    for (int c = 0; c < kNumClasses; ++c) cap += ((int64_t)p->class_cand[c] + kTile - 1) / kTile;
    e = e != hipSuccess ? e : dalloc(p, &p->items, (size_t)std::max<int64_t>(cap, 1));
  }
  e = e != hipSuccess ? e : dalloc(p, &p->d_wa, 1);
  e = e != hipSuccess ? e : dalloc(p, &p->d_energy, 1);
  if (e != hipSuccess) {
    shgo_plan_destroy(p);
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "device allocation failed");
  }
  // the key counters start at zero; every k_scan_keys clears them again after reading
  e = hipMemset(pr.key_count, 0, sizeof(int32_t) * kNumKeys);
  std::vector<int64_t> poff_h(b->n_shells);
  for (int s = 0; s < b->n_shells; ++s) poff_h[s] = b->prim_offset[s];
  std::vector<Nuc> nh(n->n_nuclei);
  for (int c = 0; c < n->n_nuclei; ++c)
    nh[c] = Nuc{n->position[3 * c], n->position[3 * c + 1], n->position[3 * c + 2], n->charge[c]};
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpy(d, h, bytes, hipMemcpyHostToDevice);
  };
  up(center, b->center, 3 * sizeof(double) * b->n_shells);
  up(l, b->l, sizeof(int32_t) * b->n_shells);
  up(nprim, b->n_prim, sizeof(int32_t) * b->n_shells);
  up(poff, poff_h.data(), sizeof(int64_t) * b->n_shells);
  up(bfo, bf.data(), sizeof(int64_t) * b->n_shells);
  up(expo, b->exponent, sizeof(double) * np);
  up(coef, b->coef, sizeof(double) * np);
  up(p->nuc, nh.data(), sizeof(Nuc) * nh.size());
  if (!full) {
    up(dpa, pa, sizeof(int32_t) * n_pairs);
    up(dpb, pb, sizeof(int32_t) * n_pairs);
    up(dblk, blk.data(), sizeof(int64_t) * n_pairs);
  }
  if (e != hipSuccess) {
    shgo_plan_destroy(p);
    return fail(ctx, SHGO_ERR_DEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  }
  p->bs = DevBasis{center, l, nprim, poff, expo, coef, w, bfo, b->n_shells, nbf};
  pr.pa = dpa;
  pr.pb = dpb;
  pr.blk_off = dblk;
  e = upload_args(p, nullptr);
  if (e != hipSuccess) {
    shgo_plan_destroy(p);
    return fail(ctx, SHGO_ERR_DEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  }
  *out = p;
  return SHGO_OK;
}

// Gradient launches, one kernel per class present in the plan.
template <int LA, int LB>
shgo_status grad_class(shgo_plan* p, const GradArgs& ga, hipStream_t st, bool launch) {
  const int c = class_id(LA, LB);
  if (p->class_cand[c] == 0) return SHGO_OK;
  const size_t lds = grad_lds_bytes<LA, LB>(p->n_nuc);
  if (!launch) {
    if (lds > 163840) return fail(p->ctx, SHGO_ERR_INVALID_ARG, "too many nuclei for the gradient kernel's LDS");
    if (lds > 65536 && hipFuncSetAttribute((const void*)k_grad<LA, LB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds) != hipSuccess)
      return fail(p->ctx, SHGO_ERR_DEVICE, "hipFuncSetAttribute failed for the gradient kernel");
    if (p->grad_occ[c] == 0) {  // workgroups that fit on a CU at once (registers, LDS), at least 1
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_grad<LA, LB>, kGradThreads, lds) !=
          hipSuccess)
        nb = 2;
      p->grad_occ[c] = std::max(1, std::min(nb, 8));
    }
    return SHGO_OK;
  }
  const int64_t waves_needed = p->class_cand[c];
  const int per_block = kGradThreads / 64;
  // one round of resident workgroups; the kernel strides over the class's pairs
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((waves_needed + per_block - 1) / per_block,
                                                                 (int64_t)p->grad_occ[c] * p->ctx->n_cu));
  hipLaunchKernelGGL((k_grad<LA, LB>), dim3(blocks), dim3(kGradThreads), lds, st, ga);
  return SHGO_OK;
}

template <int LA, int LB>
shgo_status grad_all(shgo_plan* p, const GradArgs& ga, hipStream_t st, bool launch) {
  if constexpr (LA <= SHGO_LMAX) {
    const shgo_status s = grad_class<LA, LB>(p, ga, st, launch);
    if (s != SHGO_OK) return s;
    if constexpr (LB < LA)
      return grad_all<LA, LB + 1>(p, ga, st, launch);
    else
      return grad_all<LA + 1, 0>(p, ga, st, launch);
  }
  return SHGO_OK;
}

}  // namespace

extern "C" {

const char* shgo_status_string(shgo_status s) {
  switch (s) {
    case SHGO_OK: return "ok";
    case SHGO_ERR_INVALID_ARG: return "invalid argument";
    case SHGO_ERR_UNSUPPORTED_L: return "unsupported angular momentum";
    case SHGO_ERR_NOT_FINITE: return "non-finite input";
    case SHGO_ERR_OUT_OF_MEMORY: return "out of device memory";
    case SHGO_ERR_DEVICE: return "device error";
    case SHGO_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* shgo_last_error(const shgo_context* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

shgo_status shgo_create(int device, shgo_context** out) {
  if (!out) return SHGO_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SHGO_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SHGO_ERR_DEVICE;
  shgo_context* c = new shgo_context();
  c->device = device;
  std::vector<double> tab = boys_table();
  if (hipMalloc(&c->boys_tab, tab.size() * sizeof(double)) != hipSuccess) {
    delete c;
    return SHGO_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(c->boys_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->boys_tab);
    delete c;
    return SHGO_ERR_DEVICE;
  }
  int n_cu = 0, per_cu = 0;
  if (hipFuncSetAttribute((const void*)k_integrals, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(double) * kLdsDoubles)) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrals, kIntegralThreads,
                                                   sizeof(double) * kLdsDoubles) != hipSuccess) {
    shgo_destroy(c);
    return SHGO_ERR_DEVICE;
  }
  c->n_cu = n_cu;
  c->grid = std::max(1, n_cu * std::max(1, per_cu));
  *out = c;
  return SHGO_OK;
}

void shgo_destroy(shgo_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->boys_tab) (void)hipFree(ctx->boys_tab);
  delete ctx;
}

shgo_status shgo_validate(const shgo_basis* basis, const shgo_nuclei* nuclei, double screen, char* msg,
                          size_t msg_len) {
  shgo_context tmp;
  const shgo_status s = validate(&tmp, basis, nuclei, screen);
  if (msg && msg_len > 0) {
    const std::string& m = s == SHGO_OK ? std::string() : tmp.err;
    const size_t n = std::min(msg_len - 1, m.size());
    std::memcpy(msg, m.data(), n);
    msg[n] = 0;
  }
  return s;
}

int64_t shgo_nbf(const shgo_basis* b) {
  if (!b || b->n_shells < 0 || (b->n_shells > 0 && !b->l)) return -1;
  int64_t n = 0;
  for (int s = 0; s < b->n_shells; ++s) {
    if (b->l[s] < 0 || b->l[s] > SHGO_LMAX) return -1;
    n += 2 * b->l[s] + 1;
  }
  return n;
}

shgo_status shgo_plan_matrix(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei, double screen,
                             shgo_plan** plan) {
  return make_plan(ctx, basis, nuclei, 1, 0, nullptr, nullptr, screen, plan);
}

shgo_status shgo_plan_pairs(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei, int64_t n_pairs,
                            const int32_t* pair_a, const int32_t* pair_b, double screen, shgo_plan** plan) {
  return make_plan(ctx, basis, nuclei, 0, n_pairs, pair_a, pair_b, screen, plan);
}

void shgo_plan_destroy(shgo_plan* p) {
  if (!p) return;
  if (p->ctx) (void)hipSetDevice(p->ctx->device);
  drop_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t ev : p->events) (void)hipEventDestroy(ev);
  for (void* q : p->allocs) (void)hipFree(q);
  delete p;
}

int64_t shgo_plan_output_size(const shgo_plan* p) { return p ? p->out_size : -1; }
int64_t shgo_plan_integrals(const shgo_plan* p) { return p ? p->integrals : -1; }

shgo_status shgo_execute(shgo_plan* p, double* out, void* stream) {
  if (!p) return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!out && p->out_size > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  if (p->n_cand == 0) return SHGO_OK;
  enqueue(p, out, (hipStream_t)stream, true);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

shgo_status shgo_execute_graph(shgo_plan* p, double* out, void* stream) {
  if (!p) return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!out && p->out_size > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  if (p->n_cand == 0) return SHGO_OK;
  if (!p->gexec || p->graph_out != out) {
    drop_graph(p);
    if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(ctx, SHGO_ERR_DEVICE, "hipStreamCreate failed");
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(ctx, SHGO_ERR_DEVICE, "hipStreamBeginCapture failed");
    enqueue(p, out, p->cap_stream, false);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(p->cap_stream, &g) != hipSuccess || !g)
      return fail(ctx, SHGO_ERR_DEVICE, "hipStreamEndCapture failed");
    p->graph = g;
    if (hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      drop_graph(p);
      return fail(ctx, SHGO_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    p->graph_out = out;
  }
  if (hipGraphLaunch(p->gexec, (hipStream_t)stream) != hipSuccess)
    return fail(ctx, SHGO_ERR_DEVICE, "hipGraphLaunch failed");
  return SHGO_OK;
}

shgo_status shgo_execute_overlap(shgo_plan* p, double* out, void* stream) {
  if (!p) return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!out && p->out_size > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  if (p->n_cand == 0) return SHGO_OK;
  hipStream_t st = (hipStream_t)stream;
  // the plan's pair build (primitive weights, class-sorted pairs, output destinations), as for V
  const int tb = 256;
  const int cb = (int)((p->n_cand + kClassifyThreads - 1) / kClassifyThreads);
  const int wb = (int)((p->n_shells + kClassifyThreads - 1) / kClassifyThreads);
  hipLaunchKernelGGL(k_classify, dim3(cb + wb), dim3(kClassifyThreads), 0, st, p->bs, p->pr, cb);
  hipLaunchKernelGGL(k_scan_keys, dim3(1), dim3(1024), 0, st, p->pr, p->meta, p->item_off, p->items, p->queue);
  const int nb = (int)((p->n_cand + tb - 1) / tb);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(tb), 0, st, p->bs, p->pr);
  hipLaunchKernelGGL(k_overlap, dim3(nb), dim3(tb), 0, st, p->bs, p->pr, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

shgo_status shgo_plan_autotune(shgo_plan* p, double* out, int32_t rounds, void* stream, double* ms, int32_t* chosen) {
  if (!p || rounds < 1 || rounds > 1000) return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!out && p->out_size > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  for (int i = 0; i < kTuneCandidates; ++i)
    if (ms) ms[i] = -1.0;
  if (chosen) *chosen = 0;
  if (p->n_cand == 0) return SHGO_OK;
  hipStream_t st = (hipStream_t)stream;
  drop_graph(p);
  // 1. one timed run with the model weights and the default tiles: each class's measured time per
  //    unit of the items' estimate (iterations of the longest tile x tiles / busy wavefronts)
  ClassMeta base = p->meta;
  model_weights(p->n_nuc, p->meta.weight);
  for (int c = 0; c < kNumClasses; ++c) p->meta.tiles[c] = p->def_tiles[c];
  const ClassMeta model = p->meta;
  const int64_t nmax = max_items(p);
  unsigned long long* ticks = nullptr;
  if (hipMalloc(&ticks, sizeof(unsigned long long) * (size_t)std::max<int64_t>(nmax, 1)) != hipSuccess)
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "tuning buffer");
  std::vector<unsigned long long> th((size_t)std::max<int64_t>(nmax, 1));
  std::vector<int32_t> it((size_t)std::max<int64_t>(nmax, 1)), koff(kNumKeys + 1);
  int32_t n_items = 0;
  hipError_t e = upload_args(p, ticks);
  if (e == hipSuccess) {
    enqueue(p, out, st, false);
    e = hipStreamSynchronize(st);
  }
  if (e == hipSuccess) e = hipMemcpy(&n_items, p->item_off, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess && (n_items < 0 || n_items > nmax)) e = hipErrorUnknown;
  if (e == hipSuccess && n_items > 0) {
    e = hipMemcpy(th.data(), ticks, sizeof(unsigned long long) * (size_t)n_items, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(it.data(), p->items, sizeof(int32_t) * (size_t)n_items, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(koff.data(), p->pr.key_off, sizeof(int32_t) * koff.size(), hipMemcpyDeviceToHost);
  }
  (void)hipFree(ticks);
  if (e != hipSuccess) {
    p->meta = base;
    (void)upload_args(p, nullptr);
    return fail(ctx, SHGO_ERR_DEVICE, std::string("tuning run failed: ") + hipGetErrorString(e));
  }
  double sum_ns[kNumClasses] = {0}, units[kNumClasses] = {0};
  for (int q = 0; q < n_items; ++q) {
    const int c = it[q] >> 24, blk = it[q] & 0xffffff;
    if (c < 0 || c >= kNumClasses) continue;
    const int T = model.tiles[c];
    const int start = koff[c * kKeysPerClass], end = koff[(c + 1) * kKeysPerClass];
    const int tiles = (end - start + kTile - 1) / kTile;
    const int nt = std::min(T, tiles - blk * T);
    const int last = std::min(start + (blk * T + nt) * kTile, end) - 1;
    int m = 0;
    while (m + 1 < kKeysPerClass && koff[c * kKeysPerClass + m + 1] <= last) ++m;
    m = std::max(m, 1);
    const int tasks = nt * kClassGroups[c] * std::max(1, (m + kSliceIters - 1) / kSliceIters);
    sum_ns[c] += 10.0 * (double)th[(size_t)q];
    units[c] += (double)m * nt / std::min(8, tasks);
  }
  // measured weights, scaled like the model's (largest 1024); classes without items keep theirs
  float measured[kNumClasses];
  double mx = 0.0;
  for (int c = 0; c < kNumClasses; ++c)
    if (units[c] > 0.0) mx = std::max(mx, sum_ns[c] / units[c]);
  for (int c = 0; c < kNumClasses; ++c)
    measured[c] = units[c] > 0.0 && mx > 0.0 ? (float)std::max(1.0, 1024.0 * sum_ns[c] / units[c] / mx) : model.weight[c];
  // 2. candidates: the model weights; the measured weights; the measured weights with twice the
  //    default tiles where the LDS allows; the measured weights with one tile per item; the
  //    measured weights with half the default tiles
  ClassMeta cand[kTuneCandidates];
  for (int v = 0; v < kTuneCandidates; ++v) {
    cand[v] = model;
    if (v > 0)
      for (int c = 0; c < kNumClasses; ++c) cand[v].weight[c] = measured[c];
  }
  for (int c = 0; c < kNumClasses; ++c) {
    if (2 * model.tiles[c] <= class_max_tiles(c)) cand[2].tiles[c] = 2 * model.tiles[c];
    cand[3].tiles[c] = 1;
    cand[4].tiles[c] = std::max(1, model.tiles[c] / 2);
  }
  // 3. time each candidate and keep the fastest
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    p->meta = base;
    (void)upload_args(p, nullptr);
    return fail(ctx, SHGO_ERR_DEVICE, "hipEventCreate failed");
  }
  auto time_schedule = [&](const ClassMeta& m, double& per) {
    p->meta = m;
    hipError_t r = upload_args(p, nullptr);
    if (r != hipSuccess) return r;
    enqueue(p, out, st, false);  // warm
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < rounds; ++k) enqueue(p, out, st, false);
    (void)hipEventRecord(e1, st);
    r = hipEventSynchronize(e1);
    float t = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&t, e0, e1);
    per = (double)t / rounds;
    return r;
  };
  int best = 0;
  double best_ms = 0.0;
  for (int v = 0; v < kTuneCandidates && e == hipSuccess; ++v) {
    double per = 0.0;
    e = time_schedule(cand[v], per);
    if (e != hipSuccess) break;
    if (ms) ms[v] = per;
    if (v == 0 || per < best_ms) {
      best = v;
      best_ms = per;
    }
  }
  // 4. refine the kept candidate class by class: one tile more or less, twice or half the tiles,
  //    each change kept only if it is more than 0.5% faster in a second timing beside a fresh
  //    timing of the incumbent; at most three passes over the classes
  ClassMeta cur = cand[best];
  double cur_ms = best_ms;
  for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
    bool changed = false;
    for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
      if (p->class_cand[c] == 0) continue;
      const int T = cur.tiles[c], mx = class_max_tiles(c);
      const int opt[4] = {std::min(mx, T + 1), std::max(1, T - 1), std::min(mx, 2 * T), std::max(1, T / 2)};
      for (int o = 0; o < 4 && e == hipSuccess; ++o) {
        if (opt[o] == T || (o >= 2 && opt[o] == opt[o - 2])) continue;
        ClassMeta trial = cur;
        trial.tiles[c] = opt[o];
        double t1 = 0.0, t0 = 0.0, t2 = 0.0;
        e = time_schedule(trial, t1);
        if (e != hipSuccess || !(t1 < 0.995 * cur_ms)) continue;
        e = time_schedule(cur, t0);
        if (e == hipSuccess) e = time_schedule(trial, t2);
        if (e != hipSuccess) break;
        if (t2 < 0.995 * t0) {
          cur = trial;
          cur_ms = t2;
          changed = true;
          break;
        }
        cur_ms = t0;
      }
    }
    if (!changed) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->meta = e == hipSuccess ? cur : base;
  const hipError_t e2 = upload_args(p, nullptr);
  if (e != hipSuccess || e2 != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "tuning runs failed");
  if (chosen) *chosen = best;
  return SHGO_OK;
}

shgo_status shgo_execute_grad(shgo_plan* p, const double* D, double* dE_dnuclei, double* dE_dcenters,
                              double* energy, void* stream) {
  if (!p) return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!p->full) return fail(ctx, SHGO_ERR_INVALID_ARG, "the gradient needs a matrix plan (shgo_plan_matrix)");
  if ((p->nbf > 0 && !D) || (p->n_nuc > 0 && !dE_dnuclei) || (p->n_shells > 0 && !dE_dcenters))
    return fail(ctx, SHGO_ERR_INVALID_ARG, "null gradient argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  double* e_out = energy ? energy : p->d_energy;
  GradArgs ga{p->bs, p->pr, p->nuc, p->n_nuc, ctx->boys_tab, D, dE_dnuclei, dE_dcenters, e_out};
  shgo_status s = grad_all<0, 0>(p, ga, st, false);  // LDS limits, before any device work
  if (s != SHGO_OK) return s;
  const int tb = 256;
  auto blocks = [&](int64_t n) { return (int)std::max<int64_t>(1, (n + tb - 1) / tb); };
  if (p->n_nuc > 0) hipLaunchKernelGGL(k_fill_f64, dim3(blocks(3 * p->n_nuc)), dim3(tb), 0, st, dE_dnuclei, (int64_t)3 * p->n_nuc);
  if (p->n_shells > 0)
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks(3 * p->n_shells)), dim3(tb), 0, st, dE_dcenters, (int64_t)3 * p->n_shells);
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(tb), 0, st, e_out, (int64_t)1);
  if (p->n_cand > 0 && p->n_nuc > 0) {
    // shell-pair build (a1), as for the integrals
    const int cb = (int)((p->n_cand + kClassifyThreads - 1) / kClassifyThreads);
    const int wb = (int)((p->n_shells + kClassifyThreads - 1) / kClassifyThreads);
    hipLaunchKernelGGL(k_classify, dim3(cb + wb), dim3(kClassifyThreads), 0, st, p->bs, p->pr, cb);
    hipLaunchKernelGGL(k_scan_keys, dim3(1), dim3(1024), 0, st, p->pr, p->meta, p->item_off, p->items, p->queue);
    hipLaunchKernelGGL(k_scatter, dim3(blocks(p->n_cand)), dim3(tb), 0, st, p->bs, p->pr);
    s = grad_all<0, 0>(p, ga, st, true);
    if (s != SHGO_OK) return s;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

int32_t shgo_max_tiles(int32_t class_id) {
  return class_id >= 0 && class_id < kNumClasses ? class_max_tiles(class_id) : -1;
}

shgo_status shgo_plan_get_schedule(const shgo_plan* p, float* weight, int32_t* tiles) {
  if (!p || !weight || !tiles) return SHGO_ERR_INVALID_ARG;
  for (int c = 0; c < kNumClasses; ++c) {
    weight[c] = p->meta.weight[c];
    tiles[c] = p->meta.tiles[c];
  }
  return SHGO_OK;
}

shgo_status shgo_plan_set_schedule(shgo_plan* p, const float* weight, const int32_t* tiles) {
  if (!p || !weight || !tiles) return SHGO_ERR_INVALID_ARG;
  for (int c = 0; c < kNumClasses; ++c) {
    if (!(weight[c] >= 1.0f && weight[c] <= 1.0e6f))
      return fail(p->ctx, SHGO_ERR_INVALID_ARG, "weight[c] must be within 1..1e6");
    if (tiles[c] < 1 || tiles[c] > class_max_tiles(c))
      return fail(p->ctx, SHGO_ERR_INVALID_ARG, "tiles[c] must be within 1..shgo_max_tiles(c)");
  }
  if (hipSetDevice(p->ctx->device) != hipSuccess) return fail(p->ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  for (int c = 0; c < kNumClasses; ++c) {
    p->meta.weight[c] = weight[c];
    p->meta.tiles[c] = tiles[c];
  }
  drop_graph(p);
  const hipError_t e = upload_args(p, nullptr);
  if (e != hipSuccess) return fail(p->ctx, SHGO_ERR_DEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

shgo_status shgo_plan_set_timing(shgo_plan* p, int32_t n_slots) {
  if (!p || n_slots < 0 || n_slots > 4096) return SHGO_ERR_INVALID_ARG;
  if (hipSetDevice(p->ctx->device) != hipSuccess) return fail(p->ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  for (hipEvent_t ev : p->events) (void)hipEventDestroy(ev);
  p->events.clear();
  p->slots = 0;
  p->exec_count = 0;
  std::vector<hipEvent_t> evs((size_t)n_slots * SHGO_NUM_PHASES * 2, nullptr);
  for (auto& ev : evs) {
    if (hipEventCreate(&ev) != hipSuccess) {
      for (auto& e2 : evs)
        if (e2) (void)hipEventDestroy(e2);
      return fail(p->ctx, SHGO_ERR_DEVICE, "hipEventCreate failed");
    }
  }
  p->events = std::move(evs);
  p->slots = n_slots;
  return SHGO_OK;
}

shgo_status shgo_plan_phase_ms(shgo_plan* p, double* ms, int32_t* count) {
  if (!p || !ms || !count) return SHGO_ERR_INVALID_ARG;
  const int64_t n = std::min<int64_t>(p->exec_count, p->slots);
  *count = (int32_t)n;
  for (int ph = 0; ph < SHGO_NUM_PHASES; ++ph) {
    ms[ph] = 0.0;
    for (int64_t sl = 0; sl < n; ++sl) {
      float t = 0.f;
      // a phase starts where the previous one ended (phase 0 at its own start event)
      const size_t e1 = ((size_t)sl * SHGO_NUM_PHASES + ph) * 2 + 1;
      const size_t e0 = ph == 0 ? e1 - 1 : e1 - 2;
      if (hipEventElapsedTime(&t, p->events[e0], p->events[e1]) != hipSuccess)
        return fail(p->ctx, SHGO_ERR_DEVICE, "hipEventElapsedTime failed (stream not synchronised?)");
      ms[ph] += t;
    }
  }
  return SHGO_OK;
}

shgo_status shgo_boys(shgo_context* ctx, int64_t n, const double* T, int32_t mmax, double* F, void* stream) {
  if (!ctx) return SHGO_ERR_INVALID_ARG;
  if (n < 0 || mmax < 0 || mmax > 13 || (n > 0 && (!T || !F)))
    return fail(ctx, SHGO_ERR_INVALID_ARG, "bad Boys arguments (0 <= mmax <= 13)");
  if (n == 0) return SHGO_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  const int tb = 256;
  const int nb = (int)((n + tb - 1) / tb);
  switch (mmax) {
#define SHGO_BOYS_CASE(M) \
  case M: hipLaunchKernelGGL(k_boys<M>, dim3(nb), dim3(tb), 0, st, n, T, F, (const double*)ctx->boys_tab); break;
    SHGO_BOYS_CASE(0) SHGO_BOYS_CASE(1) SHGO_BOYS_CASE(2) SHGO_BOYS_CASE(3) SHGO_BOYS_CASE(4)
    SHGO_BOYS_CASE(5) SHGO_BOYS_CASE(6) SHGO_BOYS_CASE(7) SHGO_BOYS_CASE(8) SHGO_BOYS_CASE(9)
    SHGO_BOYS_CASE(10) SHGO_BOYS_CASE(11) SHGO_BOYS_CASE(12) SHGO_BOYS_CASE(13)
#undef SHGO_BOYS_CASE
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

}  // extern "C"
