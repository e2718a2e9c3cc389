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
//   a1  k_prim_weights, k_classify, k_scan_keys, k_scatter: per-shell normalisation, shell-pair
//       enumeration, screening, counting sort by class (LA >= LB) and surviving primitive pairs.
//   a2-a8  k_class<LA,LB>: one workgroup = 64 shell pairs x Q wavefronts; wavefront g owns the
//       |M| families of group g. Work is done in the frame whose z axis is A->B, where the shift
//       of Eq. 7 keeps m (only Y^lambda_0 of a z-directed vector survives). Per primitive pair and
//       nucleus (nuclei read through the scalar cache): C = Q(c - P), Boys F_m, real solid
//       harmonics S^L_M(C), W(L,M,k) += Z G_{L,k} S^L_M in registers; then the product-rule and
//       shift coefficients map W onto the block V' (LDS, atomic adds); finally the block is
//       rotated back with D^T = Z(phi) J^T Z(theta) J and written out.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "shgo.h"
#include "generated/shgo_classes.inc"

namespace {

// ---------------------------------------------------------------------------------------------
// Constants and small types
// ---------------------------------------------------------------------------------------------
constexpr int kBoysOrders = 22;    // F_0..F_21 stored per grid point (mmax <= 14 with 8 Taylor terms)
constexpr int kBoysPoints = 481;   // grid t_i = i/16, i = 0..480
constexpr double kBoysTcut = 30.0; // below: table + downward recursion; above: asymptote + upward
constexpr int kNumClasses = SHGO_NUM_CLASSES;
static_assert(kNumClasses == (SHGO_LMAX + 1) * (SHGO_LMAX + 2) / 2, "class count");
constexpr int kKeysPerClass = 256;
constexpr int kNumKeys = kNumClasses * kKeysPerClass;

__host__ __device__ constexpr int class_id(int la, int lb) { return la * (la + 1) / 2 + lb; }

struct alignas(32) Nuc {
  double x, y, z, Z;
};

struct DevBasis {
  const double* center;    // [n][3]
  const int32_t* l;        // [n]
  const int32_t* nprim;    // [n]
  const int64_t* prim_off; // [n]
  const double* expo;      // [nprim total]
  const double* coef;      // [nprim total]
  double* w;               // [nprim total] normalised weights (written by k_prim_weights)
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
  int32_t* key_fill;       // [kNumKeys]
  int32_t* key_off;        // [kNumKeys + 1]
  double screen;
};

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
  const double e = exp(-t);
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
    const double it = 1.0 / t;
    const double f0 = 0.88622692545275801365 * sqrt(it);  // sqrt(pi)/2 / sqrt(t)
    const double corr = 0.5 * e * it * fma(it, fma(it, 0.75, -0.5), 1.0);
    F[0] = f0 - corr;
    const double h = 0.5 * it;
#pragma unroll
    for (int m = 0; m < M; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * h;
  }
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
// <phi_k|phi_k'> = n_k n_k' / (a_k + a_k')^{l+3/2}, n_k = (2 a_k)^{(l+3/2)/2}.
__global__ void k_prim_weights(DevBasis b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.n_shells) return;
  const int l = b.l[s], K = b.nprim[s];
  const int64_t o = b.prim_off[s];
  const double q = l + 1.5;
  double dfac = 1.0;
  for (int i = 2 * l - 1; i > 1; i -= 2) dfac *= i;
  const double cn = sqrt(ldexp(1.0, l) / (dfac * 5.5683279968317078453));  // pi^{3/2}
  double ss = 0.0;
  for (int k = 0; k < K; ++k) {
    const double ak = b.expo[o + k], nk = pow(2.0 * ak, 0.5 * q), dk = b.coef[o + k];
    for (int j = 0; j < K; ++j) {
      const double aj = b.expo[o + j], nj = pow(2.0 * aj, 0.5 * q);
      ss += dk * b.coef[o + j] * nk * nj / pow(ak + aj, q);
    }
  }
  const double inv = 1.0 / sqrt(ss);
  for (int k = 0; k < K; ++k) {
    const double ak = b.expo[o + k];
    b.w[o + k] = b.coef[o + k] * cn * pow(2.0 * ak, 0.5 * q) * inv;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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
  return exp(-a * b / (a + b) * R2) > screen;
}

__global__ void k_classify(DevBasis bs, DevPairs pr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pr.n_cand) return;
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
  const int key = class_id(L1, L2) * kKeysPerClass + min(ns, kKeysPerClass - 1);
  pr.key[i] = key;
  atomicAdd(&pr.key_count[key], 1);
}

// Exclusive scan of key_count into key_off (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024) k_scan_keys(DevPairs pr) {
  __shared__ int part[1024];
  constexpr int per = (kNumKeys + 1023) / 1024;
  const int t = threadIdx.x;
  int loc[per];
  int s = 0;
  for (int j = 0; j < per; ++j) {
    const int k = t * per + j;
    loc[j] = k < kNumKeys ? pr.key_count[k] : 0;
    s += loc[j];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int j = 0; j < per; ++j) {
    const int k = t * per + j;
    if (k < kNumKeys) pr.key_off[k] = run;
    run += loc[j];
  }
  if (t == 1023) pr.key_off[kNumKeys] = part[1023];
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
  const int slot = pr.key_off[key] + atomicAdd(&pr.key_fill[key], 1);
  const bool sw = bs.l[a] < bs.l[b];
  pr.s1[slot] = sw ? b : a;
  pr.s2[slot] = sw ? a : b;
  pr.orig[slot] = (int32_t)i;
  pr.nsurv[slot] = key % kKeysPerClass;
}

// ---------------------------------------------------------------------------------------------
// a2-a8: the class kernel
// ---------------------------------------------------------------------------------------------
struct ClassArgs {
  DevBasis bs;
  DevPairs pr;
  const Nuc* __restrict__ nuc;
  int32_t n_nuc;
  const double* __restrict__ boys_tab;
  double* __restrict__ out;
};

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
__device__ __forceinline__ bool next_prim(const PairState& ps, const ClassArgs& ca, int& i, int& j) {
  const double R2 = ps.R * ps.R;
  while (true) {
    ++j;
    if (j >= ps.K2) {
      j = 0;
      ++i;
    }
    if (i >= ps.K1) return false;
    if (keep_prim(ca.bs.expo[ps.o1 + i], ca.bs.expo[ps.o2 + j], R2, ca.pr.screen)) return true;
  }
}

template <int LA, int LB, int G>
__device__ __forceinline__ void run_group(const PairState& ps, const ClassArgs& ca, int wave_iters,
                                          double* __restrict__ Vp) {
  using Grp = GroupOf<LA, LB, G>;
  constexpr int LM = LA + LB;
  int pi = 0, pj = -1;
  for (int it = 0; it < wave_iters; ++it) {
    const bool have = ps.active && next_prim(ps, ca, pi, pj);
    if (have) {
      const double a = ca.bs.expo[ps.o1 + pi], b = ca.bs.expo[ps.o2 + pj];
      const double p = a + b, ip = 1.0 / p;
      const double Px = (a * ps.A[0] + b * ps.B[0]) * ip;
      const double Py = (a * ps.A[1] + b * ps.B[1]) * ip;
      const double Pz = (a * ps.A[2] + b * ps.B[2]) * ip;
      double W[Grp::NW];
#pragma unroll
      for (int q = 0; q < Grp::NW; ++q) W[q] = 0.0;
      for (int c = 0; c < ca.n_nuc; ++c) {
        const Nuc n = ca.nuc[c];
        const double cx = n.x - Px, cy = n.y - Py, cz = n.z - Pz;
        const double u = fma(ps.cp, cx, ps.sp * cy);
        const double x = fma(ps.ct, u, -ps.st * cz);
        const double y = fma(-ps.sp, cx, ps.cp * cy);
        const double z = fma(ps.st, u, ps.ct * cz);
        const double r2 = fma(cx, cx, fma(cy, cy, cz * cz));
        const double t = p * r2;
        double F[LM + 1];
        boys<LM>(t, F, ca.boys_tab);
        double ZF[LM + 1];
#pragma unroll
        for (int m = 0; m <= LM; ++m) ZF[m] = n.Z * F[m];
        double tj[LB + 1];
        tj[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LB; ++k) tj[k] = tj[k - 1] * t * (1.0 / k);
        Grp::step(W, x, y, z, r2, ZF, tj);
      }
      // prefactor -w_a w_b exp(-mu R^2) and 2 pi k!/p^{k+1}
      const double K = exp(-a * b * ip * ps.R * ps.R);
      const double pre = -ca.bs.w[ps.o1 + pi] * ca.bs.w[ps.o2 + pj] * K;
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
__device__ __forceinline__ void dispatch_group(int g, const PairState& ps, const ClassArgs& ca, int wave_iters,
                                               double* Vp) {
  if constexpr (G < ClassInfo<LA, LB>::Q) {
    if (g == G) {
      run_group<LA, LB, G>(ps, ca, wave_iters, Vp);
      return;
    }
    dispatch_group<LA, LB, G + 1>(g, ps, ca, wave_iters, Vp);
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

template <int LA, int LB>
__global__ void __launch_bounds__((64 * ClassInfo<LA, LB>::Q)) k_class(ClassArgs ca) {
  constexpr int Q = ClassInfo<LA, LB>::Q;
  constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NAB = NA * NB;
  extern __shared__ double Vs[];  // [64][NA][NB]
  const int cls = class_id(LA, LB);
  const int start = ca.pr.key_off[cls * kKeysPerClass];
  const int end = ca.pr.key_off[(cls + 1) * kKeysPerClass];
  const int base = start + blockIdx.x * 64;
  if (base >= end) return;  // uniform over the workgroup
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  for (int i = threadIdx.x; i < 64 * NAB; i += 64 * Q) Vs[i] = 0.0;

  PairState ps;
  const int slot = base + lane;
  ps.active = slot < end;
  const int sl = ps.active ? slot : end - 1;
  ps.s1 = ca.pr.s1[sl];
  ps.s2 = ca.pr.s2[sl];
  ps.nsurv = ps.active ? ca.pr.nsurv[sl] : 0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    ps.A[x] = ca.bs.center[3 * ps.s1 + x];
    ps.B[x] = ca.bs.center[3 * ps.s2 + x];
  }
  ps.o1 = ca.bs.prim_off[ps.s1];
  ps.o2 = ca.bs.prim_off[ps.s2];
  ps.K1 = ca.bs.nprim[ps.s1];
  ps.K2 = ca.bs.nprim[ps.s2];
  frame_of(ps);
  // the number of primitive-pair iterations of this wavefront (keys cap at 255; the cap only
  // costs idle iterations, every lane still visits all of its surviving pairs)
  int iters = ps.active ? (ps.nsurv >= kKeysPerClass - 1 ? ps.K1 * ps.K2 : ps.nsurv) : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) iters = max(iters, __shfl_xor(iters, off));
  __syncthreads();

  double* Vp = Vs + lane * NAB;
  dispatch_group<LA, LB, 0>(wave, ps, ca, iters, Vp);
  __syncthreads();

  // rotate back: V = D_a^T V' D_b with D^T = Z(phi) J^T Z(theta) J; rows first, then columns
  double cth[LA + 1], sth[LA + 1], cph[LA + 1], sph[LA + 1];
  angles<LA>(ps.ct, ps.st, cth, sth);
  angles<LA>(ps.cp, ps.sp, cph, sph);
  for (int r = wave; r < NA; r += Q) {
    double v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) v[j] = Vp[r * NB + j];
    Rot<LB>::apply(v, cth, sth, cph, sph);
#pragma unroll
    for (int j = 0; j < NB; ++j) Vp[r * NB + j] = v[j];
  }
  __syncthreads();
  if (!ps.active) return;
  for (int col = wave; col < NB; col += Q) {
    double v[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) v[i] = Vp[i * NB + col];
    Rot<LA>::apply(v, cth, sth, cph, sph);
    if (ca.pr.full) {
      const int64_t r0 = ca.bs.bf_off[ps.s1], c0 = ca.bs.bf_off[ps.s2], n = ca.bs.nbf;
      if (ps.s1 != ps.s2) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          ca.out[(r0 + i) * n + c0 + col] = v[i];
          ca.out[(c0 + col) * n + r0 + i] = v[i];
        }
      } else {
        // diagonal block: the upper triangle is mirrored so that V is exactly symmetric
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          if (i <= col) {
            ca.out[(r0 + i) * n + c0 + col] = v[i];
            ca.out[(c0 + col) * n + r0 + i] = v[i];
          }
        }
      }
    } else {
      const int o = ca.pr.orig[slot];
      const int64_t bo = ca.pr.blk_off[o];
      const bool sw = ca.pr.pa[o] != ps.s1;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        if (sw)
          ca.out[bo + (int64_t)col * NA + i] = v[i];
        else
          ca.out[bo + (int64_t)i * NB + col] = v[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------
// Boys table F_m(i/16), m < kBoysOrders, by the convergent series in long double.
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

using LaunchFn = void (*)(const ClassArgs&, int grid, hipStream_t);

template <int LA, int LB>
void launch_class(const ClassArgs& ca, int grid, hipStream_t st) {
  constexpr int Q = ClassInfo<LA, LB>::Q;
  const size_t lds = (size_t)64 * (2 * LA + 1) * (2 * LB + 1) * sizeof(double);
  hipLaunchKernelGGL((k_class<LA, LB>), dim3(grid), dim3(64 * Q), lds, st, ca);
}

template <int LA, int LB>
hipError_t prepare_class() {
  const size_t lds = (size_t)64 * (2 * LA + 1) * (2 * LB + 1) * sizeof(double);
  return hipFuncSetAttribute((const void*)k_class<LA, LB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

struct ClassTable {
  LaunchFn launch[kNumClasses];
  hipError_t (*prepare[kNumClasses])();
  ClassTable() {
    fill<0, 0>();
  }
  template <int LA, int LB>
  void fill() {
    if constexpr (LA <= SHGO_LMAX) {
      launch[class_id(LA, LB)] = &launch_class<LA, LB>;
      prepare[class_id(LA, LB)] = &prepare_class<LA, LB>;
      if constexpr (LB < LA)
        fill<LA, LB + 1>();
      else
        fill<LA + 1, 0>();
    }
  }
};

const ClassTable& class_table() {
  static ClassTable t;
  return t;
}

}  // namespace

struct shgo_context {
  int device = 0;
  double* boys_tab = nullptr;
  std::string err;
};

struct shgo_plan {
  shgo_context* ctx = nullptr;
  int full = 0;
  int32_t n_shells = 0, n_nuc = 0;
  int64_t nbf = 0, n_cand = 0, out_size = 0, integrals = 0;
  double screen = 0.0;
  int class_cand[kNumClasses] = {0};  // candidate pairs per class (grid bound)
  std::vector<void*> allocs;
  DevBasis bs{};
  DevPairs pr{};
  Nuc* nuc = nullptr;
  // per-class kernel timing (off when slots == 0)
  int32_t slots = 0;
  int64_t exec_count = 0;
  std::vector<hipEvent_t> events;  // [slots][kNumClasses][2]
};

namespace {

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
  e = e != hipSuccess ? e : dalloc(p, &pr.key_fill, (size_t)kNumKeys);
  e = e != hipSuccess ? e : dalloc(p, &pr.key_off, (size_t)kNumKeys + 1);
  if (e != hipSuccess) {
    shgo_plan_destroy(p);
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "device allocation failed");
  }
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
  *out = p;
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
  const ClassTable& ct = class_table();
  for (int k = 0; k < kNumClasses; ++k)
    if (ct.prepare[k]() != hipSuccess) {
      (void)hipFree(c->boys_tab);
      delete c;
      return SHGO_ERR_DEVICE;
    }
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
  hipStream_t st = (hipStream_t)stream;
  if (p->n_cand == 0) return SHGO_OK;
  const int tb = 256;
  auto blocks = [&](int64_t n) { return (int)((n + tb - 1) / tb); };
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(kNumKeys)), dim3(tb), 0, st, p->pr.key_count, (int64_t)kNumKeys, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(kNumKeys)), dim3(tb), 0, st, p->pr.key_fill, (int64_t)kNumKeys, 0);
  if (p->n_shells > 0) hipLaunchKernelGGL(k_prim_weights, dim3(blocks(p->n_shells)), dim3(tb), 0, st, p->bs);
  hipLaunchKernelGGL(k_classify, dim3(blocks(p->n_cand)), dim3(tb), 0, st, p->bs, p->pr);
  hipLaunchKernelGGL(k_scan_keys, dim3(1), dim3(1024), 0, st, p->pr);
  hipLaunchKernelGGL(k_scatter, dim3(blocks(p->n_cand)), dim3(tb), 0, st, p->bs, p->pr);
  ClassArgs ca{p->bs, p->pr, p->nuc, p->n_nuc, ctx->boys_tab, out};
  const ClassTable& ct = class_table();
  const int slot = p->slots > 0 ? (int)(p->exec_count % p->slots) : -1;
  for (int c = kNumClasses - 1; c >= 0; --c) {
    const int n = p->class_cand[c];
    if (n == 0) continue;
    if (slot >= 0) (void)hipEventRecord(p->events[((size_t)slot * kNumClasses + c) * 2], st);
    ct.launch[c](ca, (n + 63) / 64, st);
    if (slot >= 0) (void)hipEventRecord(p->events[((size_t)slot * kNumClasses + c) * 2 + 1], st);
  }
  p->exec_count++;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

shgo_status shgo_plan_set_timing(shgo_plan* p, int32_t n_slots) {
  if (!p || n_slots < 0 || n_slots > 4096) return SHGO_ERR_INVALID_ARG;
  if (hipSetDevice(p->ctx->device) != hipSuccess) return fail(p->ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  for (hipEvent_t ev : p->events) (void)hipEventDestroy(ev);
  p->events.clear();
  p->slots = 0;
  p->exec_count = 0;
  std::vector<hipEvent_t> evs((size_t)n_slots * kNumClasses * 2);
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

shgo_status shgo_plan_class_ms(shgo_plan* p, double* ms, int32_t* count) {
  if (!p || !ms || !count) return SHGO_ERR_INVALID_ARG;
  const int64_t n = std::min<int64_t>(p->exec_count, p->slots);
  *count = (int32_t)n;
  for (int c = 0; c < kNumClasses; ++c) {
    ms[c] = 0.0;
    if (p->class_cand[c] == 0) continue;
    for (int64_t s = 0; s < n; ++s) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p->events[((size_t)s * kNumClasses + c) * 2], p->events[((size_t)s * kNumClasses + c) * 2 + 1]) !=
          hipSuccess)
        return fail(p->ctx, SHGO_ERR_DEVICE, "hipEventElapsedTime failed (stream not synchronised?)");
      ms[c] += t;
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
