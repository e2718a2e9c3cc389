// Internal header of the MI355X (gfx950) nuclear-attraction library: constants, the device
// data layout, device helpers shared by the kernels (exponential, Boys function, pair frame),
// the plan and context objects and the launch functions each translation unit provides.
//
// Method (arXiv:2404.16245): Gaussian product (Eq. 5), shift of both solid harmonics to the
// product center P with the vector-coupling coefficients (Eqs. 7-8), product rule of solid
// harmonics (the supplement's Eq. 4), one-center Coulomb integral by Hobson's theorem and the
// Boys function (Eqs. 11-12, each r^{2k} Y^L_M term of the product rule giving
// Y^L_M(c-P) 2 pi k!/p^{k+1} sum_j T^j/j! F_{L+j}(T)), sum over nuclei, contraction.
//
// Translation units:
//   shgo_pairs.hip      a1: normalisation, enumeration, screening, class sort (k_classify,
//                       k_scan_keys, k_scatter); the Boys test kernels; fill kernel
//   shgo_integrals.hip  a2-a8: the persistent integral kernel (k_integrals)
//   shgo_overlap.hip    the overlap matrix S (k_overlap)
//   shgo_grad.hip       the adjoint kernels of the gradient (k_grad<LA, LB>)
//   shgo_api.hip        host side: the C ABI, plans, the autotuner
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "shgo.h"
#include "schedule.h"
#include "generated/shgo_meta.inc"

static_assert(shgo_sched::kLmax == SHGO_LMAX, "schedule and ABI disagree on the highest l");
static_assert(shgo_sched::kNumClasses == SHGO_NUM_CLASSES, "schedule and ABI disagree on the class count");

// ---------------------------------------------------------------------------------------------
// Double-float arithmetic (the mixed-precision coupling)
// ---------------------------------------------------------------------------------------------
// A double-float is an unevaluated sum h + l of two binary32 numbers with |l| <= ulp(h) / 2, about
// 48 significant bits. Products and sums use the error-free transformations: TwoProd (the
// rounding error of a * b is exactly fma(a, b, -a * b)) and Knuth's TwoSum (the rounding error of
// a + b from six additions), each followed by a renormalisation (Fast2Sum). Contraction of a
// product into a later sum is switched off in them, since it would change the rounding the
// transformations rely on. Global, like the generated class code that uses them.
struct df {
  float h, l;
};
__device__ __forceinline__ df df_zero() { return df{0.0f, 0.0f}; }
__device__ __forceinline__ df df_split(double x) {
  const float h = (float)x;
  return df{h, (float)(x - (double)h)};
}
__device__ __forceinline__ double df_value(df a) { return (double)a.h + (double)a.l; }
__device__ __forceinline__ df df_renorm(float s, float e) {
#pragma clang fp contract(off)
  const float h = s + e;
  return df{h, e - (h - s)};
}
// a * b: TwoProd of the high parts and the first-order cross terms
__device__ __forceinline__ df df_mul(df a, df b) {
#pragma clang fp contract(off)
  const float p = a.h * b.h;
  const float e = __builtin_fmaf(a.h, b.h, -p) + __builtin_fmaf(a.h, b.l, a.l * b.h);
  return df_renorm(p, e);
}
// a + b: TwoSum of the high parts and the sum of the low parts
__device__ __forceinline__ df df_add(df a, df b) {
#pragma clang fp contract(off)
  const float s = a.h + b.h;
  const float bb = s - a.h;
  const float e = ((a.h - (s - bb)) + (b.h - bb)) + (a.l + b.l);
  return df_renorm(s, e);
}
// c + a * b: TwoProd, then TwoSum of the product's high part into c
__device__ __forceinline__ df df_fma(df a, df b, df c) {
#pragma clang fp contract(off)
  const float p = a.h * b.h;
  const float pe = __builtin_fmaf(a.h, b.h, -p) + __builtin_fmaf(a.h, b.l, a.l * b.h);
  const float s = c.h + p;
  const float bb = s - c.h;
  const float e = ((c.h - (s - bb)) + (p - bb)) + (c.l + pe);
  return df_renorm(s, e);
}

namespace shgo_impl {

using namespace shgo_sched;

// ---------------------------------------------------------------------------------------------
// Constants and device data layout
// ---------------------------------------------------------------------------------------------
// Boys table: one row per (order M, grid point t_i = i/16) holding the Taylor coefficients of F_M
// about t_i, F_{M+k}(t_i)/k! for k < 8, then e^{-t_i} as the sum of two doubles (high, low part).
constexpr int kBoysMaxM = 15;      // highest order a kernel evaluates (l_a + l_b + 1 for the gradient)
constexpr int kBoysPoints = 1153;  // grid t_i = i/16, i = 0..1152
constexpr int kBoysRow = 10;       // doubles per row
constexpr int kBoysRowLoad = 10;   // doubles a kernel reads of a row
constexpr double kBoysTcut = 72.0; // below: table; above: asymptotic form (e^{-t} < 6e-32)
constexpr int kPrefetchMaxW = 32;  // groups up to this many W doubles prefetch the next nucleus
constexpr int kClassifyThreads = 1024;
constexpr int kGradThreads = 256;

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
  const int32_t* by_l;     // [SHGO_LMAX + 2] first entry of each l, then [n] the shells by l, then primitive count
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

struct WorkArgs {
  DevBasis bs;
  DevPairs pr;
  const Nuc* __restrict__ nuc;
  int32_t n_nuc;
  const double* __restrict__ boys_tab;
  int32_t* __restrict__ queue;     // [0]: next work item
  int32_t* __restrict__ item_off;  // [0]: number of work items
  int32_t* __restrict__ items;     // work items, longest first: class << 24 | tile block
  unsigned long long* __restrict__ item_ns;  // per item: start and duration (10 ns ticks) when profiling, else null
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

// Grid index of t (clamped to the table) and the first double of its row of order M.
__device__ __forceinline__ int boys_index(double t) { return (int)(fmin(t, kBoysTcut) * 16.0 + 0.5); }
__device__ __forceinline__ const double* boys_row_ptr(const double* tab, int M, int i) {
  return tab + ((size_t)M * kBoysPoints + i) * kBoysRow;
}

// F_0..F_M(t) from the row of order M at the grid point t_i nearest t (the clamped index of
// boys_index) and no divergent branch. Below kBoysTcut: the Taylor series of F_M about t_i,
// F_M(t_i + h) = sum_k F_{M+k}(t_i) (-h)^k / k!, |h| <= 1/32 (the row holds the coefficients with
// their 1/k!), and e^{-t} = e^{-t_i} e^{-h} with e^{-h} by its Taylor polynomial of degree 7 (the
// remainder is below 3e-17) and e^{-t_i} carried in two parts (about one rounding in all).
// Above: the leading asymptotic term Gamma(M+1/2) / (2 t^{M+1/2}) (the neglected part, about
// e^{-t} t^{M-1/2} / Gamma(M+1/2) relative, is below 2e-16 for M <= 15 at t = 72) and e^{-t}
// taken as 0.
// The two are selected per lane; then the downward recursion F_m = (2t F_{m+1} + e^{-t})/(2m+1),
// stable for every t.
template <int M>
__device__ __forceinline__ void boys_row(double t, const double (&row)[kBoysRowLoad], double (&F)[M + 1]) {
  static_assert(M <= kBoysMaxM, "order beyond the table");
  const int i = boys_index(t);
  const double d = 0.0625 * (double)i - t;  // t_i - t = -h
  double f = row[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) f = fma(f, d, row[k]);
  double q = add_vs(mul_vs(d, 1.9841269841269841270e-04), 1.3888888888888888889e-03);  // 1/7!, 1/6!
  q = fma_vvs(q, d, 8.3333333333333333333e-03);  // 1/5!
  q = fma_vvs(q, d, 4.1666666666666666667e-02);  // 1/4!
  q = fma_vvs(q, d, 1.6666666666666666667e-01);  // 1/3!
  q = fma(q, d, 0.5);
  q = fma(q, d, 1.0);
  q = fma(q, d, 1.0);
  // 1/sqrt(t) from the hardware estimate and two Newton steps (each doubles the bits)
  double rs = __builtin_amdgcn_rsq(t);
  rs = rs * fma(-0.5 * t * rs, rs, 1.5);
  rs = rs * fma(-0.5 * t * rs, rs, 1.5);
  const double fa = half_gamma_half(M) * rs * pow_n<M>(rs * rs);
  const bool tab_ok = t < kBoysTcut;
  F[M] = tab_ok ? f : fa;
  const double e = tab_ok ? fma(row[8], q, row[9] * q) : 0.0;
  const double t2 = 2.0 * t;
#pragma unroll
  for (int m = M - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (2 * m + 1));
}


__device__ __forceinline__ bool keep_prim(double a, double b, double R2, double screen) {
  if (!(screen > 0.0)) return true;
  return exp_neg(a * b / (a + b) * R2) > screen;
}
// The same decision as keep_prim, without the exponential and the division away from the
// threshold: with L = -ln(screen), a pair with a b R^2 below (L - d)(a + b) is kept and one above
// (L + d)(a + b) dropped for certain (d = 1e-9 max(L, 1) is far wider than the rounding of either
// side); only those in between take keep_prim's own test. lo = L - d, hi = L + d (screen_band).
struct ScreenBand {
  double lo, hi;
};
__device__ __forceinline__ ScreenBand screen_band(double screen) {
  if (!(screen > 0.0)) return {0.0, 0.0};
  const double L = -log(screen), d = 1e-9 * fmax(fabs(L), 1.0);
  return {L - d, L + d};
}
__device__ __forceinline__ bool keep_prim_banded(double a, double b, double R2, double screen, ScreenBand band) {
  if (!(screen > 0.0)) return true;
  const double x = a * b * R2, s = a + b;
  if (x < band.lo * s) return true;
  if (x > band.hi * s) return false;
  return keep_prim(a, b, R2, screen);
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

}  // namespace shgo_impl

// ---------------------------------------------------------------------------------------------
// Host objects (the opaque types of the C ABI)
// ---------------------------------------------------------------------------------------------
struct shgo_context {
  int device = 0;
  int n_cu = 0;
  int grid = 0;  // workgroups of the persistent kernel resident on the device at once
  double* boys_tab = nullptr;
  std::string err;
  // the plan of the last single call (shgo_nuclear_attraction, _grad) and the inputs it was made
  // from: a repeated call with the same inputs reuses it (device copies, tuned schedule, graph)
  shgo_plan* call_plan = nullptr;
  std::vector<char> call_key;
  // this device's address of the library's static scratch array (shgo_nuclear_attraction_noalloc)
  void* scratch = nullptr;
  // the two-electron call's buffers, kept for the next call and grown as needed (freed by
  // shgo_destroy): its device workspace, a pinned host copy of the workspace's index part, and
  // host scratch for the quartets' pairs and sort keys
  shgo_plan* eri_plan = nullptr;  // the pair plan of the last call's basis (uploaded basis, weights)
  std::vector<char> eri_key;      // and the bytes of that basis
  void* eri_dev = nullptr;
  size_t eri_dev_bytes = 0;
  void* eri_pin = nullptr;
  size_t eri_pin_bytes = 0;
  std::vector<int32_t> eri_tmp;
};

struct shgo_plan {
  shgo_context* ctx = nullptr;
  int full = 0;
  int32_t n_shells = 0, n_nuc = 0;
  int32_t max_nprim = 0;        // the longest contraction of the basis
  int32_t l_first[SHGO_LMAX + 2] = {0};  // host copy of the first SHGO_LMAX + 2 entries of bs.by_l
  int64_t nbf = 0, n_cand = 0, out_size = 0;
  int64_t integrals = 0;        // sum of (2la+1)(2lb+1) over the kept shell pairs
  int64_t kept_pairs = 0;       // shell pairs that keep at least one primitive pair
  int64_t kept_prim_pairs = 0;  // primitive pairs that survive screening
  double screen = 0.0;
  int32_t precision = SHGO_PREC_FP64;
  int class_cand[shgo_sched::kNumClasses] = {0};  // candidate pairs per class (bounds the sorted counts)
  int32_t def_tiles[shgo_sched::kNumClasses] = {0};  // default tiles per work item of each class
  int32_t grad_occ[shgo_sched::kNumClasses] = {0};    // resident workgroups per CU of each class's gradient kernel
  // the one device workspace every array below is carved from (plan_host.h: plan_layout); owned
  // by the plan unless it lives in the library's static scratch array
  void* block = nullptr;
  size_t block_bytes = 0;
  bool owns_block = true;
  shgo_impl::DevBasis bs{};
  shgo_impl::DevPairs pr{};
  shgo_impl::Nuc* nuc = nullptr;
  // persistent-kernel workspace
  shgo_impl::ClassMeta meta{};
  int32_t* queue = nullptr;     // head of the persistent kernel's work queue
  int32_t* item_off = nullptr;  // [0]: number of work items
  int32_t* items = nullptr;     // work items, longest first (capacity: one tile per item)
  shgo_impl::WorkArgs* d_wa = nullptr;  // the integral kernel's arguments, in device memory
  double* d_energy = nullptr;  // gradient: E when the caller does not ask for it
  // captured graph of one evaluation (shgo_execute_graph) and its output buffer
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* graph_out = nullptr;
  hipStream_t cap_stream = nullptr;
  // the autotune-cache file the schedule was last read from or written to (single calls)
  std::string schedule_file;
  // phase timing (off when slots == 0): events [slot][phase][start, end]
  int32_t slots = 0;
  int64_t exec_count = 0;
  std::vector<hipEvent_t> events;
};

namespace shgo_impl {

// ---------------------------------------------------------------------------------------------
// Launch functions (each defined in the translation unit of its kernels)
// ---------------------------------------------------------------------------------------------
// shgo_pairs.hip
void launch_pair_build(const shgo_plan* p, hipStream_t st);
// the pair build's primitive weights alone (k_classify's weight workgroups)
void launch_weights(const shgo_plan* p, hipStream_t st);
void launch_fill(double* ptr, int64_t n, hipStream_t st);
hipError_t launch_boys(int mmax, int64_t n, const double* T, double* F, const double* tab, hipStream_t st);
// shgo_integrals.hip and shgo_integrals_mixed.hip: the two forms of the integral kernel; the
// plan's precision picks one (launch_integrals, shgo_api.hip). The setup checks the kernel's LDS
// and threads against the launch and gives its workgroups per CU.
void launch_integrals_fp64(const shgo_plan* p, double* out, hipStream_t st);
void launch_integrals_mixed(const shgo_plan* p, double* out, hipStream_t st);
hipError_t integrals_setup_fp64(int* per_cu, std::string* why);
hipError_t integrals_setup_mixed(int* per_cu, std::string* why);
void launch_integrals(const shgo_plan* p, double* out, hipStream_t st);
// shgo_overlap.hip
void launch_overlap(const shgo_plan* p, double* out, hipStream_t st);
// shgo_cart.hip: the Cartesian (McMurchie-Davidson) route, one kernel per class present; shells
// up to l = cart_lmax()
int cart_lmax();
hipError_t launch_cartesian(const shgo_plan* p, double* out, hipStream_t st);
// shgo_eri.hip: two-electron blocks of validated host quartets [n][4] at host offsets into the
// device buffer out, after the plan's pair build (the primitive weights); allocates its own
// workspace, waits for the stream and frees it. Shells up to l = eri_lmax()
int eri_lmax();
hipError_t run_eri(const shgo_plan* p, const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets,
                   const int64_t* offsets, double* out, hipStream_t st);
// shgo_grad.hip: validate (launch = false: LDS limits, occupancy) or launch every class present
shgo_status grad_classes(shgo_plan* p, const GradArgs& ga, hipStream_t st, bool launch);

// host helpers of shgo_api.hip
shgo_status fail(shgo_context* ctx, shgo_status s, const std::string& msg);

}  // namespace shgo_impl
