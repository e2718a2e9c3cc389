// Overlap matrix S on MI355X (gfx950), Eqs. 4-10: the plan's class-sorted shell pairs, the pair
// frame, the rotation back and the output layout of V.
#include "shgo_internal.h"

#include "generated/shgo_rot.inc"

namespace shgo_impl {
namespace {

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

// The lanes of a pair: lane i of the pair's NA = 2 la + 1 lanes owns row i of its block. With the
// frame block diagonal, the laboratory block is V = Dt_a S' Dt_b^T (Dt = Rot, the rotation back),
//   V[i][j] = sum_m Dt_a[i][m + la] S'(m) Dt_b[j][m + lb],
// so row i is Rot<lb> applied to x[m + lb] = Dt_a[i][m + la] S'(m), and row i of Dt_a is the
// inverse rotation of the unit vector e_i. The pair's primitive pairs are split over its lanes
// and summed across them.
struct OvlSched {
  int64_t slot_first[kNumClasses + 1];  // class-sorted slots of class c: [slot_first[c], slot_first[c+1])
  int64_t wave_first[kNumClasses + 1];  // wavefronts of class c: [wave_first[c], wave_first[c+1])
  int32_t l_first[SHGO_LMAX + 2];       // a matrix plan's shells of l: entries [l_first[l], l_first[l+1]) of by_l
};

__host__ __device__ constexpr int ovl_pairs_per_wave(int la) { return 64 / (2 * la + 1); }

__device__ __forceinline__ void stage_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LA, int LB>
__device__ __forceinline__ void overlap_rows(const DevBasis& bs, const DevPairs& pr, const OvlSched& sc, int64_t slot0,
                                             double* __restrict__ stg, int64_t* __restrict__ sd,
                                             double* __restrict__ out) {
  constexpr int C = class_id(LA, LB);
  const int64_t slot_end = sc.slot_first[C + 1];
  constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, P = ovl_pairs_per_wave(LA);
  const int lane = threadIdx.x & 63;
  const int q = lane / NA, row = lane - q * NA;
  const int64_t slot = slot0 + q;
  const bool active = q < P && slot < slot_end;
  // the pair: a matrix plan's k-th pair of the class from the shells ordered by l and primitive
  // count (every shell of l = LA with every shell of l = LB; for LA = LB the pairs i <= j of the
  // list, each written with its mirror), else the pair build's slot
  int s1 = 0, s2 = 0;
  int64_t d0 = 0, d1 = 0;
  if (active) {
    if (pr.full) {
      const int32_t* const list = bs.by_l + SHGO_LMAX + 2;
      const int fa = sc.l_first[LA], fb = sc.l_first[LB], nb = sc.l_first[LB + 1] - fb;
      const int k = (int)(slot - sc.slot_first[C]);
      int i, j;
      if (LA == LB) {
        tri_pair(k, nb, i, j);
      } else {
        i = k / nb;
        j = k - i * nb;
      }
      s1 = list[fa + i];
      s2 = list[fb + j];
      d0 = bs.bf_off[s1];
      d1 = bs.bf_off[s2];
    } else {
      s1 = pr.s1[slot];
      s2 = pr.s2[slot];
      d0 = pr.dst0[slot];
      d1 = pr.dst1[slot];
    }
  }
  PairState ps;
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
  // G[lam] = sum over the primitive pairs of w_a w_b e^{-mu R^2} p^{-3/2} t_a^(la-lam) t_b^(lb-lam) p^{-lam};
  // since t_a t_b p = -mu R^2, each step down in lam multiplies the term by -mu R^2
  double g[LB + 1];
#pragma unroll
  for (int lam = 0; lam <= LB; ++lam) g[lam] = 0.0;
  const int64_t o1 = active ? bs.prim_off[s1] : 0, o2 = active ? bs.prim_off[s2] : 0;
  const int K1 = active ? bs.nprim[s1] : 0, K2 = active ? bs.nprim[s2] : 0;
  for (int idx = row; idx < K1 * K2; idx += NA) {
    const int i = idx / K2, j = idx - i * K2;
    const double a = bs.expo[o1 + i], b = bs.expo[o2 + j];
    const double p = a + b, ip = 1.0 / p, mr2 = a * b * ip * R * R;
    double u = bs.w[o1 + i] * bs.w[o2 + j] * exp_neg(mr2) * ip * sqrt(ip);
    const double ta = b * R * ip;
#pragma unroll
    for (int k = 0; k < LA - LB; ++k) u *= ta;
#pragma unroll
    for (int k = 0; k < LB; ++k) u *= ip;
    g[LB] += u;
#pragma unroll
    for (int lam = LB - 1; lam >= 0; --lam) {
      u *= -mr2;
      g[lam] += u;
    }
  }
  // G summed over the pair's lanes, in one order on every lane (all lanes take part), then
  // S'(m) = sum_lam cf[m][lam] G[lam]
  double gt[LB + 1];
#pragma unroll
  for (int lam = 0; lam <= LB; ++lam) {
    double t = 0.0;
    for (int k = 0; k < NA; ++k) t += __shfl(g[lam], (q * NA + k) & 63);
    gt[lam] = t;
  }
  double tot[LB + 1];
#pragma unroll
  for (int m = 0; m <= LB; ++m) {
    double t = 0.0;
#pragma unroll
    for (int lam = m; lam <= LB; ++lam) t = fma(cf[m][lam], gt[lam], t);
    tot[m] = t;
  }
  double cth[LA + 1], sth[LA + 1], cph[LA + 1], sph[LA + 1];
  angles<LA>(ps.ct, ps.st, cth, sth);
  angles<LA>(ps.cp, ps.sp, cph, sph);
  double y[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) y[k] = k == row ? 1.0 : 0.0;
  RotInv<LA>::apply(y, cth, sth, cph, sph);  // row `row` of Dt_a
  double x[NB];
#pragma unroll
  for (int m = -LB; m <= LB; ++m) x[m + LB] = y[m + LA] * tot[m < 0 ? -m : m];
  Rot<LB>::apply(x, cth, sth, cph, sph);  // row `row` of the laboratory block
  // rows through the wavefront's LDS stage: entry (q NA + row) NB + j is pair q's (row, j), so
  // consecutive lanes then store consecutive columns of one row
#pragma unroll
  for (int j = 0; j < NB; ++j) stg[lane * NB + j] = x[j];
  if (row == 0) {
    sd[2 * q] = d0;
    sd[2 * q + 1] = d1;
  }
  stage_sync();
  const int64_t n = bs.nbf;
  const int64_t pairs = slot_end - slot0 < P ? slot_end - slot0 : P;
  for (int k = lane; k < pairs * NA * NB; k += 64) {
    const int qq = k / (NA * NB), r = (k - qq * NA * NB) / NB, j = k - (qq * NA + r) * NB;
    const int64_t e0 = sd[2 * qq], e1 = sd[2 * qq + 1];
    if (pr.full) {
      if (e0 != e1 || r <= j) out[(e0 + r) * n + e1 + j] = stg[k];
    } else if (e1 == 0) {
      out[e0 + r * NB + j] = stg[k];  // the listed orientation (s1, s2), row-major
    }
  }
  stage_sync();
  if (!active) return;
  if (pr.full) {
    // the mirror; a shell with itself writes each entry once per orientation
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (d0 != d1 || row <= j) out[(d1 + j) * n + d0 + row] = x[j];
  } else if (d1 != 0) {
    // the listed pair is (s2, s1): the transposed block
#pragma unroll
    for (int j = 0; j < NB; ++j) out[d0 + j * NA + row] = x[j];
  }
}

template <int LA, int LB, int LMAXK>
__device__ __forceinline__ void overlap_dispatch(int c, int64_t gw, const DevBasis& bs, const DevPairs& pr,
                                                 const OvlSched& sc, double* __restrict__ stg, int64_t* __restrict__ sd,
                                                 double* __restrict__ out) {
  if constexpr (LA <= LMAXK) {
    constexpr int C = class_id(LA, LB);
    if (c == C) {
      const int64_t slot0 = sc.slot_first[C] + (gw - sc.wave_first[C]) * ovl_pairs_per_wave(LA);
      overlap_rows<LA, LB>(bs, pr, sc, slot0, stg, sd, out);
      return;
    }
    if constexpr (LB < LA)
      overlap_dispatch<LA, LB + 1, LMAXK>(c, gw, bs, pr, sc, stg, sd, out);
    else
      overlap_dispatch<LA + 1, 0, LMAXK>(c, gw, bs, pr, sc, stg, sd, out);
  }
}

// The wavefronts of the classes la = LMIN..LMAXK (consecutive class ids), each wavefront on
// ovl_pairs_per_wave(la) consecutive class-sorted pairs of one class (from k_scatter; s1 has the
// higher l): the kernel is register-allocated for its largest class only.
template <int LMIN, int LMAXK>
__global__ void __launch_bounds__(256) k_overlap(DevBasis bs, DevPairs pr, OvlSched sc, double* __restrict__ out) {
  constexpr int C0 = class_id(LMIN, 0), C1 = class_id(LMAXK + 1, 0);
  __shared__ double s_stage[4][64 * (2 * LMAXK + 1)];
  __shared__ int64_t s_dst[4][128];
  const int64_t gw = sc.wave_first[C0] + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= sc.wave_first[C1]) return;
  int c = C0;  // the class whose wavefronts hold gw (wave-uniform; static indices only)
#pragma unroll
  for (int k = C0 + 1; k < C1; ++k) c += gw >= sc.wave_first[k] ? 1 : 0;
  overlap_dispatch<LMIN, 0, LMAXK>(c, gw, bs, pr, sc, s_stage[threadIdx.x >> 6], s_dst[threadIdx.x >> 6], out);
}

}  // namespace

// Three launches over ranges of la (la <= 2, 3..4, 5..SHGO_LMAX), so that the small classes are not
// register-allocated for the largest block.
void launch_overlap(const shgo_plan* p, double* out, hipStream_t st) {
  OvlSched sc;
  for (int l = 0; l < SHGO_LMAX + 2; ++l) sc.l_first[l] = p->l_first[l];
  sc.slot_first[0] = 0;
  sc.wave_first[0] = 0;
  for (int la = 0, c = 0; la <= SHGO_LMAX; ++la)
    for (int lb = 0; lb <= la; ++lb, ++c) {
      const int64_t per = ovl_pairs_per_wave(la);
      sc.slot_first[c + 1] = sc.slot_first[c] + p->class_cand[c];
      sc.wave_first[c + 1] = sc.wave_first[c] + (p->class_cand[c] + per - 1) / per;
    }
  auto blocks = [&](int c0, int c1) {
    return dim3((unsigned)((sc.wave_first[c1] - sc.wave_first[c0] + 3) / 4));
  };
  constexpr int c3 = class_id(3, 0), c5 = class_id(5, 0);
  if (sc.wave_first[c3] > 0)
    hipLaunchKernelGGL((k_overlap<0, 2>), blocks(0, c3), dim3(256), 0, st, p->bs, p->pr, sc, out);
  if (sc.wave_first[c5] > sc.wave_first[c3])
    hipLaunchKernelGGL((k_overlap<3, 4>), blocks(c3, c5), dim3(256), 0, st, p->bs, p->pr, sc, out);
  if (sc.wave_first[kNumClasses] > sc.wave_first[c5])
    hipLaunchKernelGGL((k_overlap<5, SHGO_LMAX>), blocks(c5, kNumClasses), dim3(256), 0, st, p->bs, p->pr, sc, out);
}

}  // namespace shgo_impl
