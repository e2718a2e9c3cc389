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

}  // namespace

void launch_overlap(const shgo_plan* p, double* out, hipStream_t st) {
  const int tb = 256;
  hipLaunchKernelGGL(k_overlap, dim3((int)((p->n_cand + tb - 1) / tb)), dim3(tb), 0, st, p->bs, p->pr, out);
}

}  // namespace shgo_impl
