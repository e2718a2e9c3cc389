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
// consecutive lanes on consecutive entries, then a column at a time for the mirror. Each
// wavefront has its own stage of 64 (2 l_max + 1) doubles and 64 destination pairs.
struct OvlStage {
  double* stg;
  int64_t* d0;
  int64_t* d1;
};

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
                                             const OvlStage& sg, double* __restrict__ out) {
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
    const int lane = threadIdx.x & 63;
    double* const stg = sg.stg;
    sg.d0[lane] = d0;
    sg.d1[lane] = d1;
    const int64_t n = bs.nbf;
    // rows i of every block: entry k = p NB + j is block p's (i, j)
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
      for (int j = 0; j < NB; ++j) stg[lane * NB + j] = V[i * NB + j];
      ovl_wave_sync();
      for (int k = lane; k < 64 * NB; k += 64) {
        const int q = k / NB, j = k - q * NB;
        const int64_t e0 = sg.d0[q], e1 = sg.d1[q];
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
          const int64_t e0 = sg.d0[q], e1 = sg.d1[q];
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

template <int LA, int LB, bool kStaged, int LMAXK>
__device__ __forceinline__ void overlap_dispatch(int c, const DevBasis& bs, const DevPairs& pr, int slot, bool active,
                                                 const OvlStage& sg, double* __restrict__ out) {
  if constexpr (LA <= LMAXK) {
    if (c == class_id(LA, LB)) {
      overlap_pair<LA, LB, kStaged>(bs, pr, slot, active, sg, out);
      return;
    }
    if constexpr (LB < LA)
      overlap_dispatch<LA, LB + 1, kStaged, LMAXK>(c, bs, pr, slot, active, sg, out);
    else
      overlap_dispatch<LA + 1, 0, kStaged, LMAXK>(c, bs, pr, slot, active, sg, out);
  }
}

// One thread per class-sorted shell pair in the slots [begin, end) (from k_scatter; s1 has the
// higher l), whose classes all have la <= LMAXK: the kernel is register-allocated for its largest
// class only. A wavefront whose active lanes all hold one class (all but those at class
// boundaries) stores through LDS; the others store lane by lane.
template <int LMAXK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_overlap(DevBasis bs, DevPairs pr, int64_t begin, int64_t end, double* __restrict__ out) {
  __shared__ double s_stage[4][64 * (2 * LMAXK + 1)];
  __shared__ int64_t s_d0[4][64], s_d1[4][64];
  const int w = threadIdx.x >> 6;
  const OvlStage sg{s_stage[w], s_d0[w], s_d1[w]};
  const int64_t slot = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = slot < end;
  const int c = active ? class_id(bs.l[pr.s1[slot]], bs.l[pr.s2[slot]]) : -1;
  const int c0 = __shfl(c, 0);  // lanes past the last pair come after the active ones
  if (c0 < 0) return;           // no active lane in this wavefront
  if (__all(!active || c == c0)) {
    overlap_dispatch<0, 0, true, LMAXK>(c0, bs, pr, (int)(active ? slot : 0), active, sg, out);
  } else if (active) {
    overlap_dispatch<0, 0, false, LMAXK>(c, bs, pr, (int)slot, true, sg, out);
  }
}

}  // namespace

// The class-sorted slots fall into three ranges of la (classes are sorted by id, and the ids of
// la <= 2, la = 3..4 and la = 5..SHGO_LMAX are contiguous): one launch each, so that the small
// classes are not register-allocated for the largest block.
void launch_overlap(const shgo_plan* p, double* out, hipStream_t st) {
  const int tb = 256;
  int64_t first[kNumClasses + 1];
  first[0] = 0;
  for (int c = 0; c < kNumClasses; ++c) first[c + 1] = first[c] + p->class_cand[c];
  const int64_t b1 = first[class_id(3, 0)], b2 = first[class_id(5, 0)], b3 = first[kNumClasses];
  auto grid = [&](int64_t n) { return dim3((unsigned)((n + tb - 1) / tb)); };
  if (b1 > 0) hipLaunchKernelGGL(k_overlap<2>, grid(b1), dim3(tb), 0, st, p->bs, p->pr, (int64_t)0, b1, out);
  if (b2 > b1) hipLaunchKernelGGL(k_overlap<4>, grid(b2 - b1), dim3(tb), 0, st, p->bs, p->pr, b1, b2, out);
  if (b3 > b2)
    hipLaunchKernelGGL(k_overlap<SHGO_LMAX>, grid(b3 - b2), dim3(tb), 0, st, p->bs, p->pr, b2, b3, out);
}

}  // namespace shgo_impl
