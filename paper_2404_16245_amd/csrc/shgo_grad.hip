// Adjoint kernels of the gradient of E = sum_ij D_ij V_ij on MI355X (gfx950): dE/d(nuclear
// positions) and dE/d(shell centers), through Eq. 5, the shift of Eqs. 7-8, the product rule and the
// Boys function (Hobson's theorem, Eq. 3, raises and lowers l).
#include "shgo_internal.h"

#include "generated/shgo_rot.inc"
#include "generated/shgo_grad.inc"

namespace shgo_impl {
namespace {

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
          // Boys F_0..F_{LM+1} without a divergent branch, as in the integral kernel: the row of the
          // nearest grid point (index clamped to the table), or the asymptote above kBoysTcut,
          // selected per lane
          double row[kBoysRowLoad];
          {
            const double* __restrict__ r = boys_row_ptr(ga.boys_tab, LM + 1, boys_index(T));
#pragma unroll
            for (int k = 0; k < kBoysRowLoad; ++k) row[k] = r[k];
          }
          double F[LM + 2];
          boys_row<LM + 1>(T, row, F);
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
  // eight rounds of resident workgroups (the hardware starts each as one finishes, which evens out
  // the pairs' uneven costs: 35.0 -> 32.0 ms on the 500-atom molecule against one round, no further
  // gain at sixteen); the kernel strides over the class's pairs
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((waves_needed + per_block - 1) / per_block,
                                                                 (int64_t)8 * p->grad_occ[c] * p->ctx->n_cu));
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

shgo_status grad_classes(shgo_plan* p, const GradArgs& ga, hipStream_t st, bool launch) {
  return grad_all<0, 0>(p, ga, st, launch);
}

}  // namespace shgo_impl
