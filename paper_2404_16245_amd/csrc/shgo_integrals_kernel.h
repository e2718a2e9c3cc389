// a2-a8 of the nuclear-attraction path on MI355X (gfx950): the persistent integral kernel,
// templated on the arithmetic of the coupling (Mixed: binary32 with error-free transformations,
// else binary64). shgo_integrals.hip and shgo_integrals_mixed.hip each instantiate one form, so
// that the two compile in parallel.
//
// Work item = (class, block of up to T tiles of kTile class-sorted shell pairs). Every workgroup
// (one per CU, eight wavefronts) pulls items from one queue (longest first). Its wavefronts take
// the item's (tile, slice, group) tasks from an LDS counter, run the group's primitive-pair and
// nucleus loops for the tile's pairs (one pair per lane) and add the group's part of each block V'
// into the item's accumulator in LDS. Work is done in the frame whose z axis is A->B, where the
// shift of Eq. 7 keeps m (only Y^lambda_0 of a z-directed vector survives). Per primitive pair and
// nucleus (nuclei read through the scalar cache): C = c - P in the frame, Boys F_m, monic
// solid-harmonic recurrences, W(L,M,k) += Z G_{L,k} Q in registers; then the product-rule and
// shift coefficients map W onto the block V' (atomic adds into LDS). After a workgroup barrier
// each tile's blocks are rotated back to the laboratory frame, D^T = Z(phi) J^T Z(theta) J, by all
// wavefronts and written with coalesced stores. Nothing crosses a workgroup: no global atomics on
// partial sums and no device-scope fences.
#pragma once
#include "shgo_internal.h"

#define SHGO_ACC_STRIDE (shgo_sched::kAccStride)  // doubles between entries of a tile accumulator
#include "generated/shgo_rot.inc"
#include "generated/shgo_classes.inc"

namespace shgo_impl {
namespace {

static_assert(kTile == 64, "a tile is one pair per lane of a wavefront");

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
template <int LA, int LB, int G, bool Mixed>
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
      // nucleus loop: geometry in the pair frame, the Boys row of the nucleus's T, then the group's step
      double nx = 0.0, ny = 0.0, nz = 0.0, nr2 = 0.0, nt = 0.0, nZ = 0.0, nrow[kBoysRowLoad];
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
        const double* __restrict__ r = boys_row_ptr(wa->boys_tab, LM, boys_index(nt));  // index 0 .. kBoysPoints - 1
#pragma unroll
        for (int k = 0; k < kBoysRowLoad; ++k) nrow[k] = r[k];
      };
      auto nucleus = [&](double x, double y, double z, double r2, double t, double Zc,
                         const double (&row)[kBoysRowLoad]) {
        double F[LM + 1];
        boys_row<LM>(t, row, F);
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
          double row[kBoysRowLoad];
#pragma unroll
          for (int k = 0; k < kBoysRowLoad; ++k) row[k] = nrow[k];
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
      if constexpr (Mixed && LA <= kMixedLmax)
        Grp::couple_mixed(W, ta, tb, Vp);
      else
        Grp::couple(W, ta, tb, Vp);
    }
  }
}

template <int LA, int LB, int G, bool Mixed>
__device__ __forceinline__ void dispatch_group(int g, const PairState& ps, WAP wa, int it0, int it1, int c0, int c1,
                                               double* Vp) {
  if constexpr (G < ClassInfo<LA, LB>::Q) {
    if (g == G) {
      run_group<LA, LB, G, Mixed>(ps, wa, it0, it1, c0, c1, Vp);
      return;
    }
    dispatch_group<LA, LB, G + 1, Mixed>(g, ps, wa, it0, it1, c0, c1, Vp);
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
template <int LA, int LB, bool Mixed>
__device__ __attribute__((noinline)) void process_block(int b, const WorkArgs* wa_ptr, double* __restrict__ out,
                                                        int* task_ctr, int* next_item) {
  const WAP wa = uniform_args(wa_ptr);
  constexpr int Q = ClassInfo<LA, LB>::Q;
  constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NAB = NA * NB;
  constexpr int cls = class_id(LA, LB);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const ItemGeom ig = item_geom(wa->pr.key_off, cls, wa->meta.tiles[cls], b);
  const int start = ig.start, end = ig.end, t0 = ig.t0, nt = ig.nt;
  double* const acc = s_lds + acc_offset(NAB, 0);
  double* const frm = s_lds + frames_offset(NAB, nt);
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
      if (it >= kKeysPerClass - 1) it = pair_iters(it, wa->bs.nprim[wa->pr.s1[slot]], wa->bs.nprim[wa->pr.s2[slot]]);
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
    int t, g, it0, it1;
    if (!decode_task(task, Q, nt, s_tile_iters, t, g, it0, it1)) break;
    PairState ps;
    load_pair<LA, LB>(ps, wa, start + (t0 + t) * kTile + lane, end);
    if (g == 0 && it0 == 0) {
      double* const f = frm + t * 4 * kTile + lane;
      f[0] = ps.ct;
      f[kTile] = ps.st;
      f[2 * kTile] = ps.cp;
      f[3 * kTile] = ps.sp;
    }
    dispatch_group<LA, LB, 0, Mixed>(g, ps, wa, it0, it1, 0, n_nuc, acc + acc_offset(NAB, t) + lane);
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
            const int64_t o = out_index_matrix(pass, r0, c0, i, col, n);
            if (o >= 0) out[o] = acc[acc_entry(NAB, tp, i * NB + col)];
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
          out[bo + e] = acc[acc_entry(NAB, tp, list_source_entry(e, dst[2 * tp + 1] != 0, NA, NB))];
        }
      }
    }
  }
  if (threadIdx.x == 0) *next_item = next;
}

template <int LA, int LB, bool Mixed>
__device__ __forceinline__ void dispatch_class(int c, int j, const WorkArgs* wa, double* out, int* task_ctr,
                                               int* next_item) {
  if constexpr (LA <= SHGO_LMAX) {
    if (c == class_id(LA, LB)) {
      process_block<LA, LB, Mixed>(j, wa, out, task_ctr, next_item);
      return;
    }
    if constexpr (LB < LA)
      dispatch_class<LA, LB + 1, Mixed>(c, j, wa, out, task_ctr, next_item);
    else
      dispatch_class<LA + 1, 0, Mixed>(c, j, wa, out, task_ctr, next_item);
  }
}

// Every workgroup loops: take the next item, run it with its eight wavefronts; the loop ends
// once the queue is drained.
template <bool Mixed>
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
    unsigned long long* const tick = wa->item_ns;  // [item][start, duration] in wall-clock ticks
    const unsigned long long t0 = tick ? wall_clock64() : 0ull;
    dispatch_class<0, 0, Mixed>(item >> 24, item & 0xffffff, wa_ptr, out, &s_task, &s_item);
    if (tick && threadIdx.x == 0) {
      tick[2 * q] = t0;
      tick[2 * q + 1] = wall_clock64() - t0;
    }
    __syncthreads();
  }
}

template <bool Mixed>
void launch_integrals_impl(const shgo_plan* p, double* out, hipStream_t st) {
  // dynamic LDS: the largest tiles x (accumulator + frames) over the plan's classes
  size_t lds = sizeof(double);
  for (int c = 0; c < kNumClasses; ++c)
    if (p->class_cand[c] > 0) lds = std::max(lds, sizeof(double) * (size_t)item_lds_doubles(class_nab(c), p->meta.tiles[c]));
  hipLaunchKernelGGL(k_integrals<Mixed>, dim3(p->ctx->grid), dim3(kIntegralThreads), lds, st, (const WorkArgs*)p->d_wa,
                     out);
}

// Launch guard and occupancy of the persistent kernel: its static LDS (read from the code object)
// plus the largest dynamic LDS a work item uses must fit the CU's 160 KB; workgroups per CU.
template <bool Mixed>
hipError_t integrals_setup_impl(int* per_cu, std::string* why) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_integrals<Mixed>);
  if (e != hipSuccess) return e;
  if (fa.sharedSizeBytes + sizeof(double) * (size_t)kLdsDoubles > (size_t)kLdsBytes) {
    *why = "integral kernel: static LDS " + std::to_string(fa.sharedSizeBytes) + " B + dynamic " +
           std::to_string(sizeof(double) * kLdsDoubles) + " B exceed the CU's " + std::to_string(kLdsBytes) + " B";
    return hipErrorInvalidConfiguration;
  }
  if (fa.maxThreadsPerBlock < kIntegralThreads) {
    *why = "integral kernel: compiled for fewer threads per workgroup than it is launched with";
    return hipErrorInvalidConfiguration;
  }
  e = hipFuncSetAttribute((const void*)k_integrals<Mixed>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(double) * kLdsDoubles));
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_integrals<Mixed>, kIntegralThreads,
                                                      sizeof(double) * kLdsDoubles);
}

}  // namespace
}  // namespace shgo_impl
