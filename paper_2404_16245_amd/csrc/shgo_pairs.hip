// a1 of the nuclear-attraction path on MI355X (gfx950): per-shell primitive normalisation,
// shell-pair enumeration, screening, counting sort by class and surviving primitive pairs, the
// cost-sorted work-item list of the integral kernel and each pair's output destination (Eq. 1,
// Eq. 5). Also the device Boys-function test kernel and a fill kernel.
#include "shgo_internal.h"

namespace shgo_impl {
namespace {

// ---------------------------------------------------------------------------------------------
// Normalisation, enumeration, screening, class sort
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
// G lanes per shell (64 / G shells per wavefront; G = 1, 2, 4 or 8 from the plan's longest
// contraction, so that a lane sums about eight of the K^2 terms of the norm): a butterfly inside
// the group leaves the same total on its G lanes, then lane k mod G writes w_k. Lanes past the
// last shell take part in the butterfly with nothing to add.
constexpr int kWeightLanesMax = 8;
__host__ __device__ constexpr int weight_lanes(int max_nprim) {
  return max_nprim * max_nprim <= 8 ? 1 : max_nprim * max_nprim <= 16 ? 2 : max_nprim * max_nprim <= 32 ? 4 : 8;
}
__device__ void prim_weights_of(const DevBasis& b, int s, int sub, int G) {
  const bool on = s < b.n_shells;
  const int l = on ? b.l[s] : 0, K = on ? b.nprim[s] : 0;
  const int64_t o = on ? b.prim_off[s] : 0;
  double ss = 0.0;
  for (int t = sub; t < K * K; t += G) {
    const int k = t / K, j = t - k * K;
    const double ak = b.expo[o + k], aj = b.expo[o + j];
    ss += b.coef[o + k] * b.coef[o + j] * pow_half_q(2.0 * ak, l) * pow_half_q(2.0 * aj, l) / pow_q(ak + aj, l);
  }
#pragma unroll
  for (int off = kWeightLanesMax / 2; off > 0; off >>= 1)
    if (off < G) ss += __shfl_xor(ss, off);
  if (!on) return;
  double dfac = 1.0;
  for (int i = 2 * l - 1; i > 1; i -= 2) dfac *= i;
  const double cn = sqrt(ldexp(1.0, l) / (dfac * 5.5683279968317078453));  // pi^{3/2}
  const double inv = 1.0 / sqrt(ss);
  for (int k = sub; k < K; k += G) b.w[o + k] = b.coef[o + k] * cn * pow_half_q(2.0 * b.expo[o + k], l) * inv;
}


// Classification in workgroups of 1024 candidates: the key of each candidate, its rank among
// the workgroup's candidates with the same key (LDS atomics), and one global atomic per
// (workgroup, key) that reserves the workgroup's range inside the key's bucket. Workgroups from
// classify_blocks on compute the shells' normalised primitive weights instead, a group of lanes
// per shell (independent work, in the same launch).
__global__ void __launch_bounds__(kClassifyThreads) k_classify(DevBasis bs, DevPairs pr, int classify_blocks,
                                                               int weight_lanes) {
  if ((int)blockIdx.x >= classify_blocks) {
    const int G = weight_lanes;
    const int s = ((int)blockIdx.x - classify_blocks) * (kClassifyThreads / G) + (int)(threadIdx.x / G);
    prim_weights_of(bs, s, threadIdx.x % G, G);
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
    const int K1 = bs.nprim[s1], K2 = bs.nprim[s2];
    if (!(pr.screen > 0.0)) {
      ns = K1 * K2;
    } else {
      const ScreenBand band = screen_band(pr.screen);
      for (int p = 0; p < K1; ++p) {
        const double a = bs.expo[o1 + p];
        for (int q = 0; q < K2; ++q) ns += keep_prim_banded(a, bs.expo[o2 + q], R2, pr.screen, band);
      }
    }
    key = pair_key(class_id(L1, L2), ns);
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

// Cost bucket of work item i: the class c whose items start at or below i, the item's block blk
// of tiles, and four buckets per octave of its estimate (schedule.h: item_iters, item_cost).
__device__ int item_bucket(int i, const int* ioff, const int* koff, const ClassMeta& meta, int& c, int& blk) {
  c = class_of_item(i, ioff);
  blk = i - ioff[c];
  const ItemGeom g = item_geom(koff, c, meta.tiles[c], blk);
  const int m = item_iters(koff, c, g);
  const float cost = item_cost(meta.weight[c], m, g.nt, item_tasks(g.nt, meta.groups[c], m));
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
    citems[t] = class_items(koff[(t + 1) * kKeysPerClass] - koff[t * kKeysPerClass], meta.tiles[t]);
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
  pr.nsurv[slot] = key_survivors(key);
  if (pr.full) {
    pr.dst0[slot] = bs.bf_off[sw ? b : a];
    pr.dst1[slot] = bs.bf_off[sw ? a : b];
  } else {
    pr.dst0[slot] = pr.blk_off[i];
    pr.dst1[slot] = sw ? 1 : 0;
  }
}

// Boys function F_0..F_M(t) exactly as the integral and gradient kernels evaluate it: the row of
// order M at the nearest grid point, the index clamped to the table, then boys_row.
template <int M>
__global__ void k_boys(int64_t n, const double* __restrict__ T, double* __restrict__ F,
                       const double* __restrict__ tab) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = T[i];
  const double* __restrict__ r = boys_row_ptr(tab, M, boys_index(t));  // index 0 .. kBoysPoints - 1
  double row[kBoysRowLoad];
#pragma unroll
  for (int k = 0; k < kBoysRowLoad; ++k) row[k] = r[k];
  double f[M + 1];
  boys_row<M>(t, row, f);
#pragma unroll
  for (int m = 0; m <= M; ++m) F[i * (M + 1) + m] = f[m];
}

__global__ void k_fill_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace

void launch_pair_build(const shgo_plan* p, hipStream_t st) {
  // key_count is zero here: cleared at plan creation and by every k_scan_keys after reading it
  const int cb = (int)((p->n_cand + kClassifyThreads - 1) / kClassifyThreads);
  const int G = weight_lanes(p->max_nprim);
  const int wb = (int)((p->n_shells + kClassifyThreads / G - 1) / (kClassifyThreads / G));
  hipLaunchKernelGGL(k_classify, dim3(cb + wb), dim3(kClassifyThreads), 0, st, p->bs, p->pr, cb, G);
  hipLaunchKernelGGL(k_scan_keys, dim3(1), dim3(1024), 0, st, p->pr, p->meta, p->item_off, p->items, p->queue);
  const int tb = 256;
  hipLaunchKernelGGL(k_scatter, dim3((int)((p->n_cand + tb - 1) / tb)), dim3(tb), 0, st, p->bs, p->pr);
}

void launch_weights(const shgo_plan* p, hipStream_t st) {
  const int G = weight_lanes(p->max_nprim);
  const int wb = (int)((p->n_shells + kClassifyThreads / G - 1) / (kClassifyThreads / G));
  if (wb > 0) hipLaunchKernelGGL(k_classify, dim3(wb), dim3(kClassifyThreads), 0, st, p->bs, p->pr, 0, G);
}

void launch_fill(double* ptr, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int tb = 256;
  hipLaunchKernelGGL(k_fill_f64, dim3((int)((n + tb - 1) / tb)), dim3(tb), 0, st, ptr, n);
}

hipError_t launch_boys(int mmax, int64_t n, const double* T, double* F, const double* tab, hipStream_t st) {
  const int tb = 256;
  const int nb = (int)((n + tb - 1) / tb);
  switch (mmax) {
#define SHGO_BOYS_CASE(M) \
  case M: hipLaunchKernelGGL(k_boys<M>, dim3(nb), dim3(tb), 0, st, n, T, F, tab); break;
    SHGO_BOYS_CASE(0) SHGO_BOYS_CASE(1) SHGO_BOYS_CASE(2) SHGO_BOYS_CASE(3) SHGO_BOYS_CASE(4)
    SHGO_BOYS_CASE(5) SHGO_BOYS_CASE(6) SHGO_BOYS_CASE(7) SHGO_BOYS_CASE(8) SHGO_BOYS_CASE(9)
    SHGO_BOYS_CASE(10) SHGO_BOYS_CASE(11) SHGO_BOYS_CASE(12) SHGO_BOYS_CASE(13) SHGO_BOYS_CASE(14) SHGO_BOYS_CASE(15)
#undef SHGO_BOYS_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace shgo_impl
