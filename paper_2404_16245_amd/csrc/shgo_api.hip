// Host side of the MI355X (gfx950) nuclear-attraction library: the C ABI of include/shgo.h,
// contexts, plans (one device workspace each), the single-call entry points and the autotuner.
#include "shgo_internal.h"

#include <cstdio>
#include <cstring>

#include "plan_host.h"

#include <memory>
#include <mutex>

namespace shgo_impl {

// Workspace of shgo_nuclear_attraction_noalloc: a file-scope device array, one copy per GPU, held
// until the process ends. In host code its name stands for nothing on the device: kernels and
// copies use the address hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t kScratchBytes = SHGO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {nullptr};

// The device address of `scratch` on `device` (current), looked up once per device.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}
}  // namespace

shgo_status fail(shgo_context* ctx, shgo_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

namespace {

// Boys table (rows of kBoysRow doubles, order M major): F_{M+k}(t_i)/k! for k < 8, e^{-t_i} as a
// high and a low double, with
// F_m(t) = e^{-t} sum_j (2t)^j / ((2m+1)(2m+3)...(2m+2j+1)) summed in long double (positive terms).
std::vector<double> boys_table() {
  constexpr int kOrders = kBoysMaxM + 8;
  std::vector<double> tab((size_t)(kBoysMaxM + 1) * kBoysPoints * kBoysRow, 0.0);
  std::vector<long double> F(kOrders);
  for (int i = 0; i < kBoysPoints; ++i) {
    const long double t = (long double)i / 16.0L;
    const long double et = expl(-t);
    for (int m = 0; m < kOrders; ++m) {
      long double term = 1.0L / (2 * m + 1), sum = term;
      for (int k = 1; k < 4000; ++k) {
        term *= 2.0L * t / (2 * m + 2 * k + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
      }
      F[m] = et * sum;
    }
    for (int M = 0; M <= kBoysMaxM; ++M) {
      double* row = &tab[((size_t)M * kBoysPoints + i) * kBoysRow];
      long double fact = 1.0L;
      for (int k = 0; k < 8; ++k) {
        if (k > 0) fact *= k;
        row[k] = (double)(F[M + k] / fact);
      }
      row[8] = (double)et;
      row[9] = (double)(et - (long double)row[8]);
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

constexpr int kTuneCandidates = 5;

void drop_graph(shgo_plan* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->graph_out = nullptr;
}


// The integral kernel's arguments (device copy, read through the scalar cache). item_ns turns the
// per-item timing of the kernel on (tuning runs) or off (null).
hipError_t upload_args(shgo_plan* p, unsigned long long* item_ns) {
  const WorkArgs wa{p->bs, p->pr, p->nuc, p->n_nuc, p->ctx->boys_tab, p->queue, p->item_off, p->items, item_ns, p->meta};
  return hipMemcpy(p->d_wa, &wa, sizeof(WorkArgs), hipMemcpyHostToDevice);
}

// Work items of the queue for the plan's candidate counts (an upper bound of the device count).
int64_t max_items_of(const shgo_plan* p) {
  int64_t n = 0;
  for (int c = 0; c < kNumClasses; ++c) n += class_items(p->class_cand[c], p->meta.tiles[c]);
  return n;
}

// The integral kernel of the plan's precision.
void launch_integrals(const shgo_plan* p, double* out, hipStream_t st) {
  if (p->precision == SHGO_PREC_MIXED)
    launch_integrals_mixed(p, out, st);
  else
    launch_integrals_fp64(p, out, st);
}

// The launches of one evaluation on `st`: pair build (a1), then the persistent integral kernel.
// With `timed`, HIP events bracket the two phases (never inside a graph capture).
void enqueue(shgo_plan* p, double* out, hipStream_t st, bool timed) {
  const int slot = timed && p->slots > 0 ? (int)(p->exec_count % p->slots) : -1;
  auto mark = [&](int phase, int edge) {
    if (slot >= 0) (void)hipEventRecord(p->events[((size_t)slot * SHGO_NUM_PHASES + phase) * 2 + edge], st);
  };
  mark(0, 0);
  launch_pair_build(p, st);
  mark(0, 1);  // also the start of phase 1: three event records per timed execution
  launch_integrals(p, out, st);
  mark(1, 1);
  if (slot >= 0) p->exec_count++;
}


// Point every device array of the plan into its workspace block (plan_host.h: plan_layout).
void carve(shgo_plan* p, const shgo_host::PlanLayout& L, char* base, int full) {
  using namespace shgo_host;
  auto at = [&](Buf b) { return (void*)(base + L.off[b]); };
  p->bs.center = (const double*)at(kCenter);
  p->bs.l = (const int32_t*)at(kL);
  p->bs.nprim = (const int32_t*)at(kNprim);
  p->bs.prim_off = (const int64_t*)at(kPoff);
  p->bs.bf_off = (const int64_t*)at(kBfOff);
  p->bs.by_l = (const int32_t*)at(kByL);
  p->bs.expo = (const double*)at(kExpo);
  p->bs.coef = (const double*)at(kCoef);
  p->bs.w = (double*)at(kW);
  p->bs.n_shells = p->n_shells;
  p->bs.nbf = p->nbf;
  p->nuc = (Nuc*)at(kNuc);
  DevPairs& pr = p->pr;
  pr.n_cand = p->n_cand;
  pr.full = full;
  pr.screen = p->screen;
  pr.pa = full ? nullptr : (const int32_t*)at(kPa);
  pr.pb = full ? nullptr : (const int32_t*)at(kPb);
  pr.blk_off = full ? nullptr : (const int64_t*)at(kBlk);
  pr.key = (int32_t*)at(kKey);
  pr.s1 = (int32_t*)at(kS1);
  pr.s2 = (int32_t*)at(kS2);
  pr.orig = (int32_t*)at(kOrig);
  pr.nsurv = (int32_t*)at(kNsurv);
  pr.rank = (int32_t*)at(kRank);
  pr.key_count = (int32_t*)at(kKeyCount);
  pr.key_off = (int32_t*)at(kKeyOff);
  pr.dst0 = (int64_t*)at(kDst0);
  pr.dst1 = (int64_t*)at(kDst1);
  p->queue = (int32_t*)at(kQueue);
  p->item_off = (int32_t*)at(kItemOff);
  p->items = (int32_t*)at(kItems);
  p->d_wa = (WorkArgs*)at(kArgs);
  p->d_energy = (double*)at(kEnergy);
}

// Host arithmetic of a plan: validation, counts, workspace layout, default schedule. Touches no
// device; `p` receives the counts and the schedule.
shgo_status plan_host_part(shgo_context* ctx, const shgo_basis* b, const shgo_nuclei* n, int full, int64_t n_pairs,
                           const int32_t* pa, const int32_t* pb, double screen, size_t scratch_limit, shgo_plan* p,
                           shgo_host::PlanCounts* pc_out, shgo_host::PlanLayout* lay_out) {
  std::string msg;
  shgo_status st = shgo_host::validate_inputs(b, n, screen, &msg);
  if (st == SHGO_OK) st = shgo_host::validate_pairs(b, full, n_pairs, pa, pb, &msg);
  if (st != SHGO_OK) return fail(ctx, st, msg);
  shgo_host::PlanCounts pc = shgo_host::plan_counts(b, full, n_pairs, pa, pb, screen);
  st = shgo_host::check_class_sizes(pc, &msg);
  if (st != SHGO_OK) return fail(ctx, st, msg);
  const shgo_host::PlanLayout lay = shgo_host::plan_layout(pc, b->n_shells, n->n_nuclei, full, sizeof(Nuc), sizeof(WorkArgs));
  if (scratch_limit > 0 && lay.total > scratch_limit)
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "device workspace of " + std::to_string(lay.total) +
                                                 " bytes exceeds the scratch limit of " + std::to_string(scratch_limit));
  p->ctx = ctx;
  p->full = full;
  p->n_shells = b->n_shells;
  for (int32_t i = 0; i < b->n_shells; ++i) p->max_nprim = std::max(p->max_nprim, b->n_prim[i]);
  for (int l = 0; l < SHGO_LMAX + 2; ++l) p->l_first[l] = pc.by_l[(size_t)l];
  p->n_nuc = n->n_nuclei;
  p->screen = screen;
  p->nbf = pc.nbf;
  p->n_cand = pc.n_cand;
  p->out_size = pc.out_size;
  p->integrals = pc.integrals;
  p->kept_pairs = pc.kept_pairs;
  p->kept_prim_pairs = pc.kept_prim_pairs;
  for (int c = 0; c < kNumClasses; ++c) p->class_cand[c] = (int)pc.class_cand[c];
  // persistent-kernel schedule: tiles per work item and the model weight of each class
  model_weights(n->n_nuclei, p->meta.weight);
  double slices[kNumClasses];
  shgo_host::mean_slices(b, full, n_pairs, pa, pb, slices);
  for (int c = 0; c < kNumClasses; ++c) {
    p->def_tiles[c] = shgo_host::default_tiles(c, slices[c]);
    p->meta.tiles[c] = p->def_tiles[c];
    p->meta.groups[c] = kClassGroups[c];
  }
  *pc_out = std::move(pc);
  *lay_out = lay;
  return SHGO_OK;
}

// Copies of the host inputs into the plan's workspace on `st` (synchronous copies when st is
// the null stream and `async` is false), and the cleared key counters.
hipError_t upload_inputs(shgo_plan* p, const shgo_basis* b, const shgo_nuclei* n, const shgo_host::PlanCounts& pc,
                         const int32_t* pa, const int32_t* pb, hipStream_t st) {
  hipError_t e = hipSuccess;
  auto up = [&](const void* d, const void* h, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync((void*)d, h, bytes, hipMemcpyHostToDevice, st);
  };
  const size_t ns = (size_t)b->n_shells, np = (size_t)pc.n_prims;
  up(p->bs.center, b->center, 24 * ns);
  up(p->bs.l, b->l, 4 * ns);
  up(p->bs.nprim, b->n_prim, 4 * ns);
  up(p->bs.prim_off, b->prim_offset, 8 * ns);
  up(p->bs.bf_off, pc.bf_off.data(), 8 * ns);
  up(p->bs.by_l, pc.by_l.data(), 4 * pc.by_l.size());
  up(p->bs.expo, b->exponent, 8 * np);
  up(p->bs.coef, b->coef, 8 * np);
  // nuclei {x, y, z, Z}: positions and charges strided into the 32-byte records
  if (e == hipSuccess && n->n_nuclei > 0) {
    e = hipMemcpy2DAsync(p->nuc, sizeof(Nuc), n->position, 3 * sizeof(double), 3 * sizeof(double),
                         (size_t)n->n_nuclei, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync((char*)p->nuc + 3 * sizeof(double), sizeof(Nuc), n->charge, sizeof(double), sizeof(double),
                           (size_t)n->n_nuclei, hipMemcpyHostToDevice, st);
  }
  if (!p->full) {
    up(p->pr.pa, pa, 4 * (size_t)p->n_cand);
    up(p->pr.pb, pb, 4 * (size_t)p->n_cand);
    up(p->pr.blk_off, pc.blk_off.data(), 8 * (size_t)p->n_cand);
  }
  // the key counters start at zero; every k_scan_keys clears them again after reading
  if (e == hipSuccess) launch_fill((double*)p->pr.key_count, (int64_t)kNumKeys / 2, st);
  // the primitive weights depend on the basis alone: computed here once (every pair build
  // computes them again, to the same values)
  if (e == hipSuccess) launch_weights(p, st);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

shgo_status make_plan(shgo_context* ctx, const shgo_basis* b, const shgo_nuclei* n, int full, int64_t n_pairs,
                      const int32_t* pa, const int32_t* pb, double screen, size_t scratch_limit, shgo_plan** out) {
  if (!ctx || !out) return fail(ctx, SHGO_ERR_INVALID_ARG, "null context or output pointer");
  *out = nullptr;
  shgo_plan* p = new shgo_plan();
  shgo_host::PlanCounts pc;
  shgo_host::PlanLayout lay;
  shgo_status st = plan_host_part(ctx, b, n, full, n_pairs, pa, pb, screen, scratch_limit, p, &pc, &lay);
  if (st != SHGO_OK) {
    delete p;
    return st;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete p;
    return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  }
  if (hipMalloc(&p->block, lay.total) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(lay.total) + " bytes failed");
  }
  p->block_bytes = lay.total;
  p->owns_block = true;
  carve(p, lay, (char*)p->block, full);
  hipError_t e = upload_inputs(p, b, n, pc, pa, pb, nullptr);
  if (e == hipSuccess) e = upload_args(p, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    shgo_plan_destroy(p);
    return fail(ctx, SHGO_ERR_DEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  }
  *out = p;
  return SHGO_OK;
}

// Bytes that identify a single call's inputs (plan reuse): the basis, the nuclei, the screen.
std::vector<char> call_key(const shgo_basis* b, const shgo_nuclei* n, double screen) {
  std::vector<char> k;
  auto put = [&](const void* src, size_t bytes) {
    const char* c = (const char*)src;
    k.insert(k.end(), c, c + bytes);
  };
  int64_t np = 0;
  for (int s = 0; s < b->n_shells; ++s) np = std::max<int64_t>(np, b->prim_offset[s] + b->n_prim[s]);
  put(&b->n_shells, sizeof(b->n_shells));
  put(&n->n_nuclei, sizeof(n->n_nuclei));
  put(&screen, sizeof(screen));
  put(b->center, 24 * (size_t)b->n_shells);
  put(b->l, 4 * (size_t)b->n_shells);
  put(b->n_prim, 4 * (size_t)b->n_shells);
  put(b->prim_offset, 8 * (size_t)b->n_shells);
  put(b->exponent, 8 * (size_t)np);
  put(b->coef, 8 * (size_t)np);
  put(n->position, 24 * (size_t)n->n_nuclei);
  put(n->charge, 8 * (size_t)n->n_nuclei);
  return k;
}

// The context's matrix plan for a single call with these inputs: reused when the inputs are
// byte-identical to the last call's, else made anew (the old one freed once the device is idle).
shgo_status call_plan(shgo_context* ctx, const shgo_basis* b, const shgo_nuclei* n, const shgo_options& o,
                      shgo_plan** out, bool* fresh) {
  std::string msg;
  shgo_status st = shgo_host::validate_options(&o, &msg);
  if (st != SHGO_OK) return fail(ctx, st, msg);
  st = shgo_host::validate_inputs(b, n, o.screen_threshold, &msg);
  if (st != SHGO_OK) return fail(ctx, st, msg);
  std::vector<char> key = call_key(b, n, o.screen_threshold);
  *fresh = false;
  if (ctx->call_plan && key == ctx->call_key) {
    if (o.scratch_limit_bytes > 0 && ctx->call_plan->block_bytes > o.scratch_limit_bytes)
      return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "device workspace of " + std::to_string(ctx->call_plan->block_bytes) +
                                                   " bytes exceeds the scratch limit of " +
                                                   std::to_string(o.scratch_limit_bytes));
    *out = ctx->call_plan;
    return SHGO_OK;
  }
  shgo_plan* p = nullptr;
  st = make_plan(ctx, b, n, 1, 0, nullptr, nullptr, o.screen_threshold, o.scratch_limit_bytes, &p);
  if (st != SHGO_OK) return st;
  if (ctx->call_plan) {
    (void)hipDeviceSynchronize();
    shgo_plan_destroy(ctx->call_plan);
  }
  ctx->call_plan = p;
  ctx->call_key = std::move(key);
  *out = p;
  *fresh = true;
  return SHGO_OK;
}

// Schedule file of the single call's autotune cache: a header line, then one line per class
// "class weight tiles". Returns 0 when the file does not exist, 1 when it was read, -1 when it
// exists but is not a schedule.
int read_schedule(const char* path, float* w, int32_t* t) {
  FILE* f = std::fopen(path, "r");
  if (!f) return 0;
  char head[64] = {0};
  int nc = 0;
  bool ok = std::fscanf(f, "%63s %d", head, &nc) == 2 && std::strcmp(head, "shgo-schedule") == 0 && nc == kNumClasses;
  for (int c = 0; ok && c < kNumClasses; ++c) {
    int ci = -1;
    ok = std::fscanf(f, "%d %f %d", &ci, &w[c], &t[c]) == 3 && ci == c;
  }
  std::fclose(f);
  return ok ? 1 : -1;
}

bool write_schedule(const char* path, const float* w, const int32_t* t) {
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "shgo-schedule %d\n", kNumClasses);
  for (int c = 0; c < kNumClasses; ++c) std::fprintf(f, "%d %.9g %d\n", c, (double)w[c], t[c]);
  return std::fclose(f) == 0;
}


}  // namespace
}  // namespace shgo_impl

using namespace shgo_impl;

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
  std::string why;
  // both forms of the integral kernel: launch guard, dynamic LDS, workgroups per CU (the same
  // launch bounds; the grid takes the smaller occupancy)
  int per_cu_mixed = 0;
  hipError_t ge = integrals_setup_fp64(&per_cu, &why);
  if (ge == hipSuccess) ge = integrals_setup_mixed(&per_cu_mixed, &why);
  per_cu = std::min(per_cu, per_cu_mixed);
  if (ge != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    if (!why.empty()) std::fprintf(stderr, "shgo_create: %s\n", why.c_str());
    shgo_destroy(c);
    return why.empty() ? SHGO_ERR_DEVICE : SHGO_ERR_INTERNAL;
  }
  c->n_cu = n_cu;
  c->grid = std::max(1, n_cu * std::max(1, per_cu));
  if (scratch_address(device, &c->scratch) != hipSuccess) {
    std::fprintf(stderr, "shgo_create: hipGetSymbolAddress of the scratch array failed\n");
    shgo_destroy(c);
    return SHGO_ERR_DEVICE;
  }
  *out = c;
  return SHGO_OK;
}

void shgo_destroy(shgo_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->call_plan) {
    (void)hipDeviceSynchronize();
    shgo_plan_destroy(ctx->call_plan);
  }
  if (ctx->boys_tab) (void)hipFree(ctx->boys_tab);
  if (ctx->eri_plan) shgo_plan_destroy(ctx->eri_plan);
  if (ctx->eri_dev) (void)hipFree(ctx->eri_dev);
  if (ctx->eri_pin) (void)hipHostFree(ctx->eri_pin);
  delete ctx;
}

shgo_status shgo_validate(const shgo_basis* basis, const shgo_nuclei* nuclei, double screen, char* msg,
                          size_t msg_len) {
  std::string err;
  const shgo_status s = shgo_host::validate_inputs(basis, nuclei, screen, &err);
  if (msg && msg_len > 0) {
    const std::string m = s == SHGO_OK ? std::string() : err;
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
  return make_plan(ctx, basis, nuclei, 1, 0, nullptr, nullptr, screen, 0, plan);
}

shgo_status shgo_plan_pairs(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei, int64_t n_pairs,
                            const int32_t* pair_a, const int32_t* pair_b, double screen, shgo_plan** plan) {
  return make_plan(ctx, basis, nuclei, 0, n_pairs, pair_a, pair_b, screen, 0, plan);
}

void shgo_plan_destroy(shgo_plan* p) {
  if (!p) return;
  if (p->ctx) (void)hipSetDevice(p->ctx->device);
  drop_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t ev : p->events) (void)hipEventDestroy(ev);
  if (p->owns_block && p->block) (void)hipFree(p->block);
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
  // a matrix plan's pairs are enumerated by class from the shells ordered by l and the primitive
  // weights were computed with the plan, so the kernels alone run; a pair plan's pairs come from
  // its pair build, as for V
  if (!p->full) launch_pair_build(p, st);
  launch_overlap(p, out, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

shgo_status shgo_execute_cartesian(shgo_plan* p, double* out, void* stream) {
  if (!p) return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!out && p->out_size > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  for (int c = 0; c < kNumClasses; ++c)
    if (p->class_cand[c] > 0 && class_la(c) > cart_lmax())
      return fail(ctx, SHGO_ERR_UNSUPPORTED_L,
                  "the Cartesian route takes shells up to l = " + std::to_string(cart_lmax()));
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  if (p->n_cand == 0) return SHGO_OK;
  hipStream_t st = (hipStream_t)stream;
  launch_pair_build(p, st);
  hipError_t e = launch_cartesian(p, out, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

// The quartets' block sizes, checked: SHGO_ERR_INVALID_ARG for a shell index out of range,
// SHGO_ERR_UNSUPPORTED_L for a shell above the two-electron path's l, at the first quartet that
// has one. Each quartet's first double in the output into offsets (when given), the total into
// *total.
static shgo_status eri_sizes(const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets, int64_t* offsets,
                             int64_t* total, std::string* err) {
  const int32_t nsh = basis->n_shells;
  std::vector<int32_t> dim((size_t)std::max(nsh, 1));
  for (int32_t sh = 0; sh < nsh; ++sh) dim[(size_t)sh] = basis->l[sh] > eri_lmax() ? -1 : 2 * basis->l[sh] + 1;
  int64_t t = 0;
  for (int64_t q = 0; q < n_quartets; ++q) {
    int64_t size = 1;
    for (int i = 0; i < 4; ++i) {
      const int32_t sh = quartets[4 * q + i];
      if (sh < 0 || sh >= nsh) {
        *err = "shell index out of range";
        return SHGO_ERR_INVALID_ARG;
      }
      if (dim[(size_t)sh] < 0) {
        *err = "the two-electron path takes shells up to l = " + std::to_string(eri_lmax());
        return SHGO_ERR_UNSUPPORTED_L;
      }
      size *= dim[(size_t)sh];
    }
    if (offsets) offsets[q] = t;
    t += size;
  }
  *total = t;
  return SHGO_OK;
}

shgo_status shgo_eri_output_size(const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets, int64_t* size) {
  if (size) *size = 0;
  if (!basis || !size || n_quartets < 0 || (n_quartets > 0 && !quartets)) return SHGO_ERR_INVALID_ARG;
  const shgo_nuclei none{0, nullptr, nullptr};
  std::string err;
  shgo_status s = shgo_host::validate_inputs(basis, &none, 0.0, &err);
  if (s != SHGO_OK) return s;
  int64_t total = 0;
  s = eri_sizes(basis, n_quartets, quartets, nullptr, &total, &err);
  if (s == SHGO_OK) *size = total;
  return s;
}

shgo_status shgo_eri_blocks(shgo_context* ctx, const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets,
                            double* out, void* stream) {
  if (!ctx) return SHGO_ERR_INVALID_ARG;
  if (!basis || n_quartets < 0 || (n_quartets > 0 && (!quartets || !out)))
    return fail(ctx, SHGO_ERR_INVALID_ARG, "null basis, quartets or output, or a negative count");
  const shgo_nuclei none{0, nullptr, nullptr};
  std::string err;
  shgo_status s = shgo_host::validate_inputs(basis, &none, 0.0, &err);
  if (s != SHGO_OK) return fail(ctx, s, err);
  std::unique_ptr<int64_t[]> offsets(new int64_t[(size_t)std::max<int64_t>(n_quartets, 1)]);
  int64_t total = 0;
  s = eri_sizes(basis, n_quartets, quartets, offsets.get(), &total, &err);
  if (s != SHGO_OK) return fail(ctx, s, err);
  if (n_quartets == 0 || basis->n_shells == 0) return SHGO_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  // a pair plan of one pair uploads the basis and computes its primitive weights; the context
  // keeps it for the next call with a byte-identical basis
  std::vector<char> key = call_key(basis, &none, 0.0);
  if (!ctx->eri_plan || key != ctx->eri_key) {
    if (ctx->eri_plan) {
      shgo_plan_destroy(ctx->eri_plan);  // the last call waited for its stream
      ctx->eri_plan = nullptr;
    }
    const int32_t zero = 0;
    shgo_plan* np = nullptr;
    s = make_plan(ctx, basis, &none, 0, 1, &zero, &zero, 0.0, 0, &np);
    if (s != SHGO_OK) return s;
    ctx->eri_plan = np;
    ctx->eri_key = std::move(key);
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = run_eri(ctx->eri_plan, basis, n_quartets, quartets, offsets.get(), out, st);
  if (e == hipErrorOutOfMemory) return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "no device memory for the two-electron workspace");
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("two-electron evaluation failed: ") + hipGetErrorString(e));
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
  const int64_t nmax = max_items_of(p);
  unsigned long long* ticks = nullptr;
  if (hipMalloc(&ticks, 2 * sizeof(unsigned long long) * (size_t)std::max<int64_t>(nmax, 1)) != hipSuccess)
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "tuning buffer");
  std::vector<unsigned long long> th(2 * (size_t)std::max<int64_t>(nmax, 1));
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
    e = hipMemcpy(th.data(), ticks, 2 * sizeof(unsigned long long) * (size_t)n_items, hipMemcpyDeviceToHost);
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
    const ItemGeom g = item_geom(koff.data(), c, model.tiles[c], blk);
    const int m = item_iters(koff.data(), c, g);
    const int tasks = item_tasks(g.nt, kClassGroups[c], m);
    sum_ns[c] += 10.0 * (double)th[2 * (size_t)q + 1];
    units[c] += (double)m * g.nt / std::min(kWaves, tasks);
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
  shgo_status s = grad_classes(p, ga, st, false);  // LDS limits, before any device work
  if (s != SHGO_OK) return s;
  launch_fill(dE_dnuclei, (int64_t)3 * p->n_nuc, st);
  launch_fill(dE_dcenters, (int64_t)3 * p->n_shells, st);
  launch_fill(e_out, 1, st);
  if (p->n_cand > 0 && p->n_nuc > 0) {
    launch_pair_build(p, st);  // shell-pair build (a1), as for the integrals
    s = grad_classes(p, ga, st, true);
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
  if (n < 0 || mmax < 0 || mmax > kBoysMaxM || (n > 0 && (!T || !F)))
    return fail(ctx, SHGO_ERR_INVALID_ARG, "bad Boys arguments (0 <= mmax <= " + std::to_string(kBoysMaxM) + ")");
  if (n == 0) return SHGO_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  const hipError_t e = launch_boys(mmax, n, T, F, ctx->boys_tab, (hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}


void shgo_options_default(shgo_options* o) {
  if (!o) return;
  o->precision = SHGO_PREC_FP64;
  o->screen_threshold = 0.0;
  o->use_graph = 0;
  o->autotune_cache = nullptr;
  o->scratch_limit_bytes = 0;
}

shgo_status shgo_check_call(const shgo_basis* basis, const shgo_nuclei* nuclei, const shgo_options* options,
                            shgo_plan_info* info, char* msg, size_t msg_len) {
  shgo_options o;
  shgo_options_default(&o);
  if (options) o = *options;
  std::string err;
  shgo_status s = shgo_host::validate_options(&o, &err);
  if (s == SHGO_OK) s = shgo_host::validate_inputs(basis, nuclei, o.screen_threshold, &err);
  if (s == SHGO_OK) s = shgo_host::validate_pairs(basis, 1, 0, nullptr, nullptr, &err);
  if (s == SHGO_OK) {
    const shgo_host::PlanCounts pc = shgo_host::plan_counts(basis, 1, 0, nullptr, nullptr, o.screen_threshold);
    s = shgo_host::check_class_sizes(pc, &err);
    if (s == SHGO_OK) {
      const shgo_host::PlanLayout lay =
          shgo_host::plan_layout(pc, basis->n_shells, nuclei->n_nuclei, 1, sizeof(Nuc), sizeof(WorkArgs));
      if (info) {
        info->candidate_pairs = pc.n_cand;
        info->kept_pairs = pc.kept_pairs;
        info->kept_prim_pairs = pc.kept_prim_pairs;
        info->integrals = pc.integrals;
        info->output_size = pc.out_size;
        info->nbf = pc.nbf;
        info->workspace_bytes = lay.total;
      }
      if (o.scratch_limit_bytes > 0 && lay.total > o.scratch_limit_bytes) {
        s = SHGO_ERR_OUT_OF_MEMORY;
        err = "device workspace of " + std::to_string(lay.total) + " bytes exceeds the scratch limit of " +
              std::to_string(o.scratch_limit_bytes);
      }
    }
  }
  if (msg && msg_len > 0) {
    const std::string m = s == SHGO_OK ? std::string() : err;
    const size_t k = std::min(msg_len - 1, m.size());
    std::memcpy(msg, m.data(), k);
    msg[k] = 0;
  }
  return s;
}

shgo_status shgo_nuclear_attraction(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                                    const shgo_options* options, double* V, void* stream) {
  if (!ctx) return SHGO_ERR_INVALID_ARG;
  shgo_options o;
  shgo_options_default(&o);
  if (options) o = *options;
  if (!basis || !nuclei) return fail(ctx, SHGO_ERR_INVALID_ARG, "null basis or nuclei");
  if (!V && shgo_nbf(basis) > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  // a schedule file is read (or found absent or malformed) before any device work
  float w[kNumClasses];
  int32_t t[kNumClasses];
  const int r = o.autotune_cache ? read_schedule(o.autotune_cache, w, t) : 0;
  if (r < 0) return fail(ctx, SHGO_ERR_INVALID_ARG, std::string("not a schedule file: ") + o.autotune_cache);
  shgo_plan* p = nullptr;
  bool fresh = false;
  shgo_status s = call_plan(ctx, basis, nuclei, o, &p, &fresh);
  if (s != SHGO_OK) return s;
  s = shgo_plan_set_precision(p, o.precision);
  if (s != SHGO_OK) return s;
  if (o.autotune_cache && p->n_cand > 0 && p->schedule_file != o.autotune_cache) {
    if (r > 0) {
      s = shgo_plan_set_schedule(p, w, t);
      if (s != SHGO_OK) return s;
    } else {
      s = shgo_plan_autotune(p, V, 5, stream, nullptr, nullptr);
      if (s != SHGO_OK) return s;
      if (!write_schedule(o.autotune_cache, p->meta.weight, p->meta.tiles))
        return fail(ctx, SHGO_ERR_INVALID_ARG, std::string("cannot write the autotune cache ") + o.autotune_cache);
    }
    p->schedule_file = o.autotune_cache;
  }
  return o.use_graph ? shgo_execute_graph(p, V, stream) : shgo_execute(p, V, stream);
}

shgo_status shgo_nuclear_attraction_grad(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                                         const shgo_options* options, const double* D, double* dE_dnuclei,
                                         double* dE_dcenters, void* stream) {
  if (!ctx) return SHGO_ERR_INVALID_ARG;
  shgo_options o;
  shgo_options_default(&o);
  if (options) o = *options;
  if (o.precision != SHGO_PREC_FP64) return fail(ctx, SHGO_ERR_INVALID_ARG, "the gradient is evaluated in FP64 only");
  shgo_plan* p = nullptr;
  bool fresh = false;
  const shgo_status s = call_plan(ctx, basis, nuclei, o, &p, &fresh);
  if (s != SHGO_OK) return s;
  return shgo_execute_grad(p, D, dE_dnuclei, dE_dcenters, nullptr, stream);
}

shgo_status shgo_plan_item_profile(shgo_plan* p, double* out, int32_t max_items, int32_t* items, double* start_us,
                                   double* duration_us, int32_t* n_items, void* stream) {
  if (!p || !n_items || max_items < 0 || (max_items > 0 && (!items || !start_us || !duration_us)))
    return SHGO_ERR_INVALID_ARG;
  shgo_context* ctx = p->ctx;
  if (!out && p->out_size > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  *n_items = 0;
  if (p->n_cand == 0) return SHGO_OK;
  hipStream_t st = (hipStream_t)stream;
  drop_graph(p);
  const int64_t nmax = std::max<int64_t>(max_items_of(p), 1);
  unsigned long long* ticks = nullptr;
  if (hipMalloc(&ticks, 2 * sizeof(unsigned long long) * (size_t)nmax) != hipSuccess)
    return fail(ctx, SHGO_ERR_OUT_OF_MEMORY, "profiling buffer");
  int32_t n = 0;
  std::vector<unsigned long long> th(2 * (size_t)nmax);
  std::vector<int32_t> it((size_t)nmax);
  hipError_t e = upload_args(p, ticks);
  if (e == hipSuccess) {
    enqueue(p, out, st, false);
    e = hipStreamSynchronize(st);
  }
  if (e == hipSuccess) e = hipMemcpy(&n, p->item_off, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess && (n < 0 || n > nmax)) e = hipErrorUnknown;
  if (e == hipSuccess && n > 0) {
    e = hipMemcpy(th.data(), ticks, 2 * sizeof(unsigned long long) * (size_t)n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(it.data(), p->items, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost);
  }
  (void)hipFree(ticks);
  const hipError_t e2 = upload_args(p, nullptr);
  if (e != hipSuccess || e2 != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "profiling run failed");
  unsigned long long t0 = ~0ull;
  for (int q = 0; q < n; ++q) t0 = std::min(t0, th[2 * (size_t)q]);
  *n_items = n;
  for (int q = 0; q < std::min(n, max_items); ++q) {
    items[q] = it[(size_t)q];
    start_us[q] = 0.01 * (double)(th[2 * (size_t)q] - t0);  // wall clock: 100 MHz
    duration_us[q] = 0.01 * (double)th[2 * (size_t)q + 1];
  }
  return SHGO_OK;
}

shgo_status shgo_nuclear_attraction_noalloc(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                                            const shgo_options* options, double* V, void* stream) {
  if (!ctx) return SHGO_ERR_INVALID_ARG;
  shgo_options o;
  shgo_options_default(&o);
  if (options) o = *options;
  if (!basis || !nuclei) return fail(ctx, SHGO_ERR_INVALID_ARG, "null basis or nuclei");
  std::string msg;
  shgo_status st = shgo_host::validate_options(&o, &msg);
  if (st != SHGO_OK) return fail(ctx, st, msg);
  if (o.precision != SHGO_PREC_FP64 || o.use_graph || o.autotune_cache)
    return fail(ctx, SHGO_ERR_INVALID_ARG, "the allocation-free call takes FP64, no graph and no autotune cache");
  if (!V && shgo_nbf(basis) > 0) return fail(ctx, SHGO_ERR_INVALID_ARG, "null output");
  if (!ctx->scratch) return fail(ctx, SHGO_ERR_DEVICE, "no scratch address for this device");
  const size_t limit = o.scratch_limit_bytes > 0 ? std::min(o.scratch_limit_bytes, kScratchBytes) : kScratchBytes;
  // the plan lives on the stack and its workspace in the static scratch: nothing is allocated
  shgo_plan p;
  shgo_host::PlanCounts pc;
  shgo_host::PlanLayout lay;
  st = plan_host_part(ctx, basis, nuclei, 1, 0, nullptr, nullptr, o.screen_threshold, limit, &p, &pc, &lay);
  if (st != SHGO_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
  if (p.n_cand == 0) return SHGO_OK;
  p.owns_block = false;
  p.block = ctx->scratch;
  p.block_bytes = lay.total;
  carve(&p, lay, (char*)ctx->scratch, 1);
  hipStream_t st_ = (hipStream_t)stream;
  // inputs, cleared key counters and the kernel's arguments into the scratch on the caller's
  // stream; the wait lets the host arrays go once the call returns
  hipError_t e = upload_inputs(&p, basis, nuclei, pc, nullptr, nullptr, st_);
  const WorkArgs wa{p.bs, p.pr, p.nuc, p.n_nuc, ctx->boys_tab, p.queue, p.item_off, p.items, nullptr, p.meta};
  if (e == hipSuccess) e = hipMemcpyAsync(p.d_wa, &wa, sizeof(WorkArgs), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  enqueue(&p, V, st_, false);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SHGO_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return SHGO_OK;
}

shgo_status shgo_plan_get_info(const shgo_plan* p, shgo_plan_info* info) {
  if (!p || !info) return SHGO_ERR_INVALID_ARG;
  info->candidate_pairs = p->n_cand;
  info->kept_pairs = p->kept_pairs;
  info->kept_prim_pairs = p->kept_prim_pairs;
  info->integrals = p->integrals;
  info->output_size = p->out_size;
  info->nbf = p->nbf;
  info->workspace_bytes = p->block_bytes;
  return SHGO_OK;
}

shgo_status shgo_plan_set_precision(shgo_plan* p, int32_t precision) {
  if (!p) return SHGO_ERR_INVALID_ARG;
  if (precision != SHGO_PREC_FP64 && precision != SHGO_PREC_MIXED)
    return fail(p->ctx, SHGO_ERR_INVALID_ARG, "unknown precision");
  if (precision != p->precision) {
    if (hipSetDevice(p->ctx->device) != hipSuccess) return fail(p->ctx, SHGO_ERR_DEVICE, "hipSetDevice failed");
    drop_graph(p);  // a captured graph holds the other form's kernel
    p->precision = precision;
  }
  return SHGO_OK;
}

}  // extern "C"
