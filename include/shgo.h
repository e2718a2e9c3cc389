/* shgo.h -- C ABI of the MI355X (gfx950) library for one-electron nuclear-attraction integrals
 * over contracted solid-harmonic Gaussian orbitals (SHGOs).
 *
 * Method: Hu, Peslherbe, Ooi and Hu, "Computationally Efficient Molecular Integrals of Solid
 * Harmonic Gaussian Orbitals Using Quantum Entanglement of Angular Momentum" (arXiv:2404.16245).
 * A shell is a center, an angular momentum l and K primitives (exponents, contraction
 * coefficients) as in Eq. 1; nuclei are point charges at positions c (the operator of Eq. 11).
 * The result is V_{(a,ma),(b,mb)} = -sum_c Z_c int chi_{a,ma}(r) chi_{b,mb}(r) / |r - c| d^3r
 * in the real solid-harmonic basis (Eq. 2 normalisation, order m = -l..l; l = 1 is y, z, x).
 * Every step of the evaluation -- primitive normalisation, shell-pair enumeration, screening,
 * class sort, Gaussian product (Eq. 5), shift to P (Eqs. 7-8), product rule (supplement Eq. 4),
 * one-center integral with the Boys function (Eqs. 11-12), sum over nuclei, contraction and
 * scatter -- runs in device kernels; the host only validates and copies inputs at plan time.
 *
 * Conventions
 *   - Units are atomic (bohr, hartree).
 *   - Basis functions are numbered shell by shell: index = offset(shell) + m + l.
 *   - Primitive normalisation N(l,a)^2 = 2^l (2a)^{l+3/2} / ((2l-1)!! pi^{3/2}); the caller's
 *     contraction coefficients multiply normalised primitives and the contracted shell is
 *     renormalised to unit self-overlap (the paper names N in Eq. 1 but does not give it).
 *   - Ownership: the caller owns every buffer passed in. Plan creation copies the host inputs
 *     to device memory owned by the plan; nothing passed in is retained.
 *   - Streams: stream arguments are hipStream_t values (NULL = the null stream). Work is
 *     enqueued asynchronously; the caller synchronises.
 *   - Errors: every call that can fail returns shgo_status (SHGO_OK == 0); the context keeps a
 *     message for the last failure (shgo_last_error). Validation happens on the host before any
 *     device work and nothing is written on a validation error. After SHGO_ERR_DEVICE the
 *     output contents are unspecified.
 *   - A context or plan is not thread-safe; use one per host thread.
 */
#ifndef SHGO_H
#define SHGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHGO_LMAX 7 /* highest supported angular momentum of a shell */

typedef enum {
  SHGO_OK = 0,
  SHGO_ERR_INVALID_ARG = 1,   /* null pointer, negative count, exponent <= 0, bad index */
  SHGO_ERR_UNSUPPORTED_L = 2, /* l < 0 or l > SHGO_LMAX */
  SHGO_ERR_NOT_FINITE = 3,    /* NaN or Inf in a coordinate, exponent, coefficient or charge */
  SHGO_ERR_OUT_OF_MEMORY = 4, /* device allocation failed */
  SHGO_ERR_DEVICE = 5,        /* HIP runtime or kernel launch error */
  SHGO_ERR_INTERNAL = 6
} shgo_status;

typedef struct shgo_context shgo_context; /* device tables (Boys interpolation table) */
typedef struct shgo_plan shgo_plan;       /* device copies of one basis + nuclei + workspace */

/* Basis set in host memory (read during plan creation only). */
typedef struct {
  int32_t n_shells;
  const double* center;       /* [n_shells][3] */
  const int32_t* l;           /* [n_shells], 0..SHGO_LMAX */
  const int32_t* n_prim;      /* [n_shells], >= 1 */
  const int64_t* prim_offset; /* [n_shells], first primitive of each shell in exponent/coef */
  const double* exponent;     /* [total primitives], > 0 */
  const double* coef;         /* [total primitives], coefficients of normalised primitives */
} shgo_basis;

/* Point nuclei in host memory (read during plan creation only). */
typedef struct {
  int32_t n_nuclei;        /* >= 0; zero nuclei gives V = 0 */
  const double* position;  /* [n_nuclei][3] */
  const double* charge;    /* [n_nuclei] (Z) */
} shgo_nuclei;

/* Arithmetic of the integral evaluation.
 *   SHGO_PREC_FP64   binary64 throughout.
 *   SHGO_PREC_MIXED  the product rule (Supplement Eq. 4) and the shift back to the two centers
 *                    (Eq. 7, Eq. 11) of each primitive pair -- the coupling of the nucleus sums
 *                    W(L,M,k) into the block -- in binary32 double-float arithmetic (every value an
 *                    unevaluated pair hi + lo of floats; products by TwoProd, sums by TwoSum) for
 *                    classes with both l <= 4; the nucleus sums (Eq. 11 last line, Eq. 12), the
 *                    Boys function, exp(-mu R^2) (Eq. 5), the contraction prefactors and the sum
 *                    over primitive pairs stay binary64, and so does the coupling of classes with
 *                    an l above 4. Measured against the FP64 oracle: about 1e-12 absolute and
 *                    1e-11 RMS relative per element (1e-10 in the worst elements of the 200-atom
 *                    molecule). On MI355X binary32 scalar arithmetic issues at the binary64 rate
 *                    (packed binary32 is not used), so the mixed form is slower than FP64 here. */
typedef enum { SHGO_PREC_FP64 = 0, SHGO_PREC_MIXED = 1 } shgo_precision;

/* Options of the single-call entry points (shgo_nuclear_attraction, shgo_nuclear_attraction_grad).
 * shgo_options_default fills: FP64, no screening, no graph, no autotune cache, no scratch limit. */
typedef struct {
  int32_t precision;          /* shgo_precision */
  double screen_threshold;    /* drop primitive pairs with exp(-ab/(a+b)|A-B|^2) <= it; 0 keeps all */
  int32_t use_graph;          /* nonzero: replay the evaluation as a captured HIP graph (V only) */
  const char* autotune_cache; /* NULL, or the path of a schedule file for the call's plan: read
                                 if it exists (a file that is not a schedule: SHGO_ERR_INVALID_ARG
                                 before any device work), else the plan is autotuned and the file
                                 written; done once per plan and path (V only) */
  size_t scratch_limit_bytes; /* 0: no limit; else SHGO_ERR_OUT_OF_MEMORY, before any device work,
                                 when the call's device workspace would exceed it */
} shgo_options;

void shgo_options_default(shgo_options* options);

/* Create a context on HIP device `device` (tables are built on the host and uploaded).
 * Returns SHGO_ERR_DEVICE if the device cannot be used. */
shgo_status shgo_create(int device, shgo_context** ctx);
void shgo_destroy(shgo_context* ctx);

const char* shgo_status_string(shgo_status s);
const char* shgo_last_error(const shgo_context* ctx);

/* Number of basis functions sum_s (2 l_s + 1); -1 on invalid input. Host only. */
int64_t shgo_nbf(const shgo_basis* basis);

/* The host-side validation that plan creation performs, without touching a device.
 * Returns the status plan creation would return for these inputs and, when msg is not NULL,
 * copies a NUL-terminated message of at most msg_len bytes into it. */
shgo_status shgo_validate(const shgo_basis* basis, const shgo_nuclei* nuclei, double screen, char* msg,
                          size_t msg_len);


/* V = -sum_c Z_c int chi_a chi_b / |r - c| (Eq. 11 with the Boys function of Eq. 12), the full
 * symmetric nbf x nbf matrix in one call: validates, copies the inputs to the device, builds the
 * shell pairs, and evaluates on `stream` into the device buffer V (nbf * nbf doubles, row-major,
 * every element written). The context keeps the plan of its last call: a call with byte-identical
 * inputs and options reuses it (no copies; its tuned schedule and captured graph); a call with
 * others first waits for the device, then replaces it.
 *   options  NULL: shgo_options_default.
 * Errors before any device work, with V untouched: SHGO_ERR_INVALID_ARG / _UNSUPPORTED_L /
 * _NOT_FINITE as for shgo_validate; SHGO_ERR_OUT_OF_MEMORY when the workspace would exceed
 * options->scratch_limit_bytes or the device allocation fails. */
shgo_status shgo_nuclear_attraction(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                                    const shgo_options* options, double* V, void* stream);

/* dE/d(nuclear positions) and dE/d(shell centers) of E = sum_ij D_ij V_ij in one call (the adjoint
 * of Eq. 11 through Eq. 5, the shift of Eqs. 7-8, the product rule and the Boys function):
 *   D            device, nbf x nbf row-major
 *   dE_dnuclei   device [n_nuclei][3], overwritten
 *   dE_dcenters  device [n_shells][3], overwritten
 * Plan reuse, options and errors as for shgo_nuclear_attraction (use_graph and autotune_cache do
 * not apply; precision must be SHGO_PREC_FP64). */
shgo_status shgo_nuclear_attraction_grad(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                                         const shgo_options* options, const double* D, double* dE_dnuclei,
                                         double* dE_dcenters, void* stream);

/* The single call of shgo_nuclear_attraction without any device allocation, for callers that
 * cannot allocate (work under HIP graph capture setup, tight serving loops, harnesses that forbid
 * hipMalloc). Its whole workspace -- device copies of the inputs, keys, sorted pairs, work queue and
 * kernel arguments, plan_host layout -- lives in one static device array of
 * SHGO_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; it calls no hipMalloc, hipFree
 * or allocating library routine. It copies the inputs on `stream` and waits for that stream before
 * launching (so the host arrays may go when it returns); V is then written asynchronously.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race, and must be ordered by the caller.
 * options: FP64 only, use_graph = 0, autotune_cache = NULL (SHGO_ERR_INVALID_ARG otherwise); the
 * default schedule; scratch_limit_bytes, when nonzero, caps the workspace further.
 * SHGO_ERR_OUT_OF_MEMORY, before any device work, when the workspace (shgo_check_call's
 * workspace_bytes) exceeds the array (about 800,000 candidate shell pairs). Other errors as for
 * shgo_nuclear_attraction. */
#define SHGO_NOALLOC_SCRATCH_BYTES (32u << 20)
shgo_status shgo_nuclear_attraction_noalloc(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                                            const shgo_options* options, double* V, void* stream);

/* Plan for the full symmetric matrix V (nbf x nbf, row-major) over every shell pair a <= b.
 * screen > 0 drops primitive pairs with exp(-ab/(a+b) |A-B|^2) <= screen (0 keeps all; a pair
 * whose primitive pairs are all dropped gives a zero block).  Validates the inputs, copies them
 * to the device and allocates the plan's workspace. Size limits (SHGO_ERR_INVALID_ARG): at most
 * 2^31 - 1 candidate shell pairs in all and 2^30 in one (l_a, l_b) class. */
shgo_status shgo_plan_matrix(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                             double screen, shgo_plan** plan);

/* Plan for an explicit list of shell pairs (pair_a[i], pair_b[i]), host arrays of n_pairs
 * shell indices. The output holds the blocks back to back in list order, block i being
 * (2 l_a + 1) x (2 l_b + 1) row-major (rows follow shell pair_a[i]). The same size limits as
 * for shgo_plan_matrix apply to the list. */
shgo_status shgo_plan_pairs(shgo_context* ctx, const shgo_basis* basis, const shgo_nuclei* nuclei,
                            int64_t n_pairs, const int32_t* pair_a, const int32_t* pair_b, double screen,
                            shgo_plan** plan);

void shgo_plan_destroy(shgo_plan* plan);

/* Number of doubles the plan writes (nbf*nbf for a matrix plan, sum of block sizes otherwise). */
int64_t shgo_plan_output_size(const shgo_plan* plan);

/* Number of integrals one execution computes: sum of (2 l_a + 1)(2 l_b + 1) over the plan's shell
 * pairs that keep at least one primitive pair (all of them without screening; unique pairs a <= b
 * for a matrix plan). The other shell pairs' blocks are written as zeros. */
int64_t shgo_plan_integrals(const shgo_plan* plan);

/* Sizes of a plan. kept_*: after screening (the same rule as the kernels, evaluated on the host). */
typedef struct {
  int64_t candidate_pairs;  /* shell pairs of the plan (a <= b, or the list) */
  int64_t kept_pairs;       /* shell pairs with at least one surviving primitive pair */
  int64_t kept_prim_pairs;  /* surviving primitive pairs */
  int64_t integrals;        /* as shgo_plan_integrals */
  int64_t output_size;      /* as shgo_plan_output_size */
  int64_t nbf;
  size_t workspace_bytes;   /* the plan's device workspace */
} shgo_plan_info;
shgo_status shgo_plan_get_info(const shgo_plan* plan, shgo_plan_info* info);

/* The host-side checks of a single call (shgo_nuclear_attraction / _grad with these inputs and
 * options), without touching a device: input validation, the options, and the scratch limit
 * against the device workspace the call needs. When `info` is not NULL and the inputs are valid,
 * it receives the sizes of the matrix plan the call would make. Returns the status the call would
 * return before any device work; `msg` (or NULL) receives a NUL-terminated message of at most
 * msg_len bytes. */
shgo_status shgo_check_call(const shgo_basis* basis, const shgo_nuclei* nuclei, const shgo_options* options,
                            shgo_plan_info* info, char* msg, size_t msg_len);

/* Run the whole evaluation on `stream`, writing the plan's output into the device buffer `out`
 * (shgo_plan_output_size doubles; every element is written). Allocates nothing. */
shgo_status shgo_execute(shgo_plan* plan, double* out, void* stream);

/* Arithmetic of the plan's integral evaluation (shgo_execute, shgo_execute_graph):
 * SHGO_PREC_FP64 (the default) or SHGO_PREC_MIXED (see shgo_precision). SHGO_ERR_INVALID_ARG for
 * an unknown value. A change drops the plan's captured graph (the next shgo_execute_graph captures
 * the other kernel). The overlap and gradient evaluations are FP64 whatever the setting. */
shgo_status shgo_plan_set_precision(shgo_plan* plan, int32_t precision);

/* The overlap matrix S of the plan's shells (Eqs. 4-10: the Gaussian product, the shift of both
 * harmonics to P, and the single-center overlap, which the orthogonality of the harmonics
 * reduces to one term per (lambda, m)), over every primitive pair (the plan's screening threshold
 * does not apply), written into the device buffer `out` in the layout shgo_execute gives V:
 * nbf x nbf row-major for a matrix plan, the listed blocks for a pair plan. The nuclei play no
 * part. Runs on `stream`, allocates nothing; SHGO_ERR_INVALID_ARG for a null plan or output. */
shgo_status shgo_execute_overlap(shgo_plan* plan, double* out, void* stream);

/* The same V as shgo_execute by the Cartesian route the paper compares against (Table 1, the
 * Cartesian column): McMurchie-Davidson over Cartesian Gaussians -- the Hermite expansion of each
 * primitive-pair product about P, the Hermite Coulomb integrals R_tuv from the Boys function
 * summed over nuclei, their contraction -- then the transform to the real solid harmonics of the
 * plan's basis (Eq. 1 normalisation and contraction, the plan's screening). Provided to compare
 * the two routes on one GPU; shells up to l = 4 (SHGO_ERR_UNSUPPORTED_L otherwise, before any
 * device work). Writes the layout shgo_execute writes, on `stream`, allocating nothing; FP64. */
shgo_status shgo_execute_cartesian(shgo_plan* plan, double* out, void* stream);

/* Two-electron Coulomb integrals (ab|cd) = int int chi_a chi_b (r1) chi_c chi_d (r2) / |r1 - r2| over
 * the basis (Eq. 1 normalisation and contraction), by the solid-harmonic route of Eqs. 13-15: the
 * Gaussian product of each pair, the shifts to P and Q (Eq. 7) and the product rule (Supplement
 * Eq. 4) in the pair frames, and the two-center integral between the pairs' terms in closed form
 * (Hobson's theorem on the solid-harmonic gradients, the product rule applied to them, the Boys
 * function of pq/(p+q) |P-Q|^2). No screening.
 *   quartets   host [n_quartets][4] shell indices (a, b, c, d), any order within each pair
 *   out        device, the blocks in quartet order, each (2la+1)(2lb+1)(2lc+1)(2ld+1) doubles
 *              row-major in the listed shell order (a slowest)
 * Shells up to l = 2 (SHGO_ERR_UNSUPPORTED_L otherwise); SHGO_ERR_INVALID_ARG for a shell index
 * out of range; both before any device work. Uploads the basis (kept by the context for the next
 * call with a byte-identical basis), the quartets' distinct shell pairs and their
 * per-primitive-pair records (the pairs' expansions, built once per pair) to a device workspace
 * that the context keeps for its next call, with a pinned host copy of its index part (each grown
 * when a call needs more, freed by shgo_destroy; SHGO_ERR_OUT_OF_MEMORY if it cannot be
 * allocated), runs on `stream` and waits for it before returning. */
shgo_status shgo_eri_blocks(shgo_context* ctx, const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets,
                            double* out, void* stream);

/* Doubles that shgo_eri_blocks writes for these quartets: the sum over them of
 * (2la+1)(2lb+1)(2lc+1)(2ld+1), into *size. Host only (no context, no device). The same checks
 * as shgo_eri_blocks, in the same order: SHGO_ERR_INVALID_ARG for a null basis or size, a
 * negative count, null quartets with a positive count or a shell index out of range;
 * SHGO_ERR_UNSUPPORTED_L for a shell above l = 2. *size is 0 unless SHGO_OK. */
shgo_status shgo_eri_output_size(const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets, int64_t* size);

/* Gradient of E = sum_ij D_ij V_ij (the nuclear-attraction matrix of Eq. 11, differentiated
 * through Eq. 5, the shift of Eqs. 7-8, the product rule and the Boys function; an adjoint
 * kernel, not finite differences) with respect to the nuclear positions and the shell centers.
 * Matrix plans only (SHGO_ERR_INVALID_ARG for a pair plan).
 *   D            device, nbf x nbf row-major (any matrix; only D_ij V_ij enters E)
 *   dE_dnuclei   device [n_nuclei][3], overwritten
 *   dE_dcenters  device [n_shells][3], overwritten
 *   energy       device [1], overwritten with E, or NULL
 * Runs on `stream` and allocates nothing. The work needs 8 (3 n_nuclei + 4 S) bytes of LDS per
 * workgroup, S a per-class layout of at most ~2.9k doubles; SHGO_ERR_INVALID_ARG if that
 * exceeds the 160 KB of a CU (about 2,800 nuclei for l <= 6, 1,300 with l = 7 shells), before
 * any device work. */
shgo_status shgo_execute_grad(shgo_plan* plan, const double* D, double* dE_dnuclei, double* dE_dcenters,
                              double* energy, void* stream);

/* The same evaluation as a captured HIP graph. The first call for a given `out` captures the
 * launches of shgo_execute on a private stream and instantiates the graph (HIP allocates then);
 * later calls with the same `out` only launch it on `stream`. A call with another `out`, and
 * shgo_plan_set_schedule / shgo_plan_autotune, replace the graph. The graph holds no memset
 * nodes (buffers are cleared by fill kernels) and no timing events. */
shgo_status shgo_execute_graph(shgo_plan* plan, double* out, void* stream);

/* Work schedule of the persistent launch, one entry per class id c = la(la+1)/2 + lb (la >= lb).
 * A work item is a block of tiles[c] tiles of 64 class-sorted shell pairs, run by one workgroup:
 * its eight wavefronts take (tile, slice of at most 8 primitive-pair iterations, group) tasks and
 * add into one LDS accumulator. Items are dispatched longest first, by the estimate
 * weight[c] x (primitive-pair iterations of the item's longest tile) x (its tiles) / (the
 * wavefronts its tasks keep busy, at most 8).
 *   weight[36] relative time of one primitive-pair iteration of a tile of the class, 1..1e6 (the
 *              default comes from an operation-count model, largest 1024)
 *   tiles[36]  tiles per work item of each class, 1 <= tiles[c] <= shgo_max_tiles(c) (the LDS of
 *              a work item holds per tile (2la+1)(2lb+1) x 65 accumulator doubles and 256 frame
 *              doubles, at most 20448 doubles in all). A new plan's default is the fewest tiles
 *              that give the eight wavefronts eight tasks, from the class's groups and its mean
 *              slices per pair, ceil(K_a K_b / 8) capped at 8, over its candidate pairs.
 * get copies the plan's schedule out; set validates (SHGO_ERR_INVALID_ARG) and installs one, e.g. a
 * schedule saved from an earlier autotune of the same workload. Results do not depend on the
 * schedule beyond rounding. */
#define SHGO_NUM_CLASSES 36
int32_t shgo_max_tiles(int32_t class_id); /* -1 for an invalid class id */
shgo_status shgo_plan_get_schedule(const shgo_plan* plan, float* weight, int32_t* tiles);
shgo_status shgo_plan_set_schedule(shgo_plan* plan, const float* weight, const int32_t* tiles);

/* Autotuner of the batched launch. Runs the plan once with the model weights, the default tiles
 * and per-item timing, which measures each class's time per unit of the item estimate; builds
 * SHGO_TUNE_CANDIDATES schedules -- 0: the model weights with the default tiles; 1: the measured
 * weights with the default tiles; 2: the measured weights with twice the default tiles where the
 * LDS allows; 3: the measured weights with one tile per item; 4: the measured weights with half the
 * default tiles (at least one) -- times `rounds` executions of each on `stream` (the call
 * synchronizes the stream), and keeps the fastest. It then refines that schedule class by class
 * (one tile more or less, twice or half a class's tiles; a change is kept when it is more than
 * 0.5% faster, confirmed by a second timing beside the incumbent's; at most three passes) and installs
 * the result.
 * ms[SHGO_TUNE_CANDIDATES] (or NULL) receives each candidate's milliseconds per execution, *chosen
 * (or NULL) the index of the candidate the refinement started from. `out` is written as by
 * shgo_execute. */
#define SHGO_TUNE_CANDIDATES 5
shgo_status shgo_plan_autotune(shgo_plan* plan, double* out, int32_t rounds, void* stream, double* ms,
                               int32_t* chosen);

/* Per-item profile of the persistent launch: runs one execution of the plan (written to `out`)
 * with each work item timed on the device wall clock, synchronizes `stream`, and returns the
 * number of items in *n_items and, for the first max_items of them in dispatch order, the item
 * (class << 24 | tile block), its start relative to the first item's (microseconds) and its
 * duration (microseconds). Allocates a timing buffer. Shows how far the longest items set the
 * kernel's length. */
shgo_status shgo_plan_item_profile(shgo_plan* plan, double* out, int32_t max_items, int32_t* items, double* start_us,
                                   double* duration_us, int32_t* n_items, void* stream);

/* Phase timing. With n_slots > 0, every later shgo_execute records HIP events at the bounds of
 * its two phases -- 0: pair build (normalisation, enumeration, screening, class sort, work
 * queue), 1: the integral kernel (one persistent launch over every class); three events per
 * execution, the end of phase 0 being the start of phase 1 -- cycling through n_slots sets of
 * events; n_slots = 0 turns recording off. */
#define SHGO_NUM_PHASES 2
shgo_status shgo_plan_set_timing(shgo_plan* plan, int32_t n_slots);

/* After the caller has synchronised the stream: per phase, the summed milliseconds over the
 * recorded executions still held in the slots (ms[SHGO_NUM_PHASES]) and how many those are. */
shgo_status shgo_plan_phase_ms(shgo_plan* plan, double* ms, int32_t* count);

/* Boys function F_m(t) = int_0^1 u^{2m} exp(-t u^2) du for m = 0..mmax (the radial factor of
 * Eq. 12), evaluated by the device routine the integral kernels use.  T: device array of n
 * values t >= 0; F: device array [n][mmax+1].  mmax <= 15 (2 SHGO_LMAX + 1). */
shgo_status shgo_boys(shgo_context* ctx, int64_t n, const double* T, int32_t mmax, double* F, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SHGO_H */
