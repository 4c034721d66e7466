/*
 * dsfft.h -- C ABI of the MI355X (gfx950) batched power-of-two FFT whose every
 * radix-2 stage runs the dual-select six-FMA butterfly.
 *
 * Method: M. A. Bergach, "Dual-Select FMA Butterfly for FFT: Eliminating Twiddle
 * Factor Singularities with Bounded Precomputed Ratios", arXiv 2604.00567.
 *
 * Transform (Sec. I, eq. (1)): forward and unnormalised,
 *     X[k] = sum_{n<N} x[n] W^{nk},   W = exp(-j 2 pi / N),
 * computed as log2(N) radix-2 Stockham DIT passes; pass s (span L = 2^s) pairs
 * a = Y[r][j] with b = Y[r + N/L][j] and forms A = a + W^{jN/L} b, B = a - W^{jN/L} b
 * with exactly six FMAs (eqs. (berg-s)-(berg-B) on the cosine path,
 * eqs. (lf-s)-(lf-B) on the sine path, each FMA rounded once in the working
 * precision).  The twiddle table decides the path per twiddle (Algorithm 1).
 *
 * Data layout: interleaved complex, transform-contiguous.  Element n of
 * transform b sits at index b*N + n; an element is (re, im) as two binary16
 * values (FFT_F16 and FFT_F16_F32, 4 bytes) or two binary32 values (FFT_F32,
 * 8 bytes).
 * Input and output use the same layout, output in natural frequency order.
 *
 * Pointers named in/out are device pointers (HBM), owned by the caller and
 * aligned to the element size.  in == out (in place) is allowed; partial overlap is not.
 * Streams are hipStream_t values passed as void* (NULL = the null stream).
 *
 * Errors: functions returning int give FFT_OK (0) or a negative code; those
 * returning a pointer give NULL on error.  fft_last_error() returns a
 * thread-local message for the last error on the calling thread.  No call
 * aborts the process on a user error.
 */
#ifndef DSFFT_H
#define DSFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FFT_OK = 0, FFT_EINVAL = -1, FFT_ENOMEM = -2, FFT_EHIP = -3, FFT_EUNSUPPORTED = -4 };

/*
 * Storage and arithmetic precision of data and table.  FFT_F16_F32 (plans
 * only; the precision variant the paper's discussion of mixed precision
 * suggests, Sec. VI): binary16 storage in HBM, binary32 butterflies with the
 * binary32 table.  Each input element is widened exactly, every pass computes
 * in binary32 (LDS exchanges and the two-pass intermediate included), and each
 * output element is rounded once, to nearest even, to binary16: the result is
 * the FFT_F32 transform of the widened input, rounded once.  Uneven batches and
 * serving slots take FFT_F16 or FFT_F32.
 */
typedef enum { FFT_F16 = 0, FFT_F32 = 1, FFT_F16_F32 = 2 } fft_dtype;

/*
 * Twiddle-table kind (Sec. II-III):
 *   FFT_TABLE_DUAL_SELECT  Algorithm 1: per twiddle, cosine factorisation
 *                          (mult cos, ratio tan) when |cos| >= |sin|, else the
 *                          sine one (mult sin, ratio cot); |ratio| <= 1 (Theorem).
 *   FFT_TABLE_LINZER_FEIG  sine factorisation everywhere, sin clamped to +1e-7
 *                          where |sin| < 1e-7 (the clamp named in Sec. I).
 *   FFT_TABLE_COSINE       cosine factorisation everywhere (Sec. II-C).
 *   FFT_TABLE_LF_W0_EXEMPT Linzer-Feig with the W^0 entry taken on the cosine
 *                          path (no clamp needed); a finite comparison table.
 */
typedef enum {
    FFT_TABLE_DUAL_SELECT = 0,
    FFT_TABLE_LINZER_FEIG = 1,
    FFT_TABLE_COSINE = 2,
    FFT_TABLE_LF_W0_EXEMPT = 3
} fft_table_kind;

/* Transform direction, as the sign of the exponent: FFT_FORWARD computes
 * X[k] = sum_n x[n] exp(-j 2 pi n k / N) (eq. (1)); FFT_INVERSE computes
 * x[n] = sum_k X[k] exp(+j 2 pi n k / N), unnormalised (a round trip returns
 * N times the input).  The inverse uses the same butterflies and kernels with
 * the table built by the same rules from the conjugate twiddles W^{-k}: on
 * the cosine path (mult, ratio) becomes (mult, -ratio), on the sine path
 * (-mult, -ratio).  The paper uses the inverse only for its round-trip error
 * (Sec. V); which inverse it uses is not stated, this one is the reading. */
enum { FFT_FORWARD = -1, FFT_INVERSE = 1 };

typedef struct fft_plan fft_plan;     /* opaque; immutable after creation   */
typedef struct fft_batch fft_batch;   /* opaque uneven-size batch plan      */
typedef struct fft_serve_slot fft_serve_slot;   /* one in-flight serving launch */

/* Message for the last error on this thread ("" if none).  Never NULL. */
const char* fft_last_error(void);

/*
 * Builds a plan for `batch` transforms of size n (power of two, 2 <= n <= 2^20,
 * batch >= 1).  Generates the table of `kind` in FP64 on the host (Algorithm 1:
 * theta = -(2 pi k)/N, cos/sin, the |cos| >= |sin| select, the ratio division),
 * rounds mult and ratio once to `dtype`, and uploads it to HBM (shared across
 * plans of the same dtype and kind).  Chooses the kernel configuration (tuned
 * record if one exists, else a fixed rule) and, for n beyond one workgroup's
 * LDS, a two-pass schedule with a plan-owned workspace.
 * Returns NULL on error (FFT_EINVAL for bad arguments, FFT_ENOMEM, FFT_EHIP).
 */
fft_plan* fft_plan_create(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind);

/* Same, in the given direction (FFT_FORWARD or FFT_INVERSE; anything else is
 * FFT_EINVAL).  fft_plan_create(...) is fft_plan_create_dir(..., FFT_FORWARD). */
fft_plan* fft_plan_create_dir(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind,
                              int direction);

/*
 * Enqueues the plan's batched transform (forward FFT, or the inverse for a
 * plan made with FFT_INVERSE) out = FFT(in) on `stream` and returns
 * without synchronising.  in/out: device pointers of batch*n elements each.
 * A plan must not run concurrently on two streams (its workspace is shared).
 * Returns FFT_OK, FFT_EINVAL (null plan/pointer, misalignment, partial overlap)
 * or FFT_EHIP (launch failure; message in fft_last_error()).
 */
int fft_execute(fft_plan* plan, const void* in, void* out, void* stream);

/* Size of the library's fixed device scratch array (64 MiB per GPU). */
#define FFT_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate device memory while they run transforms
 * (code under HIP graph capture, tight serving loops, hosts that forbid
 * hipMalloc): fft_execute with no allocation of any kind.  The result is
 * bit-identical to fft_execute's (same kernels).  A two-pass plan's
 * intermediate goes through the library's fixed device array of
 * FFT_SCRATCH_BYTES per GPU, floor(FFT_SCRATCH_BYTES / (n * w)) transforms at
 * a time (w = 4 bytes for FFT_F16, 8 for FFT_F32 and FFT_F16_F32), instead of
 * the plan's workspace; single-pass plans use no scratch.  The array is
 * allocated with the library's code on each GPU and held until the process
 * ends; its device address is looked up on the first call with a device
 * current.  Every element of the scratch is written before it is read, so no
 * clearing is needed.  All calls on one GPU share its array: two calls of
 * two-pass plans that overlap in time on one GPU (on different streams, or
 * from different threads) race and give wrong results; calls on one stream
 * are ordered and safe.  The plan's device must be current.
 * Returns FFT_OK, FFT_EINVAL (as fft_execute; also a plan of another device,
 * or one transform whose intermediate exceeds FFT_SCRATCH_BYTES) or FFT_EHIP.
 */
int fft_execute_scratch(fft_plan* plan, const void* in, void* out, void* stream);

/* Frees the plan.  A two-pass plan that owns its workspace first waits until
 * the device has finished all work enqueued so far (its launches may still use
 * the workspace); other plans hold no device memory that their launches read
 * or write (twiddle tables are shared and live until the process ends), so
 * they return at once and launches already enqueued complete normally.
 * NULL-safe. */
void fft_destroy(fft_plan* plan);

/*
 * Host-only (no GPU needed): the table of `kind` for size n rounded to `dtype`,
 * k in [0, n/2).  mult_out/ratio_out receive n/2 values of the dtype's storage
 * type (uint16 binary16 bits or float), path_out n/2 bytes (0 cosine, 1 sine).
 * Any output pointer may be NULL.  Returns FFT_OK or FFT_EINVAL.
 */
int fft_table_build(int64_t n, fft_dtype dtype, fft_table_kind kind,
                    void* mult_out, void* ratio_out, uint8_t* path_out);

/* Same for a direction (FFT_FORWARD or FFT_INVERSE). */
int fft_table_build_dir(int64_t n, fft_dtype dtype, fft_table_kind kind, int direction,
                        void* mult_out, void* ratio_out, uint8_t* path_out);

/* The plan's parameters and its kernel choice, for tests and reports.
 * config_out receives a NUL-terminated description (up to `cap` bytes):
 * "mode:nu=2^a,e=2^b,upw=U,r=[r0,r1,r2],stg=S,lane=L,pipe=P,t=T,lds=B"
 * (mode small / cols / rows; a unit of 2^a points, 2^b elements per lane, U
 * units per workgroup, register passes of radix 2^r0, 2^r1, 2^r2; S = 1:
 * 16-byte LDS-staged I/O; L = 1: last two stages across lanes; T threads and
 * B bytes of LDS per workgroup), then ",upl=K" when a lane holds K units,
 * ",enc=select" / ",enc=branch" for the path-encoding variants, and for a
 * two-pass plan " | rows:... | chunk=C" (its second kernel, and the
 * transforms per workspace chunk).  P says where
 * twiddles come from besides per-lane table loads: 1 persistent workgroups
 * with a second register set, 2 the next pass's twiddles loaded a pass
 * ahead, 3 an LDS copy for the passes many lanes share (a whole transform's
 * middle pass, a column unit's later passes, a row unit's first pass), 4 an
 * LDS copy for every pass after the first, 5 as 3 plus 2 for the last pass.
 * All variants produce bit-identical results. */
int fft_plan_info(const fft_plan* plan, int64_t* n, int64_t* batch, int* dtype, int* kind,
                  char* config_out, size_t cap);

/* Bytes of device workspace the plan uses (0 for single-pass sizes). */
int fft_plan_workspace_bytes(const fft_plan* plan, size_t* bytes);

/*
 * Replaces the plan-owned workspace by caller memory (device pointer of at
 * least fft_plan_workspace_bytes bytes, 16-byte aligned), e.g. from torch's
 * allocator; the plan's own workspace is freed once the device has finished
 * the work enqueued so far.  The caller keeps its memory alive while the plan
 * may run.
 */
int fft_plan_set_workspace(fft_plan* plan, void* dev_ptr, size_t bytes);

/*
 * Same as fft_plan_create but with an explicit kernel choice, for the tuner and
 * for tests that compare configurations: variant_a / variant_b index the
 * compiled configurations for the size (single kernel, or the column / row
 * kernels of the two-pass schedule); two_pass = 1 forces the two-pass schedule
 * where a single kernel would fit.  Returns NULL (FFT_EUNSUPPORTED) when no
 * such configuration exists.
 */
fft_plan* fft_plan_create_variant(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind,
                                  int variant_a, int variant_b, int two_pass);

/*
 * Radix-4 form of the method (Sec. VI, generality: in a radix-r butterfly each
 * twiddle multiplication picks its own bounded-ratio factorisation).  A plan
 * for the same transform computed in the canonical radix-4 order: when log2 n
 * is odd, one radix-2 stage of span 2 (the six-FMA butterfly of W^0) comes
 * first; then radix-4 Stockham DIT stages of span L = 4, 16, ... (or 8, 32,
 * ...) up to n.  The stage of span L combines, for r < n/L and j < L/4, the
 * four span-L/4 results a, b, c, d at residues r + p n/L (p < 4) into
 *   Y[r][j] = (a + W2 c) + (W1 b + W3 d),    Y[r][j + L/2]  = (a + W2 c) - (W1 b + W3 d),
 *   Y[r][j + L/4] = (a - W2 c) - i (W1 b - W3 d), Y[r][j + 3L/4] = (a - W2 c) + i (W1 b - W3 d)
 * (W1 = W_L^j, W2 = W1^2, W3 = W1^3; the inverse swaps the last two places)
 * with 22 FMAs, each rounded once: W^k x = m_k h_k(x) through the table entry
 * of W^k (mult m_k, ratio t_k, path by Algorithm 1's rules for `kind`; two FMAs
 * each), u = a +- m2 h_c, and the odd pair W1 b +- W3 d = M (h_big +- rho
 * h_small) with M the larger of |m1|, |m3| and rho = smaller / larger computed
 * in FP64 and rounded once (|rho| <= 1), then Y = u +- M g.  Results differ
 * from the radix-2 plans (another rounding order); they equal the oracle's
 * radix-4 emulation bit for bit.  Whole transforms only: n = 2 .. 2^13
 * (FFT_EUNSUPPORTED beyond, and for FFT_F16_F32).  `variant` = -1 takes the
 * default configuration, else the variant-th radix-4 configuration of the
 * size (fft_config_count_radix4).  Executed with fft_execute.  NULL on error.
 */
fft_plan* fft_plan_create_radix4(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind,
                                 int direction, int variant);

/* Number of compiled radix-4 configurations for (n, dtype) (0 for
 * FFT_F16_F32).  FFT_EINVAL for n not a power of two in [2, 2^20], a null
 * count or an unknown dtype. */
int fft_config_count_radix4(int64_t n, fft_dtype dtype, int* count);

/*
 * Host-only radix-4 table export for size n (4 <= n <= 2^20, power of two):
 * mult_out / ratio_out / path_out receive the rounded entries of W^k for
 * k < 3n/4 (as fft_table_build, which stops at n/2), rho_out / sel_out per
 * column j < n/4 of the last stage the rounded rho and the choice of the outer
 * multiplier (1: m(W^j), 0: m(W^3j)).  Any output pointer may be NULL.
 */
int fft_table_build_radix4(int64_t n, fft_dtype dtype, fft_table_kind kind, int direction,
                           void* mult_out, void* ratio_out, uint8_t* path_out, void* rho_out,
                           uint8_t* sel_out);

/*
 * Autotuner: times every compiled configuration for (n, dtype) -- register-
 * pass radices (fusion depth), units per workgroup (LDS tile), elements per
 * lane (waves per transform), LDS staging, cross-lane tail, single-kernel or
 * two-pass -- on `batch` synthetic transforms with HIP events (`reps` timed
 * executions each), accepts a candidate only if its output is bit-identical
 * to the first configuration that runs (the default one, unless it fails),
 * and records the fastest: later
 * fft_plan_create calls for this (n, dtype) in the process use it, and the
 * record is appended to the file named by the DSFFT_TUNE_FILE environment
 * variable (read back at the first plan creation of a process).  `report`
 * receives a JSON array of the candidates' timings (up to `cap` bytes).
 */
int fft_tune(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind, int reps,
             char* report, size_t cap);

/* The recorded tuning choice for (n, dtype); FFT_EINVAL if none. */
int fft_tuned_choice(int64_t n, fft_dtype dtype, int* variant_a, int* variant_b, int* two_pass);

/* Number of compiled configurations for (n, dtype): *single for the
 * one-kernel schedule, *cols and *rows for the two kernels of the two-pass one
 * (each output may be NULL).  FFT_EINVAL for n not a power of two in
 * [2, 2^20] or an unknown dtype. */
int fft_config_count(int64_t n, fft_dtype dtype, int* single, int* cols, int* rows);

/*
 * Uneven-size batch: `count` transforms with sizes n[i] (powers of two,
 * 2 .. 2^18), packed back to back in the order given (transform i starts at
 * element sum_{j<i} n[j]).  Every transform is computed exactly as
 * fft_plan_create would (same butterflies, same table), but all of them run
 * in two persistent work-queue kernels: sizes up to 2^14 as whole-transform
 * work items, larger ones as the column items and row items of the two-pass
 * schedule.  The first kernel runs every column item and every
 * whole-transform item, the second every row item; the launch boundary
 * orders each transform's row items after its column items.  Binary16
 * transforms of 2^16 and 2^15 points (256 and 128 KiB, more than the batch
 * kernel's LDS) run whole in two list kernels of their own, one transform per
 * 1024-thread workgroup, over lists of their offsets, concurrently with the
 * first (graph branches with no dependency: the transforms are disjoint).  The
 * launches form one HIP graph built at the first execute and replayed by
 * every execute (the kernels leave their work-queue counters at zero for the
 * next replay); new data pointers are set on the graph's kernel nodes.  The
 * batch owns a workspace of the summed sizes of its two-pass transforms.
 * Returns NULL on error.
 */
fft_batch* fft_batch_create(const int64_t* n, int64_t count, fft_dtype dtype, fft_table_kind kind);

/* Same, with the tuner's choice per size class: choice_1024 / choice_4096
 * select the alternative configuration (0 or 1) for N = 2^10 / 2^12. */
fft_batch* fft_batch_create_tuned(const int64_t* n, int64_t count, fft_dtype dtype,
                                  fft_table_kind kind, int choice_1024, int choice_4096);

/* Same, with a choice per size class: alt[m] = 1 takes the alternative
 * configuration of the 2^m-point class (alt has 15 entries, m = 0 .. 14;
 * classes 2^7 .. 2^12 have one: another radix split, units per workgroup and
 * elements per lane), 0 its default; NULL takes every default. */
fft_batch* fft_batch_create_classes(const int64_t* n, int64_t count, fft_dtype dtype,
                                    fft_table_kind kind, const int32_t* alt);

/* Tuner for the uneven batch: for each size class with an alternative
 * configuration (2^7 .. 2^12), times a batch of that class alone with both
 * (2^24 elements, `reps` graph replays, outputs required to be bit-identical)
 * and sets alt_out[m] (15 entries) to 1 where the alternative is faster, for
 * fft_batch_create_classes. */
int fft_batch_tune_classes(fft_dtype dtype, fft_table_kind kind, int reps, int32_t* alt_out);

/* The 2^10 and 2^12 choices of fft_batch_tune_classes (0 or 1 each), for
 * fft_batch_create_tuned. */
int fft_batch_tune(fft_dtype dtype, fft_table_kind kind, int reps, int* choice_1024,
                   int* choice_4096);

/* Enqueues the whole uneven batch on `stream` (device pointers, packed
 * layout, element-aligned; in == out allowed).  Async. */
int fft_batch_execute(fft_batch* batch, const void* in, void* out, void* stream);

/* Total elements of the packed layout. */
int fft_batch_elements(const fft_batch* batch, int64_t* elements);

/* Work items, persistent grid size (the larger of the two kernels') and
 * workspace bytes of the batch. */
int fft_batch_info(const fft_batch* batch, int64_t* items, int64_t* grid, size_t* workspace_bytes);

/* Waits until the device has finished the work enqueued so far (the batch's
 * launches included), then frees it.  NULL-safe. */
void fft_batch_destroy(fft_batch* batch);

/* The work list an uneven batch of sizes n[0..count) and `dtype` would run
 * (host only, no device call), for inspection and tests.  Transforms are
 * packed in order (offsets are prefix sums).  items_out receives 8 int64 per
 * item: config id, units, first unit (whole-transform items: first index into
 * offs_out; column and row items: first column or row), log2 of the
 * column/row count, phase (0: first kernel, 1: second kernel), large-transform
 * index (-1 for whole-transform items), input offset, output offset (column
 * items write, and row items read, the workspace).  The first *phase0 items
 * are phase 0.  offs_out receives the transform offsets of the
 * whole-transform items, list_out those of the transforms run by the list
 * kernels (binary16 2^16-point transforms first, then 2^15-point ones, each
 * in input order).  nitems, phase0, noffs, nlist and ws_elems (workspace elements) are
 * always set; with all output pointers NULL the call only reports the sizes;
 * FFT_EINVAL when a capacity is too small. */
int fft_batch_work_list(const int64_t* n, int64_t count, fft_dtype dtype, int64_t* items_out,
                        int64_t item_cap, int64_t* nitems, int64_t* phase0, int64_t* offs_out,
                        int64_t offs_cap, int64_t* noffs, int64_t* list_out, int64_t list_cap,
                        int64_t* nlist, int64_t* ws_elems);

/*
 * Serving slot: the device and pinned buffers for one in-flight launch of the
 * uneven-batch kernels over the requests admitted in one scheduling step of a
 * continuous-batching server (the same butterflies and tables as every other
 * entry point).  Capacities: max_items work items, max_transforms
 * whole transforms (work items and list kernels together), max_large
 * transforms that take the column/row split (binary16 2^17 and 2^18 points,
 * binary32 2^15 and up), and ws_bytes of workspace for them.  Returns NULL on
 * error.
 */
fft_serve_slot* fft_serve_slot_create(fft_dtype dtype, fft_table_kind kind, int64_t max_items,
                                      int64_t max_transforms, int max_large, size_t ws_bytes);

/*
 * Enqueues requests r < nreq on `stream`: batch[r] transforms of n[r] points
 * (powers of two, 2 .. 2^18) each, transformed in place at element offsets
 * off[r] + j * n[r] of the device buffer `data`.  First waits for the slot's
 * previous launch.  FFT_ENOMEM if the step exceeds the slot's capacities.
 */
int fft_serve_slot_launch(fft_serve_slot* slot, const int64_t* n, const int64_t* batch,
                          const int64_t* off, int64_t nreq, void* data, void* stream);

/* 1 if the slot's last launch has finished (or none was made), 0 if running,
 * negative on error. */
int fft_serve_slot_query(fft_serve_slot* slot);

/* Waits for the slot's last launch, then frees it.  NULL-safe. */
void fft_serve_slot_destroy(fft_serve_slot* slot);

/*
 * Native serving loops (the continuous-batching server and its comparison)
 * over an arrival trace.  Requests r < count arrive at t[r] seconds (non-
 * decreasing, from the loop's start) and ask for batch[r] transforms of n[r]
 * points (powers of two, 2 .. 2^18) in dtype[r] (FFT_F16 or FFT_F32); their
 * data are generated on the device (fft_serve_fill, keyed by the seed and the
 * request's position among the requests of its precision, in arrival order),
 * transformed forward with the `kind` table and, when out_dev is not NULL,
 * copied to out_dev + out_off[r] bytes (for checks).  done_t[r] receives the
 * host time, in seconds from the loop's start, at which the request's
 * completion was observed.
 *   FFT_SERVE_CONTINUOUS  `slots` in-flight steps on as many streams.  Each
 *       turn retires finished steps, then admits waiting requests in arrival
 *       order into every free slot while each fits the HBM budget (request bytes
 *       in and out, plus workspace for split transforms, on top of the bytes in
 *       flight) and the slot's capacities (slot_bytes of data per precision,
 *       max_transforms whole transforms, max_large split ones, max_items work
 *       items of the slot's kernels as their work list would hold them,
 *       max_step_requests requests), generates the step's data and runs
 *       one step per precision: the serving-slot kernels (fft_serve_slot_launch),
 *       or for a step of at most direct_max requests one cached-plan launch per
 *       request (two-pass plans on a workspace of the slot); with split_direct
 *       the step's split transforms (those the slot kernels would split into
 *       column and row items) take their cached plans in every step.  Steps on
 *       different slots overlap on the device.
 *   FFT_SERVE_PER_REQUEST one cached plan (per shape and stream) and one launch
 *       per request, round-robin over `slots` streams, admitted in arrival
 *       order under the same budget (request data in a ring of
 *       max(slot_bytes, largest request) bytes per stream).
 * Returns FFT_OK, FFT_EINVAL (bad arguments, or a request that can never be
 * admitted), FFT_ENOMEM or FFT_EHIP; stats (may be NULL) receives the steps,
 * direct steps, mean requests per step, peak bytes in flight, peak concurrent
 * steps and the wall time from the first arrival to the last completion.
 */
enum { FFT_SERVE_CONTINUOUS = 0, FFT_SERVE_PER_REQUEST = 1 };
typedef struct {
    int mode;                  /* FFT_SERVE_CONTINUOUS or FFT_SERVE_PER_REQUEST */
    int slots;                 /* in-flight steps (continuous) or streams (per request), 1 .. 64 */
    int kind;                  /* fft_table_kind */
    int direct_max;            /* continuous: plan-launched steps of at most this many requests */
    int max_step_requests;
    int max_large;             /* split transforms per step and precision */
    int64_t max_transforms;    /* whole transforms per step and precision */
    int64_t max_items;         /* work items per step and precision */
    size_t budget_bytes;       /* HBM admission budget */
    size_t slot_bytes;         /* data bytes per slot and precision (continuous); ring size (per request) */
    uint64_t seed;             /* payload generator key */
    int split_direct;          /* continuous: nonzero = split transforms always run through their
                                  cached plans (two-pass ones on the slot's workspace), after the
                                  step's whole-size requests, whose completion is observed on an
                                  event of its own; zero = they run in the slot's kernels with
                                  the rest */
} fft_serve_config;
typedef struct {
    int64_t steps, direct_steps;
    double mean_requests_per_step;
    uint64_t max_inflight_bytes;
    int max_concurrent;
    double wall_s;
} fft_serve_stats;
int fft_serve_run(const fft_serve_config* cfg, const double* t, const int64_t* n, const int64_t* batch,
                  const int32_t* dtype, int64_t count, double* done_t, fft_serve_stats* stats,
                  void* out_dev, const int64_t* out_off);

/* The payload generator of the serving loops: complex elements first ..
 * first + elems - 1 of precision `dtype`'s stream, written to `data` (device,
 * interleaved re/im): each is one Box-Muller pair of N(0, 1) values from a
 * Philox4x32-10 draw keyed by `seed` and the element's index, rounded once to
 * the precision.  Enqueued on `stream`. */
int fft_serve_fill(fft_dtype dtype, void* data, int64_t elems, uint64_t first, uint64_t seed, void* stream);

/* Host only: the requests the continuous loop would admit into one step, from
 * position `head` of a trace whose requests have all arrived, with
 * inflight_bytes already in flight (the rule of FFT_SERVE_CONTINUOUS above).
 * taken receives up to cfg->max_step_requests request indices, *ntaken their
 * number, *inflight_out the bytes in flight after them.  Returns FFT_EINVAL
 * for a null argument, a negative head or count, a size that is not a power
 * of two in [2, 2^18], a batch below 1 or a dtype other than FFT_F16/FFT_F32. */
int fft_serve_admit(const int64_t* n, const int64_t* batch, const int32_t* dtype, int64_t count,
                    int64_t head, size_t inflight_bytes, const fft_serve_config* cfg, int64_t* taken,
                    int64_t* ntaken, size_t* inflight_out);

#ifdef __cplusplus
}
#endif

#endif /* DSFFT_H */
