/*
 * mont_ntt.h -- C ABI of libmont's number-theoretic transforms and
 * polynomial products modulo word-size Fourier primes (AMD MI355X, gfx950).
 *
 * Every butterfly multiplies an ordinary residue by a twiddle factor kept in
 * Montgomery form and reduces with REDC (Meng, arXiv:1609.00999, section 3.1,
 * Algorithm 2, R = 2^32), so REDC(x * w R) = x w mod P.  Primes P = c 2^k + 1
 * (Fourier primes, section 3.1) have roots of unity of order 2^n for n <= k.
 * The paper uses this arithmetic inside modular FFT and polynomial-product
 * libraries (sections 1 and 5); the transforms themselves are the textbook
 * radix-2 ones:
 *   forward:  X_j = sum_i x_i w^(i * rev(j)), natural order in, bit-reversed
 *             order out (decimation in frequency);
 *   inverse:  x_i = N^-1 sum_j X_j w^(-i * rev(j)), bit-reversed in, natural
 *             out (decimation in time);
 * with w = g^((P-1)/N) and g the smallest primitive root modulo P.
 *
 * Conventions are those of mont.h: d_* are device pointers owned by the
 * caller, stream is a hipStream_t (NULL = null stream), calls are
 * asynchronous on it, validation happens before anything is enqueued, and
 * coefficients are ordinary residues in [0, P) (not Montgomery form).
 */
#ifndef MONT_NTT_H
#define MONT_NTT_H

#include "mont.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque context: per-prime constants and resident twiddle tables. */
typedef struct ntt_ctx ntt_ctx;

/*
 * ntt_ctx_create -- per prime: section 3.1 constants, the smallest primitive
 * root g, and device-resident twiddle tables (forward and inverse, 2^L words
 * each with L = min(log2_nmax, v2(P-1))), generated on the device by REDC
 * products of repeated squares.  Allocates device memory (8 * 2^L bytes per
 * prime) and synchronizes the device.  primes: host array of nprimes
 * (1..64) odd primes < 2^31.  log2_nmax in [1, 23] (transforms up to 2^23;
 * MONT_EINVAL above).  The context is
 * read-only afterwards and may be shared by streams and threads.
 * Errors: MONT_EINVAL (bad prime or argument), MONT_ENOMEM, MONT_EHIP.
 */
MONT_API mont_status ntt_ctx_create(const uint32_t* primes, int nprimes, int log2_nmax, ntt_ctx** out);

/* Frees the context's device memory (synchronizes the device first). */
MONT_API mont_status ntt_ctx_destroy(ntt_ctx* ctx);

/*
 * ntt_ctx_prime -- introspection for prime prime_id: its parameters, the root
 * w of order 2^log2_max used by the tables (ordinary residue), log2_max, and
 * device pointers to the tables (entry h + i, h = 2^s, i < h, holds the
 * Montgomery form of w_{2h}^i, respectively w_{2h}^-i, with w_{2h} =
 * w^(2^log2_max / 2h); entry 0 is unused).  Any output pointer may be NULL.
 */
MONT_API mont_status ntt_ctx_prime(const ntt_ctx* ctx, int prime_id, mont_params* prm, uint32_t* root,
                                   uint32_t* log2_max, const uint32_t** d_twf, const uint32_t** d_twi);

/* ntt_ctx_read_twiddles -- synchronous copy of prime prime_id's forward and
 * inverse tables (2^log2_max words each) into HOST arrays h_fwd and h_inv. */
MONT_API mont_status ntt_ctx_read_twiddles(const ntt_ctx* ctx, int prime_id, uint32_t* h_fwd, uint32_t* h_inv);

/*
 * ntt_forward / ntt_inverse -- in-place transform of d_x[0 .. 2^log2n) with the
 * root of order 2^log2n (see above for orders).  ntt_inverse includes the
 * factor N^-1, so ntt_inverse(ntt_forward(x)) = x.  Values must be in [0, P).
 * Errors: MONT_EINVAL, MONT_ENOROOT (log2n above the prime's table).
 */
MONT_API mont_status ntt_forward(const ntt_ctx* ctx, int prime_id, uint32_t* d_x, uint32_t log2n, void* stream);
MONT_API mont_status ntt_inverse(const ntt_ctx* ctx, int prime_id, uint32_t* d_x, uint32_t log2n, void* stream);

/*
 * ntt_polymul -- product of two polynomials modulo prime prime_id, with plain
 * kernel launches (one for lengths up to 2^13, three above):
 *   d_out[k] = sum_{i+j=k} d_a[i] d_b[j] mod P,  k = 0 .. da+db,
 * for d_a of da+1 and d_b of db+1 coefficients in [0, P).  The transform
 * length is N = 2^n, the least power of two >= da+db+1.  d_scratch must hold
 * ntt_polymul_scratch_bytes(da, db) bytes (0 when N <= 2^13, else 8N) and be
 * 16-byte aligned (MONT_EINVAL otherwise); d_out must not overlap the inputs.
 * Errors: MONT_EINVAL, MONT_ERANGE
 * (da+db+1 > 2^31), MONT_ENOROOT (N above the prime's table), MONT_ENOMEM
 * (scratch too small).
 */
MONT_API size_t ntt_polymul_scratch_bytes(uint32_t da, uint32_t db);
MONT_API mont_status ntt_polymul(const ntt_ctx* ctx, int prime_id, const uint32_t* d_a, uint32_t da,
                                 const uint32_t* d_b, uint32_t db, uint32_t* d_out, void* d_scratch,
                                 size_t scratch_bytes, void* stream);

/*
 * ntt_polymul_noalloc -- ntt_polymul for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same launches and the same result, with the transform
 * scratch taken from a static 16 MiB device array that the library holds on
 * each device until the process ends, so the call allocates nothing and
 * takes no scratch argument.  Limit: transform length N <= 2^21 (da+db+1 <=
 * 2^21); longer products return MONT_ENOMEM.  The array's device address is
 * looked up when ntt_ctx_create runs on the device; the call must be made
 * with the context's device current (MONT_EINVAL otherwise).  Every call on
 * one device shares that one array, so calls that overlap on a device (on
 * different streams, or from several threads without ordering) race and
 * give wrong results; calls ordered on one stream are safe.  The scratch
 * needs no clearing: each call writes it before reading it.  Errors: those
 * of ntt_polymul, MONT_ENOMEM above the limit, MONT_EHIP if the array's
 * address could not be looked up.
 */
MONT_API mont_status ntt_polymul_noalloc(const ntt_ctx* ctx, int prime_id, const uint32_t* d_a, uint32_t da,
                                         const uint32_t* d_b, uint32_t db, uint32_t* d_out, void* stream);

/* One product of a batch: operands at d_in + a_off (da+1 words) and
 * d_in + b_off (db+1 words), result at d_out + c_off (da+db+1 words). */
typedef struct polymul_desc {
  uint32_t prime_id;
  uint32_t da, db;
  uint32_t reserved; /* must be 0 */
  uint64_t a_off, b_off, c_off;
} polymul_desc;

/* Opaque batch plan: the product descriptors and the ordered task list,
 * resident on the device. */
typedef struct ntt_plan ntt_plan;

/*
 * ntt_plan_create -- plans a batch of `count` products of uneven lengths,
 * each with its own prime, for ONE persistent launch.  Products with N <=
 * 2^13 are single tasks; longer ones are split into column tiles of both
 * operands, row blocks (forward rows, pointwise product, inverse rows) and
 * inverse column tiles, with per-product completion counters.  A longer
 * product whose length L = da+db+1 lies just above h = N/2 (both operands
 * shorter than h, and the top m = L - h coefficients of each operand having
 * a product of length <= N/4) is computed as the cyclic product of length h
 * plus the product of those top coefficients, and a fix-up pass after the
 * launch subtracts the wrapped part and stores the top coefficients; this
 * cuts about a quarter of such a product's butterflies.  The result is the
 * same.  Tasks are
 * ordered so that every prerequisite precedes its dependants: forward column
 * tiles, half the single tasks, row blocks, the other half, inverse column
 * tiles, each group longest-first, or shuffled within groups when
 * order_seed != 0 (for determinism tests).  descs is a host array; it is
 * copied.  Allocates device memory for the plan (not for the data).
 * Errors: MONT_EINVAL, MONT_ERANGE, MONT_ENOROOT, MONT_ENOMEM, MONT_EHIP.
 */
MONT_API mont_status ntt_plan_create(const ntt_ctx* ctx, const polymul_desc* descs, int count, uint32_t order_seed,
                                     ntt_plan** out);

/*
 * ntt_plan_reserve -- a reusable plan with room for max_products products and
 * max_tasks tasks (device arrays plus pinned host staging), for callers that
 * plan a new batch often (a serving loop).  It holds no batch until
 * ntt_plan_update.  ntt_plan_task_count(da, db) gives the tasks one product
 * adds (both parts of a split product).  Errors: MONT_EINVAL, MONT_ENOMEM.
 */
MONT_API mont_status ntt_plan_reserve(const ntt_ctx* ctx, int max_products, uint32_t max_tasks, ntt_plan** out);
MONT_API uint32_t ntt_plan_task_count(uint32_t da, uint32_t db);

/*
 * ntt_plan_update -- replans a reserved plan for a new batch (same rules and
 * task order as ntt_plan_create) and uploads it asynchronously on `stream`;
 * executions of the plan must be enqueued on the same stream, after this
 * call, so that they see the new lists.  A plan of at most 4 internal
 * products, 384 tasks and no split products is not uploaded: its lists travel
 * in the arguments of each execution's launch.  Blocks only until the
 * previous update's upload has left the staging buffers.  Errors: MONT_EINVAL (not a
 * reserved plan, bad descriptor), MONT_ERANGE (beyond the reserved capacity,
 * or a product too long), MONT_ENOROOT, MONT_EHIP.
 */
MONT_API mont_status ntt_plan_update(ntt_plan* plan, const polymul_desc* descs, int count, uint32_t order_seed,
                                     void* stream);

/* Host time of the last ntt_plan_update on a reserved plan, in
 * microseconds: us[0] planning, us[1] waiting for the previous upload to
 * leave the staging block, us[2] the upload call (0 when the lists travel in
 * the launch arguments), us[3] the whole call.  A diagnostic for callers that
 * budget host latency (a serving loop).  Errors: MONT_EINVAL. */
MONT_API mont_status ntt_plan_update_times(const ntt_plan* plan, uint32_t* us);

/* Sizes a caller needs: scratch bytes, task count, the minimum lengths (in
 * words) of d_in and d_out, and the default persistent grid (resident
 * workgroups on the device).  Any output pointer may be NULL. */
MONT_API mont_status ntt_plan_info(const ntt_plan* plan, size_t* scratch_bytes, uint32_t* ntasks,
                                   uint64_t* in_words, uint64_t* out_words, int* default_grid);

/* The work one execution of the plan performs: REDC operations (three
 * transforms of (N/2) log2 N butterflies, N pointwise products and db+1
 * operand scalings per product as planned, after splitting, less the
 * butterflies whose twiddle is 1, which run without a product: N (1 - 2^-r)
 * per transform, r the size of the register round that holds stage 0, so
 * the count depends on the plan's radix, ntt_plan_shape) and the number of
 * split products.  Either output pointer may be NULL. */
MONT_API mont_status ntt_plan_work(const ntt_plan* plan, uint64_t* redc, uint32_t* split_products);

/* The launch shape the plan's persistent launch takes: threads per
 * workgroup, log2 of the register-round radix, grid multiplier.  Chosen when
 * the plan is created or updated: the shape tuned for a transform length
 * when at least 90 % of the plan's butterflies are at that length, else the
 * default shape (ntt_tune_set, ntt_tune_set_length).  Any output pointer may
 * be NULL.  Errors: MONT_EINVAL (plan NULL). */
MONT_API mont_status ntt_plan_shape(const ntt_plan* plan, int* threads, int* radix_log, int* grid_mult);

/*
 * ntt_plan_execute -- zeroes the scratch header with a fill kernel, then runs
 * the whole batch in one persistent launch of `grid` workgroups (0 = the
 * default) that take tasks from a device counter, then (if the plan split a
 * product) one fix-up kernel.  Waits on another task's completion spin at
 * most spin_limit sleeps (0 = 2^24); on expiry the launch records a timeout,
 * skips the dependent tasks and drains.  d_scratch must
 * hold the plan's scratch bytes; d_in and d_out the plan's word counts.  The
 * result is identical for every grid size and task order.  Enqueues two or
 * three kernels and no memset or allocation, so the call may be captured in a
 * HIP graph.  d_scratch must be 16-byte aligned (MONT_EINVAL otherwise).  Calls
 * that share a scratch buffer must not overlap.
 */
MONT_API mont_status ntt_plan_execute(const ntt_plan* plan, const uint32_t* d_in, uint32_t* d_out, void* d_scratch,
                                      size_t scratch_bytes, int grid, uint32_t spin_limit, void* stream);

/* Synchronizes `stream` and reports whether the last execution on d_scratch
 * completed (MONT_OK) or timed out in a dependency wait (MONT_ETIMEOUT). */
MONT_API mont_status ntt_plan_status(const ntt_plan* plan, const void* d_scratch, void* stream);

/*
 * ntt_plan_status_async -- enqueues on `stream` a copy of the status word of
 * the last execution on d_scratch into the host word *h_status, without
 * waiting: once the stream has passed this point, *h_status is 0 (the
 * execution completed) or nonzero (a dependency wait gave up, as
 * MONT_ETIMEOUT from ntt_plan_status).  Enqueue it after ntt_plan_execute on
 * the same stream.  h_status should be pinned host memory (hipHostMalloc);
 * the caller owns it and must not read it before the stream has passed the
 * copy.  A plan with no products writes 0 at once.  Errors: MONT_EINVAL,
 * MONT_EHIP.
 */
MONT_API mont_status ntt_plan_status_async(const ntt_plan* plan, const void* d_scratch, uint32_t* h_status,
                                           void* stream);

/* Frees the plan's device memory (synchronizes the device first). */
MONT_API mont_status ntt_plan_destroy(ntt_plan* plan);

/*
 * One-call batches: the batch of uneven products, each with its own prime,
 * in ONE call whose descriptors live in DEVICE memory.  A planning kernel
 * (one workgroup) turns d_descs into the records and the task list a plan
 * holds, inside d_scratch: the same split rule as ntt_plan_create and its
 * phase task order (forward column tiles, half the single tasks, row
 * blocks, the other half, inverse column tiles, each phase longest first,
 * products of one length grouped by prime).  Then one persistent launch runs
 * every task and, for split products, one fix-up launch follows.  The call
 * performs no host-device copy and no allocation, so it can be captured in a
 * HIP graph, and every replay plans whatever descriptors d_descs then holds
 * (the same count).  Each product's result equals ntt_polymul's.
 *
 * ntt_scratch_bytes -- bytes of d_scratch that ntt_polymul_batch needs for
 * these `count` descriptors (a HOST array here, with the values the device
 * copy will hold): a header, per-product records and counters, the task
 * list, 2N words for each product of N > 2^13 after splitting, the
 * outputs of top parts, and one word per 1024 coefficients that a two-part
 * product's fix-up rewrites.  Returns 0 if ctx is NULL or a descriptor is invalid
 * (prime_id out of range, reserved != 0, da+db+1 > 2^31, N above the prime's
 * table).  Pure host arithmetic, for admission by footprint.
 *
 * ntt_polymul_batch -- d_descs: `count` polymul_desc records in device
 * memory (8-byte aligned); operands and outputs at the offsets they give in
 * d_in and d_out (words; the caller guarantees they lie inside the buffers
 * and that outputs do not overlap inputs or each other); d_scratch:
 * scratch_bytes bytes, 16-byte aligned, caller-owned.  Host checks: NULL
 * pointers, alignment, count < 0 (MONT_EINVAL) and scratch_bytes below the
 * fixed part of the layout (MONT_ENOMEM).  Errors only the descriptors show
 * (invalid descriptor, or scratch smaller than ntt_scratch_bytes) are found
 * by the planning kernel: it records them in the scratch header and no
 * product is computed; ntt_batch_status reports them.  Asynchronous on
 * `stream`; calls sharing a scratch buffer must not overlap.
 *
 * ntt_batch_status -- synchronizes `stream` and returns the outcome of the
 * last ntt_polymul_batch on d_scratch: MONT_OK, MONT_ETIMEOUT (a dependency
 * wait gave up), or the planning error (MONT_EINVAL, MONT_ERANGE,
 * MONT_ENOROOT, MONT_ENOMEM).
 */
MONT_API size_t ntt_scratch_bytes(const ntt_ctx* ctx, const polymul_desc* descs, int count);
MONT_API mont_status ntt_polymul_batch(const ntt_ctx* ctx, const polymul_desc* d_descs, int count,
                                       const uint32_t* d_in, uint32_t* d_out, void* d_scratch, size_t scratch_bytes,
                                       void* stream);
MONT_API mont_status ntt_batch_status(const void* d_scratch, void* stream);

/*
 * Launch-shape tuning of the transform kernels (used by the autotuner):
 * threads per workgroup (256, 512 or 1024), the largest number of radix-2
 * stages a lane keeps in registers between LDS exchanges (3 or 4), and the
 * default persistent grid as a multiple (1, 2 or 4) of the workgroups that
 * fit on the device at once.  Process-wide, read when a launch is enqueued;
 * never changes results.  Returns MONT_EINVAL for values outside those sets.
 */
MONT_API mont_status ntt_tune_set(int threads, int radix_log, int grid_mult);
MONT_API mont_status ntt_tune_get(int* threads, int* radix_log, int* grid_mult);

/*
 * Per-length launch shapes (the autotuner's per-length buckets): the shape
 * for transforms of length 2^log2n (log2n in [0, 23]).  Plain launches
 * (ntt_forward, ntt_inverse, ntt_polymul and its variants) use the shape of
 * their length; a plan takes, when it is created or updated, the shape of
 * the length that carries at least 90 % of its butterflies, or else the
 * default of ntt_tune_set; ntt_polymul_batch uses that default.  threads == 0 removes the entry (the default
 * applies again).  ntt_tune_get_length reports the shape in force for the
 * length.  Never changes results.  Errors: MONT_EINVAL.
 */
MONT_API mont_status ntt_tune_set_length(int log2n, int threads, int radix_log, int grid_mult);
MONT_API mont_status ntt_tune_get_length(int log2n, int* threads, int* radix_log, int* grid_mult);

#ifdef __cplusplus
}
#endif

#endif /* MONT_NTT_H */
