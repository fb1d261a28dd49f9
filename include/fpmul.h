/*
 * fpmul.h -- C ABI of the MI355X (gfx950) library that multiplies long bit
 * polynomials in GF(2)[x] with the Frobenius-partition additive FFT of
 * Chen, Cheng, Kuo, Li and Yang, "Multiplying boolean Polynomials with
 * Frobenius Partitions in Additive Fast Fourier Transform" (arXiv 1803.11301).
 *
 * Data layout (all entry points)
 *   A bit polynomial of length L bits is ceil(L / 64) 64-bit words; bit k
 *   (the coefficient of x^k) is bit (k % 64) of word (k / 64), little-endian.
 *   Bits at or above L in the last input word are ignored.
 *
 * Memory ownership
 *   Every data pointer below is a DEVICE pointer (memory of the GPU the
 *   context was made for, e.g. allocated by torch).  The caller owns it; the
 *   library never frees it.  The library owns its own workspace and constant
 *   tables, held by the context.
 *
 * Errors
 *   Every int-returning call returns 0 on success or a negative errno-style
 *   code: POLYMUL_EINVAL (bad argument: null or host pointer, overlapping
 *   output, length beyond the limit), POLYMUL_ENOMEM (workspace above the
 *   context's cap, or a failed device allocation), POLYMUL_EIO (a HIP runtime
 *   error).  polymul_last_error() gives the message of the last failure on
 *   the calling thread.  A failed call leaves its output undefined.
 *
 * Threading and streams
 *   A context owns one workspace, so calls on one context must be ordered:
 *   issue them from one host thread, on one stream (or synchronise between
 *   streams).  Different contexts are independent.
 */
#ifndef FPMUL_H
#define FPMUL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POLYMUL_OK 0
#define POLYMUL_EIO (-5)
#define POLYMUL_ENOMEM (-12)
#define POLYMUL_EINVAL (-22)

/* Largest product length in bits over GF(2^64): n <= (m/2) 2^(m/2) with
 * m = 64 (Sec. 3.1, the bound that follows Prop. 2; the partition needs
 * l < m/2).  Longer products run over GF(2^128) (m = 128, whose bound
 * 64 * 2^64 no length reaches). */
#define POLYMUL_M64_MAX_PRODUCT_BITS (1ull << 37)
/* Largest product length polymul and polymul_ex accept.  Device memory is
 * the practical limit: a product with a transform of n bits holds a
 * workspace of four buffers of at least n/8 bytes each besides its operands
 * and output (on one MI355X, 288 GB, n = 2^38 is the largest that fits), and
 * a workspace that cannot be allocated gives POLYMUL_ENOMEM. */
#define POLYMUL_MAX_PRODUCT_BITS (1ull << 62)
/* Largest product length the product server accepts. */
#define POLYMUL_SERVER_MAX_PRODUCT_BITS POLYMUL_M64_MAX_PRODUCT_BITS

typedef struct polymul_ctx polymul_ctx;

/*
 * polymul -- C = A * B in GF(2)[x]  (Alg. 5, FP_Polymul).
 *
 * a_bits, b_bits: device words of A (len_a bits) and B (len_b bits).
 * out: device words, at least ceil((len_a + len_b - 1) / 64); exactly
 *      len_a + len_b - 1 bits are written and the rest of the last word is
 *      zeroed.  If len_a or len_b is 0 the product is empty and nothing is
 *      written.  out must not overlap a_bits or b_bits.
 * The same pointer and length for both operands make a square: a product
 * of more than 2^16 bits then takes one forward transform, squared
 * pointwise (Alg. 5 with both transforms equal).
 * Uses a context owned by the library for the current HIP device and that
 * device's null stream; returns after the result is in out.
 * len_a + len_b - 1 > POLYMUL_MAX_PRODUCT_BITS -> POLYMUL_EINVAL.
 */
int polymul(const uint64_t *a_bits, uint64_t len_a, const uint64_t *b_bits, uint64_t len_b,
            uint64_t *out);

/*
 * polymul_ctx_create -- context for GPU `device`: uploads the constant tables
 * (Cantor basis, Encode matrix and its inverse, butterfly multiplier tables)
 * and holds a workspace that grows on demand up to workspace_cap bytes
 * (0 = no cap beyond device memory).
 */
int polymul_ctx_create(polymul_ctx **ctx, int device, size_t workspace_cap);
int polymul_ctx_destroy(polymul_ctx *ctx);

/*
 * polymul_ex -- same product as polymul(), stream-ordered on `stream`
 * (a hipStream_t; NULL = null stream).  Returns once the work is enqueued;
 * the result is in out when the stream reaches that point.
 */
int polymul_ex(polymul_ctx *ctx, const uint64_t *a_bits, uint64_t len_a,
               const uint64_t *b_bits, uint64_t len_b, uint64_t *out, void *stream);

/* Largest product length, in bits, of polymul_ex_noalloc. */
#define POLYMUL_NOALLOC_MAX_PRODUCT_BITS (1ull << 25)

/*
 * polymul_ex_noalloc -- polymul_ex for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and stream semantics as
 * polymul_ex; the call itself allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  Its workspace is a file-scope device array of
 * the library (about 17 MiB, one copy per GPU, held until the process ends),
 * whose address polymul_ctx_create looks up; ctx supplies the constant tables
 * uploaded then.  Products longer than POLYMUL_NOALLOC_MAX_PRODUCT_BITS
 * (len_a + len_b - 1 bits, or an operand longer than that) return
 * POLYMUL_EINVAL.  Every call on one GPU shares that GPU's array and leaves
 * its contents behind (no call depends on what an earlier one left): calls
 * that overlap on one GPU (two streams, or two host threads) race and must be
 * serialised by the caller.
 */
int polymul_ex_noalloc(polymul_ctx *ctx, const uint64_t *a_bits, uint64_t len_a,
                       const uint64_t *b_bits, uint64_t len_b, uint64_t *out, void *stream);

/* Largest product length, in bits, of one item of polymul_batch. */
#define POLYMUL_BATCH_MAX_PRODUCT_BITS (1ull << 22)

/*
 * polymul_batch -- count independent products C_k = A_k * B_k (Alg. 5 each)
 * in one stream-ordered launch on `stream`.  Every workgroup takes whole
 * products from a queue ordered by size (largest first) and chooses the
 * transform depth of each product on the device from its two lengths.
 *
 * All arrays are DEVICE memory owned by the caller:
 *   a_pool, b_pool: operand words; item k's A starts at word a_word_off[k] of
 *                   a_pool and has len_a[k] bits (same layout as polymul),
 *                   likewise B in b_pool.
 *   out_pool:       item k's product is written at word out_word_off[k]:
 *                   ceil((len_a[k] + len_b[k] - 1) / 64) words, tail bits of
 *                   the last word zeroed; nothing is written for an empty
 *                   operand.  Output ranges must not overlap each other or
 *                   the operands.
 *   len_a, len_b, a_word_off, b_word_off, out_word_off: count entries each.
 *   status:         optional (may be NULL), count int32: 0 when item k was
 *                   computed (or empty), POLYMUL_EINVAL when its product is
 *                   longer than max_product_bits (its output is untouched).
 * max_product_bits: an upper bound on len_a[k] + len_b[k] - 1, at most
 *                   POLYMUL_BATCH_MAX_PRODUCT_BITS; it sizes the per-workgroup
 *                   workspace (4 buffers of 2^ceil(log2 max_product_bits) bits
 *                   per resident workgroup).
 * The offsets are trusted: the library checks that every array is device
 * memory but not that the ranges fit their pools.  Returns 0 once the work
 * is enqueued, POLYMUL_EINVAL for a bad argument, POLYMUL_ENOMEM when the
 * workspace would exceed the context's cap.
 */
int polymul_batch(polymul_ctx *ctx, uint32_t count, const uint64_t *a_pool, const uint64_t *a_word_off,
                  const uint64_t *len_a, const uint64_t *b_pool, const uint64_t *b_word_off, const uint64_t *len_b,
                  uint64_t *out_pool, const uint64_t *out_word_off, uint64_t max_product_bits, int32_t *status,
                  void *stream);

/* Largest transform (log2 of its bits) that the m = 32 field supports. */
#define POLYMUL_SMALL_FIELD_MAX_LOG2N 20

/*
 * polymul_set_small_field -- the m = 32 variant of Sec. 3 for small products
 * (the field size limit n < (m/2) 2^(m/2) gives 2^20 bits for m = 32):
 * batch items whose transform has at most 2^max_log2n bits (polymul_batch,
 * the batched launches of the server, and polymul_ex products of at most
 * 2^16 bits, which run as one-item batches) are computed over GF(2^32)
 * instead of GF(2^64).  The product is the same either way.  0 keeps every
 * item on GF(2^64).  Default: 20.  Affects launches enqueued afterwards (a
 * server created later on ctx takes the value at its creation).
 * Returns 0, or POLYMUL_EINVAL for a null ctx or max_log2n outside [0, 20].
 */
int polymul_set_small_field(polymul_ctx *ctx, int max_log2n);

/* Smallest transform (log2 of its bits) of the m = 128 field: n_p = n / 128
 * values need n >= 128. */
#define POLYMUL_LARGE_FIELD_MIN_LOG2N 7

/*
 * polymul_set_large_field -- the m = 128 variant of Sec. 3 (GF(2^128), l_m = 7):
 * products of polymul_ex / polymul whose transform has at least 2^min_log2n
 * bits are computed over GF(2^128).  Transforms above 2^37 bits always are,
 * since GF(2^64) cannot hold them.  The product is the same either way; a
 * smaller threshold exists to run the m = 128 path on products of any size.
 * Default: 38.  Products of the server (which admits at most 2^37 bits) and
 * batch items are not affected.  The first m = 128 product on a context
 * builds and uploads its constant tables (2 MiB, synchronously).
 * Returns 0, or POLYMUL_EINVAL for a null ctx or min_log2n outside [7, 38].
 */
int polymul_set_large_field(polymul_ctx *ctx, int min_log2n);

/*
 * Schedule tuner for the fused path (transforms of 2^22 .. 2^31 bits).  The
 * product of one transform length can be computed under several schedules
 * of the same kernels: the bottom butterfly pass of layers 0..6 or 0..5
 * (Alg. 2), the layers above it split into passes of up to 7 layers in any
 * way whose lowest pass has at least 12 minus the bottom's layers, and the
 * row and zeta kernels of BasisCvt (Alg. 1) with 1, 2, 4 or 8 and 4, 8, 16
 * or 32 workgroups per CU (the inverse row kernel with four times the row
 * grid, up to one row group per workgroup; below 2^26-bit transforms the
 * butterflies take a fixed split and only the grids are searched).
 * polymul_tune times them on ctx's device for 2^log2n-bit
 * transforms (operands of 2^(log2n-1) bits from a fixed generator; the path
 * is data-oblivious), by coordinate descent from the default with `reps`
 * timed products per choice (1..100), keeps the fastest in ctx (a choice
 * other than the default only if, timed again alternately with the default
 * three times each, its median is 0.5% faster), checks
 * that it gives the default schedule's product word for word
 * (POLYMUL_EIO otherwise, the previous choice kept), appends the line
 * "<arch> cu=<CUs> log2n=<k> upper=<a,b,..> rows=<r> zeta=<z> ms=<t>" to
 * cache_path when it is not NULL, and writes a one-line report (default
 * and tuned ms) into report (may be NULL).  It allocates device memory for
 * its operands and may grow ctx's workspace; it runs on a private stream
 * and returns when done.  Tune before creating servers or graphs on ctx:
 * they read ctx's schedules when they launch (graphs: when captured).
 * polymul_tune_load applies every line of cache_path written for this
 * device's architecture and CU count (a later line for the same length
 * wins; malformed or invalid lines are skipped) and reports how many it
 * applied.  polymul_tune_get writes the schedule ctx uses for 2^log2n-bit
 * transforms as such a line (ms=0).
 */
int polymul_tune(polymul_ctx *ctx, int log2n, int reps, const char *cache_path, char *report,
                 size_t report_len);
int polymul_tune_load(polymul_ctx *ctx, const char *cache_path, int *applied);
int polymul_tune_get(polymul_ctx *ctx, int log2n, char *buf, size_t buflen);

/*
 * Captured launch chains.  polymul_graph_create records the kernels of the
 * product polymul_ex would run for these operands and this output (Alg. 5,
 * FP_Polymul, over GF(2^64)) into a HIP graph, once, on a private stream;
 * polymul_graph_launch replays it on `stream` (a hipStream_t; NULL = null
 * stream) with one call instead of one launch per kernel.  The pointers are
 * DEVICE memory owned by the caller and are baked into the graph: every
 * replay reads a_bits and b_bits as they are when it runs and writes out.
 * The graph owns its workspace (allocated by create, freed by destroy), so
 * later calls on ctx do not disturb it; replays of one graph that overlap
 * in time (two streams) race on that workspace.  Products of at most
 * POLYMUL_M64_MAX_PRODUCT_BITS bits with two non-empty operands; errors as
 * polymul_ex.  The kernels follow the same schedule as polymul_ex, so the
 * result is the same product.
 *
 * polymul_batch_graph_create records the two launches of polymul_batch
 * (the size-ordering plan and the persistent batch kernel) for these device
 * arrays.  Lengths and offsets are read from the arrays on the device at
 * every replay, so the caller may rewrite them between replays (count and
 * max_product_bits stay fixed, every product at most max_product_bits).
 *
 * polymul_graph_destroy waits for the device to finish, then frees the
 * graph and its workspace.
 */
typedef struct polymul_graph polymul_graph;
int polymul_graph_create(polymul_ctx *ctx, const uint64_t *a_bits, uint64_t len_a,
                         const uint64_t *b_bits, uint64_t len_b, uint64_t *out, polymul_graph **graph);
int polymul_batch_graph_create(polymul_ctx *ctx, uint32_t count, const uint64_t *a_pool,
                               const uint64_t *a_word_off, const uint64_t *len_a, const uint64_t *b_pool,
                               const uint64_t *b_word_off, const uint64_t *len_b, uint64_t *out_pool,
                               const uint64_t *out_word_off, uint64_t max_product_bits, int32_t *status,
                               polymul_graph **graph);
int polymul_graph_launch(polymul_graph *graph, void *stream);
int polymul_graph_destroy(polymul_graph *graph);

/*
 * Resident operands (transform reuse).  A product's forward transform of A
 * (BasisCvt, Encode, Butterfly of Alg. 5) depends on A and the transform
 * length only, so an operand that is multiplied many times can keep it on the
 * device: polymul_resident_create computes A's transform once at the length
 * of the longest product it will serve, max_product_bits (len_a <=
 * max_product_bits <= POLYMUL_M64_MAX_PRODUCT_BITS), into device memory
 * owned by the resident object (2^ceil(log2 max_product_bits) bits; the
 * call returns when it is done; a_bits may be reused afterwards).
 * polymul_resident_mul computes C = A * B for any B with len_a + len_b - 1 <=
 * max_product_bits, stream-ordered like polymul_ex, running only B's
 * forward transform, the pointwise products and the inverse steps (same
 * output rules as polymul).  polymul_submit_resident queues the same
 * product on a server (always as a launch of its own; see below).
 * polymul_resident_destroy waits for the device and frees the transform.
 * Errors: POLYMUL_EINVAL for null pointers, lengths out of range or an
 * operand on another device, POLYMUL_ENOMEM when the transform does not fit.
 */
typedef struct polymul_resident polymul_resident;
int polymul_resident_create(polymul_ctx *ctx, const uint64_t *a_bits, uint64_t len_a,
                            uint64_t max_product_bits, polymul_resident **res);
int polymul_resident_destroy(polymul_resident *res);
int polymul_resident_mul(polymul_ctx *ctx, const polymul_resident *res, const uint64_t *b_bits,
                         uint64_t len_b, uint64_t *out, void *stream);

/*
 * Product server: continuous batching of product requests on one GPU.
 *
 * polymul_server_create -- a server on `ctx`'s device (ctx must outlive it).
 *   It allocates one device arena of hbm_budget_bytes (>= 1 MiB) at creation
 *   and nothing afterwards, and runs max_slots (1..64) launch slots, each a
 *   HIP stream.  A scheduler thread admits waiting requests whenever a slot
 *   is free and the request's workspace fits in what is left of the arena:
 *   waiting products of at most 2^20 bits (up to 512 of them) go out
 *   together as one batched launch (as polymul_batch), a larger product runs
 *   alone (as polymul_ex); polymul_server_set_policy changes both limits.  A later request may pass an earlier one that
 *   does not fit yet; one passed 64 times blocks later ones until it fits.
 *   Each slot has a launcher thread that enqueues the slot's kernels, so
 *   launches on different slots are issued side by side and overlap on the
 *   device.
 * polymul_submit -- queues C = A * B (same arguments and rules as polymul,
 *   with products of at most POLYMUL_SERVER_MAX_PRODUCT_BITS bits;
 *   device pointers the caller keeps alive and unmodified until the ticket is
 *   done; the server copies nothing) and returns its ticket.  A product whose
 *   workspace exceeds the whole arena is refused with POLYMUL_ENOMEM.
 * polymul_submit_resident -- queues C = A * B for a resident operand A
 *   (polymul_resident_create on the server's device; it must outlive the
 *   ticket): only B's transform is computed.  It runs as a launch of its own
 *   on the workspace of the resident transform length; same rules as
 *   polymul_submit otherwise.
 * polymul_poll -- *done = 1 once the ticket's product is in out; then returns
 *   the product's result code (0, or the error of its launch).  Polling does
 *   not release the ticket.
 * polymul_wait -- blocks until the ticket is done, returns its result code
 *   and releases the ticket: afterwards the server no longer knows it (poll,
 *   wait and ticket_times then return POLYMUL_EINVAL).  Every ticket is
 *   released by exactly one wait (or wait_times), which returns at once for
 *   a ticket already done; the server keeps nothing of released tickets.
 * polymul_wait_times -- polymul_wait that also stores the ticket's times
 *   (as polymul_ticket_times; any pointer may be NULL) before releasing it.
 * polymul_ticket_times -- host steady-clock times (ns since server creation)
 *   at which a ticket not yet released was submitted, launched and seen
 *   complete (0 for a step not reached yet).
 * polymul_server_tickets -- *count = tickets submitted and not yet released.
 * polymul_server_destroy -- finishes every submitted request, then frees the
 *   arena, streams and thread.
 * submit, poll, wait and ticket_times may be called from any host thread.
 */
typedef struct polymul_server polymul_server;
int polymul_server_create(polymul_server **srv, polymul_ctx *ctx, size_t hbm_budget_bytes, uint32_t max_slots);
int polymul_server_destroy(polymul_server *srv);
/*
 * polymul_server_set_policy -- before the first submit: products of at most
 * batch_limit_bits bits (<= POLYMUL_BATCH_MAX_PRODUCT_BITS) are grouped into
 * batched launches of at most max_batch requests (1..4096); larger products
 * run alone.  Defaults: 2^20 bits, 512 requests.  POLYMUL_EINVAL after the
 * first submit or for values out of range.
 */
int polymul_server_set_policy(polymul_server *srv, uint64_t batch_limit_bits, uint32_t max_batch);
int polymul_submit(polymul_server *srv, const uint64_t *a_bits, uint64_t len_a, const uint64_t *b_bits,
                   uint64_t len_b, uint64_t *out, uint64_t *ticket);
int polymul_submit_resident(polymul_server *srv, const polymul_resident *res, const uint64_t *b_bits,
                            uint64_t len_b, uint64_t *out, uint64_t *ticket);
int polymul_poll(polymul_server *srv, uint64_t ticket, int *done);
int polymul_wait(polymul_server *srv, uint64_t ticket);
int polymul_wait_times(polymul_server *srv, uint64_t ticket, uint64_t *submit_ns, uint64_t *start_ns,
                       uint64_t *done_ns);
int polymul_ticket_times(polymul_server *srv, uint64_t ticket, uint64_t *submit_ns, uint64_t *start_ns,
                         uint64_t *done_ns);
int polymul_server_tickets(polymul_server *srv, uint64_t *count);

/*
 * polymul_addfft -- the modified additive FFT of Sec. 3.4: BasisCvt (Alg. 1),
 * Encode (Alg. 4) and Butterfly (Alg. 2) at alpha = v_{l+32}.  Evaluates A
 * (len_a bits, len_a <= 2^log2n) at the n/64 points of the Frobenius
 * partition Sigma = v_{l+32} + V_l, l = log2n - 6 (Eq. 6, Eq. 8).
 * values: device, 2^(log2n-6) words; word j is A(v_{l+32} + j) with j read
 * as Cantor coordinates.  Each value is a GF(2^64) element in the library's
 * multiplication representation: the tower over V_8 = span(v_0 .. v_7)
 * (a subfield, Sec. 2.2) by v_8, v_16 and v_32, where bit 8k + u is the
 * coefficient of v_u * W_k and W_k is the product of v_8, v_16, v_32 for
 * the set bits 0, 1, 2 of k.  (Any representation gives the same product;
 * this one is chosen for the device, see polymul_pointwise.)
 * 6 <= log2n <= 37.
 */
int polymul_addfft(polymul_ctx *ctx, const uint64_t *a_bits, uint64_t len_a, int log2n,
                   uint64_t *values, void *stream);

/*
 * polymul_iaddfft -- inverse of polymul_addfft for the same log2n:
 * iButterfly, Decode and iBasisCvt (the inverse steps of Alg. 5).  Reads 2^(log2n-6)
 * values, writes the first out_bits bits (<= 2^log2n) of the polynomial of
 * degree < 2^log2n they determine (Prop. 2), zeroing the rest of the last
 * word.  values is not modified.
 */
int polymul_iaddfft(polymul_ctx *ctx, const uint64_t *values, int log2n, uint64_t *out,
                    uint64_t out_bits, void *stream);

/*
 * polymul_pointwise -- fc[j] = fa[j] * fb[j] in GF(2^64) for the
 * 2^(log2n-6) values of two transforms of the same log2n (the pointwise step
 * of Alg. 5), in the representation polymul_addfft writes.  With it a
 * transform can be computed once and reused: A * B_k for several B_k is
 * addfft(A) once, addfft(B_k), pointwise, iaddfft; A^2 is addfft(A),
 * pointwise(fa, fa), iaddfft.  fc may be fa or fb; otherwise it must not
 * overlap them.  6 <= log2n <= 37.
 */
int polymul_pointwise(polymul_ctx *ctx, const uint64_t *fa, const uint64_t *fb, int log2n, uint64_t *fc,
                      void *stream);

/*
 * polymul_basiscvt -- Alg. 1 alone: monomial -> novelpoly coefficients of a
 * bit polynomial of len bits, written as 2^log2n bits (log2n >= ceil(log2
 * len), zero-padded).  inverse != 0 runs iBasisCvt on 2^log2n bits instead.
 * out receives ceil(2^log2n / 64) words and must not overlap in.
 */
int polymul_basiscvt(polymul_ctx *ctx, const uint64_t *in, uint64_t len, int log2n, int inverse,
                     uint64_t *out, void *stream);

/*
 * polymul_profile_enable -- per-kernel timing: when on, every kernel the
 * context launches is bracketed by HIP events recorded on its launch stream.
 * Enabling or disabling clears the counters.
 */
int polymul_profile_enable(polymul_ctx *ctx, int on);

/*
 * polymul_profile_report -- waits for the recorded events and writes one line
 * per kernel name, "name launches total_ms\n", NUL-terminated, into buf
 * (buflen bytes; POLYMUL_EINVAL if it does not fit).
 */
int polymul_profile_report(polymul_ctx *ctx, char *buf, size_t buflen);

/* Message of the last failure on this thread ("" if none). */
const char *polymul_last_error(void);

/* Library version string. */
const char *polymul_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FPMUL_H */
