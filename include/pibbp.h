/*
 * pibbp.h -- C ABI of the MI355X bit-extraction library for pi.
 *
 * The library evaluates BBP-type formulas at a bit position n (Sze, "The Two
 * Quadrillionth Bit of pi is 0!", section 3): for every series j of the
 * formula and every index k it forms the term
 *
 *     t_{j,k} = floor(2^P * frac(2^E / M)),   E = n - 1 + c_j - step*k,
 *                                             M = a_j*k + b_j,
 *
 * (the A_k of eq (3.3) when E >= 0, computed with a modular exponentiation
 * and a division; the B_k of eq (3.3) when E < 0) and adds
 * sign_j * alt^k * t_{j,k} modulo 2^P. Formulas: Bellard's (eq (1.2); step
 * 10, alternating signs, seven series) and the BBP formula (eq (1.1), in the
 * odd-denominator form of eq (3.1); step 4, four series). Every result is
 * exact: integer arithmetic, plus binary64 operations on integer-valued
 * doubles that are proven never to round.
 *
 * Conventions shared by every call:
 *  - n is the 1-based position of the first result bit after the radix point
 *    (the abstract's footnote: the 8 bits starting at position 9 are 0x3F).
 *  - A P-bit sum S is returned in L = ceil(P/64) little-endian uint64 limbs,
 *    LEFT-ALIGNED: the limbs hold S * 2^(64L-P), so the first result bit is the
 *    most significant bit of limb L-1 and the low 64L-P bits are zero.
 *  - Pointers named out/status/workspace are DEVICE pointers owned by the
 *    caller; the library never frees them. Query tables are HOST pointers.
 *  - Calls are asynchronous on `stream`: argument validation is synchronous
 *    and returns an error code; results are ready when the stream is.
 *  - Limits: 1 <= P <= PI_MAX_P; the modulus a_j*k+b_j of every index a call
 *    sums below 2^54, and n + P below 2^62 (otherwise PI_EUNSUPPORTED).
 *  - Calls on one device share internal scratch per stream; calls on
 *    different streams may overlap, calls on one stream are serialized.
 */
#ifndef PIBBP_H
#define PIBBP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define PI_API __attribute__((visibility("default")))
#else
#define PI_API
#endif

/* Formulas: eq (1.1) (as written in eq (3.1)) and eq (1.2). */
enum { PI_BBP = 0, PI_BELLARD = 1 };

/* A single series j of a formula, for pi_sum_slice. Bellard's series, in the
 * order of eq (1.2): 0: +2^2/(10k+1), 1: -1/(10k+3), 2: -2^-4/(10k+5),
 * 3: -2^-4/(10k+7), 4: +2^-6/(10k+9), 5: -2^-1/(4k+1), 6: -2^-6/(4k+3).
 * BBP series, in the order of eq (3.1): 0: +2^2/(8k+1), 1: -2^-1/(2k+1),
 * 2: -1/(8k+5), 3: -2^-1/(4k+3). */
#define PI_TERM(formula, j) ((formula) * 16 + (j))

/* Return codes. PI_UNCERTAIN is a status, not an error: the bits were
 * computed exactly, but the guard window (section 3.1) cannot prove that they
 * are pi's bits; a larger P can. */
enum {
  PI_OK = 0,
  PI_UNCERTAIN = 1,
  PI_EINVAL = -1,
  PI_ENOMEM = -2,
  PI_EDEVICE = -3,
  PI_EUNSUPPORTED = -4,
  PI_ESCRATCH = -5
};

#define PI_MAX_P 1088u

/* Result status written by pi_extract_ex and pi_extract_batch (device memory). */
typedef struct {
  int32_t code;     /* PI_OK when certified, PI_UNCERTAIN otherwise */
  int32_t reserved; /* 0 */
  uint64_t nterms;  /* N: indices summed (head terms plus tail terms before the stop) */
} pi_status;

/* nbits bits of pi starting at 1-based position n, with P = nbits + 64 (the
 * 64 guard bits are what certification, section 3.1, examines).
 *   out: device uint64[ceil((nbits+64)/64)], the left-aligned P-bit sum S.
 * Returns PI_OK or an error; certification is reported by pi_extract_ex. */
PI_API int pi_extract(int formula, uint64_t n, uint32_t nbits, uint64_t *out, hipStream_t stream);

/* As pi_extract with an explicit precision P >= nbits (e.g. P = 96 for 64
 * result bits) and an optional device pi_status (may be NULL).
 * The tail of each series is summed up to its stop index: the first E < 0
 * index whose P-bit truncation is 0 (every later term is smaller).
 *   out: device uint64[ceil(P/64)]. status: device pi_status or NULL. */
PI_API int pi_extract_ex(int formula, uint64_t n, uint32_t nbits, uint32_t P, uint64_t *out,
                  pi_status *status, hipStream_t stream);

/* pi_extract_ex for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and status, bit for bit; the kernels' scratch (the
 * query's 2*ceil(P/64) carry-save counters and the head launch's chunk
 * counter, at most 35 64-bit words) is a static device array of 64 words
 * instead of the library's per-stream arena, so the call allocates nothing
 * and never waits. Each device holds one such array, shared by every call on
 * it: calls that overlap on one device (on different streams, or from
 * different host threads) race and must not be issued; calls on one stream
 * are ordered and safe. Every call clears what it uses with a kernel (no
 * hipMemsetAsync). PI_ESCRATCH if a query needed more than the array (not
 * possible within PI_MAX_P); other errors as pi_extract_ex. */
PI_API int pi_extract_noalloc(int formula, uint64_t n, uint32_t nbits, uint32_t P, uint64_t *out,
                              pi_status *status, hipStream_t stream);

/* One summand of eq (3.1), restricted to an index range, as in the
 * partition/compute split of section 4.1: the sum over k in [k0, k1) of
 * sign_j * alt^k * t_{j,k} modulo 2^P, for term = PI_TERM(formula, j). Head
 * and tail indices may both be in the range; tail terms past the stop index
 * are zero. Sums over disjoint ranges add up (mod 2^P) to the full sum.
 *   out: device uint64[ceil(P/64)], left-aligned. */
PI_API int pi_sum_slice(int term, uint64_t n, uint64_t k0, uint64_t k1, uint32_t P, uint64_t *out,
                 hipStream_t stream);

/* pi_sum_slice that also reports, in status->nterms, how many indices of
 * [k0, k1) are summed before the series' stop index (every head index, and
 * the tail indices whose truncated term is nonzero); status->code is PI_OK.
 * Summed over a partition of a query's index set these counts give the N of
 * pi_extract_ex. status: device pi_status or NULL. */
PI_API int pi_sum_slice_ex(int term, uint64_t n, uint64_t k0, uint64_t k1, uint32_t P,
                           uint64_t *out, pi_status *status, hipStream_t stream);

/* The sum of `count` partial sums kept between calls (section 4 persists the
 * partial sums of jobs and adds them at the end): parts is a device array of
 * count x ceil(P/64) left-aligned limbs, e.g. pi_sum_slice outputs over a
 * partition of a query's index set. out receives their sum mod 2^P, and
 * status (device, may be NULL) its certification for the top nbits with
 * N = nterms and nseries series (4 for BBP, 7 for Bellard), as in
 * pi_extract_ex. */
PI_API int pi_combine(const uint64_t *parts, int count, uint32_t P, uint32_t nbits,
                      uint32_t nseries, uint64_t nterms, uint64_t *out, pi_status *status,
                      hipStream_t stream);

/* A query of a batch. out_offset is in uint64 limbs from the batch's `out`;
 * the query writes ceil(P/64) limbs there. */
typedef struct {
  int32_t formula;
  uint32_t nbits;
  uint32_t P;
  uint32_t reserved; /* 0 */
  uint64_t n;
  uint64_t out_offset;
} pi_query;

/* Many extractions in one submission: the head terms of every query of up
 * to 6 limbs (P <= 384) go through one persistent launch, whose chunks each
 * run at their own query's limb count, and those of larger queries through
 * one launch per limb count (8, 12, 17); each query keeps its partial sum on
 * the device, and one finalize launch per group writes every result.
 * Each query's result is bit-identical to pi_extract_ex on its own.
 *   q: host array[count]. out: device, packed per out_offset.
 *   status: device pi_status[count] or NULL.
 *   workspace: device memory of at least pi_workspace_size(q, count) bytes,
 *   or NULL to use the library's per-stream scratch. */
PI_API int pi_extract_batch(const pi_query *q, int count, uint64_t *out, pi_status *status,
                     void *workspace, size_t ws_bytes, hipStream_t stream);

/* A planned batch that can be launched many times, e.g. captured once into a
 * HIP graph and replayed. pi_batch_create plans the queries, allocates the
 * plan's own device memory and uploads its tables (synchronously);
 * pi_batch_launch then only enqueues kernels on `stream` (clear the counters,
 * then per launch group of pi_extract_batch one head and one finalize
 * launch): it never
 * allocates, copies from the host or waits, so it can be captured. Every
 * launch writes the results again into the out/status given at creation.
 * Launches of one plan must not overlap (they share its counters).
 * pi_batch_destroy waits for the plan's last eager launch (an event recorded
 * on its stream, not the whole device) and frees the plan; a plan captured
 * into a graph must outlive every replay of that graph. */
typedef struct pi_batch pi_batch;
PI_API int pi_batch_create(const pi_query *q, int count, uint64_t *out, pi_status *status,
                           pi_batch **plan);
PI_API int pi_batch_launch(pi_batch *plan, hipStream_t stream);
PI_API void pi_batch_destroy(pi_batch *plan);

/* Bytes of device workspace pi_extract_batch needs for these queries. */
PI_API size_t pi_workspace_size(const pi_query *q, int count);

/* Number of head terms (E >= 0 indices) of an extraction: sum over series of
 * floor((n-1+c_j)/step)+1 where that is positive. Host-only arithmetic. */
PI_API uint64_t pi_head_terms(int formula, uint64_t n);

/* One head segment of a plan: series j, index range [kb, ke), the arithmetic
 * of its moduli M = a_j k + b_j (cls: 22, 27, 29, 31: R = 2^32 Montgomery,
 * M below 2^cls; 33, 42, 48, 51: exact binary64, M below 2^cls; 64:
 * R = 2^62 Montgomery, M below 2^54), the indices each lane takes per chunk
 * (run), its chunk count (chunks of 256 * run indices) and, for cls 64, the
 * exponent bits folded into the ladder's start value (pre). */
typedef struct {
  uint32_t j, cls, run, pre;
  uint64_t kb, ke, nchunks;
} pi_segment;

/* The head segments that pi_extract_ex (series_mask 0x7f, k0 = 0,
 * k1 = UINT64_MAX) or pi_sum_slice (series_mask 1 << j) would launch for this
 * query, under the current arithmetic mode and tuning: the partition of
 * section 4 (jobs of series and modulus range, tasks of 256 * run indices)
 * as this library plans it. Host work only; nothing is launched. Mask bits
 * past the formula's series count are ignored. *count receives the number of
 * segments; segs (host, max_segs entries) receives them, or PI_EINVAL is
 * returned when max_segs is too small (count still set). Other errors as for
 * pi_sum_slice. */
PI_API int pi_plan_head(int formula, uint32_t series_mask, uint64_t n, uint64_t k0, uint64_t k1,
                        uint32_t P, pi_segment *segs, int max_segs, int *count);

/* Launch shape of the head kernel instance for `limbs` = ceil(P/64) rounded
 * up to an instantiated count (1-6, 8, 12, 17), of the fused launch that
 * batches and serving steps use for queries of 1 to 6 limbs when limbs is
 * PI_TUNE_FUSED, or of every one when limbs is 0: wg_per_cu workgroups per CU
 * (0, the default: as many as fit, from the occupancy API; at most 64) and
 * run_cap, the most indices one lane takes per chunk (1..4096, default 2048;
 * for the fused launch, of each query in it). Results do not depend on these; only speed
 * does. The settings are process-wide (one launch shape per kernel instance
 * and device). The autotuner sets them from its cache. PI_EINVAL for limbs outside
 * -1..17 (-1 or 1..17 for pi_get_tuning), out-of-range values or NULL outputs. */
#define PI_TUNE_FUSED (-1)
PI_API int pi_set_tuning(int limbs, uint32_t wg_per_cu, uint32_t run_cap);
PI_API int pi_get_tuning(int limbs, uint32_t *wg_per_cu, uint32_t *run_cap);

/* Arithmetic of the head terms' modular exponentiation (section 4.2 names
 * successive squaring and Montgomery's method). Both modes compute the same
 * exact integers, so every result is bit-identical:
 *   PI_ARITH_FAST (default): moduli from 2^29 to 2^51 run on integer-valued
 *     binary64 numbers whose every operation is exact, for both the
 *     exponentiation and the division into P bits (fp64 FMA issues at the
 *     same rate as a 32-bit integer multiply-add and needs fewer
 *     instructions); Montgomery below and above;
 *   PI_ARITH_INTEGER: integer Montgomery arithmetic for every modulus.
 * The mode belongs to the calling host thread (each thread starts in
 * PI_ARITH_FAST) and is read when that thread plans a query (pi_extract*,
 * pi_sum_slice*, pi_extract_batch, pi_batch_create, pi_server_submit).
 * PI_EINVAL for an unknown mode. */
enum { PI_ARITH_FAST = 0, PI_ARITH_INTEGER = 1 };
PI_API int pi_set_arith(int mode);
PI_API int pi_get_arith(void);

/* Static text for a return code. */
PI_API const char *pi_strerror(int code);

/* Release the library's scratch memory on every device. */
PI_API void pi_shutdown(void);

/* ---- serving: continuous batching ------------------------------------------
 *
 * A server owns a stream-ordered pool of query slots on one device. Queries
 * are admitted while a slot can be had (the pool grows on demand within a
 * device-memory cap, see pi_server_set_memory_limit), each step gives every
 * active query a fair share of the step's head terms, and a query's
 * carry-save partial sum stays in its device slot across steps until its
 * last chunk is done; it is then finalized and its result can be polled. A query's result is bit-identical
 * to pi_extract_ex on its own, whatever else is in flight. This is the
 * one-GPU counterpart of section 4.3's admission of small jobs as cluster
 * slots free up. A server is not thread-safe; use one per host thread. */
typedef struct pi_server pi_server;

/* A finished query, copied to the host by pi_server_poll. */
typedef struct {
  uint64_t tag;        /* the caller's tag from pi_server_submit */
  int32_t code;        /* PI_OK when certified, PI_UNCERTAIN otherwise */
  uint32_t P;
  uint64_t nterms;     /* N, as in pi_status */
  uint64_t limbs[17];  /* left-aligned S in the first ceil(P/64) limbs */
} pi_result;

/* PI_BUSY: pi_server_submit found no free slot; submit again after a step. */
#define PI_BUSY 2

/* Create a server on the current device and `stream`.
 *   max_active: the most queries admitted at once (slots are allocated as
 *   admission needs them, within the memory cap); step_terms: head terms per
 *   step (the step's budget, shared fairly by the active queries). */
PI_API int pi_server_create(uint32_t max_active, uint64_t step_terms, hipStream_t stream,
                            pi_server **out);

/* Cap the device memory the server's query slots may take (bytes; the
 * default is a quarter of the device memory free at creation). Slots are
 * allocated on demand, doubling the pool, only while the cap and the
 * device's free memory (the last eighth is never taken) allow: admission is
 * by device memory. Lowering the cap below what is in use admits nothing new
 * until enough queries finish. */
PI_API int pi_server_set_memory_limit(pi_server *s, size_t bytes);

/* depth 1 (the default): pi_server_step returns with its step still running
 * and the host plans the next one meanwhile; a query submitted then joins
 * the step after next. depth 0: pi_server_step waits for its own step, so a
 * query submitted after it returns joins the next step, while the device
 * idles during planning. Higher throughput against lower latency; results
 * are the same. PI_EINVAL for other depths. */
PI_API int pi_server_set_pipeline(pi_server *s, int depth);

/* Admit one query (host struct; out_offset is ignored). Returns PI_OK,
 * PI_BUSY when no slot can be had (max_active or the memory cap reached), or
 * an argument error. */
PI_API int pi_server_submit(pi_server *s, const pi_query *q, uint64_t tag);

/* Withdraw an admitted query that is still being summed (section 4 lets
 * running jobs be killed and the computation be resumed later; here one
 * query is dropped and may be submitted again): it takes no part in the
 * steps that follow, its slot is freed at once and no result is delivered
 * for it. Chunks of it that a step already queued still run, into the freed
 * slot, and the slot's next user clears it with a kernel queued behind them.
 * Submitting the same query again starts it afresh. Host work only; nothing
 * waits. With several active queries under one tag, the earliest submitted
 * is withdrawn. PI_EINVAL when none is active under the tag: its last chunks
 * already ran (its result is on the way), it was delivered, or the tag is
 * unknown. */
PI_API int pi_server_cancel(pi_server *s, uint64_t tag);

/* Plan and enqueue one step on the server's stream, then wait for the
 * previous step (pipelined, the default: the host plans the next step while
 * the device runs this one) or for this one (depth 0), and deliver the
 * finished queries' results; with nothing left to plan it waits for every
 * step in flight. *finished (may be NULL) receives the number of results
 * delivered. */
PI_API int pi_server_step(pi_server *s, uint32_t *finished);

/* Move up to `max` completed results to `out` (host); *count receives how
 * many. */
PI_API int pi_server_poll(pi_server *s, pi_result *out, uint32_t max, uint32_t *count);

/* Queries admitted whose results have not been delivered yet. */
PI_API uint32_t pi_server_active(const pi_server *s);

/* The most queries the server admits at once: max_active, or fewer when
 * the memory cap allows fewer slots. */
PI_API uint32_t pi_server_capacity(const pi_server *s);

PI_API void pi_server_destroy(pi_server *s);

#ifdef __cplusplus
}
#endif
#endif
