/*
 * rs.h -- C ABI of the MI355X (gfx950) novel-polynomial-basis Reed-Solomon
 * erasure codec: the transform Psi_h^l and its inverse, the formal
 * derivative, and the (n, k) encoder and erasure decoder built on them
 * (Lin, Chung, Han, "Novel Polynomial Basis and Its Application to
 * Reed-Solomon Erasure Codes", arXiv:1404.3458).
 *
 * Library: librs_nb.so (HIP, hand-written gfx950 kernels).  No torch or HIP
 * type appears in these signatures: device buffers are plain pointers and a
 * stream is an opaque hipStream_t passed as void* (NULL = the null stream).
 *
 * Conventions fixed by this library where the paper leaves a choice:
 *   - field GF(2^r), r in {8, 16}; field polynomial 0x11D (r = 8) or 0x1100B
 *     (r = 16); primitive element alpha = 2 (it only enters the locator's
 *     logarithms and never changes an output);
 *   - symbols: r = 8 -> one byte; r = 16 -> a little-endian 16-bit word.  Bit
 *     b of a symbol is the coefficient of x^b.  Row t of a buffer starts at
 *     byte t * row_bytes; symbol c of a row is at byte c * (r / 8);
 *   - points: omega_i = sum_j i_j v_j over the basis v (Sec. 2.1);
 *   - codeword rows: message row i is the point omega_i (eq. F(i)=m_i);
 *     parity row t is the point omega_{k'+t} where k' = pow2ceil(k);
 *   - shortening (Sec. 5 allows any k through zero padding): the mother code
 *     is (n', k') with n' = pow2ceil(k' + n - k) <= 2^r; points
 *     omega_k..omega_{k'-1} carry virtual zero symbols and points
 *     omega_{k'+n-k}..omega_{n'-1} are never stored;
 *   - nb_fft output b is [D](omega_b + omega_l) for any shift l < 2^r (the
 *     definition of Psi_h^l in Sec. 3); these are consecutive points only
 *     when h divides l.
 *
 * Ownership and ordering: data pointers are device memory owned by the
 * caller and must stay valid until the stream reaches the call.  Host arrays
 * (erasure masks, descriptors) are copied before the call returns.  Work is
 * stream-ordered; calls that share a context but run on different streams
 * use separate per-stream scratch.  Argument errors are returned before any
 * work is queued, with no partial writes.  Device faults surface as
 * RS_EDEVICE from the next call or from rs_sync().
 */
#ifndef RS_NB_H
#define RS_NB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_ctx rs_ctx;

enum {
    RS_OK = 0,
    RS_EINVAL = -1,    /* null pointer or invalid argument */
    RS_EFIELD = -2,    /* r not in {8, 16} */
    RS_EBASIS = -3,    /* basis not F2-independent or out of range */
    RS_ESHAPE = -4,    /* h or (n, k) not supported: see each call */
    RS_ETOOMANY = -5,  /* more than n - k erasures */
    RS_EALIGN = -6,    /* row length not a multiple of the symbol size */
    RS_ENOMEM = -7,    /* device or pinned host allocation failed */
    RS_EDEVICE = -8    /* a HIP call or kernel failed */
};

/* Create a context on the current HIP device (Sec. 2.1, 2.2, 3.5, 4.2 and
 * the appendix).  basis: r field elements v_0..v_{r-1}, F2-independent, each
 * < 2^r; NULL selects v_j = 2^j (omega_i = i).  Builds, on the device, the
 * skew-factor table W_i(omega_{b 2^{i+1}}) / W_i(omega_{2^i}) for every level
 * i < r (2^r - 1 factors, Sec. 3.5), the derivative table B of eq. B and its
 * inverses, the log/exp tables and the Walsh-Hadamard transforms of the
 * logarithm vector L_N for every N = 2^t <= 2^r (appendix).  The context owns
 * only these tables and per-stream scratch; free it with rs_free. */
int rs_init(int r, const uint32_t *basis, rs_ctx **out);
void rs_free(rs_ctx *ctx);

/* Algorithm 1.  msg: k rows, parity: n - k rows, each row_bytes long,
 * row-major and contiguous, device memory, not overlapping.  Writes the n - k
 * parity rows of the systematic codeword (message rows are the codeword's
 * first k rows and are not copied).  1 <= k < n, n' <= 2^r (RS_ESHAPE);
 * row_bytes a multiple of r/8 (RS_EALIGN); row_bytes == 0 is a no-op. */
int rs_encode(rs_ctx *ctx, int n, int k, const void *msg, void *parity,
              size_t row_bytes, void *stream);

/* Algorithm 2.  shards: n rows (device); erasure_mask: n host bytes, nonzero
 * = erased (the erased rows of shards are never read).  On return every row
 * of out (n rows, device) holds the codeword: erased rows recovered,
 * surviving rows copied unless out == shards (in place).  Any number of
 * erasures e <= n - k is accepted (RS_ETOOMANY otherwise); e == 0 copies. */
int rs_decode(rs_ctx *ctx, int n, int k, const uint8_t *erasure_mask,
              const void *shards, void *out, size_t row_bytes, void *stream);

/* rs_decode without any allocation, for callers that cannot allocate (code
 * under HIP graph capture, serving loops that must not call hipMalloc,
 * harnesses that forbid it): arguments, results and errors as rs_decode,
 * but the call's device arena (stripe descriptors, point bitmaps, the
 * locator's per-point tables: at most 32 KiB) lives in a fixed array of the
 * library in each GPU's memory, held until the process ends, and the
 * host-built part of it reaches the device as a kernel argument, so the call
 * allocates no device or pinned host memory and queues no host-to-device
 * copy.  Only mother codes of n' <= 256 points (the single-kernel decodes)
 * fit; larger ones return RS_ESHAPE.  Every call on a GPU shares that GPU's
 * array, which keeps the last call's contents: calls on one stream are
 * ordered, calls that overlap on one GPU (other streams, other contexts,
 * other threads) race and must be ordered by the caller. */
int rs_decode_static(rs_ctx *ctx, int n, int k, const uint8_t *erasure_mask,
                     const void *shards, void *out, size_t row_bytes, void *stream);

/* Transform Psi_h^l (Sec. 3.2) and its inverse (Sec. 3.3), in place on h
 * rows of `data` (device); each column of symbols is one coefficient vector
 * (nb_fft input) or one evaluation vector (nb_ifft input).  h a power of two,
 * 1 <= h <= 2^r; l < 2^r. */
int nb_fft(rs_ctx *ctx, int h, uint32_t l, void *data, size_t row_bytes, void *stream);
int nb_ifft(rs_ctx *ctx, int h, uint32_t l, void *data, size_t row_bytes, void *stream);

/* Formal derivative (Sec. 4.2): replaces each column's coefficients of
 * [D_h](x) by those of [D_h]'(x), in place; h as for nb_fft. */
int nb_derivative(rs_ctx *ctx, int h, void *data, size_t row_bytes, void *stream);

/* Product in the novel basis (Sec. 6.1, Table 1): for each column, out holds the 2h
 * coefficients of [A_h](x) [B_h](x), computed as the inverse transform
 * Psi_2h^l of the point-by-point product of the transforms Psi_2h^l of A and
 * B padded with h zero coefficients (the last output coefficient is zero).
 * a and b: h rows; out: 2h rows, overlapping neither (RS_EINVAL).  h a power
 * of two with 2h <= 2^r (RS_ESHAPE); l < 2^r (any l: the 2h points
 * omega_b + omega_l are distinct, and the product does not depend on l).
 * Uses the stream's scratch of the context (2h rows). */
int nb_polymul(rs_ctx *ctx, int h, uint32_t l, const void *a, const void *b, void *out, size_t row_bytes,
               void *stream);

/* Degree (Sec. 6.1, Table 1): deg[c] (device, one int32 per column) = the largest j < h
 * whose coefficient in column c is nonzero (deg X_j = j), or -1.
 * 1 <= h <= 2^r (any h). */
int nb_degree(rs_ctx *ctx, int h, const void *data, size_t row_bytes, int32_t *deg, void *stream);

/* Basis conversion in place, each column a polynomial of degree < h: novel
 * -> monomial coefficients of x^0 .. x^(h-1), and back.  Computed level by
 * level from X_{i + 2^(t-1)} = X_i What_{t-1} (Definition 1) and the
 * monomials of What_{t-1}, which sit at the degrees 2^m (Sec. 2.2):
 * O(h lg^2 h) operations per column.  h a power of two <= 2^r.
 * nb_to_monomial uses the stream's scratch of the context (h rows). */
int nb_to_monomial(rs_ctx *ctx, int h, void *data, size_t row_bytes, void *stream);
int nb_from_monomial(rs_ctx *ctx, int h, void *data, size_t row_bytes, void *stream);

/* One stripe of a batch.  Encode: in = k message rows, out = n - k parity
 * rows.  Decode: in = n shard rows, out = n rows (may equal in). */
typedef struct rs_stripe_desc {
    int32_t n, k;
    uint64_t row_bytes;
    const void *in;
    void *out;
} rs_stripe_desc;

/* Batched Algorithm 1 / Algorithm 2 over `count` independent stripes of
 * possibly different (n, k) and row lengths, queued as a few launches.
 * masks: for decode, the stripes' erasure masks concatenated in descriptor
 * order (sum of n bytes, host).  Every descriptor is validated as for the
 * single-stripe call before any work is queued. */
int rs_encode_batch(rs_ctx *ctx, const rs_stripe_desc *descs, int count, void *stream);
int rs_decode_batch(rs_ctx *ctx, const rs_stripe_desc *descs, const uint8_t *masks,
                    int count, void *stream);

/* Reusable batch plans (the batched calls above, planned once).  A plan
 * validates its stripes, builds their descriptors and point bitmaps and
 * allocates their scratch once, on the context's device; a decode plan also
 * runs the erasure locator once (Algorithm 2 step 1 depends only on the
 * erasure patterns, which the plan fixes), so its launches run steps 2-6
 * only.  rs_plan_launch queues only kernels and device-to-device copies (no
 * host-to-device copy, no allocation), so a launch can be captured in a HIP
 * graph and replayed.
 * The buffers the descriptors name must stay valid for the plan's life; their
 * contents may change between launches (a decode plan fixes the erasure
 * pattern).  Launches of one plan must be ordered (one stream, or events):
 * the plan's scratch rows live in its own device memory.  Errors as for
 * the batched calls; RS_ENOMEM if the plan's device memory cannot be
 * allocated. */
typedef struct rs_plan rs_plan;
int rs_plan_encode_batch(rs_ctx *ctx, const rs_stripe_desc *descs, int count, rs_plan **out);
int rs_plan_decode_batch(rs_ctx *ctx, const rs_stripe_desc *descs, const uint8_t *masks, int count,
                         rs_plan **out);
int rs_plan_launch(rs_plan *plan, void *stream);
/* Completion timestamps of the stripes of a plan (the per-stripe timing of a
 * batch): each later launch first sets ts[0] to the device's real-time
 * counter; every workgroup of every kernel of the launch then raises a slot
 * of its own to the counter as its waves finish (a vector atomic maximum),
 * and a last kernel of the launch sets ts[1 + i] to the latest slot of the
 * workgroups that worked on stripe i, so ts[1 + i] - ts[0] is when stripe i
 * was done.  ts[1 + i] is 0 when no kernel works on the stripe (no columns;
 * a decode without erasures, which is nothing in place and a copy
 * otherwise).  dev_ts: count + 1 device uint64 (NULL stops the stamps);
 * clock_khz (may be NULL) receives the counter's rate.  The first call with
 * a non-NULL dev_ts allocates the plan's slots (8 bytes per workgroup of its
 * launches, freed with the plan): RS_ENOMEM if they cannot be allocated.  A
 * graph captured from the plan keeps the setting it was captured with. */
int rs_plan_set_timestamps(rs_plan *plan, uint64_t *dev_ts, int *clock_khz);
/* Waits for the device, then frees the plan (NULL is a no-op). */
void rs_plan_free(rs_plan *plan);

/* Serving: a request loop with continuous batching.  Requests are admitted
 * first-in first-out while the bytes they keep in flight (codeword rows,
 * scratch of codes over more than 256 points, locator tables) fit the budget;
 * admitted requests are grouped into encode and decode batches (at most
 * max_batch requests each) and queued on one of nstreams streams of default
 * priority, so batches formed while others run overlap on the device.  A
 * scheduler thread owned by the server does the grouping, launching and
 * completion tracking; results are bit-identical to the single calls.
 * Completion times are CLOCK_MONOTONIC nanoseconds taken when the batch's
 * event is observed complete.  Buffers must stay valid until the request's
 * completion is returned; requests whose buffers overlap are the caller's
 * race.  A request larger than the budget is admitted alone, and nothing
 * else is admitted while it is in flight.  The server's streams do not
 * follow any stream of the caller's unless a request names one (`after`). */
typedef struct rs_server rs_server;
enum { RS_OP_ENCODE = 0, RS_OP_DECODE = 1 };
typedef struct rs_request {
    int32_t op;             /* RS_OP_ENCODE or RS_OP_DECODE */
    rs_stripe_desc desc;    /* as in the batched calls */
    const uint8_t *mask;    /* decode: n bytes, host, copied by rs_server_submit */
    uint64_t tag;           /* returned with the completion */
    void *after;            /* a hipStream_t or NULL: the request's kernels start only
                               after the work queued on that stream before the
                               submit (the producer of its input) has finished */
} rs_request;
typedef struct rs_completion {
    uint64_t tag;
    int32_t status;         /* RS_OK, or the error of this request's batched call
                               (a failed batch is retried request by request, so
                               a request reports its own error) */
    int64_t t_done_ns;
} rs_completion;
int rs_server_create(rs_ctx *ctx, size_t budget_bytes, int max_batch, int nstreams, rs_server **out);
/* Runs the checks the batched calls run on a descriptor (mother code
 * n' <= 2^r, 1 <= k < n, row_bytes a multiple of r/8, non-null rows, at most
 * n - k erasures) and returns their error without queueing anything, then
 * queues; never blocks on the device.  RS_EDEVICE if the `after` stream
 * cannot be marked. */
int rs_server_submit(rs_server *srv, const rs_request *req);
/* Admission record of a server, for checking the budget: bytes are the
 * in-flight bytes of the admission rule above. */
typedef struct rs_server_stats {
    uint64_t budget;              /* the budget given to rs_server_create */
    uint64_t inflight_bytes;      /* now */
    uint64_t peak_bytes;          /* largest in-flight total after any admission */
    uint64_t peak_shared_bytes;   /* the same, over admissions under the budget rule
                                     (every one but a lone oversized request) */
    uint64_t oversize_admitted;   /* requests admitted alone above the budget */
    uint64_t largest_oversize;    /* bytes of the largest of them (0 if none) */
    uint64_t admitted;            /* requests admitted */
    uint64_t batches;             /* batched calls queued */
    uint64_t retried;             /* requests rerun alone after their batch failed */
} rs_server_stats;
int rs_server_get_stats(rs_server *srv, rs_server_stats *out);
/* Returns up to `max` completions (count >= 0), waiting up to timeout_ms
 * (0: do not wait, < 0: until at least one) when none is ready. */
int rs_server_poll(rs_server *srv, rs_completion *out, int max, int timeout_ms);
/* Requests submitted and not yet returned by rs_server_poll. */
int rs_server_pending(rs_server *srv);
/* Finishes every queued request, then frees the server (NULL is a no-op). */
void rs_server_free(rs_server *srv);

/* Schedules of the pass pipelines used by codes whose transforms exceed
 * 256 points (GF(2^16) only).  Such a transform over 2^N points is split
 * into 2 to 4 parts of consecutive levels, each applied by passes over
 * groups of rows that differ only in that part's index bits: level i only
 * pairs rows j and j + 2^i (Sec. 3.2), so such a group can apply those
 * levels alone.  parts[0] is the low part (groups of consecutive rows); each
 * part has 4 to 8 levels and they sum to N.  The default is two parts,
 * ceil(N / 2) low.  op selects the encoder (N = lg k', the size of its
 * transforms) or the decoder (N = lg n').  A schedule changes only the
 * speed, never an output; calls and plans built after the change use it.
 * rs_schedule_set is the two-part form (T1 low levels; T1 = 0 restores the
 * default); rs_schedule_set_parts takes the list (nparts = 0 restores the
 * default).  rs_init applies the environment variable RS_NB_SCHEDULE, a
 * comma-separated list of "enc:N:P" and "dec:N:P" entries where P is the low
 * part's count or the counts joined by '/', low part first, optionally
 * followed by ":C" with C the column tile of rs_schedule_set_tile, and
 * returns RS_EINVAL when it is malformed.
 * Errors: RS_ESHAPE for r = 8 or N outside 9..16; RS_EINVAL for a bad op or
 * split. */
int rs_schedule_set(rs_ctx *ctx, int op, int N, int T1);
int rs_schedule_set_parts(rs_ctx *ctx, int op, int N, const int *parts, int nparts);
/* The schedule in effect for (op, N): the low part's count, or the parts
 * (parts: room for 4). */
int rs_schedule_get(rs_ctx *ctx, int op, int N, int *T1);
int rs_schedule_get_parts(rs_ctx *ctx, int op, int N, int *parts, int *nparts);
/* Column tiles of the pass pipelines of (op, N): a workgroup covers 256
 * columns (64 lanes of 4 columns each), or, in the "packed" form of the
 * two-part pipelines' passes, 128 columns with each wave's two halves
 * holding two sets of rows.  cols = 0 (the default): 256-column tiles, and
 * packed ones for rows of at most 128 columns; 128: packed tiles for every
 * row; 256: 256-column tiles for every row.  Like the level split this
 * changes only the speed, never an output.
 * Errors: RS_ESHAPE for r = 8 or N outside 9..16; RS_EINVAL for a bad op or
 * cols. */
int rs_schedule_set_tile(rs_ctx *ctx, int op, int N, int cols);
int rs_schedule_get_tile(rs_ctx *ctx, int op, int N, int *cols);

/* Wait for all work of this context on `stream`; reports deferred device
 * errors. */
int rs_sync(rs_ctx *ctx, void *stream);

/* Copy one of the context's raw tables to host memory (inspection and
 * tests).  which: RS_TAB_SKEW (2^r - 1 factors, level i at offset
 * 2^r - 2^{r-i}, entry b = W_i(omega_{b 2^{i+1}}) / W_i(omega_{2^i})),
 * RS_TAB_B and RS_TAB_BINV (2^r entries: B_j of eq. B and its inverse),
 * RS_TAB_LOG and RS_TAB_EXP (2^r entries each, Log(0) = 0).  count must be
 * at least the table length; returns the length or a negative error. */
enum { RS_TAB_SKEW = 0, RS_TAB_B = 1, RS_TAB_BINV = 2, RS_TAB_LOG = 3, RS_TAB_EXP = 4 };
int rs_get_table(rs_ctx *ctx, int which, uint32_t *host_out, size_t count);

/* Static description of an error code. */
const char *rs_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RS_NB_H */
