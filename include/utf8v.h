/*
 * utf8v -- lookup UTF-8 validation on AMD Instinct MI355X (gfx950).
 *
 * Implements the lookup algorithm of Keiser & Lemire, "Validating UTF-8 In Less
 * Than One Instruction Per Byte" (section 6): every byte is classified together
 * with its predecessor through three 16-entry nibble tables ANDed into an
 * error-class byte (section 6.1, tables following the error patterns of
 * Table 8), required third/fourth continuation bytes are checked (section
 * 6.2), the end of the input must not cut a character (section 6.3), and
 * all-ASCII spans skip the classification (section 6.4).
 *
 * What is computed.  A byte string is valid when it is a concatenation of the
 * well-formed characters of Table 1 (section 2), i.e. it breaks none of the
 * six rules of section 3 (5+ byte lead, too short, too long, overlong, too
 * large, surrogate).  The paper decides validity only; this library also
 * reports the FIRST-ERROR OFFSET: the length of the longest valid prefix made
 * of whole characters (the start of the first ill-formed character), or -1
 * when the string is valid.  The empty string is valid.
 *
 * Memory.  Every buffer pointer given to these functions must be device
 * accessible (hipMalloc memory, a torch CUDA tensor, managed or pinned host
 * memory) unless it is documented as a host pointer.  The caller owns all
 * buffers; the library never frees or retains them.  The library owns a small
 * per-(device, stream) workspace (about 8 bytes per wave of the batch grid, 128 KiB
 * on 256 compute units; created and initialised on the stream by the first call
 * that uses it, freed by utf8v_release).
 *
 * Errors.  Functions returning int return UTF8V_OK (0) or a negative status.
 * Invalid UTF-8 is a result, never an error.  No function aborts or throws.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  *_async functions only enqueue work; the others synchronize the
 * stream before returning.  Calls that overlap on one stream are ordered by
 * the stream; the library serializes its own workspace per stream.
 */
#ifndef UTF8V_H
#define UTF8V_H

#include <stdbool.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UTF8V_OK 0
#define UTF8V_EINVAL (-1)     /* NULL pointer with a non-zero size, n < 0, bad offsets, bad config */
#define UTF8V_ENOTDEVICE (-2) /* a pointer the GPU cannot access (pageable host memory) */
#define UTF8V_EHIP (-3)       /* HIP runtime error; utf8v_last_hip_error() has the code */
#define UTF8V_ENOMEM (-4)     /* workspace allocation failed */

/*
 * utf8_validate -- true iff buf[0..len) is valid UTF-8 (section 6 lookup
 * algorithm over one buffer).  buf may be NULL iff len == 0; len < 2^40.
 * Synchronous on the default stream.  On misuse it returns false and sets
 * utf8v_last_status().
 */
bool utf8_validate(const uint8_t *buf, size_t len);

/*
 * utf8v_validate_ex -- validate buf[0..len) on `stream`, wait, and store the
 * first-error offset (-1 if valid) in *first_err (a HOST pointer, may be NULL).
 * Returns 1 if valid, 0 if invalid, or a negative status.
 */
int utf8v_validate_ex(const uint8_t *buf, size_t len, int64_t *first_err, void *stream);

/*
 * utf8v_validate_async -- enqueue the validation of buf[0..len) on `stream`;
 * the first-error offset (-1 if valid) is written to *dev_first_err (a DEVICE
 * pointer to one int64) when the stream reaches it.  No host synchronization.
 */
int utf8v_validate_async(const uint8_t *buf, size_t len, int64_t *dev_first_err, void *stream);

/*
 * utf8_validate_batch -- validate n strings given in CSR form: string k is
 * data[offsets[k] .. offsets[k+1]).  offsets has n+1 entries (device memory),
 * non-decreasing, offsets[0] >= 0 (need not be 0).  Every string is a stream of
 * its own: the bytes before its start count as zero and its end gets the end
 * check (section 6.3).  Outputs (device memory, n entries each):
 *   out_flags[k]     = 1 if string k is valid UTF-8, else 0;
 *   out_first_err[k] = first-error offset RELATIVE to the string start, or -1.
 * n == 0 is a no-op; n must be below 2^31 - 64 (else UTF8V_EINVAL: the kernel counts
 * string indices in 32 bits).  Synchronous on the default stream.  Offsets are trusted:
 * decreasing or out-of-range offsets give undefined results (use
 * utf8v_check_offsets first when they come from untrusted input).
 */
int utf8_validate_batch(const uint8_t *data, const int64_t *offsets, int64_t n,
                        uint8_t *out_flags, int64_t *out_first_err);

/* utf8v_validate_batch_async -- as utf8_validate_batch, enqueued on `stream`. */
int utf8v_validate_batch_async(const uint8_t *data, const int64_t *offsets, int64_t n,
                               uint8_t *out_flags, int64_t *out_first_err, void *stream);

/*
 * utf8v_validate_batch_graph -- as utf8v_validate_batch_async, launched as one
 * replay of a HIP graph holding the persistent validation kernel, made once per
 * (device, stream) and launch configuration.  Each call sets the kernel node's
 * arguments to this batch and launches the graph, so any batch shape replays the
 * same graph; replays already enqueued keep their own arguments.  The call must
 * not itself be made under stream capture (UTF8V_EINVAL): a capture would keep
 * this call's arguments in the caller's graph.  To capture a batch validation,
 * capture utf8v_validate_batch_async instead.
 */
int utf8v_validate_batch_graph(const uint8_t *data, const int64_t *offsets, int64_t n,
                               uint8_t *out_flags, int64_t *out_first_err, void *stream);

/*
 * utf8v_validate_batch_noalloc -- as utf8v_validate_batch_async, for callers that
 * cannot allocate memory (code under stream capture, tight serving loops): it never
 * calls hipMalloc or any other allocating routine, on any call.  The batch kernel's
 * cross-wave slots (one 64-bit word per wave of the persistent grid) live in a fixed
 * device array of 16384 words (128 KiB) that the library holds on every GPU it runs
 * on until the process ends; a launch configuration whose grid (compute units x
 * batch_waves_per_cu) needs more words is rejected with UTF8V_EINVAL.  The array is
 * zero when idle and every finished call leaves it zero.  All calls on one GPU share
 * it: calls that overlap on one GPU (on different streams, or from different threads
 * without ordering) race and must not be made.  Inputs, outputs and results are those
 * of utf8_validate_batch; n == 0 is a no-op.
 */
int utf8v_validate_batch_noalloc(const uint8_t *data, const int64_t *offsets, int64_t n,
                                 uint8_t *out_flags, int64_t *out_first_err, void *stream);

/*
 * utf8v_copy_validate -- enqueue one pass that copies src[0..len) to dst and
 * validates it (first-error offset to *dev_first_err, as utf8v_validate_async):
 * every byte is read once, for both jobs.  src may be device memory or pinned
 * host memory (then this is a validating host-to-device copy over PCIe); dst
 * device memory.  dst and src must have the same address modulo 16 and must not
 * overlap (else UTF8V_EINVAL).
 */
int utf8v_copy_validate(uint8_t *dst, const uint8_t *src, size_t len, int64_t *dev_first_err, void *stream);

/* ---- error classes ------------------------------------------------------------------ */

/*
 * Which rule of section 3 the first ill-formed character breaks, from a
 * first-error offset computed by the functions above:
 *   UTF8V_CLASS_NONE 0 (valid), 1 five or more header bits (rule a), 2 too short
 *   (rule b), 3 too long (rule c), 4 overlong (rule d), 5 too large (rule e),
 *   6 surrogate (rule f).
 * A character can break several rules (C0 alone is both a two-byte lead without
 * its continuation and an overlong lead); the malformed rules a, c, b rank first,
 * because only a complete sequence decodes to a code point, then d, e, f.
 */
#define UTF8V_CLASS_NONE 0
#define UTF8V_CLASS_FIVE_PLUS 1
#define UTF8V_CLASS_TOO_SHORT 2
#define UTF8V_CLASS_TOO_LONG 3
#define UTF8V_CLASS_OVERLONG 4
#define UTF8V_CLASS_TOO_LARGE 5
#define UTF8V_CLASS_SURROGATE 6

/*
 * utf8v_error_class -- enqueue: *dev_class (device uint8) = class of buf's
 * first error, given its first-error offset in *dev_first_err (device int64, as
 * written by utf8v_validate_async).
 */
int utf8v_error_class(const uint8_t *buf, size_t len, const int64_t *dev_first_err, uint8_t *dev_class,
                      void *stream);

/*
 * utf8v_error_classes -- enqueue: out_class[k] = class of string k's first
 * error, from first_err[k] as written by the batch functions (relative offsets,
 * -1 = valid).  All arrays in device memory; n == 0 is a no-op.
 */
int utf8v_error_classes(const uint8_t *data, const int64_t *offsets, int64_t n, const int64_t *first_err,
                        uint8_t *out_class, void *stream);

/* ---- streams: one byte sequence fed in chunks --------------------------------------- */

/*
 * A stream validates the concatenation of the chunks fed to it, as one buffer
 * (section 6: the previous input carries over; section 6.3: the end check is
 * applied once, at finish).  Splitting the bytes anywhere -- inside a
 * character, into empty or one-byte chunks -- gives the same result as
 * validating them whole.  The state (first-error offset and the last 8 bytes)
 * lives on the device, so updates are asynchronous and ordered by the HIP
 * stream they are enqueued on; use one HIP stream per utf8v_stream and call it
 * from one host thread at a time.  Streams are limited to 2^40 - 1 bytes.
 */
typedef struct utf8v_stream utf8v_stream;

/* Create an empty stream on the current device (its reset is enqueued on `stream`). */
int utf8v_stream_create(utf8v_stream **out, void *stream);

/*
 * Enqueue the validation of the next chunk (device memory, len bytes; may be
 * NULL iff len == 0).  The chunk must stay unchanged until the call is done on
 * `stream`.  Offsets reported later are stream positions.
 */
int utf8v_stream_update(utf8v_stream *s, const uint8_t *chunk, size_t len, void *stream);

/*
 * Apply the end check, wait, and report: *first_err (host, may be NULL) = the
 * stream's first-error offset (start of the first ill-formed character), or -1.
 * Returns 1 if valid, 0 if invalid, or a negative status.  The stream may be fed
 * further afterwards (a later finish checks the longer stream's end).
 */
int utf8v_stream_finish(utf8v_stream *s, int64_t *first_err, void *stream);

/* Enqueue a reset to the empty stream. */
int utf8v_stream_reset(utf8v_stream *s, void *stream);

/* Bytes fed since creation or the last reset (host-side count), -1 for NULL. */
int64_t utf8v_stream_position(const utf8v_stream *s);

/* Free the stream.  No call on it may be in flight. */
int utf8v_stream_destroy(utf8v_stream *s);

/*
 * utf8v_check_offsets -- 1 if offsets[0..n] (device memory) is non-decreasing
 * with offsets[0] >= 0, else 0; negative status on error.  Synchronous.
 */
int utf8v_check_offsets(const int64_t *offsets, int64_t n, void *stream);

/* ---- serving: continuous batching of requests ---------------------------------------- */

/*
 * A server validates requests -- each one a CSR batch of strings, with the
 * semantics of utf8_validate_batch -- submitted at any time from any thread.  A
 * scheduler thread admits pending requests in submission order into a device ring
 * of budget_bytes and launches them together as one batch as soon as one of
 * max_inflight batch slots is free (continuous batching; consecutive batches use
 * alternating streams and overlap on the GPU).  Per batch it copies the payloads
 * and offsets straight from the requests' pinned host memory into the ring,
 * validates them in one launch and writes every request's results back into its
 * host arrays.  A request's results do not depend on what it is batched with.
 */
typedef struct {
  uint64_t budget_bytes;      /* device ring (admission budget), default 8 GiB */
  uint64_t max_batch_bytes;   /* payload bytes per batch (and per request), default 64 MiB */
  int64_t max_batch_strings;  /* strings per batch incl. one separator per request, default 4 Mi */
  int32_t max_batch_requests; /* requests per batch, default 4096 */
  int32_t max_inflight;       /* batches on the GPU at once, 1..64, default 4 */
  int32_t streams;            /* streams the batches alternate over, 1..8, default 2 */
  int32_t max_pending;        /* submitted but unfinished requests, default 262144 */
} utf8v_server_config;

typedef struct utf8v_server utf8v_server;

/* Fill *cfg with the defaults above. */
int utf8v_server_default_config(utf8v_server_config *cfg);

/*
 * Create a server on the current device (allocates the ring, pinned staging and
 * streams; starts the scheduler thread).  UTF8V_EINVAL if a limit is out of range
 * or the budget cannot hold the largest batch the limits allow.
 */
int utf8v_server_create(const utf8v_server_config *cfg, utf8v_server **out);

/*
 * Submit one request: strings data[offsets[k] .. offsets[k+1]), k < n.  offsets
 * (n+1 entries) must be pinned host memory (read by the host and the GPU); data,
 * out_flags and out_first_err pinned host or device memory.  All four must stay
 * valid until the request is done.  Results: as utf8_validate_batch.  *ticket
 * identifies the request.  Blocks only while max_pending requests are unfinished.
 * UTF8V_EINVAL for a request larger than the batch limits.
 */
int utf8v_server_submit(utf8v_server *srv, const uint8_t *data, const int64_t *offsets, int64_t n,
                        uint8_t *out_flags, int64_t *out_first_err, uint64_t *ticket);

/*
 * 1 if the request is done (its results are in place; *done_ns, if not NULL,
 * gets the utf8v_clock_ns() time it was seen done), 0 if not yet, < 0 on error.
 */
int utf8v_server_poll(utf8v_server *srv, uint64_t ticket, int64_t *done_ns);

/* Wait until the request is done; as poll otherwise (returns UTF8V_OK when done). */
int utf8v_server_wait(utf8v_server *srv, uint64_t ticket, int64_t *done_ns);

/* out4 = {requests done, batches launched, largest batch (requests), ring bytes}. */
int utf8v_server_stats(utf8v_server *srv, int64_t *out4);

/* Finish every submitted request, stop the scheduler and free everything. */
int utf8v_server_destroy(utf8v_server *srv);

/* Monotonic clock used for done times, in nanoseconds. */
int64_t utf8v_clock_ns(void);

/*
 * utf8v_serve_replay -- open-loop load generator for measurements.  Request i
 * (nreq of them, arrival_ns non-decreasing, relative to the start) is pool entry
 * pick[i] of npool requests given as parallel arrays (pinned host memory as for
 * utf8v_server_submit).  It is submitted at its arrival time, whether or not
 * earlier requests are done, and latency_ns[i] = (time its results are on the
 * host) - (its arrival time).  mode 0: through a server made with cfg;
 * mode 1: one synchronous launch per request, in arrival order (copy in,
 * validate, copy out, wait).  *span_ns (may be NULL) = last completion - first
 * arrival.  Results land in the pool's result arrays (the same values for every
 * repetition of an entry).
 */
int utf8v_serve_replay(const utf8v_server_config *cfg, int mode, const uint8_t *const *req_data,
                       const int64_t *const *req_offsets, const int64_t *req_n, uint8_t *const *req_flags,
                       int64_t *const *req_errs, int npool, const int64_t *arrival_ns, const int32_t *pick,
                       int64_t nreq, int64_t *latency_ns, int64_t *span_ns);

/* ---- tuning ------------------------------------------------------------------------- */

typedef struct {
  int32_t unroll;            /* single buffer: dwordx4 loads per lane per tile, 1, 2, 4 or 8 */
  int32_t waves_per_cu;      /* single buffer: persistent waves per compute unit, >= 1 */
  int32_t ascii;             /* 1: skip classification of all-ASCII wave tiles (section 6.4; tested per
                                tile of `unroll` KiB, with an exponential back-off after a non-ASCII one) */
  int32_t batch_waves_per_cu; /* batch: persistent one-wave workgroups per compute unit, 1..64 */
  int32_t batch_ascii;       /* batch: 1 = skip the classification of all-ASCII wave tiles (section 6.4,
                                with the same back-off as the single-buffer kernel) */
  int32_t batch_unroll;      /* batch: 1 KiB slabs per wave tile (the bytes a lane checks per tile / 16),
                                4 or 8; an 8 KiB tile halves the per-tile work on long strings and needs
                                twice the LDS per wave */
} utf8v_config;

/* Read / replace the launch configuration of the calling process (all devices). */
int utf8v_get_config(utf8v_config *cfg);
int utf8v_set_config(const utf8v_config *cfg);

/*
 * utf8v_autotune_single -- time every single-buffer launch configuration
 * (unroll 2/4/8 x waves per CU 8..40 x ASCII skip off/on) on the sample buffers
 * bufs[i][0..lens[i]) (device memory; bufs and lens are host arrays of nbufs),
 * in `rounds` interleaved rounds, and keep the one with the least median time:
 * it becomes the process configuration and is stored in *best.  times_ms (host,
 * may be NULL) receives up to max_times per-candidate medians in candidate order.
 * Returns the number of candidates, or a negative status (configuration unchanged).
 * Results never depend on the configuration; only speed does.
 */
int utf8v_autotune_single(const uint8_t *const *bufs, const size_t *lens, int nbufs, int rounds,
                          utf8v_config *best, float *times_ms, int max_times);

/*
 * utf8v_autotune_batch -- the same for the batch kernel: persistent grid (4..64
 * one-wave workgroups per CU) x section 6.4 ASCII test (off/on) x wave tile (4 or
 * 8 KiB), on a sample CSR batch (device memory, with output arrays of n entries the
 * timing runs overwrite).
 */
int utf8v_autotune_batch(const uint8_t *data, const int64_t *offsets, int64_t n, uint8_t *out_flags,
                         int64_t *out_first_err, int rounds, utf8v_config *best, float *times_ms, int max_times);

/* ---- diagnostics and measurement -------------------------------------------------- */

/*
 * utf8v_classify -- for positions 0..len of buf (device), write the section 6.1
 * classification byte to sc[i] and the per-position error byte (classification
 * XOR the section 6.2 requirement) to err[i]; position len is the end check on
 * a virtual zero byte.  sc and err are device arrays of len+1 bytes.  Async.
 */
int utf8v_classify(const uint8_t *buf, size_t len, uint8_t *sc, uint8_t *err, void *stream);

/*
 * utf8v_read_ceiling / utf8v_copy -- plain streaming kernels over len bytes
 * (len a multiple of 16, 16-byte aligned device buffers) used as the measured
 * memory ceiling next to the validator.  read_ceiling ORs words into *dev_out.
 */
int utf8v_read_ceiling(const uint8_t *buf, size_t len, uint32_t *dev_out, void *stream);
int utf8v_copy(const uint8_t *src, uint8_t *dst, size_t len, void *stream);

/* Status of the last call on this host thread, its message, and the last HIP error code. */
int utf8v_last_status(void);
const char *utf8v_strerror(int status);
int utf8v_last_hip_error(void);

/* Number of compute units of the current device (0 if no device). */
int utf8v_num_cus(void);

/* Free the workspaces of the calling process.  No call may be in flight. */
int utf8v_release(void);

#ifdef __cplusplus
}
#endif

#endif /* UTF8V_H */
