/*
 * falcon.h -- C ABI of the MI355X Falcon codec (lossless compression of
 * float32 / float64 arrays, arXiv 2511.04140).
 *
 * Problem statement followed (Sec. 3, Sec. 4 of the paper): a set V of n
 * floating-point values is split into chunks of 1025 values; each chunk is
 * turned into integers (Alg. 2 decimal-place detection and Eq. 3), delta +
 * zigzag coded (Eq. 4) and written with the adaptive sparse/dense bit-plane
 * layout (Sec. 3.3, Fig. 9); the variable-length chunks are packed into one
 * stream by an exclusive prefix sum of their sizes (Sec. 3.4).  Decompression
 * is the exact inverse (Sec. 4): decompress(compress(x)) reproduces every
 * bit of x, NaN payloads, infinities, -0.0 and subnormals included.
 *
 * Stream format (little-endian):
 *   bytes  0..31  header: "FLCN", version u8 = 1, dtype u8 (1 = f32,
 *                 2 = f64), u16 0, chunk length u32 = 1025, u32 0,
 *                 value count N u64, payload byte count u64
 *   bytes 32..    one u32 compressed size per chunk (ceil(N / 1025) of them)
 *   then          the chunk payloads back to back, in chunk order
 * Each chunk payload: alpha_max u8, beta_hat_max u8, z_1 (8 bytes f64,
 * 4 bytes f32), bit width w u8, ceil(w/8) scheme-flag bytes, then w rows of
 * the transposed bit-plane matrix, most significant plane first, each row
 * dense (128 bytes) or sparse (16-byte bitmap + its non-zero bytes).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     context's device); h_* are host pointers.  The caller owns every
 *     buffer.
 *   - Input arrays must be aligned to their element size; output streams
 *     to 4 bytes.
 *   - The device-resident calls (falcon_compress, falcon_compress_variant,
 *     falcon_decompress, falcon_decompress_n and the *_each loops) are
 *     asynchronous on `stream` (a hipStream_t; NULL selects the context's
 *     own stream): they check their arguments, enqueue their kernels and
 *     return.  The caller keeps its buffers (and host length pointers)
 *     valid until the work is done: until falcon_sync returns, or until the
 *     stream has passed the call.  Lengths that only the device knows (the
 *     stream length of a compression) reach host memory at falcon_sync;
 *     with FALCON_OPT_DEVICE_LENGTHS they are written in stream order to
 *     device memory instead.  Errors found on the device (a corrupt stream)
 *     are reported by falcon_sync.  With FALCON_OPT_BLOCKING every device
 *     call synchronises itself and reports its own errors.
 *   - Successive device calls on one context are ordered even when they use
 *     different streams (they share the context's scratch): a call on a new
 *     stream first waits for the previous call.
 *   - The host <-> host calls, batch calls and plan runs are synchronous.
 *   - Errors are reported as status codes; nothing unwinds across the ABI.
 *     On any error the contents of output buffers are unspecified.
 *   - A context is used by one host thread at a time; distinct contexts are
 *     independent.
 */
#ifndef FALCON_H
#define FALCON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FALCON_FLOAT32 = 1, FALCON_FLOAT64 = 2 } falcon_dtype;

typedef enum {
  FALCON_OK = 0,
  FALCON_ERR_INVALID_ARG = 1,     /* null pointer, bad dtype, misaligned buffer */
  FALCON_ERR_BUFFER_TOO_SMALL = 2,/* output capacity below what the call needs */
  FALCON_ERR_CORRUPT_STREAM = 3,  /* stream fails a structural check */
  FALCON_ERR_DEVICE = 4,          /* a HIP runtime call failed */
  FALCON_ERR_OUT_OF_MEMORY = 5    /* the context could not grow its scratch */
} falcon_status;

typedef struct falcon_ctx falcon_ctx;

/* How falcon_compress runs on the device (both give the same stream).
 *  TWO_PASS     a size pass computes every chunk's size (Sec. 3.3), a prefix
 *               scan turns the sizes into offsets (Sec. 3.4), and a write
 *               pass recomputes each chunk and writes it at its offset; no
 *               chunk waits for another.  The default.
 *  SINGLE_PASS  one launch: waves take chunks from a work queue (atomic
 *               ticket counters) and each chunk finds its offset with a
 *               decoupled look-back over the sizes published by the chunks
 *               before it (the synchronisation of Sec. 3.4), so the input
 *               is read once. */
typedef enum falcon_compress_form {
  FALCON_FORM_TWO_PASS = 0,
  FALCON_FORM_SINGLE_PASS = 1
} falcon_compress_form;

/* Context options.  A zero-initialised struct, or opts = NULL, gives the
 * defaults: asynchronous device calls, host length pointers, two passes. */
typedef struct falcon_opts {
  unsigned flags;     /* FALCON_OPT_* */
  int compress_form;  /* falcon_compress_form of falcon_compress */
} falcon_opts;

enum {
  /* every device call waits for its own work, writes its host outputs and
   * reports its own errors before returning */
  FALCON_OPT_BLOCKING = 1,
  /* out_len (falcon_compress, falcon_compress_variant) is a device pointer
   * to a size_t that the kernels write in stream order */
  FALCON_OPT_DEVICE_LENGTHS = 2
};

/* Creates a context on HIP device `device` with options opts (NULL: the
 * defaults): a stream, pinned staging and device scratch (per-chunk
 * metadata, sizes and offsets for the prefix sum, work-queue counters and
 * status words, an error word), grown on demand.  Returns
 * FALCON_ERR_INVALID_ARG for unknown option bits or form, FALCON_ERR_DEVICE
 * if the device cannot be used. */
falcon_status falcon_create(int device, const falcon_opts* opts, falcon_ctx** out);

/* Waits for the work of every device call made on ctx since the last
 * falcon_sync, writes the host lengths those calls left pending, and
 * returns the first error the device found among them: FALCON_ERR_CORRUPT_STREAM
 * when a decompressed chunk failed a check, FALCON_ERR_DEVICE when a HIP call
 * failed or a single-pass look-back gave up (which a correct run never
 * does).  FALCON_OK otherwise, also when there was nothing to wait for. */
falcon_status falcon_sync(falcon_ctx* ctx);

/* Releases everything the context owns.  NULL is ignored. */
void falcon_destroy(falcon_ctx* ctx);

/* Largest stream that compressing n values of type dt can produce:
 * 32 + ceil(n/1025) * (4 + 8211) for f64, 32 + ceil(n/1025) * (4 + 4107) for
 * f32 (the all-dense chunk of Sec. 3.3: 11 + 8 + 64 * 128 and
 * 7 + 4 + 32 * 128 bytes).  Returns 0 for an unknown dtype. */
size_t falcon_compress_bound(size_t n, falcon_dtype dt);

/* Compresses n values at d_in (device) into d_out (device, out_cap bytes).
 * Sec. 3.2-3.5 and Alg. 3: per-chunk integer conversion and adaptive
 * bit-plane encoding, the chunks packed by a prefix sum of their sizes
 * (Sec. 3.4), in the context's falcon_compress_form.  Asynchronous: *out_len
 * receives the stream length at falcon_sync (a host size_t), or in stream
 * order with FALCON_OPT_DEVICE_LENGTHS (a device size_t); the stream header
 * at d_out + 24 also holds the payload byte count once the work is done.
 * Returns FALCON_ERR_BUFFER_TOO_SMALL without launching anything if
 * out_cap < falcon_compress_bound(n, dt).  n = 0 gives a 32-byte stream. */
falcon_status falcon_compress(falcon_ctx* ctx, const void* d_in, size_t n, falcon_dtype dt,
                              void* d_out, size_t out_cap, size_t* out_len, void* stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): falcon_compress
 * (two passes, FALCON_OPT_DEVICE_LENGTHS semantics) without a context and
 * without any allocation.  Its scratch is a fixed array of about 14 MiB in
 * the library's device code; every GPU the library runs on holds its own
 * copy until the process ends.  The device is the current HIP device, and
 * `stream` (NULL: its null stream) must belong to it.  The first call on a
 * device (or falcon_create for it) takes the array's device address; that
 * call makes no allocation either.  Asynchronous: d_out receives the stream,
 * and d_out_len, if not NULL, a device size_t (8-byte aligned), receives its
 * length in stream order (the header at d_out + 24 also holds the payload
 * byte count).  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (on different streams, or from different threads)
 * race, so the caller orders them, for instance on one stream.  Nothing of
 * the array needs to start at zero.  Errors: FALCON_ERR_OUT_OF_MEMORY
 * without any launch if n exceeds 537,395,200 values (2^19 chunks of 1025),
 * the array's limit; FALCON_ERR_BUFFER_TOO_SMALL if out_cap <
 * falcon_compress_bound(n, dt); FALCON_ERR_INVALID_ARG for a null or
 * misaligned pointer or an unknown dtype; FALCON_ERR_DEVICE if a HIP call
 * fails. */
falcon_status falcon_compress_noalloc(const void* d_in, size_t n, falcon_dtype dt, void* d_out, size_t out_cap,
                                      size_t* d_out_len, void* stream);

/* Ablation variants of Sec. 5.4.2 (Fig. 12b).  Each changes one step of
 * compression and keeps the stream layout:
 *  ELF    Alg. 2 stops at the first alpha where v (x) 10^alpha is an exact
 *         integer (the trial-and-error test of Sec. 1) instead of the error
 *         bound of Thm. 4; loop limits, the recover check and exceptions are
 *         unchanged, so the stream stays lossless but alpha can come out too
 *         large (1.11 gets 3).
 *  SPARSE every bit-plane row is written sparse (16-byte bitmap + non-zero
 *         bytes), whatever its zero count.
 *  DENSE  every bit-plane row is written dense (128 bytes). */
typedef enum falcon_variant {
  FALCON_VARIANT_FALCON = 0,
  FALCON_VARIANT_ELF = 1,
  FALCON_VARIANT_SPARSE = 2,
  FALCON_VARIANT_DENSE = 3
} falcon_variant;

/* falcon_compress_bound for a variant.  SPARSE rows can take 144 bytes, so
 * its chunks reach 11 + 8 + 64 * 144 (f64) and 7 + 4 + 32 * 144 (f32); the
 * others equal falcon_compress_bound.  0 for an unknown dtype or variant. */
size_t falcon_compress_bound_variant(size_t n, falcon_dtype dt, falcon_variant v);

/* falcon_compress under variant v (arguments, errors and the stream header
 * as there; out_cap is checked against falcon_compress_bound_variant).
 * FALCON_VARIANT_FALCON is falcon_compress.  falcon_decompress reads ELF
 * and DENSE streams; a SPARSE stream decodes only if every chunk stays
 * within the f64/f32 chunk bound of falcon_compress_bound, otherwise it is
 * reported as FALCON_ERR_CORRUPT_STREAM. */
falcon_status falcon_compress_variant(falcon_ctx* ctx, const void* d_in, size_t n, falcon_dtype dt, falcon_variant v,
                                      void* d_out, size_t out_cap, size_t* out_len, void* stream);

/* Decompresses the stream of in_len bytes at d_in (device) into d_out
 * (device, out_cap_bytes bytes).  Sec. 4: scan of the size array into chunk
 * offsets, per-chunk bit-plane decoding, inverse of Eq. 4 and Eq. 3.  The
 * value count and dtype come from the stream header, which this call reads
 * to the host (one 32-byte copy that waits for the work already on `stream`)
 * and checks; *n_out (host) receives N before the call returns.  The
 * decoding is then enqueued as by falcon_decompress_n.  If out_cap_bytes is
 * below N times the element size, FALCON_ERR_BUFFER_TOO_SMALL is returned
 * before any launch and *n_out still receives N.  d_in must be 4-byte and
 * d_out element-size aligned (else FALCON_ERR_INVALID_ARG); d_out may sit
 * at any element offset inside a larger buffer.  Only d_out[0, N) is
 * written. */
falcon_status falcon_decompress(falcon_ctx* ctx, const void* d_in, size_t in_len, void* d_out,
                                size_t out_cap_bytes, size_t* n_out, void* stream);

/* Decompresses a stream that the caller knows to hold n values of type dt
 * (the count and dtype it compressed, or falcon_stream_info of its header)
 * without any host access to the stream: fully asynchronous.  The header is
 * checked on the device against n, dt and in_len, and every chunk is
 * checked (bit width, row extents inside the chunk's size, sizes summing to
 * the payload byte count); a failure is reported as
 * FALCON_ERR_CORRUPT_STREAM by falcon_sync (or at once with
 * FALCON_OPT_BLOCKING), and then the chunks that passed their checks are
 * written and the failing ones are not, so d_out[0, n) holds no defined
 * result.  On the host: FALCON_ERR_CORRUPT_STREAM if in_len cannot hold the
 * header and n chunk sizes, FALCON_ERR_BUFFER_TOO_SMALL if out_cap_bytes <
 * n times the element size, FALCON_ERR_INVALID_ARG for a null or misaligned
 * pointer or an unknown dtype; nothing is launched then. */
falcon_status falcon_decompress_n(falcon_ctx* ctx, const void* d_in, size_t in_len, size_t n, falcon_dtype dt,
                                  void* d_out, size_t out_cap_bytes, void* stream);

/* Host -> host compression through the asynchronous pipeline of Sec. 3.1
 * (Alg. 1, event-driven scheduler).  The n values at h_in (host) are cut
 * into batches of whole chunks; each of the context's pipeline streams
 * copies a batch to the device, compresses it, reads back its payload byte
 * count, and -- once every batch launched before it has been placed --
 * copies its chunk sizes and payload to their final place in h_out (host,
 * out_cap bytes).  The result is byte-identical to falcon_compress of the
 * same values.  Pinned (hipHostMalloc) buffers are transferred directly;
 * pageable ones are staged through pinned buffers the context owns.
 * Synchronous: returns when h_out is complete.  If out_cap is below
 * falcon_compress_bound(n, dt), returns FALCON_ERR_BUFFER_TOO_SMALL and
 * sets *out_len to that bound. */
falcon_status falcon_compress_host(falcon_ctx* ctx, const void* h_in, size_t n, falcon_dtype dt, void* h_out,
                                   size_t out_cap, size_t* out_len);

/* Host -> host decompression of the stream of in_len bytes at h_in (host)
 * into h_out (host, out_cap_bytes bytes).  Sec. 4: the chunk sizes are in
 * host memory, so every batch's payload offset is known before any
 * transfer (pre-allocation); the pipeline streams each copy a batch's sizes
 * and payload to the device, decode it and copy the values to their place.
 * The size array is checked on the host, every chunk on the device; errors
 * as for falcon_decompress. */
falcon_status falcon_decompress_host(falcon_ctx* ctx, const void* h_in, size_t in_len, void* h_out,
                                     size_t out_cap_bytes, size_t* n_out);

/* Sets the pipeline geometry used by the two calls above: n_streams HIP
 * streams (1..64; N_s of Alg. 1) and batch_chunks chunks of 1025 values per
 * batch (1..2^20).  Defaults: 4 streams, 2048 chunks (measured fastest on
 * MI355X; the paper's Sec. 5.1.4 setting is 16 streams, 4096 chunks).
 * Device and pinned buffers (about 2 x 16.8 MB per stream at the default
 * batch, twice that when pageable buffers are staged) are allocated on
 * first use and kept until the geometry changes or the context is
 * destroyed.  FALCON_ERR_INVALID_ARG outside the ranges. */
falcon_status falcon_set_pipeline(falcon_ctx* ctx, int n_streams, size_t batch_chunks);

/* The three schedulers of the compression pipeline that Sec. 3.1 compares
 * (Fig. 5, Fig. 12a).  All give the same stream, byte for byte.
 *  EVENT_DRIVEN   Alg. 1 (the default): each lane polls its events, and a
 *                 lane places its payload once its byte count has arrived
 *                 and every batch launched before it has been placed.
 *  SYNC_BASED     Fig. 5b: the host waits for each batch's byte count
 *                 (M-D2H) before it launches the next batch; only the
 *                 payload copy (P-D2H) of a batch overlaps the next batch.
 *  PRE_ALLOCATION Fig. 5a: every batch copies its whole worst-case output
 *                 region into a fixed slot of a pinned host buffer (about
 *                 falcon_compress_bound of the input, kept by the context
 *                 until the geometry changes or the context is destroyed),
 *                 and a host merge packs the slots into h_out. */
typedef enum falcon_scheduler {
  FALCON_SCHED_EVENT_DRIVEN = 0,
  FALCON_SCHED_SYNC_BASED = 1,
  FALCON_SCHED_PRE_ALLOCATION = 2
} falcon_scheduler;

/* Selects the scheduler falcon_compress_host uses (decompression always uses
 * pre-allocation, Sec. 4).  FALCON_ERR_INVALID_ARG for another value. */
falcon_status falcon_set_pipeline_scheduler(falcon_ctx* ctx, falcon_scheduler kind);

/* ---- Many series in one launch ----------------------------------------
 * One series of a batch call or plan.  Compression: d_in holds n values of
 * type dtype (device), d_out (device, out_cap bytes, 4-byte aligned) receives
 * the stream, out_len its length.  Decompression: d_in holds a stream of
 * in_len bytes (device, 4-byte aligned) that must hold n values of type
 * dtype (the count and dtype the caller compressed, or falcon_stream_info of
 * its header); d_out (device, out_cap bytes) receives the values, out_len = n.
 * Each series' output is byte-identical to a one-series call on it. */
typedef struct falcon_series {
  const void* d_in;
  size_t n;
  size_t in_len;
  void* d_out;
  size_t out_cap;
  falcon_dtype dtype;
  size_t out_len;
} falcon_series;

typedef enum { FALCON_OP_COMPRESS = 0, FALCON_OP_DECOMPRESS = 1 } falcon_op;

/* Plan flags: FALCON_PLAN_TUNE times every launch geometry candidate on the
 * plan's own series and keeps the fastest (compression: launch form split /
 * mixed x 8 or 16 waves per workgroup x full or half grid x two passes with
 * static striding or the single pass with its work queue; decompression:
 * form x grid), and records the choice in the context by shape class
 * (operation, dtypes present, log2 of the chunk count, log2 of the series
 * count): a later tuned plan of the same class takes the recorded geometry
 * without timing.  FALCON_PLAN_GRAPH records the plan's launches as one HIP
 * graph replayed by falcon_plan_run.  FALCON_PLAN_SINGLE_PASS makes an
 * untuned compression plan run the single-pass form (the tuner decides by
 * itself).  The one-shot batch calls compress in the context's
 * falcon_compress_form. */
enum { FALCON_PLAN_TUNE = 1, FALCON_PLAN_GRAPH = 2, FALCON_PLAN_SINGLE_PASS = 4 };

typedef struct falcon_plan falcon_plan;

typedef struct falcon_plan_info {
  int split;            /* 1: one launch per dtype; 0: one launch over both dtypes */
  int waves_per_group;  /* wavefronts per workgroup */
  int grid_percent;     /* grid as a percentage of the co-resident workgroups */
  int candidates;       /* geometries timed by the autotuner (0: not tuned) */
  float best_ms;        /* autotuner: time of the chosen geometry */
  float default_ms;     /* autotuner: time of the default geometry */
  int graph;            /* 1 if runs replay a HIP graph */
  uint64_t total_chunks;
  int form;             /* compression: 0 two passes, 1 single pass (work queue; falcon_compress_form) */
  int from_cache;       /* 1 if the geometry came from the context's record of an earlier plan of the
                           same shape class instead of timing */
} falcon_plan_info;

/* The one-series-per-launch path over count series, as a C loop: one
 * asynchronous falcon_compress (falcon_decompress_each: falcon_decompress_n)
 * per series, in order, on `stream`, each with its own launches; the stream
 * lengths are written by the kernels to device memory and read back once,
 * after a single wait at the end (s[i].out_len; decompression: s[i].n).
 * Descriptors as for the batch calls below, checked on the host before any
 * launch.  It is the baseline that batch calls and plans are measured
 * against. */
falcon_status falcon_compress_each(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream);
falcon_status falcon_decompress_each(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream);

/* Compresses count series in one launch sequence (no tuning, no graph):
 * every chunk of every series is a work item of the same size pass, one
 * scan turns the sizes of all series into offsets (Sec. 3.4, each series
 * relative to its first chunk), and the write pass places every chunk.
 * Sets each s[i].out_len.  Series are checked on the host first: a bad descriptor
 * returns FALCON_ERR_INVALID_ARG / FALCON_ERR_BUFFER_TOO_SMALL before any
 * launch.  Synchronous. */
falcon_status falcon_compress_batch(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream);

/* Decompresses count streams in one launch sequence (Sec. 4 per series):
 * headers checked on the device against the descriptors, one scan over the
 * sizes of all series, one decoding launch.  Errors as falcon_decompress;
 * FALCON_ERR_CORRUPT_STREAM if any series fails. */
falcon_status falcon_decompress_batch(falcon_ctx* ctx, falcon_series* s, size_t count, void* stream);

/* Builds a reusable plan for op over count series (1 <= count < 2^31).  The
 * plan keeps the series' device pointers, sizes and dtypes; the contents of
 * the buffers may change between runs.  It owns its scratch, so plans run
 * independently of each other and of one-series calls on the context.
 * flags: FALCON_PLAN_TUNE, FALCON_PLAN_GRAPH (above).  Tuning runs the
 * operation on the series several times (outputs are written). */
falcon_status falcon_plan_create(falcon_ctx* ctx, falcon_op op, const falcon_series* s, size_t count,
                                 unsigned flags, falcon_plan** out);

/* Runs a plan on `stream` (NULL: the plan's own) and waits for it; fills
 * s[i].out_len if s is not NULL (s must then have the plan's count). */
falcon_status falcon_plan_run(falcon_plan* p, falcon_series* s, void* stream);

/* Reports the plan's launch geometry and tuning record. */
falcon_status falcon_plan_describe(const falcon_plan* p, falcon_plan_info* info);

void falcon_plan_destroy(falcon_plan* p);

/* ---- Serving: a request loop with continuous batching ------------------
 * Clients submit compress and decompress requests on device-resident
 * inputs; a worker thread admits them in arrival order as output memory
 * frees up in a device pool of hbm_budget bytes, groups admitted requests of
 * one kind into batch launches (as falcon_compress_batch /
 * falcon_decompress_batch) on up to `lanes` streams, and keeps admitting and
 * launching arrivals while earlier batches run, so their work overlaps on
 * the device.  Each request's output is byte-identical to the one-series
 * call on it, alone or in any mix.  lanes = 1, max_batch = 1 gives the plain
 * one-request-per-launch FIFO. */
typedef struct falcon_server falcon_server;

/* Each lane also keeps the scratch of its batch launches (descriptors, chunk
 * sizes, offsets and metadata: about 36 bytes per chunk) outside the pool; a
 * batch takes requests only up to 2^22 chunks (at least one request), so this
 * stays below about 150 MB per lane. */
typedef struct falcon_server_opts {
  size_t hbm_budget;  /* bytes of the output pool (0: 64 GiB) */
  void* pool;         /* optional caller-owned device memory of hbm_budget bytes to use as the pool
                         (256-byte aligned; kept by the caller); NULL: the server allocates it */
  int lanes;          /* concurrent batch launches, 1..32 (0: 4) */
  int max_batch;      /* requests per batch launch (0: 256) */
} falcon_server_opts;

typedef struct falcon_request {
  falcon_op op;
  const void* d_in;   /* device: n values (compress) or a stream of in_len bytes holding n values */
  size_t n;
  size_t in_len;
  falcon_dtype dtype;
  uint64_t tag;       /* returned with the completion */
} falcon_request;

typedef struct falcon_completion {
  uint64_t tag;
  falcon_status status;
  void* d_out;        /* in the server's pool: the stream (compress) or the values; null on error */
  size_t out_len;     /* stream bytes (compress) or values (decompress) */
  double submit_us, admit_us, complete_us;  /* host times since the server was created */
  double dev_start_us, dev_end_us;  /* device times (HIP events) of the start and end of the batch launch the
                                       request ran in, since a reference event recorded at server creation;
                                       -1 when it ran in no batch (an error found on the host) */
  int lane;           /* the lane (stream) of that batch, -1 if none */
} falcon_completion;

/* Creates a server on ctx (opts may be NULL).  The input buffers of a
 * request must stay valid until its completion is polled.  The context must
 * not be destroyed before the server. */
falcon_status falcon_server_create(falcon_ctx* ctx, const falcon_server_opts* opts, falcon_server** out);

/* Queues a request (thread-safe; returns at once).  A request whose output
 * is larger than the whole pool completes with FALCON_ERR_OUT_OF_MEMORY; a
 * bad descriptor completes with the status the batch call would return. */
falcon_status falcon_server_submit(falcon_server* s, const falcon_request* r);

/* Moves up to max completions into out, waiting up to wait_ms for the
 * first; returns how many were moved. */
size_t falcon_server_poll(falcon_server* s, falcon_completion* out, size_t max, int wait_ms);

/* Returns a completion's output buffer to the pool. */
falcon_status falcon_server_release(falcon_server* s, void* d_out);

/* Requests submitted and not yet completed. */
uint64_t falcon_server_in_flight(const falcon_server* s);

/* Stops the worker after the work it can still do (requests that cannot be
 * admitted any more complete with FALCON_ERR_OUT_OF_MEMORY) and frees the
 * pool, including unreleased outputs. */
void falcon_server_destroy(falcon_server* s);

/* Parses a stream header held in host memory (len >= 32 bytes) and returns
 * the value count and dtype.  FALCON_ERR_CORRUPT_STREAM if the header is not
 * a version-1 Falcon header. */
falcon_status falcon_stream_info(const void* h_hdr, size_t len, size_t* n, falcon_dtype* dt);

/* Device time in milliseconds of the last falcon_compress /
 * falcon_compress_variant (all its launches: size pass, scan, write pass; or
 * the single-pass launch and the clearing of its counters) or
 * falcon_decompress / falcon_decompress_n (the scan of the size array and
 * the decoding kernel), measured with HIP events recorded on the launch
 * stream; waits for that call's work.  Intended for roofline accounting;
 * FALCON_ERR_INVALID_ARG if no call has run yet. */
falcon_status falcon_last_kernel_ms(falcon_ctx* ctx, float* ms);

/* The stages of that call separately, ms[0..2]: two-pass compression: size
 * pass, scan, write pass; single-pass compression: the whole launch, 0, 0;
 * decompression: 0, scan, decoding kernel. */
falcon_status falcon_last_stage_ms(falcon_ctx* ctx, float* ms);

/* The context keeps the events of its last FALCON_TIMED_CALLS timed calls
 * (falcon_compress, falcon_compress_variant, falcon_decompress,
 * falcon_decompress_n), so that a caller who enqueues many asynchronous
 * calls and synchronises once can still read each call's stages. */
#define FALCON_TIMED_CALLS 64

/* ms[0..2] as falcon_last_stage_ms for the timed call made `back` timed
 * calls before the last (back = 0: the last one); waits for that call's
 * work.  FALCON_ERR_INVALID_ARG if back >= FALCON_TIMED_CALLS, or if that
 * many timed calls have not been made, or that call failed before its
 * kernels were enqueued. */
falcon_status falcon_call_stage_ms(falcon_ctx* ctx, unsigned back, float* ms);

/* Static, human-readable name of a status code. */
const char* falcon_status_str(falcon_status st);

#ifdef __cplusplus
}
#endif

#endif /* FALCON_H */
