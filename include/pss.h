/*
 * pss.h -- C ABI of libpss: parallel samplesort with exact splitting (PSES)
 * on AMD MI355X (gfx950).
 *
 * The library sorts N keys ascending into a separate output array, following
 * the problem statement of Tokuue & Ishiyama, "Performance Evaluation of
 * Parallel Sortings on the Supercomputer Fugaku" (arXiv 2305.05245), Section 2:
 * the input A is cut into n_B contiguous blocks of length ceil(N/n_B), each
 * block is sorted (step 1), n_P - 1 pivots P_1..P_{n_P-1} are chosen with the
 * implicit sentinels P_0 = -inf and P_{n_P} = +inf (step 2), every sorted block
 * is cut into n_P partitions (step 3), and the k-th partitions of all blocks
 * are merged into the output at an offset that is the sum of the sizes of the
 * partitions before it (step 4).  Pivots are chosen by exact splitting
 * (Section 2.3, Eq. 1 and Eq. 2): with r_k = floor(k N / n_P),
 *     |{x < P_k}| <= r_k <= |{x <= P_k}|  and  c_k = r_k - |{x < P_k}|,
 * so every partition holds floor(N/n_P) or ceil(N/n_P) keys however many keys
 * are equal.  Of the keys equal to P_k, the c_k that go left are taken from the
 * lowest-numbered block first, earliest position first.
 *
 * Conventions for every call:
 *  - Pointers named *_in, *_out, ws, pivots, counts, split, offsets are DEVICE
 *    pointers (memory owned by the caller, e.g. torch tensors).  Host pointers
 *    are only the out-parameters of pss_create, pss_workspace_bytes,
 *    pss_plan_describe and pss_validate's arguments, which are never
 *    dereferenced.
 *  - Every call that launches work is asynchronous on `stream` (a hipStream_t
 *    passed as void*, NULL = the null stream) and returns once the work is
 *    queued.  The caller synchronises.
 *  - keys_in is never written.  Input and output must not overlap (the method
 *    is out of place: the output needs its own N elements, Section 4).
 *  - Errors are returned as status codes; nothing is thrown across the ABI.
 *    pss_last_error() gives a message for the last failing call on a context
 *    (or on the calling thread when the context is NULL).
 *  - A context is used by one host thread at a time.
 *  - Key order: unsigned/signed integers by value; float32/float64 by IEEE
 *    754-2019 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN),
 *    so the output is unique bit for bit.  Key-value sorts are stable: equal
 *    keys keep their input order.
 */
#ifndef PSS_H
#define PSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSS_U32 = 0,
  PSS_I32 = 1,
  PSS_U64 = 2,
  PSS_I64 = 3,
  PSS_F32 = 4, /* IEEE totalOrder */
  PSS_F64 = 5  /* IEEE totalOrder */
} pss_key_t;

typedef enum {
  PSS_VAL_NONE = 0, /* keys only */
  PSS_VAL_U32 = 1   /* one uint32 payload per key, stable by input index */
} pss_val_t;

typedef enum {
  PSS_OK = 0,
  PSS_ERR_INVALID = 1,     /* bad argument (null pointer, overlap, bad enum)  */
  PSS_ERR_UNSUPPORTED = 2, /* valid request outside the library's limits      */
  PSS_ERR_OOM = 3,         /* host allocation failed                          */
  PSS_ERR_HIP = 4,         /* a HIP runtime call failed (see pss_last_error)  */
  PSS_ERR_WORKSPACE = 5,   /* workspace missing or smaller than required      */
  PSS_ERR_BUDGET = 6,      /* request larger than the server's memory budget  */
  PSS_ERR_BUSY = 7,        /* request already launched: it can't be cancelled */
  PSS_ERR_CANCELLED = 8    /* request cancelled before it was launched        */
} pss_status;

typedef struct pss_ctx pss_ctx;

/* Limits of the library. */
#define PSS_MAX_KEYS ((uint64_t)2147483647u) /* n < 2^31                      */
#define PSS_MAX_BLOCKS 2048u                 /* explicit n_B                  */
#define PSS_MAX_PARTS 4194304u               /* explicit n_P                  */

/* Create a context bound to HIP device `device`.  Returns PSS_ERR_HIP when the
 * device does not exist.  *out receives the handle (NULL on failure). */
pss_status pss_create(int device, pss_ctx **out);

/* Destroy a context (NULL is allowed).  Pending work is not waited for. */
void pss_destroy(pss_ctx *ctx);

/* Static English name of a status code. */
const char *pss_status_string(pss_status s);

/* Message of the last failing call on ctx (or on this thread if ctx is NULL);
 * "" if none.  Valid until the next call on the same context or thread. */
const char *pss_last_error(const pss_ctx *ctx);

/* Argument check performed by pss_sort before anything touches the device;
 * exposed so it can be exercised without a GPU.  keys_in/keys_out/vals_* are
 * compared as addresses only.  Returns PSS_OK, PSS_ERR_INVALID,
 * PSS_ERR_UNSUPPORTED or PSS_ERR_WORKSPACE (ws_bytes below the requirement;
 * pass SIZE_MAX to skip that check). */
pss_status pss_validate(pss_key_t key, pss_val_t val, const void *keys_in, const void *keys_out,
                        const void *vals_in, const void *vals_out, uint64_t n,
                        uint32_t n_blocks, uint32_t n_parts, size_t ws_bytes);

/* Device workspace pss_sort / pss_splitters need for these arguments (bytes,
 * 256-byte aligned pieces).  Host-only arithmetic; ctx may be NULL. */
pss_status pss_workspace_bytes(const pss_ctx *ctx, pss_key_t key, pss_val_t val, uint64_t n,
                               uint32_t n_blocks, uint32_t n_parts, size_t *bytes);

/* Plan of the launches pss_sort makes for these arguments, as a
 * NUL-terminated JSON object written to buf (host memory of buf_len bytes):
 *   {"mode": "auto"|"paper", "tile": T, "part": T_m, "passes": [fan-in, ...],
 *    "block_passes": [...], "n_blocks": n_B, "n_parts": n_P, "hbm_passes": h}
 * where "passes" are the merge passes after the tile sort and "hbm_passes"
 * the number of full read+write sweeps over the keys.  Keys-only sorts use
 * tiles and merge partitions of 8192 keys and passes of at most 32 runs;
 * key-value sorts tiles and partitions of 4096 keys and passes of at most 64
 * runs (they hold 12 bytes a key in LDS).  Host-only. */
pss_status pss_plan_describe(pss_key_t key, pss_val_t val, uint64_t n, uint32_t n_blocks,
                             uint32_t n_parts, char *buf, size_t buf_len);

/*
 * Sort n keys (and, with PSS_VAL_U32, their uint32 payloads) ascending.
 *
 *   n_blocks = n_parts = 0: automatic plan.  The input is cut into LDS-sized
 *     blocks (tiles); step 1 sorts each tile; steps 2-4 are then applied level
 *     by level, each level merging groups of sorted runs with exact splitting
 *     into LDS-sized partitions, until one run remains.
 *   n_blocks > 0 and n_parts > 0: the paper's single-level method with those
 *     n_B and n_P: n_B blocks of ceil(N/n_B) keys are sorted, exact splitters
 *     P_1..P_{n_P-1} cut every block, and partition k of all blocks is merged
 *     to output offset O_k = sum of the sizes of partitions 0..k-1 (computed on
 *     the device by an exclusive scan).  A partition larger than one LDS-sized
 *     merge is merged in chunks cut at exact ranks inside it.
 *   Exactly one of n_blocks, n_parts zero: PSS_ERR_INVALID.
 *
 * keys_in: n keys of the given type, never written.  keys_out: n keys.
 * vals_in/vals_out: n uint32 each when val == PSS_VAL_U32 (ignored otherwise).
 * ws: device workspace of at least pss_workspace_bytes(...) bytes, owned by
 * the caller; its contents are scratch and may be left changed.
 * n == 0 is a no-op.  Returns PSS_OK once all launches are queued.
 */
pss_status pss_sort(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                    void *keys_out, const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                    uint32_t n_blocks, uint32_t n_parts, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pss_sort
 * with the same arguments, except that the workspace is the library's own
 * scratch array of PSS_NOALLOC_SCRATCH_BYTES (64 MiB) on ctx's device, a
 * fixed array that each GPU the library runs on holds until the process
 * ends.  The call makes no device allocation (no hipMalloc or hipFree, no
 * allocating library call); per-launch timing (pss_profile_enable) is
 * suspended for the call, since creating timing events may allocate.
 *   Limit: the workspace pss_workspace_bytes gives for these arguments must
 *     fit the scratch array (keys only: about 7 million int64 or 14 million
 *     int32 keys; with uint32 values fewer); a larger request returns
 *     PSS_ERR_WORKSPACE and launches nothing.
 *   Every call on one GPU shares that GPU's scratch array, which keeps the
 *     last call's contents (no part of it needs to start at zero).  Calls
 *     that overlap on one GPU (on different streams, or from host threads
 *     that do not order them) race on it and give wrong results.
 * Other arguments, ownership and errors as for pss_sort.
 */
#define PSS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pss_status pss_sort_noalloc(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                            void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                            uint64_t n, uint32_t n_blocks, uint32_t n_parts, void *stream);

/*
 * Steps 1-3 of the paper's method with explicit n_B, n_P (n_blocks, n_parts
 * > 0), for inspection and parity checks.  Any output may be NULL.
 *   sorted_blocks: n keys, the concatenation of the sorted blocks (step 1).
 *   pivots: n_P - 1 keys, P_k = the key of rank r_k - 1 (the smallest key v
 *     with |{x <= v}| >= r_k, one valid choice under Eq. 1); 0 when r_k = 0.
 *   counts: n_P - 1 values c_k of Eq. 2 (0 when r_k = 0).
 *   split: n_B * (n_P + 1) values, row-major [b][k]: partition k of sorted
 *     block b is [split[b][k], split[b][k+1]) (step 3).
 *   offsets: n_P + 1 values O_k (O_0 = 0, O_{n_P} = n), from the device scan.
 * Workspace as for pss_sort with the same n_blocks, n_parts.
 */
pss_status pss_splitters(pss_ctx *ctx, pss_key_t key, const void *keys_in, uint64_t n,
                         uint32_t n_blocks, uint32_t n_parts, void *sorted_blocks, void *pivots,
                         uint64_t *counts, uint64_t *split, uint64_t *offsets, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * The paper's single level with the pivots of parallel sorting by regular
 * sampling (PSRS, Section 2.3, first paragraph) instead of exact splitting,
 * for comparison: step 1 as in pss_sort with n_blocks, n_parts > 0; step 2
 * takes n_P - 1 samples from every non-empty sorted block at its positions
 * floor(j len_b / n_P), j = 1..n_P-1, sorts the samples (S, n_s = non-empty
 * blocks * (n_P - 1) keys; non-empty blocks = ceil(n / ceil(n / n_B))), and
 * takes P_k = S[floor(k n_s / n_P)]; step 3 cuts every block by value alone,
 * partition k holding the keys P_k < x <= P_{k+1} (Section 2), so partition
 * sizes follow the data (on Duplicate3-like inputs at most three partitions
 * are non-empty, Fig. 3a); step 4 merges partition k of every block into the
 * output at offset |{x <= P_k}|, cut into chunks of at most 8192 keys.  The
 * output is the same stable sort as pss_sort's.
 *   part_sizes: optional DEVICE array of n_P uint64 partition sizes.
 * Limits: at most 2^27 samples.  Workspace: pss_psrs_workspace_bytes.  Other
 * arguments, ownership and errors as for pss_sort.
 */
pss_status pss_psrs_workspace_bytes(const pss_ctx *ctx, pss_key_t key, pss_val_t val, uint64_t n,
                                    uint32_t n_blocks, uint32_t n_parts, size_t *bytes);
pss_status pss_psrs_sort(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                         void *keys_out, const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                         uint32_t n_blocks, uint32_t n_parts, uint64_t *part_sizes, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * Steps 1-3 of the PSRS variant (see pss_psrs_sort), for inspection and
 * parity checks.  Any output may be NULL (all DEVICE arrays):
 *   sorted_blocks: n keys, the sorted blocks (step 1).
 *   samples: n_s keys, the sorted regular samples S.
 *   pivots: n_P - 1 keys P_k.
 *   split: n_B * (n_P + 1) values, row-major [b][k]: the number of keys
 *     <= P_k in sorted block b (column 0 is 0, column n_P the block length).
 *   offsets: n_P + 1 values, offsets[k] = |{x <= P_k}| (0 and n at the ends).
 * Workspace as for pss_psrs_sort with the same arguments.
 */
pss_status pss_psrs_splitters(pss_ctx *ctx, pss_key_t key, const void *keys_in, uint64_t n,
                              uint32_t n_blocks, uint32_t n_parts, void *sorted_blocks,
                              void *samples, void *pivots, uint64_t *split, uint64_t *offsets,
                              void *ws, size_t ws_bytes, void *stream);

/*
 * Records sorted by a key field (Table 1: Pair, 16-byte key-index records,
 * and Particle, 96-byte records of a key and particle data, both sorted by
 * their uint64 key): n records of record_bytes bytes (an array of
 * structures) are written to records_out in ascending key order, stable
 * (equal keys keep their input order).  The keys and their input indices go
 * through the key-value sort (pss_sort with PSS_VAL_U32), then whole records
 * are gathered in that order: records move once, not once per merge pass.
 *   key / key_offset: type and byte offset of the key inside each record
 *     (aligned to the key width).
 *   record_bytes: a multiple of 4 and of the key width, 4..4096.
 *   records_in, records_out: DEVICE arrays of n * record_bytes bytes, aligned
 *     to the key width, not overlapping; records_in is never written.
 * Workspace: pss_records_workspace_bytes (about 2 (w + 4) n bytes plus the
 * key-value sort's).  Errors as for pss_sort; n < 2^31.
 */
pss_status pss_records_workspace_bytes(const pss_ctx *ctx, pss_key_t key, uint64_t n,
                                       size_t *bytes);
pss_status pss_sort_records(pss_ctx *ctx, pss_key_t key, const void *records_in,
                            void *records_out, uint64_t n, uint32_t record_bytes,
                            uint32_t key_offset, void *ws, size_t ws_bytes, void *stream);

/*
 * Batched segmented sort: sort each segment [seg_offsets[i], seg_offsets[i+1])
 * of one array independently (ascending; key-value sorts stable within the
 * segment), all segments in one fixed sequence of launches with no host round
 * trip, so the sequence can be captured once into a hipGraph and replayed.
 * The segments' shapes are read on the device: a planning kernel classifies
 * every segment (one small tile, or tiles of 8192 keys (4096 with values) plus
 * merge passes of fan-in 32 or 64 with exact splitting, the paper's steps 2-4
 * applied per segment),
 * and every later kernel finds its segment through the plan's prefix tables.
 *
 *   seg_offsets: DEVICE array of n_segs + 1 uint64, seg_offsets[0] = 0,
 *     non-decreasing, seg_offsets[n_segs] <= n (keys past the last offset are
 *     left alone, so a batch may fill a buffer sized for n only partly, with
 *     unused trailing segments empty).  Invalid offsets leave the output
 *     unspecified and set bit 16 of the device error word (pss_device_check).
 *   tuning (host, may be NULL = defaults): which segments go to the smaller
 *     tile sorts, and a bound on the longest segment that bounds the number
 *     of merge passes launched.  Chosen by the project's autotuner per
 *     workload; any valid tuning gives the same output.
 *   Other arguments as pss_sort (n keys in total, out of place, caller-owned
 *   workspace of pss_segmented_workspace_bytes bytes).
 */
typedef struct {
  uint32_t small_max_2k; /* segments with <= this many keys: 2048-key tiles, 128 threads (<= 2048) */
  uint32_t small_max_4k; /* segments with <= this many keys: 4096-key tiles, 256 threads (<= 4096) */
  uint64_t max_seg_len;  /* upper bound on any segment's length; 0 = n */
  uint32_t fan_log2;     /* runs merged per pass, as a power of two: 5 (32 runs) or 6 (64 runs,
                            fewer passes for segments of 33-64 tiles and 1025-4096 tiles, each
                            pass with one more merge round); 0 = 5 */
  uint32_t reserved;     /* 0 */
} pss_tuning;

#define PSS_MAX_SEGMENTS 16777216u

pss_status pss_segmented_workspace_bytes(const pss_ctx *ctx, pss_key_t key, pss_val_t val,
                                         uint64_t n, uint32_t n_segs, const pss_tuning *tuning,
                                         size_t *bytes);
pss_status pss_segmented_sort(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                              void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                              uint64_t n, const uint64_t *seg_offsets, uint32_t n_segs,
                              const pss_tuning *tuning, void *ws, size_t ws_bytes, void *stream);

/*
 * Capture the launch sequence of one pss_segmented_sort call (same arguments,
 * no stream) into an instantiated HIP graph.  pss_graph_launch replays it on
 * `stream`: the same kernels on the same buffers, reading whatever keys,
 * values and offsets those buffers then hold, so one graph serves every batch
 * of at most n keys in at most n_segs segments (pad unused trailing offsets
 * with the batch total).  The graph holds no memset nodes.  The caller keeps
 * every buffer alive while the graph exists.
 */
typedef struct pss_graph pss_graph;
pss_status pss_segmented_graph_create(pss_ctx *ctx, pss_key_t key, pss_val_t val,
                                      const void *keys_in, void *keys_out,
                                      const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                                      const uint64_t *seg_offsets, uint32_t n_segs,
                                      const pss_tuning *tuning, void *ws, size_t ws_bytes,
                                      pss_graph **out);
pss_status pss_graph_launch(pss_graph *graph, void *stream);
void pss_graph_destroy(pss_graph *graph);

/*
 * Serving loop.  A server sorts independent requests (each one array of keys,
 * optionally with uint32 values, sorted ascending and stably, exactly as
 * pss_sort would) that arrive at any time from any host thread.  Requests
 * wait in one first-come-first-served queue.  Each of max_streams workers owns
 * a HIP stream and an equal share of the server's device-memory budget; a
 * worker that is free takes, in arrival order, every waiting request of the
 * head request's key and value types that still fits its share (continuous
 * batching: the batch is whatever arrived while the workers were busy), and
 * sorts the batch with one segmented sort (one segment per request): a
 * gather kernel copies the requests' inputs into the batch buffer, the
 * segmented sort runs (step 1 in tiles, steps 2-4 per request), and a
 * scatter kernel copies every sorted segment to its request's outputs.  The
 * workers' streams overlap one batch's work with the next.
 *
 *   hbm_budget_bytes: all device memory the server holds (batch buffers,
 *     workspace, tables), allocated at creation and split evenly over the
 *     workers.  A request whose batch of one would not fit a worker's share
 *     is refused at submission with PSS_ERR_BUDGET.
 *   max_streams: workers (and streams), 1..16.
 *   tuning (host, may be NULL): small-segment tile choice as for
 *     pss_segmented_sort; max_seg_len is ignored (each batch uses its longest
 *     request).
 *
 * pss_request (host struct, copied at submission):
 *   keys_in, keys_out, vals_in, vals_out: DEVICE pointers owned by the caller,
 *     naturally aligned, n elements each (values only with PSS_VAL_U32), kept
 *     alive and unmodified until the request completes; out must not overlap
 *     in.  n <= PSS_MAX_KEYS; n = 0 completes at once.
 *   arrival_ns: CLOCK_MONOTONIC time of arrival in ns, the start of the
 *     request's latency; 0 = the time of submission.
 * Results are visible to any stream once pss_poll or pss_wait reports the
 * request done (the worker has synchronised its stream).
 * A batch fails as a whole (every request in it completes with the batch's
 * status, others are unaffected) when a launch or copy of it fails, or when
 * the device error word (see pss_device_check) is non-zero once the batch
 * has finished.  That word is process-wide and stays set until
 * pss_device_check clears it, so after an invariant failure every batch that
 * finishes fails too: no result is reported valid while it is set.
 *
 * pss_submit never blocks on the GPU and returns a ticket (> 0).  pss_poll
 * reports whether a ticket is done; pss_wait blocks until it is.  Both give
 * the request's status (PSS_OK, PSS_ERR_CANCELLED, or the error of its batch)
 * and, once they report done, forget the ticket (PSS_ERR_INVALID afterwards).
 * pss_cancel withdraws a request that is still queued (it then completes
 * with PSS_ERR_CANCELLED) and returns PSS_ERR_BUSY for one already launched
 * or finished.  pss_server_stats reports counters and, over requests
 * completed since creation or the last pss_server_reset_stats, the latency
 * (arrival to completion) percentiles (of the most recent 2^22 of them) and
 * keys/s (keys completed divided by the time from the first arrival to the
 * last completion).
 * pss_server_destroy cancels queued requests, waits for launched batches and
 * frees everything; no other call on the server may be in progress.
 * Every server call is thread-safe.  Error messages go to the calling
 * thread's pss_last_error(NULL).
 */
typedef struct pss_server pss_server;

typedef struct {
  pss_key_t key;
  pss_val_t val;
  const void *keys_in;
  void *keys_out;
  const uint32_t *vals_in;
  uint32_t *vals_out;
  uint64_t n;
  uint64_t arrival_ns;
} pss_request;

typedef struct {
  uint64_t submitted, completed, rejected, cancelled, failed;
  uint64_t batches, keys_completed;
  double keys_per_s;
  double latency_p50_ms, latency_p99_ms, latency_mean_ms, latency_max_ms;
  double mean_batch_requests, mean_batch_keys;
  uint64_t budget_in_use; /* bytes of the budget held by batches now running  */
  uint64_t queued;        /* requests waiting in the queue                      */
} pss_stats;

pss_status pss_server_create(pss_ctx *ctx, size_t hbm_budget_bytes, uint32_t max_streams,
                             const pss_tuning *tuning, pss_server **out);
pss_status pss_submit(pss_server *server, const pss_request *req, uint64_t *ticket);
pss_status pss_poll(pss_server *server, uint64_t ticket, int *done, pss_status *result);
pss_status pss_wait(pss_server *server, uint64_t ticket, pss_status *result);
pss_status pss_cancel(pss_server *server, uint64_t ticket);
pss_status pss_server_stats(pss_server *server, pss_stats *out);
pss_status pss_server_reset_stats(pss_server *server);
void pss_server_destroy(pss_server *server);

/*
 * How step 4 of the paper's single level (pss_sort with n_blocks > 0, and
 * pss_psrs_sort) combines the sorted segments of a partition (Section 2.2):
 *   PSS_MERGE_PAIRWISE (default): stable pairwise merge rounds in LDS, one
 *     workgroup per chunk of at most 8192 keys;
 *   PSS_MERGE_SORT: the chunk's segments are gathered and sorted as a whole
 *     (the paper's "merging by sequential sorting"), with ties broken by
 *     (block, position), so the output is the same.
 * A setting of the context; the automatic plan's merge passes always merge.
 */
typedef enum { PSS_MERGE_PAIRWISE = 0, PSS_MERGE_SORT = 1 } pss_merge_method;
pss_status pss_set_merge_method(pss_ctx *ctx, pss_merge_method method);

/*
 * Per-launch timing for measurement.  While enabled, every kernel launch that
 * a call on ctx makes is bracketed by two HIP events recorded on that call's
 * stream (a few microseconds of overhead per launch).  pss_profile_read waits
 * for the recorded events and writes a NUL-terminated JSON object to buf (host
 * memory): {"<kernel family>": {"launches": L, "ms": total milliseconds,
 * "bytes": algorithmic HBM bytes of those launches}, ...}, then forgets the
 * records.  Families: tile_sort (step 1 tiles), sample_split_search,
 * sample_merge, split_search and merge (the merge passes: steps 2-4 over
 * groups of runs), partition_search, offset_scan and partition_merge (steps
 * 2-4 of the paper's single level, with partition_sample_search and
 * partition_sample_merge when its search starts from the blocks' samples),
 * psrs_samples, psrs_sample_sort,
 * psrs_partition and psrs_chunks (regular-sampling pivots), record_keys and
 * record_gather (record sorts).
 */
pss_status pss_profile_enable(pss_ctx *ctx, int on);
pss_status pss_profile_read(pss_ctx *ctx, char *buf, size_t buf_len);

/* Restrict the per-launch timing to one kernel family (a name from the list
 * above, copied; NULL or "" = every launch), so that a measurement of one
 * kernel adds events around its launches only.  Returns PSS_ERR_INVALID for
 * a null ctx or a name longer than 63 characters. */
pss_status pss_profile_only(pss_ctx *ctx, const char *family);

/*
 * Wait for all work on ctx's device, then read and clear the library's device
 * error word into *code (host memory): 0 when every kernel found its
 * invariants intact.  Bits: 1 = splitter candidate set overflow, 2 = splitter
 * target outside its bracket, 4 = split position outside its run, 8 = merged
 * segments do not add up to their partition.  A kernel that sets a bit stops
 * before writing outside its own partition, and its output is then invalid.
 * Bit 16: segment offsets of pss_segmented_sort invalid (or a segment needing
 * more merge passes than tuning->max_seg_len allowed for).
 * Meant for tests and debugging; it synchronises the whole device.
 */
pss_status pss_device_check(pss_ctx *ctx, uint32_t *code);

/*
 * Fault injection, for tests of failure handling (process-wide, thread-safe).
 * Arms one operation of the given kind to fail: the library lets `after`
 * more operations of that kind through, then the next one is not performed
 * and its call returns the error a refusing runtime would cause, with a
 * message naming the injection; the arming is then used up.
 *   PSS_INJECT_LAUNCH: queued device work (a kernel launch, an asynchronous
 *     copy or fill) made by any call, the server's workers included; the call
 *     returns PSS_ERR_HIP and work it queued before that point stays queued.
 *   PSS_INJECT_ALLOC: a device or pinned host allocation (the serving
 *     loop's buffers at pss_server_create); the call returns PSS_ERR_BUDGET.
 *   PSS_INJECT_NONE: disarm both kinds (after is ignored).
 * after < 0 disarms the kind.  Not for production use.
 */
typedef enum { PSS_INJECT_NONE = 0, PSS_INJECT_LAUNCH = 1, PSS_INJECT_ALLOC = 2 } pss_inject_t;
pss_status pss_debug_inject(pss_inject_t what, int64_t after);

#ifdef __cplusplus
}
#endif
#endif /* PSS_H */
