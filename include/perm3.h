/*
 * perm3 -- permanents over F_3 on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libperm3.so.  Everything here is plain C: integers, pointers and
 * sizes.  Pointers marked "host" are ordinary CPU memory; pointers marked
 * "device" are HIP device allocations (for example torch tensors on cuda:0)
 * on the library's current device.  The library never frees caller memory.
 *
 * The method (Scheinerman, "Fast computation of permanents over F_3 via F_2
 * arithmetic"):
 *   - perm(A) by Ryser's identity, eq. (2), summed over row subsets visited in
 *     reflected-binary Gray-code order, so that consecutive subsets differ by
 *     one row (Section 3 and its RBC footnote);
 *   - each length-n vector over F_3 is held "bipedally" as two F_2^n words
 *     (mag, sgn) under the map phi of Section 2: 0 -> (0,0), 1 -> (1,0),
 *     -1 -> (1,1), with (0,1) a second legal zero (Definition 2.1);
 *   - a row is added or subtracted with the and/or/xor formulas of
 *     Theorem 2.1; a subset's column product is non-zero exactly when every
 *     mag bit is set, and then equals (-1)^popcount(sgn) (Section 3);
 *   - independent blocks of consecutive Gray indices are started by jumping
 *     straight to Gray state i xor (i >> 1) (Section 3.1).
 *
 * Conventions shared by every entry point:
 *   - A matrix is n x n, row-major, one byte per entry, entries in {0,1,2};
 *     the byte 2 is the element -1 of F_3.
 *   - 0 <= n <= PERM_MAX_N (63).  perm of the 0 x 0 matrix is 1.
 *   - Results are bytes in {0,1,2} (2 is -1).
 *   - Every call returns an int32_t status: PERM_OK (0) or a negative code
 *     below.  perm_strerror() names a code; perm_last_error() gives the
 *     calling thread's last message (for PERM_EDEVICE, the HIP error).
 *   - Calls are thread-safe; calls into one device context are serialised.
 *     The library lazily creates, per device, a context holding a HIP stream,
 *     work buffers, cached HIP graphs and the kernel tuning table.
 */
#ifndef PERM3_H
#define PERM3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERM_MAX_N 63

/* status codes */
#define PERM_OK        0
#define PERM_EINVAL   (-1)  /* null pointer, n or count out of range, bad range or config  */
#define PERM_EDOMAIN  (-2)  /* a matrix entry > 2, or a packed plane with a bit >= n set    */
#define PERM_ENOMEM   (-3)  /* a device or host allocation failed                           */
#define PERM_EDEVICE  (-4)  /* a HIP runtime error, or no gfx950 device                    */
#define PERM_EAGAIN   (-5)  /* the server's submission queue is full; retry later           */
#define PERM_ESTATE   (-6)  /* the object is shut down or busy                              */

/* written by the device-input entry points for a matrix that fails validation */
#define PERM_RESULT_INVALID 0xFFu

/* --------------------------------------------------------------------------
 * Single matrix.
 *
 * perm_mod3: perm(A) mod 3 (eq. 1), computed by the bipedal Gray-code Ryser
 * sum (Section 3).  A: host, n*n bytes.  *out: host, one byte in {0,1,2}.
 * Synchronous.  PERM_EINVAL for n < 0, n > 63, or a null pointer (A may be
 * null when n == 0); PERM_EDOMAIN if any entry > 2 (then perm_last_error_index()
 * is the offending byte's offset).
 */
int32_t perm_mod3(const uint8_t *A, int32_t n, uint8_t *out);

/*
 * perm_mod3_range_tally: the exact partial Ryser sum over Gray indices
 * begin <= i < end (Sections 3 and 3.1):
 *     T(begin,end) = sum_i (-1)^|g(i)| * prod_cols sum_{k in g(i)} a_{k,col},
 * with g(i) = i xor (i >> 1) a set of rows, each column sum taken in F_3 as
 * an integer in {-1,0,1}.  T is additive over ranges, and
 * perm(A) = (-1)^n * T(0, 2^n) mod 3.  Requires 0 <= begin <= end <= 2^n.
 * A: host.  *tally: host int64.  Synchronous.
 */
int32_t perm_mod3_range_tally(const uint8_t *A, int32_t n, uint64_t begin, uint64_t end,
                          int64_t *tally);

/*
 * perm_mod3_range_tally_wide: T over a range of Gray indices of a matrix of
 * up to 128 columns, two 64-bit words per plane (Section 3 names this as the
 * ambitious case past n = 64, where Gray indices outgrow 64 bits).
 *   A:         host, n*n bytes in {0,1,2}, 1 <= n <= PERM_MAX_N_WIDE
 *   begin_hi, begin_lo:  the first Gray index, begin = begin_hi * 2^64 + begin_lo
 *   count:     number of indices, 0 <= count <= PERM_WIDE_MAX_COUNT; the
 *              range [begin, begin + count) must lie inside [0, 2^n]
 *   *tally:    host int64, T(begin, begin + count) as for perm_mod3_range_tally
 * Synchronous.  For n <= 63 the value equals perm_mod3_range_tally's.  The
 * whole sum for n >= 64 (2^64 indices and more) is out of reach of one
 * device; the call is the unit a sharded run over many devices adds up.
 * PERM_EINVAL for n or count out of range, a range outside [0, 2^n] or a null
 * pointer; PERM_EDOMAIN for an entry > 2 (perm_last_error_index() = offset).
 */
#define PERM_MAX_N_WIDE 128
#define PERM_WIDE_MAX_COUNT (1ull << 62)
int32_t perm_mod3_range_tally_wide(const uint8_t *A, int32_t n, uint64_t begin_hi, uint64_t begin_lo,
                                   uint64_t count, int64_t *tally);

/* --------------------------------------------------------------------------
 * Bitsliced vectors over F_3 in device memory (Theorem 2.1 in full).
 *
 * A vector of len elements is held as ceil(len/64) word pairs:
 * planes[2w] = mag and planes[2w+1] = sgn of elements 64w .. 64w+63, element
 * e at bit e mod 64 (least significant first), under phi of Section 2:
 * 0 -> (0,0), 1 -> (1,0), -1 -> (1,1), and (0,1) is also 0.  Bits at and
 * above len in the last word are 0 after perm_f3_pack.  (Any bit order is
 * valid for perm_mod3_batch_packed's rows, since a permanent does not depend
 * on the order of the columns.)  Every pointer is device memory; planes must
 * be 16-byte aligned.  Calls are asynchronous on `stream` (a hipStream_t;
 * NULL is the legacy default stream) and return after enqueueing.
 */
#define PERM_F3_ADD 0   /* a + b, Theorem 2.1 as printed                         */
#define PERM_F3_SUB 1   /* a - b, Theorem 2.1 as printed                         */
#define PERM_F3_MUL 2   /* elementwise a * b                                     */
#define PERM_F3_DIV 3   /* elementwise a / b where b != 0; where b = 0 unspecified */
#define PERM_F3_NEG 4   /* -a (b is not read and may be NULL)                    */
#define PERM_F3_MAX_LEN (1ll << 40)

/* phi: v_dev bytes in {0,1,2} (2 = -1) -> planes_dev[2 * ceil(len/64)].  A
 * byte > 2 is packed as 0 and counted: the count is ADDED to *invalid_dev
 * (device uint64, may be NULL).  0 <= len <= PERM_F3_MAX_LEN. */
int32_t perm_f3_pack(const uint8_t *v_dev, int64_t len, uint64_t *planes_dev, uint64_t *invalid_dev,
                     void *stream);

/* psi: planes_dev -> v_dev[len] bytes in {0,1,2}; (0,1) reads as 0. */
int32_t perm_f3_unpack(const uint64_t *planes_dev, int64_t len, uint8_t *v_dev, void *stream);

/* out = a op b over `words` word pairs (out may alias a or b).  The result's
 * bits are those of Theorem 2.1's formulas, so a zero may come out as (0,1). */
int32_t perm_f3_op(int32_t op, const uint64_t *a_dev, const uint64_t *b_dev, uint64_t *out_dev, int64_t words,
                   void *stream);

/* *sum_dev (device int64) = sum over the elements of a_e * b_e as integers in
 * {-1,0,1}; the dot product over F_3 is that sum mod 3.  Bits beyond a
 * vector's length must be 0 in mag (as perm_f3_pack leaves them). */
int32_t perm_f3_dot(const uint64_t *a_dev, const uint64_t *b_dev, int64_t words, int64_t *sum_dev, void *stream);

/* --------------------------------------------------------------------------
 * Many matrices in one persistent launch.
 *
 * perm_mod3_batch: As[k] is a host pointer to the k-th n_k x n_k matrix,
 * ns: host int32[count], out: host uint8[count].  Synchronous.  The whole
 * batch is validated before anything runs; on error nothing runs and
 * perm_last_error_index() is the index of the first bad matrix.
 * 0 <= count <= PERM_MAX_BATCH.
 */
#define PERM_MAX_BATCH (1 << 22)
int32_t perm_mod3_batch(const uint8_t *const *As, const int32_t *ns, int32_t count,
                         uint8_t *out);

/*
 * perm_mod3_batch_dev: device-resident form of perm_mod3_batch.
 *   mats_dev:  device bytes, matrix k at byte offset offs_dev[k], n_k*n_k bytes
 *   offs_dev:  device int64[count]
 *   ns_dev:    device int32[count], each in [0, 63]
 *   out_dev:   device uint8[count]; a matrix with an entry > 2 or n outside
 *              [0, 63] gets PERM_RESULT_INVALID and is not computed
 *   hist_dev:  device uint64[64*3] or NULL; the counts of results 0/1/2 are
 *              ADDED at hist_dev[3*n + r] (the caller zeroes it)
 *   stream:    a hipStream_t; or NULL: the legacy default stream itself for
 *              a call of up to 64 matrices (or with graphs off); otherwise
 *              the library's stream, ordered after earlier and before later
 *              work on the legacy default stream
 * Asynchronous on `stream`: all steps (validate, pack with phi, plan, Gray
 * walk, reduce, finish) run as kernels; the call returns after enqueueing.
 * A call of up to 64 matrices is two direct launches: one kernel plans and
 * packs them and, when they hold at most 2^28 Gray indices in all, walks
 * them too; the persistent walk that follows then finds nothing to do.  The
 * launches of a larger call are captured once per (pointers, count, stream)
 * into a HIP graph and replayed afterwards.  Calls into one device are
 * ordered among themselves, whatever their streams.  Buffers must stay valid
 * until the stream reaches the call's end.
 *
 * Graph capture: a call made while the caller captures `stream` (a non-NULL
 * stream, for example inside torch.cuda.graph) records its kernels into the
 * caller's graph and returns; nothing runs until the graph is launched.  Such
 * a call gets device work buffers of its own (allocated at capture time, kept
 * until the process ends), so every replay recomputes it from whatever the
 * input buffers then hold, and replays are not ordered with other calls into
 * the library: they need not be, since they share no buffers with them.  The
 * graph holds no memset node.  The first call on a device may be a captured
 * one.
 */
int32_t perm_mod3_batch_dev(const uint8_t *mats_dev, const int64_t *offs_dev,
                             const int32_t *ns_dev, int32_t count, uint8_t *out_dev,
                             uint64_t *hist_dev, void *stream);

/*
 * perm_mod3_batch_packed: as perm_mod3_batch_dev but the matrices are
 * already bipedal.  planes_dev holds, for the r-th row of matrix k,
 * planes_dev[2*(row_off_dev[k] + r)] = mag and [.. + 1] = sgn as uint64 words
 * under phi (Section 2): element j of the row (0-based) is bit n-1-j.  Any
 * bipedal representation is accepted ((0,1) is a zero).  Bits >= n must be
 * zero in both words; a matrix violating that gets PERM_RESULT_INVALID.
 * row_off_dev: device int64[count].  Other arguments as perm_mod3_batch_dev.
 */
int32_t perm_mod3_batch_packed(const uint64_t *planes_dev, const int64_t *row_off_dev,
                                const int32_t *ns_dev, int32_t count, uint8_t *out_dev,
                                uint64_t *hist_dev, void *stream);

/*
 * perm_mod3_batch_packed_noalloc: perm_mod3_batch_packed for callers that
 * cannot allocate device memory: code recorded under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Arguments, layout, results
 * and the histogram are those of perm_mod3_batch_packed, and the same kernels
 * run, but the call allocates nothing (no hipMalloc, hipFree, host staging or
 * library graph): its work buffers (plan records, packed rows, tallies,
 * completion counts, queue counters, accumulator words) live in one static
 * device array of the library, PERM_NOALLOC_SCRATCH_BYTES bytes on every
 * device the library runs on, held until the process ends.  The array's
 * device address is looked up once per device when the library first runs
 * there (that first call makes the device's context: a stream and events,
 * no device memory).
 *   count:  0 <= count <= PERM_NOALLOC_MAX_COUNT, else PERM_EINVAL and
 *           nothing runs.
 *   stream: the kernels go on `stream` (NULL: the legacy default stream)
 *           directly; under the caller's graph capture they are recorded
 *           into the caller's graph.  The call is not ordered with other
 *           calls into the library (it shares no buffer with them).
 * Every call on one device shares that device's array, which keeps the last
 * call's contents; each call clears what must start at zero itself.  Two such
 * calls that overlap on one device (different streams without an order
 * between them, or replays of two graphs holding such calls run
 * concurrently) race on the array and give wrong results: order them.
 */
#define PERM_NOALLOC_MAX_COUNT 8192
#define PERM_NOALLOC_SCRATCH_BYTES 17212416ull
int32_t perm_mod3_batch_packed_noalloc(const uint64_t *planes_dev, const int64_t *row_off_dev,
                                       const int32_t *ns_dev, int32_t count, uint8_t *out_dev,
                                       uint64_t *hist_dev, void *stream);

/*
 * perm_mod3_from_tallies: perm(A) mod 3 of an n x n matrix from the exact
 * partial tallies T(a_k, b_k) of Gray ranges that together cover [0, 2^n)
 * exactly once (for example the shards of a long run, each from
 * perm_mod3_range_tally, possibly on different devices): by eq. (2) and the
 * additivity of T over blocks of consecutive Gray states (Section 3.1),
 * perm(A) = (-1)^n * sum_k T_k, reduced here mod 3 on the device.
 *   tallies: host int64[count], 1 <= count <= PERM_MAX_TALLIES; their true
 *            sum must fit in int64 (it does for tallies of such a cover).
 *   *out:    host byte in {0,1,2}.
 * Synchronous.  PERM_EINVAL for n outside [0, 63], count out of range or a
 * null pointer.
 */
#define PERM_MAX_TALLIES (1 << 20)
int32_t perm_mod3_from_tallies(int32_t n, const int64_t *tallies, int32_t count, uint8_t *out);

/*
 * perm_mod3_pack: the map phi of Section 2 applied to each row of A on the host:
 * planes[2r] = mag, planes[2r+1] = sgn of row r, element j at bit n-1-j
 * (so the row (1,1,0,-1) packs to mag 0xd, sgn 0x1).  A: host n*n bytes,
 * planes: host uint64[2n].  PERM_EDOMAIN on an entry > 2.
 */
int32_t perm_mod3_pack(const uint8_t *A, int32_t n, uint64_t *planes);

/* --------------------------------------------------------------------------
 * Census: how many matrices have perm 0, 1 and -1, over matrices made on the
 * device (the exact counts of Table 3 and the Monte Carlo study of Table 4).
 *
 * generator PERM_GEN_ENUMERATE: matrix t (first <= t < first + count) has
 *   entry k (row-major) equal to the k-th base-3 digit of t, least significant
 *   first; t = 0 .. 3^(n*n) - 1 lists every n x n matrix over F_3 once.
 *   Requires n <= 6 and first + count <= 3^(n*n).
 * generator PERM_GEN_SPLITMIX: entry k of matrix t is floor(3 x / 2^64) for x
 *   the (t*n*n + k + 1)-th output of SplitMix64 seeded with `key` (Steele, Lea
 *   and Flood 2014: state key + q * 0x9E3779B97F4A7C15, then its mixing
 *   function), i.e. iid uniform entries.
 * counts: host uint64[3], receives the number of matrices with perm mod 3
 * equal to 0, 1 and 2.  1 <= n <= 63.  Synchronous.  Small n walk one matrix
 * per lane; larger n are generated into device memory in chunks and walked by
 * the batch path.
 */
#define PERM_GEN_ENUMERATE 0
#define PERM_GEN_SPLITMIX  1
int32_t perm_mod3_census(int32_t n, int32_t generator, uint64_t key, uint64_t first, uint64_t count,
                         uint64_t *counts);

/* --------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * Requests (one matrix each) are admitted into device-resident slots while
 * the total admitted work (sum of 2^n Gray indices still to visit) stays
 * within work_budget and a slot is free.  The server repeatedly launches a
 * "tick": a persistent launch that visits up to `quantum` Gray indices,
 * split across the admitted requests by the policy; each request's partial
 * tally stays on the device between ticks, so requests that arrive while
 * others are running join the next tick.  A request finishes when its last
 * chunk is visited; the finishing kernel reduces its tally mod 3.
 */
typedef struct perm_server perm_server;

typedef struct {
    int32_t  max_slots;     /* device slots (admitted requests); 1..65536          */
    int32_t  queue_cap;     /* host submission queue capacity; 1..1<<24            */
    uint64_t work_budget;   /* max admitted Gray indices still to visit (0 = none) */
    uint64_t quantum;       /* Gray indices per tick (0 = library default)         */
    int32_t  policy;        /* PERM_POLICY_*                                      */
    int32_t  fast_max_n;    /* requests with n <= fast_max_n skip the slots and run
                               in batches of up to 64 (and 2^28 Gray indices) beside
                               the tick in flight, one launch each; 0 = library
                               default (28), -1 = none, else 1..28               */
    int32_t  tick_timeout_ms; /* watchdog: a tick still running after this many ms
                               fails the server, and every request it holds or has
                               queued completes with status PERM_EDEVICE; 0 = none */
    int32_t  reserved;      /* 0 */
} perm_server_cfg;

#define PERM_POLICY_SRPT 0   /* least remaining work first                         */
#define PERM_POLICY_FIFO 1   /* admission order; each tick serves the oldest first */

typedef struct {
    uint64_t tag;           /* the caller's tag from perm_server_submit          */
    int32_t  status;        /* PERM_OK or an error code for this request         */
    int32_t  n;
    uint8_t  result;        /* perm mod 3 in {0,1,2}                              */
    uint8_t  pad[7];
    uint64_t t_submit_ns;   /* CLOCK_MONOTONIC times                              */
    uint64_t t_admit_ns;
    uint64_t t_done_ns;
} perm_done;

typedef struct {
    uint64_t submitted, completed, ticks, tick_indices;
    uint64_t busy_ns;       /* wall time with at least one tick in flight         */
    int32_t  active_slots, queued;
} perm_server_stats;

/* Create a server with its own device context, stream and worker thread. */
int32_t perm_server_create(const perm_server_cfg *cfg, perm_server **out);
/* Copy A (host, n*n bytes) into the server; the caller may free A at once.
 * PERM_EAGAIN when the queue is full, PERM_EDOMAIN/EINVAL for bad input. */
int32_t perm_server_submit(perm_server *s, const uint8_t *A, int32_t n, uint64_t tag);
/* Move up to max finished requests into out (host); *got = how many.
 * Waits up to timeout_us for at least one (0 = do not wait). */
int32_t perm_server_poll(perm_server *s, perm_done *out, int32_t max, int32_t *got,
                          int64_t timeout_us);
int32_t perm_server_stats_get(perm_server *s, perm_server_stats *st);
/* Finish all admitted and queued work, stop the worker and free everything. */
int32_t perm_server_destroy(perm_server *s);

/* --------------------------------------------------------------------------
 * Tuning, timing, device facts.
 */
typedef struct {
    int32_t waves_per_simd;   /* persistent waves per SIMD (1..16)                        */
    int32_t body_log;         /* n > mid_max_n: a lane's chunk is at least 2^(body_log+1)
                                 Gray indices and the fast walk takes n >= body_log + 7
                                 (its blocks are 16 indices whatever the value): 4, 5 or 6  */
    int32_t chunk_log_max;    /* largest per-lane chunk, log2 Gray indices (8..24)        */
    int32_t tasks_per_wave;   /* target tasks per persistent wave                         */
    int32_t direct_max_n;     /* n at or below which every step is tested exactly        */
    int32_t use_graphs;       /* 1: capture device-input calls of more than 64 matrices
                                 into cached HIP graphs                                     */
    int32_t states_per_lane;  /* chunks a lane walks per task, one after another: 1, 2, 4 */
    int32_t body_log_mid;     /* body_log for direct_max_n < n <= mid_max_n: 4, 5 or 6    */
    int32_t mid_max_n;        /* see body_log_mid                                         */
    int32_t max_tasks_log;    /* a matrix is cut into at most 2^min(max_tasks_log,
                                 (n-3)/2) tasks ...                                         */
    int32_t min_task_log;     /* ... unless its tasks would then exceed 2^min_task_log Gray
                                 indices; each task ends with an atomic on its matrix's
                                 counters, and on one address those serialise (0..30)       */
    int32_t queue_task_log;   /* tasks of a call hold at least 2^queue_task_log Gray indices
                                 once its work gives every persistent wave one such task:
                                 each task after a wave's first is one atomic on the call's
                                 single queue counter, and those serialise (0..30; 0 = no
                                 floor)                                                      */
} perm_tuning;

/*
 * The context keeps one tuning per class of call.  The block decomposition of
 * Section 3.1 (how long a lane's run of consecutive Gray states is, how many
 * runs make a task, how many waves take tasks) is a free choice that does not
 * change any result; what runs fastest differs between one large matrix, one
 * small one and a batch of mixed orders.  A call's class:
 *   PERM_TUNE_SMALL  host calls of one matrix with n <= 24 (latency bound)
 *   PERM_TUNE_MID    host calls of one matrix with 25 <= n <= 31
 *   PERM_TUNE_LARGE  host calls of one matrix with n >= 32; one-matrix
 *                    device-input calls (the host does not read their order);
 *                    the 128-column walk
 *   PERM_TUNE_BATCH  calls of two or more matrices, the census, the server
 * The host calls perm_mod3 and perm_mod3_range_tally count as calls of one
 * matrix.
 */
#define PERM_TUNE_SMALL   0
#define PERM_TUNE_MID     1
#define PERM_TUNE_LARGE   2
#define PERM_TUNE_BATCH   3
#define PERM_TUNE_CLASSES 4

/* where a class's tuning came from */
#define PERM_TUNE_SRC_DEFAULT  0   /* the library's built-in defaults              */
#define PERM_TUNE_SRC_CACHE    1   /* a tuning cache file (perm_tuning_cache_load) */
#define PERM_TUNE_SRC_SET      2   /* perm_tuning_set / perm_tuning_set_class      */
#define PERM_TUNE_SRC_AUTOTUNE 3   /* perm_autotune / perm_autotune_batch          */

/* perm_tuning_get: the tuning of class PERM_TUNE_LARGE.  perm_tuning_set:
 * one tuning for every class.  Both act on the current device's context. */
int32_t perm_tuning_get(perm_tuning *t);
int32_t perm_tuning_set(const perm_tuning *t);
/* One class's tuning and its source (source may be NULL). */
int32_t perm_tuning_get_class(int32_t cls, perm_tuning *t, int32_t *source);
int32_t perm_tuning_set_class(int32_t cls, const perm_tuning *t);
/* Every class back to the built-in defaults (source PERM_TUNE_SRC_DEFAULT);
 * with with_cache != 0, then the tuning cache a new context loads (below),
 * which leaves the classes as they were when the context was made. */
int32_t perm_tuning_reset(int32_t with_cache);

/*
 * Tuning cache: a text file, one line per (device, class):
 *     <arch> <compute units> <class name> key=value ...
 * with the class names small, mid, large, batch and the keys the fields of
 * perm_tuning; '#' starts a comment.  perm_tuning_cache_load applies the lines
 * whose arch (the gcnArchName, e.g. "gfx950:sramecc+:xnack-") and compute
 * unit count equal the current device's; lines for other devices, unknown
 * keys and out-of-range tunings are skipped.  *loaded (may be NULL) = classes
 * set.  PERM_EINVAL if the file cannot be opened.
 * perm_tuning_cache_save writes the current device's classes whose source is
 * not the default, keeping every other line of an existing file; the file is
 * replaced atomically.
 * When a context is made, the library loads the file named by the environment
 * variable PERM3_TUNING_CACHE (none when it is set but empty), else the file
 * perm3_tuning.txt beside libperm3.so, if there is one.
 */
int32_t perm_tuning_cache_load(const char *path, int32_t *loaded);
int32_t perm_tuning_cache_save(const char *path);

/*
 * perm_autotune: time candidate tunings of the class a one-matrix host call
 * of order n falls in (12 <= n <= 63) on a synthetic uniform n x n matrix and
 * keep the fastest as that class's tuning (source PERM_TUNE_SRC_AUTOTUNE).
 * The search covers the persistent waves per SIMD, the per-lane chunk length
 * (chunk_log_max, tasks_per_wave, and the per-matrix task bounds), the block
 * length and the chunks per lane, by successive halving: every candidate is
 * timed once, the faster half again with twice the repetitions, and so on;
 * the class's current tuning is always a candidate.  budget_ms bounds the
 * search (the first round always completes).  Classes SMALL and MID are timed
 * by the whole call's wall time, LARGE by the walk kernel's HIP events over
 * 2^min(n, 36) Gray indices.  Writes the winner to *best.
 */
int32_t perm_autotune(int32_t n, int32_t budget_ms, perm_tuning *best);

/*
 * perm_autotune_batch: the same search for class PERM_TUNE_BATCH, timed on the
 * caller's own batch (arguments as perm_mod3_batch_packed; out_dev receives
 * the results of the last timed run).  Each candidate's time is the whole
 * call's (plan, pack, walk) by HIP events on the library's stream.
 * Synchronous.
 */
int32_t perm_autotune_batch(const uint64_t *planes_dev, const int64_t *row_off_dev, const int32_t *ns_dev,
                            int32_t count, uint8_t *out_dev, int32_t budget_ms, perm_tuning *best);

typedef struct {
    double   hot_kernel_ms;   /* Gray-walk kernel of the last call, HIP events on its stream */
    double   total_ms;        /* all launches of the last call                          */
    uint64_t indices;         /* Gray indices visited by the last call                   */
    int32_t  launches;        /* kernel launches of the last call                        */
    int32_t  graph_replayed;  /* 1 if the last call replayed a cached HIP graph          */
} perm_timing;

/* Enable (1) or disable (0) event timing of subsequent calls on this thread's device. */
int32_t perm_timing_enable(int32_t on);
int32_t perm_timing_last(perm_timing *t);

typedef struct {
    int32_t compute_units;
    int32_t simds_per_cu;
    int32_t wave_size;
    int32_t max_clock_khz;
    char    arch[64];
} perm_device_info;

int32_t perm_device_info_get(perm_device_info *info);

/* Device self-check of Theorem 2.1: for each of the count inputs
 * in[4k..4k+3] = (mag1, sgn1, mag2, sgn2) (32-bit words), writes
 * out[8k..8k+7] = (mag, sgn) of, in order: the sum by the printed addition
 * formula, the difference by the printed subtraction formula, the product,
 * and the difference as the walk forms it (the sum with the negated second
 * operand, whose sgn word is sgn2 xor mag2), each computed by the device
 * functions the kernels use.  in/out: host.  For testing. */
int32_t perm_bipedal_ops(const uint32_t *in, int32_t count, uint32_t *out);

const char *perm_strerror(int32_t code);
const char *perm_last_error(void);
int64_t     perm_last_error_index(void);
const char *perm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PERM3_H */
