/*
 * abjoin.h -- C ABI of the MI355X (gfx950) AB-join library, libabjoin.so.
 *
 * The library computes the matrix profile of an inter-time-series similarity
 * join ("Error-bounded Approximate Time Series Joins Using Compact Dictionary
 * Representations of Time Series", Sec. 2.1 Def. 7 and Sec. 3.2 Alg. 2): for
 * every length-m window i of a query series it finds the nearest neighbour,
 * under the z-normalised Euclidean distance (Def. 4), among the windows of a
 * reference.  The reference is a dictionary stored as one concatenated series
 * with segment offsets; only the windows that slide inside one segment take
 * part (Def. 8), so a plain AB-join is the one-segment case.
 *
 * Conventions shared by every entry point
 *   - Indexing is 0-based.  Window i of a series x of length n is
 *     x[i .. i+m-1], i = 0 .. n-m.
 *   - seg_bounds is a HOST array of n_seg+1 int64 offsets with
 *     seg_bounds[0] = 0 < seg_bounds[1] < ... < seg_bounds[n_seg] = n_dict.
 *     Reference window j is valid iff seg_bounds[s] <= j and
 *     j + m <= seg_bounds[s+1] for some s (Def. 8).  Segments shorter than m
 *     contribute no window.
 *   - Distance: population mean and deviation per window; d = ||z(u) - z(v)||,
 *     which equals sqrt(2 m (1 - rho)) and lies in [0, 2 sqrt(m)].
 *   - Results: P_AB[i] is the distance to the nearest valid reference window,
 *     I_AB[i] its index in the concatenated reference (ties: smallest index).
 *     A row with no valid reference window gets P = +inf, I = -1 (Alg. 2
 *     initialises the profile to +inf).
 *   - Flat windows (population variance <= 1e-10 x the variance of all finite
 *     samples of their series) are the zero vector after normalisation:
 *     flat-flat distance 0, flat vs non-flat sqrt(m).  Reference windows with a
 *     non-finite sample are not windows; query rows with one get P = NaN,
 *     I = -1.  (The paper does not cover either case.)
 *   - Device buffers are caller-owned device memory (hipMalloc or a PyTorch
 *     CUDA tensor).  The library never frees caller memory.
 *   - hip_stream: a hipStream_t cast to void*, NULL for the null stream.  Calls
 *     that take a stream are asynchronous: they enqueue work and return; the
 *     results are ready when the stream reaches that point.
 *   - Every entry point returns an abj_status.  On ABJ_EINVAL nothing has been
 *     enqueued and no output has been written.  abj_last_error() gives the
 *     text of the last failure on the calling thread.  No C++ exception
 *     crosses this interface.
 */
#ifndef ABJOIN_H
#define ABJOIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ABJ_OK = 0,
    ABJ_EINVAL = -1,    /* invalid argument; nothing enqueued, outputs untouched */
    ABJ_ENOMEM = -2,    /* device or host allocation failed */
    ABJ_EHIP = -3,      /* a HIP runtime call failed; text in abj_last_error() */
    ABJ_EBUSY = -4,     /* serving: no slot or memory for the request right now */
    ABJ_ECANCELED = -5, /* serving: the request was cancelled */
    ABJ_ETIMEOUT = -6,  /* serving: the wait timed out */
    ABJ_ENOTFOUND = -7  /* serving: unknown request id */
} abj_status;

typedef enum {
    ABJ_TIER_FP32 = 0, /* FP32 incremental-diagonal covariance, FP64 winner re-check */
    ABJ_TIER_BF16 = 1, /* BF16 MFMA on centred, scaled windows + FP64 re-check of top-K */
    ABJ_TIER_FP16 = 2  /* FP16 MFMA on centred, scaled windows + FP64 re-check of top-K */
} abj_tier;

/* opts.flags bits */
#define ABJ_FLAG_NO_REFINE 1 /* precision tiers: skip the FP64 re-check and report the distance implied by the
                                best 16-bit score (to measure the tier's error before refinement) */
#define ABJ_FLAG_PEARSON 2   /* report the Pearson correlation of the nearest window, rho = 1 - d^2 / (2m), instead
                                of d (Sec. 2 allows either measure; the nearest window is the most correlated one).
                                Flat conventions become rho = 1 (flat-flat) and 1/2 (flat vs non-flat); a row with no
                                window gets -inf; NaN rows stay NaN */

typedef struct {
    int32_t tier;     /* abj_tier */
    int32_t refine_k; /* precision tiers: candidates re-checked per row, 1..8 (0 = 4), rounded up to 1, 2,
                         4 or 8; candidates are more than 4 windows apart and the re-check computes the
                         FP64 distance of the 64 / refine_k windows around each (7 before to 8 after
                         for 4) */
    int32_t flags;    /* ABJ_FLAG_* bits; 0 for default behaviour */
    int32_t reserved; /* must be 0 */
} abj_opts;

/* Library version, (major << 16) | minor. */
int abj_version(void);

/* Text describing the last non-OK status returned on this thread. */
const char* abj_last_error(void);

/*
 * Select the GPU and create library state for it.  Optional: every entry
 * point initialises the current device on first use.  Errors: ABJ_EHIP if the
 * device does not exist.
 */
int abj_init(int device_ordinal);

/*
 * Per-window statistics of one series (the O(n) step before the pair loop):
 * FP64 prefix sums of the series minus its mean give, for each window
 * i = 0 .. n-m, the mean mu[i] and population deviation sigma[i]
 * (Def. 4's z-normalisation).  flags[i] bit 0 = flat, bit 1 = holds a
 * non-finite sample.  x, mu, sigma, flags: device pointers; mu and sigma hold
 * n-m+1 doubles, flags n-m+1 bytes.  Errors: ABJ_EINVAL if m < 2, n < m or a
 * pointer is NULL or not device memory.
 */
int abj_window_stats(const double* x, int64_t n, int32_t m, double* mu, double* sigma, uint8_t* flags,
                     void* hip_stream);

/*
 * AB-join of a query against a concatenated dictionary (Alg. 2 over the
 * windows of Def. 8; one segment = plain AB-join).
 *   query   device, n_query doubles          dict  device, n_dict doubles
 *   seg_bounds  host, n_seg+1 int64 offsets (see conventions)
 *   P_AB    device, n_query-m+1 floats (out)  I_AB  device, n_query-m+1 int64 (out)
 *   opts    NULL = FP32 tier
 * FP32 tier: 2 <= m <= 4096, |P| within 1e-3 of FP64 (windows shorter than 8
 * samples, whose nearest distances fall below the resolution of FP32 pair
 * scores, compare FP64 correlations and run at about a fifth of the rate; the bar
 * is tested for every m).  BF16 / FP16 tiers (the paper's join with 16-bit
 * window products, a speed/accuracy option of this library): m <= 256; every
 * row takes up to refine_k candidates best-first by 16-bit score (pairwise
 * more than 4 windows apart) and returns the closest window in FP64 among the
 * windows near a candidate (for refine_k <= 4: from 7 before to 8 after it);
 * the 1e-3 bar is tested for m >= 8 (shorter windows have near-equal 16-bit
 * scores by the hundred: use the FP32 tier there).
 * Errors: ABJ_EINVAL if m < 2 (or above the tier's limit), n_query < m,
 * n_dict < 1, n_seg < 1, bad seg_bounds, an unknown tier, refine_k outside
 * 0..8, unknown flag bits, nonzero reserved field, or a NULL / non-device
 * pointer; ABJ_ENOMEM / ABJ_EHIP from the runtime.  Workspace is taken from the stream-ordered allocator on
 * hip_stream and returned to it before the call's work completes.
 */
int ab_join(const double* query, int64_t n_query, const double* dict, int64_t n_dict, const int64_t* seg_bounds,
            int32_t n_seg, int32_t m, float* P_AB, int64_t* I_AB, const abj_opts* opts, void* hip_stream);

/*
 * ab_join without device allocation, for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, serving loops that
 * must not call the allocator, harnesses that forbid it).  Arguments,
 * outputs, results and errors are those of ab_join, and the results equal
 * ab_join's.  The workspace is a fixed array of ABJ_NOALLOC_SCRATCH_BYTES
 * bytes of device memory that the library holds on every GPU it runs on until
 * the process ends (abj_init sets it up for its device; otherwise the first
 * call on a device does).  The call allocates nothing.
 *   Limit: a join whose workspace exceeds the array (about 90 bytes per
 *   sample of query and dictionary, plus 8 bytes per query window and column
 *   chunk of 1,024 dictionary windows when those fit, else atomics are used;
 *   plus the 16-bit operands and candidates in the BF16 / FP16 tiers) is
 *   rejected with ABJ_EINVAL before anything is enqueued.
 *   Sharing: every call on one GPU uses that GPU's one array, and each call
 *   initialises what it reads.  Calls that overlap on one GPU (other streams
 *   or other threads before the previous call's work has completed) race on
 *   the array and give undefined results: serialise them on one stream.
 */
#define ABJ_NOALLOC_SCRATCH_BYTES (64ll << 20)
int ab_join_noalloc(const double* query, int64_t n_query, const double* dict, int64_t n_dict,
                    const int64_t* seg_bounds, int32_t n_seg, int32_t m, float* P_AB, int64_t* I_AB,
                    const abj_opts* opts, void* hip_stream);

/*
 * Self-join matrix profile of one series (the P_B of the learning phase,
 * Alg. 1, and Def. 7 with A = B): for every window i of x, the nearest window
 * j with |i - j| > excl (trivial matches excluded).  excl = m/2 (rounded down)
 * is the zone the learning phase uses; excl < 0 selects it.
 *   x   device, n doubles
 *   P   device, n-m+1 floats (out)        I  device, n-m+1 int64 (out)
 *   P64 device, n-m+1 doubles (out, may be NULL): P before rounding to FP32
 * Rows whose zone covers every window get P = +inf, I = -1.  FP32 tier only
 * (opts may be NULL; tier must be ABJ_TIER_FP32), m <= 4096.  Errors: as
 * ab_join, and ABJ_EINVAL if excl >= n-m+1.
 */
int self_join(const double* x, int64_t n, int32_t m, int64_t excl, float* P, int64_t* I, double* P64,
              const abj_opts* opts, void* hip_stream);

/* ------------------------------------------------------------------------
 * Learning phase (Sec. 3.1, Alg. 1): greedy choice of the windows of a
 * training series T_B that form the dictionary D_B.
 *
 * Every window is ranked by its self-join distance (exclusion zone m/2,
 * rounded down) minus its distance to the closest window chosen so far (the
 * element-wise minimum of the chosen windows' distance profiles, Def. 4), and
 * the lowest-ranked window is taken next, so motifs come first and repeats of
 * a motif already in the dictionary sink (Fig. 4).  A chosen window and those
 * within m/2 of it are never chosen again, nor are windows whose self-join
 * distance is not finite; ties go to the smallest index; the run ends early
 * when no window is left.  Each choice adds ceil(context * m) samples of T_B
 * (at least m, at most n) with the window in the middle, shifted back inside
 * the series at the ends; pieces that overlap or touch merge into one segment.
 *
 * Stop conditions: ABJ_STOP_SPACE_SAVING stops once the merged dictionary
 * holds at least (1 - stop_value) n samples; ABJ_STOP_EMAX stops once e_max
 * of the current dictionary (Def. 10: the largest AB-join distance of a
 * window of T_B to the dictionary, computed with the FP32 join and its FP64
 * re-check) is <= stop_value.  max_iters > 0 caps the number of steps.
 * ---------------------------------------------------------------------- */
typedef enum { ABJ_STOP_SPACE_SAVING = 0, ABJ_STOP_EMAX = 1 } abj_stop;

typedef struct {
    double context;    /* element length factor k > 0: ceil(k m) samples, at least m, at most n (paper: 1.5) */
    double stop_value; /* SPACE_SAVING: s in [0, 1]; EMAX: target >= 0 */
    int32_t stop;      /* abj_stop */
    int32_t max_iters; /* 0: no cap */
} abj_learn_opts;

/*
 *   series       device, n doubles (T_B)
 *   segments     host, 2 * max_segments int64 (out): [start, end) sample
 *                ranges of T_B, sorted; the dictionary is their concatenation
 *                and its seg_bounds are the running sums of their lengths
 *   chosen       host, max_chosen int64 (out, may be NULL): the window chosen
 *                at each step, in order
 *   dict_out     device, n doubles (out, may be NULL): the concatenated
 *                dictionary; n_dict receives its length
 *   e_max        host (out, may be NULL): e_max of the final dictionary
 *                (+inf if it is empty)
 *   p_self       device, n-m+1 doubles (out, may be NULL): P_B
 * Sizing call: with segments, chosen and dict_out all NULL nothing runs and
 * the call returns, in whichever of *n_segments, *n_chosen and *n_dict are
 * given, upper bounds that every run with these n, m and opts respects
 * (series may then be NULL): buffers of those sizes never fail the run.
 * Blocking: runs on hip_stream and synchronises it once per step.
 * Errors: ABJ_EINVAL for m outside [2, 4096], n < m, bad opts, NULL required
 * pointers or non-device buffers, and (after the run, with no output
 * written) when the segments or choices exceed max_segments / max_chosen
 * (buffers sized by the sizing call are always large enough);
 * ABJ_ENOMEM / ABJ_EHIP from the runtime.
 */
int dict_build(const double* series, int64_t n, int32_t m, const abj_learn_opts* opts, int64_t* segments,
               int32_t max_segments, int32_t* n_segments, int64_t* chosen, int32_t max_chosen, int32_t* n_chosen,
               double* dict_out, int64_t* n_dict, double* e_max, double* p_self, void* hip_stream);

/* ------------------------------------------------------------------------
 * Discords (Sec. 2: the window with the largest matrix-profile value).  For
 * K > 1 discords the rule is greedy: the largest finite value (ties: smallest
 * index), then every row within excl of it is dropped (|r - r*| <= excl), and
 * so on; excl < 0 selects m - 1, so that no two discords overlap.
 * ---------------------------------------------------------------------- */

/*
 * Greedy top-K of any profile.
 *   P       device, W floats (NaN and +-inf rows are never chosen)
 *   rows    host, K int64 (out)      values  host, K floats (out, may be NULL)
 *   n_found host (out): picks made (< K when the rows run out)
 * Blocking (synchronises hip_stream).  Errors: ABJ_EINVAL if W < 1, K < 1,
 * excl < 0 or a pointer is NULL / not device memory.
 */
int topk_discords(const float* P, int64_t W, int32_t K, int64_t excl, int64_t* rows, float* values,
                  int32_t* n_found, void* hip_stream);

typedef struct {
    int64_t rows_exact;    /* query rows joined exactly against ref */
    int32_t rounds;        /* exact-evaluation rounds */
    int32_t certified;     /* bit 0: largest P_hat - second largest > e_max (the paper's test);
                              bit 1: same with the runner-up taken as the second discord, which
                              places the exact top discord within excl of the approximate one */
} abj_discord_info;

/*
 * Exact top-K discords of a query against a reference series (the database
 * T_B, or several joined with seg_bounds as in ab_join), starting from the
 * dictionary join P_hat of the same query.  By Lemmas 1 and 2 the exact
 * profile P obeys P_hat - e_max <= P <= P_hat, so the dictionary join is an
 * upper bound and rows far below the leaders need no exact join:
 *   round 0: rows with P_hat >= (largest P_hat) - e_max, which hold the top
 *            discord, are joined exactly (1024-row bands of the FP32 engine);
 *   repeat:  greedy top-K on the mixed profile (exact where joined, P_hat
 *            elsewhere); if every pick is exact they are the exact discords
 *            (every other row's value is an upper bound); otherwise the bands
 *            of all rows at or above the smallest pick value are joined.
 *   query    device, n_query doubles       P_hat  device, n_query-m+1 floats
 *   e_max    the dictionary's bound (Def. 10); < 0 skips round 0
 *   ref, ref_bounds, n_ref_seg: as dict / seg_bounds / n_seg of ab_join
 *   rows / values / neighbors: host, K entries (out): discord rows, their
 *            exact distances, and their nearest windows in ref (values and
 *            neighbors may be NULL)
 *   info     host (out, may be NULL)
 * Exact here means the FP32 tier's join (|error| <= 1e-3 against FP64).
 * Blocking.  Errors: as ab_join for the join arguments; ABJ_EINVAL if K < 1.
 */
int discords(const double* query, int64_t n_query, int32_t m, const float* P_hat, double e_max, const double* ref,
             int64_t n_ref, const int64_t* ref_bounds, int32_t n_ref_seg, int32_t K, int64_t excl, int64_t* rows,
             float* values, int64_t* neighbors, int32_t* n_found, abj_discord_info* info, void* hip_stream);

/* ------------------------------------------------------------------------
 * Resident dictionary: the learned dictionary of the inference phase (Alg. 2
 * joins every incoming series against the same D_B) kept in library-owned
 * device memory with its per-window statistics precomputed for each window
 * length in ms[].
 * ---------------------------------------------------------------------- */
typedef struct abj_dict abj_dict;

/*
 * dict: host or device pointer to n_dict doubles (copied; the caller keeps
 * ownership).  seg_bounds: host, n_seg+1 offsets.  orig_start: host, n_seg
 * entries or NULL: where each segment starts in the series it was taken from
 * (dict_build's segments; Sec. 4.2 builds D_B from pieces of T_B), kept so
 * that join results can be mapped back; NULL makes the dictionary its own
 * source (orig_start[s] = seg_bounds[s]).  ms: host, n_ms window lengths (each
 * 2..4096, n_ms 1..16).  Errors: ABJ_EINVAL on bad sizes, bounds, a negative
 * orig_start or pointers; ABJ_ENOMEM / ABJ_EHIP from the runtime.
 */
int abj_dict_create(const double* dict, int64_t n_dict, const int64_t* seg_bounds, int32_t n_seg,
                    const int64_t* orig_start, const int32_t* ms, int32_t n_ms, abj_dict** out);
int abj_dict_free(abj_dict* d);

/*
 * Maps n dictionary indices (I_AB of a join against d) to positions in the
 * source series: out[i] = orig_start[s] + (I[i] - seg_bounds[s]) for the
 * segment s holding I[i]; an index outside [0, n_dict) (the -1 of a row with
 * no neighbour) maps to -1.  I and out are device buffers of n int64 (they
 * may be the same buffer).  Asynchronous on hip_stream.  Errors: ABJ_EINVAL
 * for a NULL dictionary, n < 0 or non-device buffers.
 */
int abj_dict_source_index(const abj_dict* d, const int64_t* I, int64_t n, int64_t* out, void* hip_stream);

/* ab_join against a resident dictionary (m must be one of its ms).  Same
 * conventions, outputs and errors as ab_join; query, P_AB, I_AB are device
 * pointers. */
int ab_join_dict(const abj_dict* d, const double* query, int64_t n_query, int32_t m, float* P_AB, int64_t* I_AB,
                 const abj_opts* opts, void* hip_stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of joins against a resident dictionary.
 * A scheduler thread admits queued requests while a slot and memory are
 * free, launches every admitted request's tiles together in one persistent
 * FP32 batch kernel (two launches in flight, in order on the server's
 * stream, so requests that arrive while one batch runs join the next), and
 * completes each request when its batch finishes: a completion thread copies
 * the results out while the next batches run.  BF16/FP16 batches take one
 * operand launch, one matrix-core sweep per window-length class (k steps of
 * 16) present in the batch and one FP64 re-check launch for all their
 * requests; the dictionary's 16-bit operand is built at the first request of
 * each window length and kept.  A batch takes
 * at most half of the slots and half of the budget (a lone request may take
 * the whole budget), so the next batch can be formed and queued while one
 * runs.  A batch costs one host-to-device copy (queries and descriptors) and
 * one device-to-host copy (all results); each of the two batch buffer sets
 * keeps a device work buffer and pinned staging that grow to the largest
 * batch it has run and are released by abj_server_destroy, so the device
 * memory held stays within twice the budget plus descriptors.
 * ---------------------------------------------------------------------- */
typedef struct abj_server abj_server;

typedef struct {
    int32_t tier;            /* abj_tier for every request */
    int32_t max_slots;       /* requests admitted at once (>= 1) */
    int64_t mem_budget;      /* device bytes for admitted requests (> 0) */
    int32_t backend;         /* 0 = GPU; 1 = host simulation (no GPU calls; dict must be NULL) */
    int32_t sim_n_ms;        /* simulation only: accepted window lengths ... */
    int32_t sim_ms[8];
    int64_t sim_dict_windows;   /* ... dictionary window count used for pair counts */
    double sim_pairs_per_s;     /* ... simulated execution rate */
} abj_server_opts;

typedef struct {
    double t_arrive; /* seconds since server creation: submit */
    double t_admit;  /* admitted (slot + memory granted) */
    double t_start;  /* its batch was launched */
    double t_done;   /* results delivered to the host buffers */
    int64_t pairs;   /* valid pairs of the request */
    int32_t status;  /* ABJ_OK, ABJ_ECANCELED, or an error code */
    int32_t batch;   /* launch the request ran in */
    double t_device_done;  /* its batch finished on the device (slot and memory released) */
} abj_req_stats;

typedef struct {
    int64_t submitted, completed, canceled, rejected, batches;
    int64_t pairs;               /* valid pairs of completed requests */
    double busy_s;               /* first launch to last completion */
    double p50_s, p99_s, max_s;  /* latency t_done - t_arrive of completed requests */
} abj_server_stats;

/* Errors: ABJ_EINVAL on bad options (or a NULL dict with backend 0). */
int abj_server_create(const abj_dict* d, const abj_server_opts* opts, abj_server** out);
/* query_host: host pointer, copied before return.  Errors: ABJ_EINVAL if
 * n_query < m or m is not a window length of the dictionary (the request is
 * rejected; others are unaffected); ABJ_ENOMEM if the request alone exceeds
 * the memory budget. */
int abj_submit(abj_server* s, const double* query_host, int64_t n_query, int32_t m, uint64_t* req_id);
/* Zero-copy form of abj_submit: the server thread reads query_host when the
 * request is launched and writes the results straight into P_host and I_host
 * (host memory, n_query-m+1 entries each) when its batch completes.  The
 * caller keeps all three buffers alive, leaves the query unchanged and does
 * not read P_host / I_host until abj_wait returns ABJ_OK (or the request is
 * canceled); abj_result still has to be called to forget the request (its
 * output pointers may then be NULL).  Same errors as abj_submit, plus
 * ABJ_EINVAL for a NULL output. */
int abj_submit_borrowed(abj_server* s, const double* query_host, int64_t n_query, int32_t m, float* P_host,
                        int64_t* I_host, uint64_t* req_id);
/* Blocks until the request is done (ABJ_OK), canceled (ABJ_ECANCELED) or the
 * timeout passes (ABJ_ETIMEOUT; timeout_ms < 0 waits forever).  ABJ_ENOTFOUND
 * for unknown ids. */
int abj_wait(abj_server* s, uint64_t req_id, int32_t timeout_ms);
/* Copies a finished request's results (n_query-m+1 entries each; either may
 * be NULL) and statistics, then forgets the request.  ABJ_EBUSY if it is not
 * finished yet. */
int abj_result(abj_server* s, uint64_t req_id, float* P_host, int64_t* I_host, abj_req_stats* st);
/* Cancels a request that has not been launched yet (ABJ_OK); a launched
 * request completes normally (ABJ_EBUSY). */
int abj_cancel(abj_server* s, uint64_t req_id);
/* Waits until no request is queued or running (ABJ_ETIMEOUT otherwise). */
int abj_server_drain(abj_server* s, int32_t timeout_ms);
int abj_server_stats_get(abj_server* s, abj_server_stats* out);
/* Stops the scheduler after the running batches finish; queued requests are
 * canceled.  Results not yet collected are discarded. */
int abj_server_destroy(abj_server* s);

/*
 * Benchmark timing.  While enabled (on != 0), every join records a HIP event
 * pair around its pair-loop kernel on the call's stream.  abj_profile_read
 * waits for the recorded events, returns the summed kernel milliseconds, the
 * number of launches and the number of valid (query window, reference window)
 * pairs they covered since the previous read, and clears the record.  Any
 * output pointer may be NULL.  Errors: ABJ_EHIP from the event calls.
 */
int abj_profile_enable(int on);
int abj_profile_read(double* kernel_ms, int64_t* launches, int64_t* pairs);

#ifdef __cplusplus
}
#endif

#endif /* ABJOIN_H */
