/*
 * wf.h -- C ABI of libwf, the anti-diagonal wavefront sweep for AMD MI355X
 * (gfx950).
 *
 * THE OPERATION
 *   An m x n grid H is computed from a per-cell input c.  Each cell depends on
 *   its north (i-1, j), west (i, j-1) and north-west (i-1, j-1) neighbours:
 *
 *       H[i][j] = c[i][j] + op(N, W, NW),      op = min  (WF_RULE_MIN)
 *                                               op = max  (WF_RULE_MAX)
 *
 *   with boundary row/column
 *       N  = i == 0 ? top[j+1] : H[i-1][j]
 *       W  = j == 0 ? left[i]  : H[i][j-1]
 *       NW = i == 0 ? top[j]   : (j == 0 ? left[i-1] : H[i-1][j-1]).
 *   top has n+1 values (top[0] is the corner H[-1][-1]), left has m values.
 *   A NULL top/left selects the default boundary: the corner is 0 and every
 *   other boundary value is "absent" (+inf for min, -inf for max; for int32
 *   INT32_MAX and INT32_MIN+1), so H[i][j] is the min (max) over all monotone
 *   lattice paths (steps S, E, SE) from (0,0) to (i,j) of the sum of c.
 *   The grid resolves in m+n-1 anti-diagonal wavefronts.
 *
 *   Source: arxiv 2501.05938 states no sweep of its own; the cell rule above
 *   is this library's reading of the task it serves.  The max rule is the
 *   one the paper's equations fix: with the three copy/compute engines as
 *   columns and stream chunks as rows it is the flow-shop recurrence whose
 *   identical-rows closed form is the streamed-time model of Eq. 2
 *   (Section 2.2).  Problem parameters follow that paper's statement of its
 *   own problem: a size (here m, n), a precision (FP32 here; its FP64 is not
 *   offered), the caller's stream, and tuning knobs in place of its threads
 *   per block and sub-system size.
 *
 * ARITHMETIC
 *   WF_F32: float32 inputs and outputs, exactly one IEEE round-to-nearest-even
 *   addition per cell after an exact min/max, so results are bit-identical to
 *   a sequential fp32 loop in any evaluation order.  Inputs must be free of
 *   NaN; a NaN input gives unspecified values and may end in WF_ETIMEDOUT.
 *   WF_I32: int32 inputs and outputs, wrapping 32-bit addition; results are
 *   exact while every partial path sum stays inside (INT32_MIN, INT32_MAX).
 *   The value INT32_MIN is reserved (never a valid result).
 *   WF_F64: float64 inputs and outputs, one IEEE round-to-nearest-even fp64
 *   addition per cell, bit-identical to a sequential fp64 loop; the paper's own
 *   computations are FP64 (its Section 2), FP32 its variant (Section 3.2).  fp64
 *   grids use 64-row bands only, n and ld_cost at most 2^22, and are not served
 *   by the server; 16 bytes of memory traffic per cell in FULL mode.
 *
 * MEMORY AND OWNERSHIP
 *   All data pointers in wf_problem are DEVICE pointers on the context's
 *   device, owned by the caller; the library reads/writes them only inside
 *   the work it enqueues and keeps no reference after that work completes.
 *   Layouts are row-major with leading dimensions in ELEMENTS (ld >= n).
 *   The context owns its workspace (handoff rows, counters, descriptor
 *   tables); the server owns the output slots it hands out.
 *
 * ASYNCHRONY
 *   wf_solve / wf_solve_batched enqueue on `stream` (a hipStream_t, or NULL
 *   for the legacy default stream) and return; results are valid once the
 *   stream's work up to that point has completed.  Errors raised by the
 *   device (watchdog) are reported by the next call on the same context.
 *
 * ERRORS
 *   Every call returns a wf_status; nothing throws or aborts across the ABI.
 *   wf_last_error() returns a thread-local message for the last failure.
 */
#ifndef WF_H
#define WF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int wf_status;
enum {
  WF_OK = 0,
  WF_PENDING = 1,        /* wf_poll: request not finished yet */
  WF_EINVAL = -1,        /* bad argument (sizes, NULL required pointer, ld < n, unknown enum) */
  WF_ENOMEM = -2,        /* device or host allocation failed */
  WF_E2BIG = -3,         /* request larger than the server's HBM budget */
  WF_EHIP = -4,          /* HIP runtime error; message kept in wf_last_error() */
  WF_ETIMEDOUT = -5,     /* device watchdog fired (a wait exceeded the limit) */
  WF_ENOTFOUND = -6,     /* unknown server ticket */
  WF_ESHUTDOWN = -7,     /* server is shutting down / was destroyed */
  WF_EUNSUPPORTED = -8   /* valid but unsupported combination */
};

enum { WF_F32 = 0, WF_I32 = 1, WF_F64 = 2 };  /* element type of cost, top, left and outputs */
enum { WF_RULE_MIN = 0, WF_RULE_MAX = 1 };    /* op of the cell rule */
enum { WF_MODE_FULL = 0, WF_MODE_EDGES = 1 }; /* FULL writes all of H; EDGES writes only last row/col/cell */
/* wf_problem.flags.  WF_COST_ABSDIFF: dynamic time warping of two sequences.  The
 * input of cell (i, j) is |seq_x[i] - seq_y[j]| (the difference rounded once in fp32;
 * the absolute value is exact), computed on the device, so only the m + n sequence
 * values are read from memory; cost and ld_cost are ignored.  WF_F32 only.  With
 * the min rule and the default boundary, H[i][j] is the DTW distance of x[0..i] and
 * y[0..j].  (The paper has no such workload: it is a second input of the same
 * cell rule.) */
enum { WF_COST_ABSDIFF = 1 };

typedef struct wf_problem {
  int64_t m, n;            /* grid rows and columns, >= 1 (0 means nothing to do); n <= 2^23 (2^22 for fp64) */
  int32_t dtype;           /* WF_F32, WF_I32 or WF_F64 */
  int32_t rule;            /* WF_RULE_MIN or WF_RULE_MAX */
  int32_t mode;            /* WF_MODE_FULL or WF_MODE_EDGES */
  int32_t flags;           /* 0 or WF_COST_ABSDIFF */
  const void* cost;        /* device, m x n, row stride ld_cost elements; required */
  int64_t ld_cost;         /* >= n and <= 2^23 (WF_EUNSUPPORTED above) */
  void* out;               /* device, m x n, row stride ld_out; required in FULL mode, ignored in EDGES */
  int64_t ld_out;
  const void* top;         /* device, n+1 values, or NULL for the default boundary */
  const void* left;        /* device, m values, or NULL for the default boundary */
  void* last_row;          /* device, n values, or NULL (required in EDGES mode unless last_col or final_cell given) */
  void* last_col;          /* device, m values, or NULL */
  void* final_cell;        /* device, 1 value, or NULL */
  const void* seq_x;       /* WF_COST_ABSDIFF: device, m values (else ignored) */
  const void* seq_y;       /* WF_COST_ABSDIFF: device, n values (else ignored) */
} wf_problem;

typedef struct wf_tuning {
  int32_t waves_per_wg;    /* compute waves per workgroup: 1 or 2 (0 = automatic) */
  int32_t max_wgs;         /* persistent workgroups per launch (0 = automatic) */
  int32_t order;           /* batched work order: 0 = automatic, 1 = grid-major, 2 = interleaved by band */
  int32_t use_graph;       /* batched: 1 = capture and replay a hipGraph, 0 = plain launch,
                              -1 = plain launch without autotuning */
  int32_t rows_per_lane;   /* grid rows each lane of a compute wave owns: 1 or 2 (0 = automatic);
                              bands are 64 * waves_per_wg * rows_per_lane rows; two waves of two
                              rows per lane are not offered (WF_EUNSUPPORTED) */
  int32_t reserved[3];     /* must be 0 */
} wf_tuning;

typedef struct wf_ctx wf_ctx;

/* Create a context on HIP device `device`.  One context per host thread, or
 * guard it with your own lock. */
wf_status wf_init(int device, wf_ctx** out);
/* Wait for the context's outstanding work and free its workspace. */
wf_status wf_destroy(wf_ctx* ctx);

/* Sweep one grid with one persistent kernel launch on `stream`. */
wf_status wf_solve(wf_ctx* ctx, const wf_problem* p, void* stream);

/* wf_solve with explicit tuning (NULL: as wf_solve): waves_per_wg and rows_per_lane pick
 * the band shape -- 64-row bands (1, 1), 128-row bands of two compute waves chained
 * through LDS (2, 1) or of one wave whose lanes own two rows each (1, 2); wf_solve takes
 * (1, 1) -- and max_wgs caps the
 * persistent workgroups; order and use_graph are ignored.  Every shape gives the same,
 * bit-identical result. */
wf_status wf_solve_tuned(wf_ctx* ctx, const wf_problem* p, const wf_tuning* t, void* stream);

/* The per-grid path: every problem swept by its own launch (as wf_solve), problem i
 * on streams[i % nstreams].  Launches on different streams may run concurrently;
 * up to 64 launches of a context are in flight before a launch waits for the
 * oldest to finish.  The stream count is the parameter the paper's model chooses
 * (wf_stream_model_choose). */
wf_status wf_solve_each(wf_ctx* ctx, const wf_problem* ps, int64_t count, void* const* streams, int32_t nstreams);

/* Sweep `count` independent grids of any sizes in one persistent launch on
 * `stream`; the bands of all grids are packed into one work list so the thin
 * first and last diagonals of one grid overlap the wide middle of another.
 * All grids of one call share dtype and rule (WF_EUNSUPPORTED otherwise).
 * Autotuning: when `t` is NULL or leaves waves_per_wg, rows_per_lane and order at 0
 * (and use_graph is not -1), the first call for a batch of a new shape class (dtype,
 * rule, modes, and the binary magnitudes of the grid count, total cells, tallest and
 * widest grid) runs the batch twice per candidate configuration (the three band
 * shapes x grid-major / interleaved order x all or half of the resident workgroups),
 * synchronously, timing the second run on `stream`, and keeps the fastest in the
 * context's tuning table (persisted to the JSON file WF_TUNE_CACHE names, if set);
 * later calls of that class use it.  Every trial writes the full, correct result.
 * With use_graph = 1 the chosen launch is captured in a hipGraph and replayed
 * when the same batch shape is solved again. */
wf_status wf_solve_batched(wf_ctx* ctx, const wf_problem* ps, int64_t count, const wf_tuning* t, void* stream);

/* For callers that cannot allocate memory: code under HIP graph capture, serving
 * loops and harnesses that forbid hipMalloc.  wf_solve_noalloc is wf_solve
 * (same kernels, same results, same asynchrony and error reporting) except that
 * the launch's control words and handoff rows live in a fixed device array of
 * WF_NOALLOC_SCRATCH_BYTES that the library holds on each device from wf_init
 * until the process ends, and the call allocates nothing: no hipMalloc, hipFree
 * or allocating library routine.  The caller still passes inputs and outputs.
 * It uses the band shape wf_solve picks (bands of 64 rows), and a problem needs
 * 256 + 4 * (ceil(m / 64) - 1) * L bytes of it, with
 * L = 64 * ceil(4 * floor((n + 66) / 4) / 64) (the handoff row of one band
 * boundary; about 4 * m * n / 64 bytes in all, 16.8 MB for 16384 x 16384); a
 * problem that needs more returns WF_E2BIG and nothing is enqueued (empty
 * problems are no-ops, as in wf_solve).  Every call on a device shares
 * that device's array, and each call re-arms what it uses on `stream` before its
 * launch: calls that overlap on one device (different streams, or different
 * contexts of one device, with no ordering between them) race on the array and
 * give wrong results.  Order them on one stream. */
#define WF_NOALLOC_SCRATCH_BYTES (32ll << 20)
wf_status wf_solve_noalloc(wf_ctx* ctx, const wf_problem* p, void* stream);

/* Traceback, the step after a sweep: the path of predecessor choices through a
 * computed grid.  Reads p->out (FULL-mode H of an m x n problem, row stride
 * p->ld_out), p->dtype, p->rule and p->top / p->left (the boundary the sweep used,
 * or NULL for the default); cost and the edge outputs are not used.  Starting at
 * (m-1, n-1) it repeatedly steps to the predecessor -- NW (i-1, j-1), N (i-1, j),
 * W (i, j-1), boundary values standing in for predecessors outside the grid --
 * whose value the rule selects (smallest for min, largest for max), the first of
 * NW, N, W on equal values, and stops when that predecessor lies outside the grid.
 * The paper states no traceback; the preference order is this library's reading.
 * Writes to `path` (device, int32, 2 * (m + n) entries) the visited cells as (i, j)
 * pairs, (m-1, n-1) first, followed by the outside predecessor the walk ended on
 * ((-1, j), (i, -1) or (-1, -1)); writes the number of visited cells (at most
 * m + n - 1) to `length` (device, one int64).  Asynchronous on `stream` like
 * wf_solve; one wave walks the grid in 64 x 64 tiles held in registers.
 * Errors: WF_EINVAL (m or n < 1, NULL out/path/length, ld_out < n). */
wf_status wf_traceback(wf_ctx* ctx, const wf_problem* p, int32_t* path, int64_t* length, void* stream);

/* Set the device watchdog of later launches on this context: a wait for a
 * neighbouring band that makes no progress for `ms` milliseconds (0 .. 3600000)
 * aborts the launch, which then drains and is reported as WF_ETIMEDOUT.  The
 * default is 2000 ms (or WF_WATCHDOG_MS from the environment at wf_init). */
wf_status wf_set_watchdog(wf_ctx* ctx, int64_t ms);

/* Wait for all work this context has enqueued and return WF_ETIMEDOUT if the
 * device watchdog fired in any of it, WF_OK otherwise.  (wf_solve and
 * wf_solve_batched report such an error too, on the first call after the
 * failed launch has finished.) */
wf_status wf_check(wf_ctx* ctx);

/* ---------------------------------------------------------------- serving */
typedef struct wf_server wf_server;

typedef struct wf_server_opts {
  int64_t hbm_budget_bytes;  /* bytes of device memory the server may hold for requests (0 = 64 GiB) */
  int32_t max_inflight;      /* launches allowed in flight at once (0 = 2), each on its own stream.  More
                                overlap host set-up with running launches, but persistent launches that
                                run together share compute units, which slows both: two measured best */
  int32_t max_batch;         /* requests per launch at most (0 = 256) */
  int32_t copy_streams;      /* streams that copy host inputs at admission, overlapping earlier launches
                                (0 = copy on the launch stream just before the launch; at most 8) */
  int32_t max_wait_skip_us;  /* a request that does not fit the budget yet may be overtaken by later,
                                smaller ones until it has waited this long (0 = 20000 us) */
  int64_t staging_bytes;     /* pinned staging for pageable host inputs when copy_streams > 0 (0 = 256 MiB) */
  int32_t reserved[2];       /* must be 0 */
} wf_server_opts;

enum {
  WF_INPUT_DEVICE = 0,       /* `input` is device memory, read in place */
  WF_INPUT_HOST = 1,         /* `input` is pageable host memory, copied into a server-owned slot */
  WF_INPUT_SEED = 2,         /* no `input`: cell (i, j) is output i*n + j of the SplitMix64 stream seeded
                                with `seed` (float32: (x >> 40) * 2^-24; int32: x & 255), generated on
                                the device into a server-owned slot */
  WF_INPUT_HOST_PINNED = 3   /* `input` is pinned host memory (hipHostMalloc), copied by DMA without staging */
};

typedef struct wf_request {
  int64_t m, n;
  int32_t dtype, rule, mode;
  int32_t input_kind;        /* WF_INPUT_*.  Device inputs must stay valid and unchanged until wf_poll
                                reports completion; host inputs may be reused once it has */
  const void* input;
  int64_t ld_input;          /* elements, >= n (ignored for WF_INPUT_SEED) */
  uint64_t seed;             /* WF_INPUT_SEED only */
  void* ready_event;         /* WF_INPUT_DEVICE: a hipEvent_t recorded after the input was written (the
                                launch waits for it on the device), or NULL when the input is already
                                complete at wf_submit; the event must not be destroyed before completion */
} wf_request;

typedef struct wf_result {
  const void* out;           /* device, server-owned; FULL mode: m x n with stride ld_out; else NULL */
  int64_t ld_out;
  const void* last_row;      /* device, server-owned, n values */
  const void* last_col;      /* device, server-owned, m values */
  const void* final_cell;    /* device, server-owned, 1 value */
  double t_submit;           /* seconds on the server's monotonic clock */
  double t_admit;
  double t_launch;
  double t_done;             /* time the server observed completion */
} wf_result;

/* Start a server thread that admits requests as device memory frees up,
 * batches the admitted ones into persistent launches on up to max_inflight
 * streams, and records completion times. */
wf_status wf_server_create(wf_ctx* ctx, const wf_server_opts* opts, wf_server** out);
/* Queue a request; never blocks on the GPU.  WF_E2BIG if it can never fit. */
wf_status wf_submit(wf_server* s, const wf_request* r, uint64_t* ticket);
/* WF_OK with *out filled when done, WF_PENDING before that. */
wf_status wf_poll(wf_server* s, uint64_t ticket, wf_result* out);
/* Free the request's slots; pointers from wf_poll become invalid. */
wf_status wf_release(wf_server* s, uint64_t ticket);
/* Drain admitted work, cancel the rest (WF_ESHUTDOWN), join the thread, free everything. */
wf_status wf_server_destroy(wf_server* s);
/* Bytes of device memory currently held for requests, and the peak so far. */
wf_status wf_server_memory(wf_server* s, int64_t* in_use, int64_t* peak);
/* Tickets whose requests have finished (done or failed) since the last call, oldest
 * first: up to `cap` are written to tickets[0..cap) and their number to *count.  Each
 * finished ticket is reported once (a ticket released before it is reported is
 * skipped); wf_poll still returns its result until it is released.  One call replaces
 * a wf_poll per pending ticket for a caller with many requests in flight.
 * WF_EINVAL: NULL server or count, cap < 0, or NULL tickets with cap > 0. */
wf_status wf_server_done(wf_server* s, uint64_t* tickets, int64_t cap, int64_t* count);

/* Latency of one step of the walk's dependency chain on this device, in ns: one wave
 * runs `steps` (16 .. 2^30) steps of N = the neighbour lane's H, H = c + min(N, NW, H)
 * with nothing else on the compute unit (synchronous; allocates a few bytes).  The
 * shortest possible sweep of an m x n grid by lanes that each own a row takes
 * (m + n - 1) such steps: the sweep's latency floor. */
wf_status wf_measure_step_ns(wf_ctx* ctx, int64_t steps, double* ns_per_step);

/* ------------------------------------------ launch-concurrency (stream) model
 * The model of arXiv 2501.05938, Sections 2.3-2.4 (Eqs. 3-7) and the selection
 * rule of Section 3, used here to choose how many streams the per-grid path
 * (wf_solve_each) spreads its launches over.  Host-only: no device call.
 *
 * A sample is one timed job: `size` is the problem size (the paper's SLAE size;
 * for the per-grid path, the cells of all grids of the job), `streams` the
 * stream count s, `t_str` its time on s streams, `t_non_str` the same job on one
 * stream, and `sum` the time of the operations the streams overlap (the paper's
 * Eq. 3; here the device time of the job's kernels run one after another).
 * All times in milliseconds. */
typedef struct wf_stream_sample {
  double size;
  int32_t streams;           /* >= 1 */
  int32_t reserved;          /* ignored */
  double t_str, t_non_str, sum;
} wf_stream_sample;

typedef struct wf_stream_model {
  double sum_slope, sum_intercept;  /* Eq. 4: sum = sum_slope * size + sum_intercept */
  double split_size;                /* Eq. 7 regimes: small for size <= split_size, big above */
  double small[3];                  /* Eq. 7 small: small[0]*size + small[1]*log10(s) + small[2] */
  double big[3];                    /* Eq. 7 big: (big[0]*size + big[1]) * log2(s^(4/3)) + big[2] */
} wf_stream_model;

typedef struct wf_fit_report {
  double r2_train, r2_test;         /* 1 - SS_res / SS_tot on each half of the 3:1 split */
  double mse_train, mse_test;       /* SS_res / samples */
  int64_t n_train, n_test;
} wf_fit_report;

/* Fit the model to `count` samples (Section 2.4).
 *   Eq. 4 is fitted on one point per distinct size (sizes in order of first
 *   appearance; its sum is the mean of that size's samples); Eq. 5 turns every
 *   sample with streams >= 2 into an overhead, and Eq. 7 is fitted per regime on
 *   those samples in input order (small: size <= split_size).
 *   Each fit is least squares on a shuffled 3:1 split: the caller passes the
 *   shuffle as a permutation of the fit's points (perm_sum: one entry per distinct
 *   size; perm_small / perm_big: one per overhead sample of that regime; a
 *   regime without samples gets zero coefficients and its permutation is not
 *   read); the first ceil(k/4) entries of a permutation are the test set.
 *   report (may be NULL) receives 3 entries: sum model, small, big.
 * Errors: WF_EINVAL for NULL pointers, invalid samples, a permutation that is not
 * one, or too few / degenerate training points. */
wf_status wf_stream_model_fit(const wf_stream_sample* samples, int64_t count, double split_size,
                              const int64_t* perm_sum, const int64_t* perm_small, const int64_t* perm_big,
                              wf_stream_model* out, wf_fit_report* report);
/* Eq. 7: the modelled overhead of s streams at `size` (NaN for a NULL model or s < 1). */
double wf_stream_model_overhead(const wf_stream_model* m, double size, int32_t s);
/* Section 3's choice: among `ncand` candidate stream counts (NULL = 1, 2, 4, 8, 16,
 * 32) the one whose gap (s-1)/s * sum_model(size) - overhead(size, s) (Eq. 6) is
 * largest and positive; 1 when no gap is positive.  gaps (may be NULL) receives
 * one gap per candidate. */
wf_status wf_stream_model_choose(const wf_stream_model* m, double size, const int32_t* candidates, int32_t ncand,
                                 int32_t* best, double* gaps);

/* ----------------------------------------------------------------- errors */
const char* wf_last_error(void);
const char* wf_status_str(wf_status s);
/* Library version string. */
const char* wf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WF_H */
