/*
 * libdpc -- exact Density Peaks Clustering on AMD Instinct MI355X (gfx950).
 *
 * The method is that of "Faster Parallel Exact Density Peaks Clustering"
 * (Huang, Yu, Shun).  Given n points in d dimensions and the three parameters
 * d_cut, rho_min and delta_min (Section 3), it computes
 *
 *   rho[i]    the density of point i: the number of points j (i itself
 *             included) with D(x_i, x_j) <= d_cut            (Definition 1);
 *   dep[i]    the dependent point of i: the nearest point of strictly higher
 *             priority, where the priority of j is the pair (rho[j], -j), so
 *             that equal densities rank the lower index higher; an equal
 *             distance is won by the smaller index            (Definition 2,
 *             and the tie rule of the write-min in Section 5, Algorithm 2);
 *   delta2[i] the squared dependent distance D(x_i, x_dep[i])^2
 *                                                              (Definition 3);
 *   label[i]  -1 for a noise point (rho < rho_min, Definition 4); otherwise
 *             the index of the cluster centre (a non-noise point with
 *             delta >= delta_min, Definition 5) reached by following
 *             dependent points: the single-linkage step of Section 6.2,
 *             Algorithm 3.
 *
 * D is the Euclidean distance.  Coordinates are int32, so D^2 is an integer
 * and is computed exactly: D <= d_cut is decided as D^2 <= floor(d_cut^2)
 * and delta >= delta_min as delta2 >= ceil(delta_min^2).  Every output is
 * therefore a unique, exactly defined integer array.
 *
 * Sentinels: the point of highest priority has dep = -1 and
 * delta2 = INT64_MAX (delta = infinity, Definition 3); so do points skipped as
 * noise when dependents are requested only for rho >= rho_min.
 *
 * Conventions shared by every call below
 *   - Array arguments are DEVICE pointers on the current HIP device.  points
 *     is int32 [n][d], row-major and contiguous.  Outputs are allocated by the
 *     caller and fully overwritten.  Indices are 0-based.
 *   - n >= 0 and 1 <= d <= 8.  n = 0 is a no-op returning DPC_OK.  n must be
 *     below 2^31.
 *   - The sum over axes of (max - min)^2 of the coordinates must not exceed
 *     2^63 - 1, so that every squared distance fits in int64; otherwise
 *     DPC_ERR_RANGE.
 *   - Work is enqueued on `stream` (0 = the null stream).  Calls that build
 *     a spatial index read the coordinate bounds back to the host once, which
 *     synchronises the stream at that point.  The library allocates its
 *     workspace stream-ordered from a memory pool of its own on the current
 *     device and releases it, also stream-ordered, before returning; it keeps
 *     no pointer to caller memory after return.  The pool keeps freed memory
 *     for later calls (up to the largest workspace used) until the process
 *     ends.  Outputs are ready when the stream's work completes.
 *   - The return value is a dpc_status.  Argument errors are detected before
 *     any GPU work is enqueued.  On any error the output contents are
 *     unspecified.  Nothing aborts the process and no exception crosses the
 *     interface.
 *   - Results are bit-identical across runs, streams and tuning choices.
 *     Concurrent calls on different streams are allowed.
 */
#ifndef LIBDPC_H
#define LIBDPC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#if defined(__GNUC__)
#define DPC_API __attribute__((visibility("default")))
#else
#define DPC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DPC_OK = 0,
    DPC_ERR_INVALID_ARG = 1, /* null pointer, n < 0, d outside [1, 8], NaN/negative d_cut, ... */
    DPC_ERR_RANGE = 2,       /* squared distances could exceed int64 */
    DPC_ERR_NOT_FOREST = 3,  /* dpc_cluster: a followed dependent edge does not rank higher */
    DPC_ERR_OOM = 4,         /* workspace allocation failed */
    DPC_ERR_HIP = 5,         /* a HIP runtime call failed */
    DPC_ERR_SCRATCH = 6      /* dpc_run_noalloc: the instance needs more than its fixed scratch */
} dpc_status;

/* dpc_run flag: compute dependents only for points with rho >= rho_min, as
 * Section 4.3, Algorithm 1 does; the others get (-1, INT64_MAX).  Labels do
 * not change. */
#define DPC_SKIP_NOISE_DEPENDENTS 1u
/* dpc_run flag: record HIP events on the call's stream around each step, for
 * dpc_last_stats.  Adds no synchronisation to the call. */
#define DPC_TIME_STAGES 2u
/* dpc_run flag: run instrumented kernels that count the work they do (slower;
 * for measurement only).  The counts are read back before the call returns. */
#define DPC_COUNT_WORK 4u
/* dpc_run flag: find dependent points with the Fenwick tree of k-d trees
 * (Section 5, Algorithm 2) instead of the priority-search k-d tree
 * (Section 4.2).  Same outputs; a different algorithm, for comparison.
 * Work counters (DPC_COUNT_WORK) then cover the density step only. */
#define DPC_FENWICK_DEPENDENTS 8u
/* dpc_run flag: find dependent points with the priority-search k-d tree
 * exactly as Section 4.2 defines it, every node storing the point of highest
 * priority in its subtree (DPC_BACKEND_PRIORITY_SEARCH_TREE below).  Same
 * outputs; not combinable with DPC_FENWICK_DEPENDENTS.  Work counters then
 * cover the density step only. */
#define DPC_PST_DEPENDENTS 16u

/* Steps of dpc_run timed by DPC_TIME_STAGES. */
enum {
    DPC_STAGE_INDEX = 0,     /* bounds (with the host read-back) and k-d tree build */
    DPC_STAGE_DENSITY = 1,   /* density kernel */
    DPC_STAGE_PRIORITY = 2,  /* priority keys and per-node maximum keys */
    DPC_STAGE_DEPENDENT = 3, /* dependent-point kernel */
    DPC_STAGE_LABELS = 4,    /* cluster labels */
    DPC_STAGES = 5
};

/* Measurements of the most recent dpc_run on the calling host thread that
 * passed DPC_TIME_STAGES and/or DPC_COUNT_WORK. */
typedef struct {
    uint32_t flags;                /* which of the two were recorded */
    double stage_ms[DPC_STAGES];   /* GPU time per step, from the events */
    int64_t density_pairs;         /* point-pair distance tests, density step */
    int64_t density_nodes;         /* node-box tests by query lanes, density step */
    int64_t density_contained;     /* points counted through whole contained nodes (Section 6.1) */
    int64_t dependent_pairs;       /* point-pair tests of higher-priority candidates, dependent step */
    int64_t dependent_nodes;       /* node-box tests by query lanes, dependent step */
    /* the same walks counted per wavefront (64 queries walk together) */
    int64_t density_wave_nodes;    /* nodes visited, density step */
    int64_t density_wave_points;   /* leaf points iterated over (some lane tests them), density step */
    int64_t dependent_wave_nodes;  /* nodes visited, dependent step */
    int64_t dependent_wave_points; /* leaf points iterated over, dependent step */
    uint64_t workspace_bytes;      /* device workspace the call allocated (each allocation rounded up to 256 B) */
} dpc_stats;

/*
 * Density (Section 3, Definition 1; Section 6.1 for the counting of whole
 * index cells that lie inside the ball).
 *   points  int32 [n][d] device, read only.
 *   d_cut   radius >= 0 (may be +inf); NaN or negative -> DPC_ERR_INVALID_ARG.
 *   rho     int32 [n] device, written: rho[i] >= 1.
 */
DPC_API int dpc_density(const int32_t *points, int64_t n, int32_t d, double d_cut,
                int32_t *rho, hipStream_t stream);

/*
 * Dependent points (Section 3, Definitions 2-3; Section 4, the priority
 * nearest-neighbour search of Algorithm 1).
 *   rho      int32 [n] device, read only: any densities (typically from
 *            dpc_density); they define the priority (rho[j], -j).
 *   rho_min  0 computes every point; > 0 skips points with rho < rho_min,
 *            which get (-1, INT64_MAX).  Negative -> DPC_ERR_INVALID_ARG.
 *   dep      int32 [n] device, written.
 *   delta2   int64 [n] device, written.
 */
DPC_API int dpc_dependent(const int32_t *points, int64_t n, int32_t d, const int32_t *rho,
                  int32_t rho_min, int32_t *dep, int64_t *delta2, hipStream_t stream);

/*
 * Cluster labels (Section 3, Definitions 4-5 and the assignment rule after
 * them; Section 6.2, Algorithm 3).  A non-noise point i with
 * delta2[i] < ceil(delta_min^2) follows dep[i]; a non-noise point with
 * delta2[i] >= ceil(delta_min^2) is a centre.  delta_min <= 0 makes every
 * non-noise point a centre; +inf leaves only points with delta2 = INT64_MAX.
 *   rho, dep, delta2  device arrays of n, read only (from the calls above or
 *                     any caller data).
 *   label             int32 [n] device, written.
 * Every followed edge must lead to an index in [0, n) of strictly higher
 * priority (which makes the graph a forest); otherwise DPC_ERR_NOT_FOREST.
 * The check reads one flag back to the host, synchronising the stream.
 */
DPC_API int dpc_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2,
                int32_t rho_min, double delta_min, int32_t *label, hipStream_t stream);

/*
 * The whole method: density, dependent points and labels, sharing one
 * spatial index (the three steps of Section 1).  flags: any combination of
 * DPC_SKIP_NOISE_DEPENDENTS, DPC_TIME_STAGES, DPC_COUNT_WORK and one of
 * DPC_FENWICK_DEPENDENTS and DPC_PST_DEPENDENTS.  Output
 * arrays as above; all four are written.
 */
DPC_API int dpc_run(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min,
            double delta_min, uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2,
            int32_t *label, hipStream_t stream);

/*
 * For callers that cannot allocate device memory: code that must not call
 * hipMalloc or a stream-ordered allocator (tight serving loops, harnesses
 * that forbid allocation).  Computes exactly what dpc_run computes, with
 * every workspace array carved from a fixed scratch area instead of the
 * library's memory pool: a static device array of DPC_NOALLOC_SCRATCH_BYTES
 * that the library's code object holds on every device it runs on, until
 * the process ends.  The call allocates no device memory and frees none.
 *   Arguments and outputs as for dpc_run (device pointers; the caller
 *   allocates the outputs).  flags: 0 or DPC_SKIP_NOISE_DEPENDENTS.  The
 *   dependent points always come from the priority-search k-d tree, whatever
 *   dpc_set_dependent_backend says.
 *   Limit: an instance fits when dpc_workspace_bytes(n, d) is at most
 *   DPC_NOALLOC_SCRATCH_BYTES (64 MiB: up to 706,560 points in 2-D,
 *   524,288 in 3-D and 262,144 in 8-D); a larger one returns
 *   DPC_ERR_SCRATCH before any GPU work.
 *   The first call on a device looks up that device's copy of the scratch
 *   (hipGetSymbolAddress, no allocation); DPC_ERR_HIP if that fails.
 *   Synchronises the stream like dpc_run (the bounds read-back).
 * Every call on one device shares that device's scratch, and the scratch
 * keeps the last call's contents: calls that overlap in time on one device
 * (on other streams or host threads) race on it and their outputs are
 * unspecified.  Order such calls on one stream or with events.
 */
#define DPC_NOALLOC_SCRATCH_BYTES (64ull << 20)
DPC_API int dpc_run_noalloc(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                            double delta_min, uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2,
                            int32_t *label, hipStream_t stream);

/*
 * Parameter sweeps (the decision-graph workflow of Section 3: the outputs for
 * many parameter values, each step reusing what does not depend on them).
 *
 * dpc_density_sweep: the density of every point for count radii, building
 * the spatial index once (it does not depend on d_cut).
 *   d_cuts  host array of count radii (each as for dpc_density).
 *   rho     int32 [count][n] device: row k is dpc_density with d_cuts[k].
 * Synchronises the stream once more at the end.
 */
DPC_API int dpc_density_sweep(const int32_t *points, int64_t n, int32_t d, const double *d_cuts, int32_t count,
                              int32_t *rho, hipStream_t stream);

/*
 * dpc_cluster_sweep: labels for count (rho_min, delta_min) pairs from one
 * (rho, dep, delta2) (delta_min touches only this step, Definition 5; rho_min
 * only the noise test of Definition 4, with dependents computed for every
 * point).
 *   rho_mins, delta_mins  host arrays of count values (each as for
 *                         dpc_cluster); 0 <= count <= 65535.
 *   label   int32 [count][n] device: row k is dpc_cluster with pair k.
 * Every followed edge of every pair is checked as in dpc_cluster
 * (DPC_ERR_NOT_FOREST); synchronises the stream once for that check.
 */
DPC_API int dpc_cluster_sweep(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2,
                              const int32_t *rho_mins, const double *delta_mins, int32_t count, int32_t *label,
                              hipStream_t stream);

/*
 * One independent clustering problem of a batch: the arguments and output
 * arrays of dpc_run, plus the instance's own status (written).
 */
typedef struct {
    const int32_t *points; /* int32 [n][d] device */
    int64_t n;
    int32_t d;
    double d_cut;
    int32_t rho_min;
    double delta_min;
    int32_t *rho;          /* int32 [n] device, written */
    int32_t *dep;          /* int32 [n] device, written */
    int64_t *delta2;       /* int64 [n] device, written */
    int32_t *label;        /* int32 [n] device, written */
    int32_t status;        /* written: the status dpc_run would return for this instance */
} dpc_instance;

/*
 * The whole method on many independent instances at once (sizes and
 * dimensions may differ).  Instances of one dimension and one arithmetic
 * share every launch: each step runs once over all of them, so the number of
 * kernel launches does not grow with the number of instances.  Every
 * instance's outputs are bit-identical to those of dpc_run with the same
 * arguments.
 *   instances  host array of count records; pointers in them are device
 *              pointers.  Each record's status is set: an invalid instance
 *              (as dpc_run would reject it) or one out of range is skipped.
 *   flags      0 or DPC_SKIP_NOISE_DEPENDENTS (applies to every instance).
 * Returns DPC_OK if every instance succeeded, otherwise the first failing
 * instance's status (or a runtime error, after which outputs are
 * unspecified).  Reads back the coordinate bounds of each dimension's
 * instances once (synchronising the stream).  When the instances span
 * several dimensions, each dimension runs on a stream and host thread that
 * the library creates for the call (default priority, on the current
 * device); those streams first wait for the work already queued on
 * `stream`, and `stream` then waits for them, so the call is ordered on
 * `stream` as a single-stream call would be.
 */
DPC_API int dpc_batch_run(dpc_instance *instances, int32_t count, uint32_t flags, hipStream_t stream);

/*
 * Upper bound on the device workspace (bytes, as the library counts them:
 * each allocation rounded up to 256 B) that dpc_run or dpc_batch_run takes
 * for an instance of n points in d dimensions; a batch takes at most the sum
 * of its instances' bounds.  The caller's inputs and outputs are not
 * included.  Host only; 0 for an invalid shape.
 */
DPC_API uint64_t dpc_workspace_bytes(int64_t n, int32_t d);

/*
 * Plans: a dpc_run recorded once and replayed.  dpc_plan_create runs dpc_run
 * on the given arguments (same outputs, same errors) and keeps its workspace
 * and its sequence of kernel launches, arguments included.  A replay
 * (dpc_plan_launch) enqueues that sequence again on any stream with no host
 * work, no allocation and no synchronisation: it reads the CURRENT contents
 * of `points` and overwrites rho, dep, delta2 and label, exactly as dpc_run
 * would for those contents, provided every coordinate still lies inside the
 * per-axis bounds measured when the plan was made.  Each replay checks this
 * on the device and records DPC_OK or DPC_ERR_RANGE in the plan's status
 * word (dpc_plan_status); after DPC_ERR_RANGE that replay's outputs are
 * unspecified (coordinates are clamped into the planned bounds, so the
 * replay stays within its buffers).  n, d, d_cut, rho_min, delta_min,
 * flags, the pointers and the leaf size are fixed at creation.
 *
 * dpc_plan_capture turns the sequence into a HIP graph (captured on the
 * given non-null stream, which must not be capturing already); later
 * dpc_plan_launch calls launch the graph.  The graph holds no memset or copy
 * nodes.  Replays of one plan that overlap in time race on its workspace and
 * outputs: order them on one stream or with events.  The caller keeps the
 * input and output buffers alive while the plan is used.
 *
 * dpc_plan_create: arguments as for dpc_run (flags: 0 or
 *   DPC_SKIP_NOISE_DEPENDENTS); *out receives the plan (NULL on error).
 *   Synchronises the stream.  The plan holds dpc_workspace_bytes(n, d) at
 *   most, until destroyed.
 * dpc_plan_launch: enqueues one replay on `stream`.
 * dpc_plan_capture: DPC_ERR_INVALID_ARG for a NULL stream or a plan already
 *   captured; DPC_ERR_HIP if capture fails (the plan stays usable uncaptured).
 * dpc_plan_status: copies the status word of the last replay (DPC_OK before
 *   any) to *status after the work on `stream` completes.
 * dpc_plan_destroy: waits for the device to go idle, then frees the plan.
 */
typedef struct dpc_plan dpc_plan; /* opaque */

DPC_API int dpc_plan_create(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                            double delta_min, uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2,
                            int32_t *label, hipStream_t stream, dpc_plan **out);
/*
 * dpc_plan_create_batch: the same for dpc_batch_run: records the batch
 *   (instances and flags as for dpc_batch_run; every record's status is
 *   set) and keeps it for replay.  Every instance must succeed, otherwise
 *   the first failing status is returned and no plan is made.  The record
 *   array itself is not kept.  A replay checks every instance against its
 *   planned bounds.  All dimensions run on `stream` (no library streams).
 */
DPC_API int dpc_plan_create_batch(dpc_instance *instances, int32_t count, uint32_t flags, hipStream_t stream,
                                  dpc_plan **out);
DPC_API int dpc_plan_launch(dpc_plan *plan, hipStream_t stream);
DPC_API int dpc_plan_capture(dpc_plan *plan, hipStream_t stream);
DPC_API int dpc_plan_status(dpc_plan *plan, hipStream_t stream, int32_t *status);
DPC_API int dpc_plan_destroy(dpc_plan *plan);

/*
 * Served clustering (the batching of dpc_batch_run applied to a stream of
 * requests).  A server owns `slots` host threads, each with a HIP stream of
 * its own on the device current at creation.  Requests wait in one queue in
 * arrival order; whenever a slot is free it takes the longest prefix of the
 * queue (at most max_batch requests) whose footprints, added to those of the
 * requests already running, stay within hbm_budget_bytes, and runs it as one
 * batch.  A request's footprint is its workspace bound (dpc_workspace_bytes)
 * plus its own device arrays: n * (4d + 20) bytes of points and outputs.  A request that
 * arrives while batches run thus joins the next batch a slot forms, and
 * several batches overlap on the device.  Every request's outputs are
 * bit-identical to those of dpc_run with the same arguments, whatever it is
 * batched with.
 */
typedef struct dpc_server dpc_server; /* opaque */

typedef struct {
    uint64_t hbm_budget_bytes; /* > 0: bound on the summed footprints of the requests in flight */
    int32_t slots;             /* 1 .. 16: batches in flight at once */
    int32_t max_batch;         /* >= 1: requests per batch */
} dpc_server_config;

typedef struct {
    int32_t done;        /* 1 once the request's outputs are written and its device work has completed */
    int32_t status;      /* when done: the dpc_status dpc_run would return for it (or a runtime error) */
    int64_t submit_ns;   /* CLOCK_MONOTONIC times of submission, admission to a batch and completion */
    int64_t admit_ns;
    int64_t done_ns;
    uint64_t footprint;  /* bytes charged against the budget while it ran: workspace bound + n * (4d + 20) */
    int32_t batch_size;  /* requests in its batch */
    int32_t slot;        /* the slot that ran it */
} dpc_request_info;

typedef struct {
    int64_t submitted;            /* requests accepted */
    int64_t completed;            /* requests done */
    int64_t rejected;             /* requests refused because their bound exceeds the whole budget */
    int64_t batches;              /* batches started */
    int64_t max_batch_seen;       /* largest batch */
    int32_t max_slots_busy;       /* most batches in flight at once */
    uint64_t max_admitted_bytes;  /* largest summed footprint of the requests in flight */
    uint64_t max_workspace_bytes; /* largest workspace a batch held */
    int64_t over_footprint;       /* batches whose workspace exceeded their summed footprint (a library bug if > 0) */
    uint64_t in_flight_bytes;     /* now: summed footprint of the requests in flight */
    int64_t queued;               /* now: requests waiting */
} dpc_server_stats;

/* Creates a server on the current device.  DPC_ERR_INVALID_ARG for a NULL
 * argument or a configuration outside the ranges above. */
DPC_API int dpc_server_create(const dpc_server_config *config, dpc_server **out);

/*
 * Queues one request: a record as for dpc_batch_run (device pointers; status
 * is ignored) and flags 0 or DPC_SKIP_NOISE_DEPENDENTS.  The arrays must stay
 * valid and untouched until the request is done.  Argument errors are
 * returned at once (no ticket); DPC_ERR_OOM if the request's footprint alone
 * exceeds the budget.  Otherwise *ticket identifies the request.
 */
DPC_API int dpc_server_submit(dpc_server *server, const dpc_instance *request, uint32_t flags, uint64_t *ticket);

/* Copies the request's state into *info without blocking.  Once a poll or
 * wait has reported it done, the ticket is forgotten (later calls with it
 * return DPC_ERR_INVALID_ARG). */
DPC_API int dpc_server_poll(dpc_server *server, uint64_t ticket, dpc_request_info *info);

/* Blocks until the request is done, then as dpc_server_poll. */
DPC_API int dpc_server_wait(dpc_server *server, uint64_t ticket, dpc_request_info *info);

/* Counters since creation. */
DPC_API int dpc_server_get_stats(dpc_server *server, dpc_server_stats *out);

/* Runs every queued request to completion, then stops the slots and frees
 * the server.  Results of requests not yet waited for are discarded. */
DPC_API int dpc_server_destroy(dpc_server *server);

/*
 * Tuning (never changes any output).  Points per k-d tree leaf, per
 * dimension: 16, 32 or 64 (the default).  Smaller leaves prune more point
 * tests and visit more nodes.  The setting is process-wide and read when a
 * call builds its index, so it applies to later calls on any thread and
 * stream.
 * dpc_set_leaf_size: DPC_ERR_INVALID_ARG for d outside [1, 8] or another size.
 * dpc_leaf_size: the current size for d (0 for an invalid d).
 */
#define DPC_LEAF_SIZES 3
DPC_API int dpc_set_leaf_size(int32_t d, int32_t leaf_points);
DPC_API int32_t dpc_leaf_size(int32_t d);

/*
 * Autotuner: runs the whole method on the given instance with each leaf size
 * (one warm-up and two timed runs each, HIP events on `stream`), keeps the
 * fastest size for dimension d (as dpc_set_leaf_size) and returns the
 * DPC_LEAF_SIZES times in ms_out[0] (16 points), ms_out[1] (32 points) and
 * ms_out[2] (64 points) and the choice in *chosen (either may be NULL).  Arguments as for dpc_run; the outputs go to
 * workspace and are discarded.  Synchronises the stream.  On failure the
 * previous setting is kept.
 */
DPC_API int dpc_autotune(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                         double delta_min, hipStream_t stream, double *ms_out, int32_t *chosen);

/*
 * Dependent-point backend per dimension.  All give the same outputs.
 *   DPC_BACKEND_PRIORITY_TREE (the default): the priority nearest-neighbour
 *     search of Section 4.2.2 on a balanced k-d tree whose nodes carry the
 *     highest priority below them (points stay in the leaves); the fastest
 *     here, and the only one the batched, served, planned and
 *     allocation-free calls use.
 *   DPC_BACKEND_FENWICK: the Fenwick tree of k-d trees (Section 5,
 *     Algorithm 2).
 *   DPC_BACKEND_PRIORITY_SEARCH_TREE: the priority-search k-d tree exactly as
 *     Section 4.2 defines it, every node storing the point of highest
 *     priority in its subtree and the rest split below it (Algorithm 1).
 * dpc_run uses the backend set for d unless DPC_FENWICK_DEPENDENTS or
 * DPC_PST_DEPENDENTS is passed; dpc_dependent and the other calls always use
 * DPC_BACKEND_PRIORITY_TREE.  The setting is process-wide.
 * dpc_set_dependent_backend: DPC_ERR_INVALID_ARG for d outside [1, 8] or an
 *   unknown backend.
 * dpc_dependent_backend: the current backend for d (-1 for an invalid d).
 * dpc_autotune_dependent: runs the whole method on the given instance with
 *   each backend (one warm-up and two timed runs each, HIP events on
 *   `stream`), keeps the fastest for dimension d and returns the times in
 *   ms_out[DPC_BACKEND_*] (DPC_BACKENDS entries) and the choice in *chosen
 *   (either may be NULL).  Arguments as for dpc_autotune.  Synchronises the
 *   stream.
 */
#define DPC_BACKEND_PRIORITY_TREE 0
#define DPC_BACKEND_FENWICK 1
#define DPC_BACKEND_PRIORITY_SEARCH_TREE 2
#define DPC_BACKENDS 3
DPC_API int dpc_set_dependent_backend(int32_t d, int32_t backend);
DPC_API int32_t dpc_dependent_backend(int32_t d);
DPC_API int dpc_autotune_dependent(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                                   double delta_min, hipStream_t stream, double *ms_out, int32_t *chosen);

/*
 * Diagnostics: copies the measurements of the calling thread's most recent
 * dpc_run made with DPC_TIME_STAGES or DPC_COUNT_WORK into *out, waiting for
 * that call's recorded events first.  DPC_ERR_INVALID_ARG if out is NULL or
 * no such call was made on this thread.  Not part of the method.
 */
DPC_API int dpc_last_stats(dpc_stats *out);

/* Static description of a status code; never NULL. */
DPC_API const char *dpc_status_str(int status);

/*
 * Host-only helper: the integer threshold used for a radius r >= 0.
 * round_up = 0 gives floor(r^2) (the d_cut rule), 1 gives ceil(r^2) (the
 * delta_min rule), both saturating at INT64_MAX; r = +inf gives INT64_MAX.
 * NaN, negative r or out == NULL -> DPC_ERR_INVALID_ARG.  No GPU work.
 */
DPC_API int dpc_square_threshold(double r, int32_t round_up, int64_t *out);

#ifdef __cplusplus
}
#endif

#endif /* LIBDPC_H */
