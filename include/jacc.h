/*
 * jacc.h — C ABI of the K-partitioned loop-nest runtime for AMD MI355X (gfx950).
 *
 * Model (after JACC, Matsumura, Garcia De Gonzalo, Pena, HiPC 2021,
 * arXiv 2110.14340):
 *   - Data regions: arrays are declared to the runtime with create / copyin /
 *     copyout routines that stand in for OpenACC data directives
 *     (Sec. "JACC", converted-code listing: jacc_create ... jacc_copyout).
 *     Any address inside a declared array resolves to it (Sec. "Automated
 *     Asynchronous Execution": data ranges are kept in an ordered tree so any
 *     address of declared data is accepted).
 *   - Parallel loops: a loop nest is launched by one call that carries its
 *     kernel, its arguments and flags (the jacc_kernel_push routine of the
 *     converted-code listing).  Here the kernel is one of a fixed set of
 *     hand-written HIP loop bodies (JACC_LOOP_*), and every argument declares
 *     the rows of dim 0 it reads or writes relative to the outer iterator.
 *   - Partitioning: the outermost dimension of every array is divided
 *     equally into K owner blocks (Sec. "Division of Multidimensional
 *     Arrays"), B_p = [floor(p*E/K), floor((p+1)*E/K)).  Partition p keeps a
 *     private device slab holding B_p widened by the array's declared halo
 *     (or the whole array for arrays declared WHOLE, which are replicated as
 *     the paper replicates allocations and host-to-device copies on every
 *     device, Sec. "Predicate-Based Filtering").  A loop runs on partition p
 *     only the iterations whose write row lies in B_p — the paper's
 *     write-predicate [a_lb, a_ub] hoisted into the launch bounds, exact for
 *     loops that write element i of dim 0 from outer iteration i.
 *   - Coherence: before a partition runs, the rows it reads that its slab
 *     does not hold in their latest version are copied from the partition
 *     that wrote them last (device-local copies).  For the stencil kinds the
 *     producing partition instead also writes the output rows that other
 *     slabs hold as halo (a write-through restricted to the holders of each
 *     row), so no copy is needed at all.  Both replace the paper's
 *     send-everything-after-each-kernel scheme with range-driven transfers.
 *   - Asynchrony: partition p's work runs on stream p (outside batches the
 *     partitions of a JACOBI2D, HEAT3D, SUM or column-banded SPMV_CSR loop
 *     instead run as one packed launch on one stream; see
 *     JACC_INIT_NO_PACK).  Cross-stream waits are inserted only for the
 *     rows actually shared (read-after-write and write-after-read),
 *     skipping waits already satisfied (the paper keeps access timestamps
 *     and the most recent synchronisation among queues, Sec. "Automated
 *     Asynchronous Execution").  The events these waits use are recorded
 *     after each partition's kernel of a loop spread over several streams;
 *     after a packed launch or a loop of one partition an event is
 *     recorded only when some other stream first waits on it.
 *
 * Conventions
 *   - Every call returns a jacc_status (0 = success, negative = error).  The
 *     library never aborts and no C++ exception crosses this boundary.
 *   - A failed HIP call makes the context sticky: every later call returns
 *     JACC_ERR_DEVICE until jacc_finalize.  jacc_last_error gives the text.
 *   - Host arrays are owned by the caller and must stay valid from enter to
 *     exit.  Device slabs are owned by the library and freed when the
 *     array's reference count reaches zero or at jacc_finalize.  Streams
 *     passed to jacc_init stay owned by the caller.
 *   - Calls return after enqueueing.  Results become visible on the host at
 *     jacc_wait, jacc_update(HOST), jacc_data_exit(COPYOUT) or a synchronous
 *     reduction.
 */
#ifndef JACC_H
#define JACC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jacc_ctx jacc_ctx; /* opaque; owned by the library */

typedef enum {
    JACC_OK = 0,
    JACC_ERR_INVALID = -1,         /* bad argument (NULL, negative size, unknown kind ...) */
    JACC_ERR_NOT_PRESENT = -2,     /* host address not inside any declared array */
    JACC_ERR_ALREADY_PRESENT = -3, /* enter of an overlapping range with a different descriptor */
    JACC_ERR_RANGE = -4,           /* access outside a slab, or partitions writing the same rows */
    JACC_ERR_ALLOC = -5,           /* the allocator returned NULL */
    JACC_ERR_DEVICE = -6,          /* a HIP call failed (sticky) */
    JACC_ERR_UNSUPPORTED = -7      /* a legal request the library does not implement */
} jacc_status;

/* Device-memory allocator.  alloc returns device memory of at least `bytes`
 * bytes aligned to 256 bytes, or NULL; free releases it.  The library calls
 * free only after every stream that used the memory has been synchronised.
 * Passing NULL to jacc_init selects hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} jacc_allocator;

typedef enum { JACC_F64 = 0, JACC_F32 = 1, JACC_I32 = 2, JACC_I64 = 3 } jacc_dtype;

/* Array descriptor.  Row-major.  part_dim is the partitioned dimension (0,
 * or 1 for a 2-D array; Sec. "Division of Multidimensional Arrays": the
 * dimension jacc_parallel_dim chooses) with extent E = extent[part_dim]; a
 * "row" is one index of that dimension: with part_dim 0 it holds
 * extent[1]*...*extent[ndim-1] contiguous elements, with part_dim 1 it is a
 * column of extent[0] elements, extent[1] apart in the host array.  Row
 * ranges everywhere in this interface (owner blocks, halos, access offsets,
 * updates) count such rows.  halo_lo/halo_hi are the largest distances (in
 * rows) below and above the owner block that loops will read.  whole = 1
 * keeps a full replica in every partition (the paper's replicated
 * allocation); whole = 2 keeps one full copy on the device that every
 * partition reads (one GPU holds all partitions, so read-only data need not
 * be duplicated): loops may only read it (a writing argument is
 * JACC_ERR_INVALID) and update(DEVICE) refreshes the one copy.
 * num_partitions: K of this array
 * (0 = the context's K; at most 64; with more partitions than the context has
 * streams, partition p runs on stream p mod the stream count).
 * A partition's slab of a part_dim 1 array holds its columns [lo, hi) as a
 * row-major block of extent[0] rows that starts at the even column lo & ~1
 * and has an even pitch ((hi - (lo & ~1) + 1) & ~1 elements), so that even
 * global columns sit on 16-byte boundaries; its transfers are strided 2-D
 * copies.  Such arrays are never whole (JACC_ERR_INVALID) and take JACOBI2D
 * loops only, with both arguments split along dimension 1 (otherwise
 * JACC_ERR_UNSUPPORTED).  By default the kernel writes each column another
 * slab keeps into that slab too (column mirrors) and the partitions run as
 * one packed launch; halo columns are pulled under JACC_INIT_LAZY, or sent
 * under JACC_INIT_EAGER.  No FILTERED output, no persistent execution, no
 * tuning or cost-model picks (JACC_ERR_UNSUPPORTED). */
typedef struct {
    int32_t dtype;
    int32_t ndim;            /* 1..4 */
    int64_t extent[4];
    int32_t halo_lo, halo_hi;
    int32_t whole;
    int32_t num_partitions;
    int32_t part_dim;        /* 0, or 1 for ndim == 2 */
    int32_t reserved;        /* must be 0 */
} jacc_array_desc;

/* data_enter clauses */
enum { JACC_COPYIN = 1, JACC_CREATE = 2, JACC_COPY = 3 };
/* data_exit clauses */
enum { JACC_COPYOUT = 1, JACC_DELETE = 2 };
/* update directions */
enum { JACC_UPDATE_HOST = 1, JACC_UPDATE_DEVICE = 2 };
/* argument access modes */
enum { JACC_READ = 1, JACC_WRITE = 2, JACC_READWRITE = 3,
       /* with JACC_WRITE: the argument is written through data-dependent
        * indices; every partition runs the whole iteration space and keeps
        * only the writes that land in its owner block (the paper's
        * predicate-based filtering: a write a[k] is guarded by
        * a_lb <= k <= a_ub, Sec. "Predicate-Based Filtering") */
       JACC_FILTERED = 4 };

/* Loop argument: the base address of a declared array, its access mode and
 * the rows of dim 0 that outer iteration i touches, [i+off_lo, i+off_hi]
 * (inclusive), or the whole array when whole != 0. */
typedef struct {
    void *host;
    int32_t mode;
    int32_t off_lo, off_hi;
    int32_t whole;
} jacc_arg;

/* Iteration space: half-open [lo[d], hi[d]) per loop dimension; dim 0 is the
 * one split among partitions. */
typedef struct {
    int32_t ndim;
    int32_t pad_;
    int64_t lo[3], hi[3];
} jacc_bounds;

/* Launch configuration.  Never changes the arithmetic of a loop body's
 * outputs (fields are bit-identical under every configuration); the order in
 * which a reduction adds its terms does depend on it.
 *   bx, by     workgroup shape in threads (bx a multiple of 64; bx*by <= 1024)
 *   tile       rows (2-D) or planes (3-D) each thread marches through;
 *              GEMM: k-slab depth staged through LDS, 16 or 32 (with bx =
 *              256 or 512 threads per 128x128 tile); SPMV_CSR: lanes per
 *              row, 4, 8 or 16 (order 2 = non-temporal col/val loads), or
 *              with order 4 (column bands) lanes per row and band, 1 to 16,
 *              by = bands per XCD (1, 2, 4, 8), rows = rows per lane (2 or 4
 *              with one lane).  The banded form copies each partition's
 *              entries once into band-major order on the device (kept until
 *              row_ptr, col or val change), runs the bands of XCD j on XCD j
 *              so that its slice of x stays in that XCD's L2, and adds each
 *              row's band sums in band order: within the SpMV bound of the
 *              plain order, and the same bits for every partition count.  It
 *              is the default when x has at least 2^20 elements, except
 *              inside batches, which capture the plain form (an explicit
 *              order 4 there returns JACC_ERR_UNSUPPORTED).
 *   vec        1 or 2 consecutive FP64 elements per lane (2 needs an even row
 *              length)
 *   persistent 1 = run the loop inside the batched persistent kernel
 *   order      workgroup-to-tile order: 1 = row-major, 2 = XCD-aware (the
 *              chip hands consecutive workgroup ids to its 8 XCDs in turn; with
 *              this order each XCD walks one contiguous band of tiles, so the
 *              rows two neighbouring tiles share meet in that XCD's L2);
 *              HEAT3D also 3 = XCD-aware with y-blocks of 8 tile rows walked
 *              through all z tiles (compact bricks per XCD)
 *   march      stencil march direction: 1 = every tile toward higher rows
 *              (planes), 2 = odd tiles toward lower ones, so that the
 *              boundary rows two neighbouring tiles share are read by both at
 *              the same time (a cache hit for the second)
 *   rows       HEAT3D: consecutive rows (dim 1) each wave holds, 1, 2, 4 or 8;
 *              the y neighbours of inner rows then come from registers.  A
 *              workgroup covers bx*vec columns and by*rows rows, and with
 *              rows > 1 has at most 256 threads.  Persistent execution takes
 *              rows = 1; JACOBI2D takes rows = 1.
 * Fields equal to 0 take the default. */
typedef struct {
    int32_t bx, by, tile, vec, persistent, order, march, rows;
} jacc_config;

/* Loop kinds (hand-written HIP loop bodies) and their arguments, in order:
 *   JACOBI2D  u_in R [-1,+1]; u_out W [0,0] (or W|FILTERED with u_in entered
 *             whole: every partition sweeps the whole box and keeps its
 *             owner rows).  2-D bounds (normally [1,N-1)^2).
 *             u_out[i][j] = 0.25*((u_in[i-1][j]+u_in[i+1][j]) + (u_in[i][j-1]+u_in[i][j+1]))
 *   HEAT3D    u_in R [-1,+1]; u_out W [0,0].  3-D bounds; scalars[0] = alpha.
 *             lap = (((x-1 + x+1) + (y-1 + y+1)) + (z-1 + z+1)) - 6*u;  u' = u + alpha*lap
 *             optional reduction: sum over the box of (u'-u)^2 (stored values)
 *   SUM       x R [0,0].  1-D bounds over dim 0 rows; whole rows are summed.
 *             reduction: sum of x (scalars[0] != 0: sum of x^2)
 *   GEMM      A R [0,0] (M x L); B R WHOLE (L x N); C W [0,0] (M x N).
 *             2-D bounds [0,M) x [0,N).  C = A*B (FP64 matrix cores)
 *   SPMV_CSR  row_ptr (int32, n+1) R [0,+1]; col (int32) R WHOLE; val (f64)
 *             R WHOLE; x R WHOLE; y W [0,0].  1-D bounds [0,n).
 *             y[i] = sum_{k=row_ptr[i]}^{row_ptr[i+1]-1} val[k]*x[col[k]]
 *   SCATTER_SQ in (f64) R WHOLE; idx (int32) R WHOLE; out (f64) W|FILTERED.
 *             1-D bounds over i.  out[idx[i]] = in[i]*in[i] (the map of the
 *             paper's OpenACC example with an indirect write); indices must be
 *             distinct; an index outside [0, rows of out) is skipped.
 *   PRED_CHAIN a (f64) W|FILTERED; b (f64) W|FILTERED; c (f64) R WHOLE; idx
 *             (int32, T x 3) R WHOLE; xs (f64, T) R WHOLE.  a and b are entered
 *             whole (replicated).  1-D bounds over t in [0, T).  The statement
 *             chain of the paper's filtering example (Sec. "Predicate-Based
 *             Filtering", Fig. conv-code): with (i, j, k) = idx[t], x = xs[t]:
 *               a[i] = x;  b[i] = a[i];  x = c[j];  a[k] = x;  b[k] = a[k];
 *             Every partition runs every iteration on its own replicas of a
 *             and b under the example's guards: a's writes and the read of c
 *             are kept where the index lies in a's or b's owner block of the
 *             partition, b's writes where it lies in b's.  Iterations must not
 *             write an element another iteration touches; an iteration with i
 *             or k outside [0, min(rows of a, rows of b)) or j outside
 *             [0, rows of c) is skipped.
 *
 * FILTERED writes into an array entered whole: partition p's owner block of
 * that array is B_p (the equal division of dim 0); after the loop B_p of
 * partition p's replica holds the array's rows and the other replicas' copies
 * of B_p are stale (they are pulled when read, or broadcast at once under
 * JACC_INIT_EAGER).  Writes a partition makes outside its owner block stay
 * private to its replica.
 *
 * Aliasing (Sec. "Predicate-Based Filtering"): when one array is passed in
 * two argument positions and one of them writes, the partition ranges cannot
 * be trusted; if every argument's array is entered whole the loop runs
 * duplicated — every partition computes the whole iteration space on its own
 * replicas without filtering, and no rows move afterwards (every replica then
 * holds the result) — otherwise the call returns JACC_ERR_RANGE. */
enum {
    JACC_LOOP_JACOBI2D = 1,
    JACC_LOOP_HEAT3D = 2,
    JACC_LOOP_SUM = 3,
    JACC_LOOP_GEMM = 4,
    JACC_LOOP_SPMV_CSR = 5,
    JACC_LOOP_SCATTER_SQ = 6,
    JACC_LOOP_PRED_CHAIN = 7
};

/* jacc_init flags */
enum {
    JACC_INIT_DRYRUN = 1u << 0, /* plan and trace only: no HIP call, fake device addresses */
    JACC_INIT_TRACE = 1u << 1,  /* record every planned operation (see jacc_trace_get) */
    JACC_INIT_SERIALIZE = 1u << 2, /* one stream for every partition, device sync after each op */
    JACC_INIT_LAZY = 1u << 3,      /* halo rows are pulled before each read (default: a stencil
                                      partition also writes the output rows other slabs hold) */
    JACC_INIT_SPLIT = 1u << 4,     /* stencil loops without a reduction: each partition first runs
                                      the rows that read only its own block, then its edge rows
                                      (which wait for the neighbours), so no partition's bulk
                                      waits on another stream; default for 2 to 4 partitions,
                                      this flag asks for it at any partition count */
    JACC_INIT_NO_SPLIT = 1u << 5,  /* never split (one launch per partition) */
    JACC_INIT_EAGER = 1u << 6,     /* the paper's coherence: after every loop each partition
                                      sends the rows it wrote to every other slab holding them
                                      (device copies on its stream); no mirror stores, no pulls */
    JACC_INIT_FORK_CAPTURE = 1u << 7, /* with JACC_INIT_DRYRUN only: plan batches with every
                                      partition on its own stream, forked from and joined
                                      into stream 0 around the capture (otherwise
                                      JACC_ERR_UNSUPPORTED: graphs are captured on one stream) */
    JACC_INIT_POISON = 1u << 8,    /* debug: after each loop launched outside a persistent
                                      group, the rows of FP64/FP32 slabs the loop left stale
                                      (another partition wrote them and this slab was not
                                      refreshed) are filled with 0xFF bytes (NaN) by a fill
                                      kernel ordered like a write, so a read the runtime should
                                      have preceded by a pull carries NaN into the results */
    JACC_INIT_MARKERS = 1u << 9,   /* roctx ranges around the host phases of each call (loop
                                      planning, copies and launches, combines; data enter, exit,
                                      update; batch capture and launch), for rocprofv3
                                      --marker-trace */
    JACC_INIT_NO_PACK = 1u << 10   /* a launch per partition on its own stream for every loop.
                                      Default: outside batches, a JACOBI2D, HEAT3D, SUM or
                                      column-banded SPMV_CSR loop of 2 to 16 row-split partitions
                                      (JACOBI2D also over arrays split along dim 1)
                                      without a FILTERED output runs all its partitions in one
                                      launch on one stream, each partition's tiles a run of the
                                      workgroups, in the loop's configuration (halo pulls before
                                      it, mirror stores inside it; reductions finalised per
                                      partition by one launch and combined in partition order,
                                      banded products combined by one launch: the same bits as a
                                      launch per partition); JACC_INIT_SPLIT, SERIALIZE,
                                      per-partition timing, and reductions whose workgroup
                                      partials of all partitions exceed the stream's buffer keep
                                      a launch per partition */
};

/* Create a context with K partitions (1 <= K <= 64; K = 0 takes the
 * environment's JACC_K).  streams: K hipStream_t handles owned by the
 * caller, or NULL to let the library create K non-blocking streams of
 * default priority.  alloc: NULL selects hipMalloc.  On success *out
 * receives the context.
 *
 * Environment (read here; flags the caller passes win):
 *   JACC_K=<1..64>            K when the K argument is 0
 *   JACC_SERIALIZE=1, JACC_TRACE=1, JACC_DEBUG_POISON=1, JACC_ROCTX=1
 *                             add JACC_INIT_SERIALIZE / _TRACE / _POISON / _MARKERS
 *   JACC_COHERENCE=lazy|eager add JACC_INIT_LAZY / _EAGER unless the caller chose one
 *   JACC_TUNE=model|off|exhaustive
 *                             what a stencil loop called with cfg = NULL outside a batch
 *                             runs: the attached model's pick (model, the default), the
 *                             library defaults (off), or jacc_tune's best non-persistent
 *                             candidate at the arrays' K, tuned once per loop signature
 *                             and kept for the context (exhaustive)
 *   JACC_TUNE_DB=<path>       timing database of the exhaustive mode
 *   JACC_MODEL_PATH=<path>    a cost-model file loaded and attached at init; a file that
 *                             does not load leaves the context without a model (the
 *                             reason in jacc_last_error) and init still succeeds
 * A malformed JACC_K, JACC_COHERENCE or JACC_TUNE value: JACC_ERR_INVALID. */
int jacc_init(jacc_ctx **out, int K, void *const *streams, const jacc_allocator *alloc,
              unsigned flags);

/* Synchronise, free every slab still present, destroy library-created
 * streams and events, and free the context.  Returns the context's sticky
 * status (JACC_OK if no device error occurred). */
int jacc_finalize(jacc_ctx *ctx);

/* Declare the array whose host copy starts at `host` (data directive entry).
 * A repeated enter of the same range with an equal descriptor increments
 * its reference count.  clause JACC_COPYIN / JACC_COPY copies every slab's
 * rows from the host; JACC_CREATE leaves device contents undefined. */
int jacc_data_enter(jacc_ctx *ctx, void *host, const jacc_array_desc *desc, int clause);

/* Leave the data region of the array containing `host`.  JACC_COPYOUT
 * gathers every row from the partition that wrote it last into the host
 * array (synchronously); JACC_DELETE discards device data.  Slabs are freed
 * when the reference count reaches zero. */
int jacc_data_exit(jacc_ctx *ctx, void *host, int clause);

/* Copy rows [row_lo, row_hi) of the array containing `host` between host and
 * device.  JACC_UPDATE_HOST gathers from the latest writers and returns
 * after the host copy is complete.  JACC_UPDATE_DEVICE scatters to every
 * slab holding the rows.  row_hi < 0 means the last row. */
int jacc_update(jacc_ctx *ctx, void *host, int dir, int64_t row_lo, int64_t row_hi);

/* Launch one loop nest over its K partitions.  kind: JACC_LOOP_*; args: the
 * kind's arguments in its documented order; scalars: kind-specific doubles;
 * reduce_slot >= 0 stores the loop's reduction in device slot reduce_slot
 * (0 <= slot < 4096; read later with jacc_reduction_get); reduce_host !=
 * NULL additionally waits and writes the value there (the paper's
 * obligatory synchronisation after an explicit reduction).  cfg: NULL takes
 * the tuned or default configuration.
 * Errors: JACC_ERR_NOT_PRESENT (an argument is not declared), JACC_ERR_RANGE
 * (a partition would touch rows outside its slab, or two partitions would
 * write the same rows — the paper's aliasing case), JACC_ERR_UNSUPPORTED
 * (arguments partitioned with different K, or an interior pointer),
 * JACC_ERR_INVALID (bad kind, bounds, argument count or config). */
int jacc_parallel_loop(jacc_ctx *ctx, int kind, const jacc_bounds *bounds, int nargs,
                       const jacc_arg *args, const double *scalars, int nscalars,
                       int reduce_slot, double *reduce_host, const jacc_config *cfg);

/* Block until every stream of the context has finished. */
int jacc_wait(jacc_ctx *ctx);

/* Wait for the loop that produced reduction slot `slot` and read it. */
int jacc_reduction_get(jacc_ctx *ctx, int slot, double *out);

/* Read reduction slots [first, first+count) into out after a full wait. */
int jacc_reduction_read(jacc_ctx *ctx, int first, int count, double *out);

/* Text of the last error on this context (library-owned; valid until the
 * next call on ctx).  jacc_last_error(NULL) gives the reason of the last
 * failed jacc_init or jacc_heat3d_noalloc on the calling thread. */
const char *jacc_last_error(const jacc_ctx *ctx);

/* ---- batches: many loop nests in one captured HIP graph ---------------------
 * The paper overlaps independent kernels through asynchronous queues to gain
 * kernel-level parallelism (Sec. "Automated Asynchronous Execution"); here a
 * whole sequence of loop calls is captured once into a hipGraph and replayed.
 *
 * jacc_batch_begin starts stream capture on stream 0: the following
 * jacc_parallel_loop calls are planned as usual (copies, launches) but
 * recorded into a single-stream graph instead of executed.  Loops whose
 * configuration has persistent = 1 are not launched one by one: they gather
 * into one persistent-kernel launch that walks a task table of all their
 * tiles, launched when a later loop touches one of their arrays or the
 * batch ends (loops on other arrays are recorded ahead of it).  No
 * data_enter/exit, update, wait or synchronous reduction is allowed inside.
 *
 * jacc_batch_end closes the capture, instantiates the graph, runs it once
 * (so the calls take effect exactly once) and returns its id.  It also plans
 * the calls a second time from the state the first execution leaves; if that
 * plan issues the same copies, waits and launches, the graph is replay-safe
 * and jacc_batch_launch may replay it `repeats` more times (otherwise it
 * returns JACC_ERR_UNSUPPORTED).  Every launch joins all streams into
 * stream 0 before the graph and forks them after it.  A graph addresses the
 * device slabs of the arrays its loops use: once one of those arrays leaves
 * the data region (jacc_data_exit down to a reference count of zero), the
 * graph is stale and jacc_batch_launch / jacc_batch_time return
 * JACC_ERR_INVALID for it (re-entering the array does not revive it). */
int jacc_batch_begin(jacc_ctx *ctx);
int jacc_batch_end(jacc_ctx *ctx, int *graph_id);
int jacc_batch_launch(jacc_ctx *ctx, int graph_id, int repeats);
/* Number of loop calls, persistent groups, and replay safety of a graph. */
int jacc_batch_info(jacc_ctx *ctx, int graph_id, int *loops, int *persistent_groups, int *replay_safe);
int jacc_batch_destroy(jacc_ctx *ctx, int graph_id);
/* Replays a replay-safe graph `warmup` times untimed, then `reps` times,
 * each timed with HIP events on stream 0; ms[0..reps) receives the times. */
int jacc_batch_time(jacc_ctx *ctx, int graph_id, int warmup, int reps, double *ms);

/* ---- configuration timing (the autotuner's measurement) --------------------
 * Runs one loop call `warmup` times, then `reps` times, each timed with HIP
 * events from a start event on stream 0 (every partition stream waits for
 * it) to an end event after all partition streams have joined stream 0.
 * ms[0..reps) receives the times in milliseconds.  A configuration with
 * persistent = 1 is timed as a one-loop batch.  The paper names auto-tuning
 * as future work (Sec. "Conclusion"); the selection rule built on these
 * samples (median, ties to the lowest candidate) lives with the tuner. */
int jacc_time_loop(jacc_ctx *ctx, int kind, const jacc_bounds *bounds, int nargs, const jacc_arg *args,
                   const double *scalars, int nscalars, const jacc_config *cfg, int warmup, int reps,
                   double *ms);

/* One timed execution of a loop call, split into its parts (the measurement
 * the adaptive rule of Sec. "Adaptive Utilization" takes: the kernel time of
 * a partition and the communication around it).  *step_ms receives the time
 * from a start event on stream 0 (every partition stream waits for it) to
 * the join of all partition streams into stream 0; kernel_ms[p], p <
 * nkernel (at most 64), the time of partition p's kernel alone, from HIP
 * events recorded on its stream right before and right after its launch
 * (after the copies and waits it needed), or 0 when partition p has no
 * iterations.  Stencil loops are not split into interior and edge launches
 * here.  JACC_ERR_UNSUPPORTED for persistent configurations and in dry-run
 * contexts. */
int jacc_time_loop_parts(jacc_ctx *ctx, int kind, const jacc_bounds *bounds, int nargs, const jacc_arg *args,
                         const double *scalars, int nscalars, const jacc_config *cfg, double *step_ms,
                         double *kernel_ms, int nkernel);

/* Device pointer of partition p's slab of the array containing `host`, and
 * the slab's first and one-past-last rows (columns for a part_dim 1 array,
 * whose storage starts at column row_lo & ~1 with the even pitch given at
 * jacc_array_desc).  For callers that run their own kernels on the data
 * (and for tests). */
int jacc_slab_info(jacc_ctx *ctx, void *host, int p, void **dev, int64_t *row_lo,
                   int64_t *row_hi);

/* ---- learned cost model -------------------------------------------------------
 * A small FP32 network that predicts the log run time of a loop nest under a
 * launch configuration from F standardised features (1 <= F <= 16):
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3),
 *   yhat = w4 . h3 + b4, with hidden width 64 and relu'(0) = 0;
 * loss = mean over a batch of (yhat - y)^2; Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) with bias correction.  Forward, backward, gradient reduction and
 * Adam run in the library's HIP kernels on the context's stream 0; host
 * arrays are copied in and out (all calls return after their results are on
 * the host).  The paper has no learned model; it names auto-tuning as
 * future work (Sec. "Conclusion").
 * Parameter vector (floats): W1 [64 x F] row-major | b1 [64] | W2 [64 x 64] |
 * b2 [64] | W3 [64 x 64] | b3 [64] | w4 [64] | b4 [1]. */
typedef struct jacc_model jacc_model;
/* Number of parameters for F features (or JACC_ERR_INVALID). */
int jacc_model_nparams(int nfeat);
/* New model on ctx with all parameters zero, scaler mean 0 / std 1. */
int jacc_model_create(jacc_ctx *ctx, int nfeat, jacc_model **out);
int jacc_model_destroy(jacc_model *m);
/* Parameters in the layout above; setting them also resets Adam's state. */
int jacc_model_set_params(jacc_model *m, const float *params, int nparams);
int jacc_model_get_params(jacc_model *m, float *params, int nparams);
/* Feature standardisation x' = (x - mean) / std applied inside the forward
 * pass (std > 0). */
int jacc_model_set_scaler(jacc_model *m, const float *mean, const float *stdev);
/* yhat[0..n) for the raw feature rows X [n x F]. */
int jacc_model_predict(jacc_model *m, const float *X, int n, float *yhat);
/* Loss and parameter gradient of the batch X [n x F], y [n] (grad: nparams
 * floats, either output may be NULL). */
int jacc_model_gradients(jacc_model *m, const float *X, const float *y, int n, float *grad, float *loss);
/* One Adam step with learning rate lr on the gradient of the last
 * jacc_model_gradients call. */
int jacc_model_adam_step(jacc_model *m, float lr);
/* Minibatch training of one network: `epochs` passes over (X, y) in an
 * order shuffled per epoch from `seed` (splitmix64 + Fisher-Yates),
 * minibatches of `batch` rows, one Adam step each.  epoch_loss[e] (optional)
 * receives the mean minibatch loss of epoch e. */
int jacc_model_fit(jacc_model *m, const float *X, const float *y, int n, int epochs, int batch, float lr,
                   uint64_t seed, float *epoch_loss);

/* ---- autotuner and learned choice of launch configurations ----------------
 * The paper names auto-tuning as future work (Sec. "Conclusion"), and its
 * adaptive rule (Sec. "Adaptive Utilization") already picks, per kernel,
 * between duplicated and distributed execution from profiled times.  Here
 * a stencil loop (JACOBI2D, HEAT3D) gets a launch configuration and a
 * partition count K.  No choice changes a field bit.
 *
 * Candidates.  For each K of a requested set (those not above the array's
 * interior rows), in this order: workgroup shapes (bx, by) in {(64,1),
 * (128,1), (256,1), (512,1), (64,4), (128,2), (256,2), (256,4)}, for HEAT3D
 * rows per wave in {1, 4} (4 only with at most 256 threads), tiles in {1, 4,
 * 16, 64}, vec in {1, 2} (2 only for an even row length); then persistent
 * execution with 256 threads, tiles {1, 4, 16}, vec {1, 2}.  order and march
 * stay 0 (the defaults).  A candidate's index in this order breaks ties.
 *
 * Features (the cost model's input, JACC_NFEATURES floats): 1 for 3-D,
 * log2 of each extent (1 for a missing third), log2 of the interior cells,
 * log2 bx, log2 by, log2 tile, vec, log2 K, persistent, log2 of the
 * workgroups one launch over the interior uses, log2 rows.
 *
 * Timing database: a text file of median-ready sample lists keyed by the
 * loop signature (kind, extents) and the candidate, in sections keyed by
 * "<gpu arch>|hip<runtime version>|<library build id>", so timings of
 * another device, runtime or build are kept in the file but never used.
 * A malformed file is an error (JACC_ERR_INVALID), never overwritten. */
typedef struct {
    jacc_config cfg;
    int32_t K;
    int32_t pad_;
} jacc_candidate;

enum { JACC_NFEATURES = 13, JACC_MAX_CANDIDATES = 1024 };

/* Candidates of a stencil loop over an array of extents extent[0..ndim)
 * (ndim 2 for JACOBI2D, 3 for HEAT3D) for the partition counts ks[0..nks)
 * (1..64 each).  Writes at most cap of them to out (out may be NULL) and
 * their number to *n. */
int jacc_candidates(int kind, const int64_t *extent, int ndim, const int *ks, int nks, jacc_candidate *out, int cap,
                    int *n);
/* The JACC_NFEATURES features of one candidate. */
int jacc_features(int kind, const int64_t *extent, int ndim, const jacc_candidate *c, float *out);
/* Build key of the timing database and of cost-model files on this context
 * ("dry|hip0|<build>" for a dry-run context); library-owned string. */
const char *jacc_build_key(jacc_ctx *ctx);

typedef struct {
    int32_t warmup;      /* untimed replays per candidate (0: 1) */
    int32_t reps;        /* timed replays per candidate (0: 5) */
    int32_t nks;         /* partition counts to search (0: the arrays' own K) */
    int32_t ks[8];
    const char *db_path; /* timing database read first and written back, or NULL */
} jacc_tune_opts;

/* Exhaustive autotuner of one stencil loop call (kind, bounds, 2 arguments
 * and scalars as for jacc_parallel_loop; the arguments must be present and
 * give the shapes and halos).  Every candidate runs on scratch replicas of
 * the two arrays entered with the candidate's K (the caller's arrays are
 * never written), as a captured graph of S sweeps alternating between the
 * two replicas, replayed `warmup` times untimed and `reps` times timed with
 * HIP events; each replay's time divided by S is a sample (S even, at most
 * 8, chosen from a one-sweep graph of the first candidate so that a replay
 * lasts about 0.1 ms: small loops are then timed by their work more than by
 * the graph launch).  Candidates already in the database are not run again.  The choice is the smallest median, ties to
 * the lowest candidate index.  *best receives it; medians (optional, `cap`
 * doubles) each candidate's median in ms and *ncand their number.
 * JACC_ERR_UNSUPPORTED for other loop kinds and in dry-run contexts. */
int jacc_tune(jacc_ctx *ctx, int kind, const jacc_bounds *bounds, int nargs, const jacc_arg *args,
              const double *scalars, int nscalars, const jacc_tune_opts *opts, jacc_candidate *best,
              double *medians, int cap, int *ncand);
/* Median of n samples (the mean of the two middle ones for even n) and the
 * index of the smallest of n values, ties to the lowest index: the
 * selection rule jacc_tune applies. */
double jacc_median(const double *samples, int n);
int jacc_argmin(const double *values, int n);

typedef struct {
    int32_t members;   /* networks whose predictions are averaged (0: 3) */
    int32_t epochs;    /* 0: 600 */
    int32_t batch;     /* 0: 256 */
    float lr;          /* 0: 1e-3 */
    uint64_t seed;     /* initial weights (He-uniform from splitmix64) and sample orders */
    int32_t holdout;   /* > 0: every holdout-th loop signature of the database is kept out of
                          training and its mean squared error reported */
    int32_t pad_;
} jacc_train_opts;

typedef struct {
    int32_t rows, signatures;  /* database rows used for training, and their loop signatures */
    float loss_first, loss_last;  /* mean training loss of the first and last epoch (member 0) */
    float heldout_mse;         /* on the held-out signatures (0 without) */
    int32_t pad_;
} jacc_train_report;

/* Trains the cost model on the GPU from every row of the timing database
 * under this context's build key (features -> log of the median ms),
 * standardising the features by their training mean and standard deviation,
 * and writes it to out_path: magic, build key, feature count, members,
 * scaler, parameters, checksum.  opts/report may be NULL. */
int jacc_model_train(jacc_ctx *ctx, const char *db_path, const char *out_path, const jacc_train_opts *opts,
                     jacc_train_report *report);
/* Loads a cost-model file and attaches it to the context (replacing any
 * attached one).  JACC_ERR_INVALID for a missing, truncated or corrupt file
 * (checksum) or one written under another build key; the context then keeps
 * no model.  While a model is attached, jacc_parallel_loop with cfg = NULL
 * on a stencil loop outside a batch uses the model's pick among the
 * non-persistent candidates at its arrays' K (cached per loop signature;
 * inside a batch only an already cached pick is used, else the defaults). */
int jacc_model_load(jacc_ctx *ctx, const char *path);
int jacc_model_unload(jacc_ctx *ctx);
/* The attached model's choice among the candidates for ks[0..nks): the
 * smallest predicted log time (mean over members; ties to the lowest index),
 * batched inference on the GPU.  pred (optional, cap floats) receives every
 * candidate's prediction and *ncand their number.  JACC_ERR_INVALID without
 * an attached model. */
int jacc_model_pick(jacc_ctx *ctx, int kind, const int64_t *extent, int ndim, const int *ks, int nks,
                    jacc_candidate *best, float *pred, int cap, int *ncand);

/* The configuration for a stencil loop call by the fallback chain
 * model -> tuner -> default: the pick of the model in model_path (loaded
 * and attached when it is not the attached one) if it loads; else, when
 * opts != NULL, jacc_tune's choice; else the library defaults (all config
 * fields 0) at the arrays' K.  *source receives 1, 2 or 3 for the three;
 * the reason a step was skipped is left in jacc_last_error. */
enum { JACC_CHOICE_MODEL = 1, JACC_CHOICE_TUNER = 2, JACC_CHOICE_DEFAULT = 3 };
int jacc_choose(jacc_ctx *ctx, int kind, const jacc_bounds *bounds, int nargs, const jacc_arg *args,
                const double *scalars, int nscalars, const char *model_path, const jacc_tune_opts *opts,
                jacc_candidate *out, int *source);

/* ---- operation trace (planning and tests) ------------------------------ */
enum {
    JACC_OP_ALLOC = 1,   /* array a, partition dst, rows [lo,hi) */
    JACC_OP_FREE = 2,
    JACC_OP_H2D = 3,     /* host rows [lo,hi) -> slab dst, on stream */
    JACC_OP_D2H = 4,     /* slab src rows [lo,hi) -> host, on stream */
    JACC_OP_COPY = 5,    /* slab src rows [lo,hi) -> slab dst, on stream (== dst) */
    JACC_OP_KERNEL = 6,  /* loop kind `kind`, partition dst, iterations [lo,hi) of dim 0 */
    JACC_OP_RECORD = 7,  /* event recorded on stream, covering its ops up to seq */
    JACC_OP_WAIT = 8,    /* stream waits for stream src up to seq */
    JACC_OP_SYNC = 9,    /* host waits for stream */
    JACC_OP_COMBINE = 10, /* reduction combine on stream into slot `kind` */
    JACC_OP_ACCESS = 11,  /* the op `seq` on stream touches slab dst of array rows
                             [lo,hi): kind 1 = read, 2 = write, 3 = write of values
                             private to that slab (a filtered loop's writes outside
                             the partition's owner block), 4 = write of the values
                             the same loop writes in the first partition's slab (a
                             duplicated loop), 5 = write of invalid values (POISON) */
    JACC_OP_JOIN = 12,    /* all streams joined: every later op is ordered after every
                             earlier op (around graph launches and timed runs) */
    JACC_OP_POISON = 13   /* stale rows [lo,hi) of slab dst of array filled with NaN bytes
                             on stream (JACC_INIT_POISON) */
};

typedef struct {
    int32_t op;
    int32_t stream;
    int32_t array;   /* array id (order of first enter), or -1 */
    int32_t src;     /* source partition / stream, or -1 */
    int32_t dst;     /* destination partition, or -1 */
    int32_t kind;    /* loop kind (KERNEL), slot (COMBINE) */
    int64_t lo, hi;  /* rows or iterations */
    int64_t seq;     /* per-stream sequence number of this op (WAIT: awaited seq) */
} jacc_trace_op;

/* Number of recorded trace entries; entry i; clear. */
int jacc_trace_len(const jacc_ctx *ctx);
int jacc_trace_get(const jacc_ctx *ctx, int i, jacc_trace_op *out);
int jacc_trace_clear(jacc_ctx *ctx);

/* Library version string (static). */
const char *jacc_version(void);

/* ---- adaptive duplicate-vs-partition choice (Sec. "Adaptive Utilization",
 * Eq. 1-3) ------------------------------------------------------------------
 * A per-loop policy record, host memory only, independent of any context.
 * It starts in JACC_ADAPT_DUPLICATE (the whole loop on one device, no
 * exchange).  jacc_adapt_observe feeds one execution of the loop in the
 * current mode: time_kernel_s (seconds of the loop body: in duplicate mode
 * the whole loop, in partitioned mode the kernel of one partition — the
 * longest one when they differ), time_comm_s (seconds of the rest of a
 * partitioned execution: exchange and synchronisation; 0 in duplicate mode)
 * and write_bytes (bytes the loop writes, > 0), and returns the mode for the
 * next execution.
 *   duplicate: the first observation is a warm-up and ignored; later ones
 *     add time/WriteSize to eff_dup (mean seconds per byte) and count Eq. 1,
 *     t_k > t_k/n + WriteSize/peak; at five the mode becomes PARTITION.
 *   partition: Eq. 2, t_k + t_c > n*t_k, and Eq. 3, t_k + t_c > eff_dup *
 *     WriteSize, are counted; when either has held five times and the mean,
 *     over every partitioned execution since the switch, of (t_k + t_c)
 *     minus the smaller right side is above zero, the mode becomes
 *     DUPLICATE_FINAL and stays there.  (Executions faster than both bounds
 *     lower that mean, so violations alone do not switch a loop off.)
 * n_parts >= 1 is the partition (device) count, peak_bytes_per_s > 0 the
 * bandwidth of one link between partitions.  Returns JACC_ERR_INVALID on bad
 * arguments, JACC_ERR_ALLOC if the record cannot be allocated.  The record
 * is not thread-safe. */
typedef struct jacc_adapt jacc_adapt;
enum { JACC_ADAPT_DUPLICATE = 0, JACC_ADAPT_PARTITION = 1, JACC_ADAPT_DUPLICATE_FINAL = 2 };
int jacc_adapt_create(jacc_adapt **out, int n_parts, double peak_bytes_per_s);
int jacc_adapt_destroy(jacc_adapt *a);
int jacc_adapt_observe(jacc_adapt *a, double time_kernel_s, double time_comm_s, double write_bytes, int *mode);
/* Current mode, eff_dup (0 before any profiled duplicate run) and counts[5]
 * = {profiled duplicate runs, Eq. 1 hits, Eq. 2 hits, Eq. 3 hits, violating
 * partitioned runs}; any output pointer may be NULL. */
int jacc_adapt_state(const jacc_adapt *a, int *mode, double *eff_dup, long long *counts);
/* Mean of (t_k + t_c) - min(n*t_k, eff_dup*WriteSize) over the partitioned
 * executions observed so far (0 before any), and their number. */
int jacc_adapt_mean_diff(const jacc_adapt *a, double *mean_diff, long long *n_partitioned);

/* ---- parallel dimension of an updated array (Sec. "Division of
 * Multidimensional Arrays") ----------------------------------------------------
 * For an array of ndim (1..16) dimensions, parallel_iters[d] and
 * sequential_iters[d] count the parallel and sequential loop iterators that
 * appear in its index expression of dimension d (>= 0).  *dim receives the
 * dimension with the most parallel iterators, then the fewest sequential
 * ones, ties going to the leftmost dimension (column_major == 0, C order) or
 * the rightmost (column_major != 0, Fortran order); -1 when no dimension has
 * a parallel iterator (the loop would have to be duplicated).  Host-only
 * planning helper: the runtime partitions dimension 0.  Returns
 * JACC_ERR_INVALID on bad arguments. */
int jacc_parallel_dim(int ndim, const int *parallel_iters, const int *sequential_iters, int column_major, int *dim);

/* ---- allocation-free heat step ----------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One heat
 * step with its residual on caller-owned device buffers, computing exactly
 * what a one-partition JACC_LOOP_HEAT3D loop with a reduction computes (same
 * loop body, launch shape and addition order, so the field and the residual
 * are bit-identical to that loop's), without a context and without any
 * allocation: the residual's workgroup partials go to a fixed array of
 * JACC_NOALLOC_MAX_PARTIALS doubles (512 KiB) that the library holds on every
 * device it runs on until the process ends.
 *   u_in, u_out  device pointers to nz x ny x nx FP64 fields, row-major with z
 *                outermost; must not overlap.  u_out's interior
 *                [1,nz-1) x [1,ny-1) x [1,nx-1) receives
 *                u + alpha*((((x-1 + x+1) + (y-1 + y+1)) + (z-1 + z+1)) - 6u);
 *                its boundary faces are not written.
 *   residual     device pointer to one double receiving the sum over the
 *                interior of (u_out - u_in)^2 of the stored values, or NULL
 *                (then no reduction and no size limit).
 *   stream       hipStream_t to enqueue on (NULL: the null stream); the call
 *                returns after enqueueing.
 * The current device is the one that runs the step; on the first call on a
 * device the library looks up that device's copy of the partials array.
 * Every call on one device shares that copy (each call overwrites the
 * partials it reads, so nothing carries over between calls), so calls with a
 * residual that may overlap in time on one device race: order them on one
 * stream or by events.  Errors (nothing is launched): JACC_ERR_INVALID for NULL or
 * overlapping fields or non-positive extents; JACC_ERR_RANGE when the
 * default launch for these extents needs more than JACC_NOALLOC_MAX_PARTIALS
 * workgroups (cubes above 1026^3) and residual != NULL; JACC_ERR_DEVICE for a
 * failed HIP call.  jacc_last_error(NULL) gives the reason. */
#define JACC_NOALLOC_MAX_PARTIALS 65536
int jacc_heat3d_noalloc(const double *u_in, double *u_out, int64_t nz, int64_t ny, int64_t nx, double alpha,
                        double *residual, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* JACC_H */
