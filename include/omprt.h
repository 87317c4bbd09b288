/*
 * omprt.h -- C ABI of an MI355X (gfx950) implementation of the data-parallel
 * core of an OpenMP device runtime: what a
 *     #pragma omp target teams distribute parallel for reduction(op:x)
 * region lowers to.  The paper this follows (Tian, Chesterfield, Doerfert,
 * Chapman, "Experience Report: Writing A Portable GPU Runtime with OpenMP
 * 5.1") describes the device runtime as the library that supplies OpenMP
 * semantics on the GPU, including the routines the compiler calls for
 * worksharing loops (sec. 1, sec. 2.1); it maps one OpenMP team to one GPU
 * thread block (sec. 3.1, "Global Shared Variables"); team-shared variables
 * live in on-chip shared memory and are uninitialised until written
 * (sec. 3.1); cross-thread communication uses device atomics, in particular
 * a wrap-around increment, and a flush that is a device fence (sec. 3.1
 * "Atomic Operations", Listing of the flush entry, sec. 3.2).
 *
 * Conventions for every entry point:
 *  - Pointers prefixed d_ are device pointers (hipMalloc / torch CUDA
 *    tensors); h_ are host pointers.  The caller owns all of them; the
 *    library never frees or retains a caller buffer beyond the call, except
 *    that buffers named by a cached batched plan must stay valid until the
 *    next omprt_reduce_batched call with a different plan, or
 *    omprt_finalize.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Device work
 *    is enqueued asynchronously and stream-ordered; no entry point
 *    synchronises the device unless it says so.  Results are visible after
 *    the stream is synchronised.
 *  - Every function returns an omprt_status and never aborts; after a
 *    non-OK status omprt_last_error() holds a message (per host thread).
 *    Device faults surface at the caller's next synchronisation.
 *  - Calls on one stream are serialised by the stream.  Different streams
 *    get different workspaces, so concurrent calls on different streams do
 *    not interfere.  Two host threads must not share one stream.
 *  - The library's own device memory (per-stream workspaces, pools, scratch,
 *    batched plans) is never freed while in use: when a call needs a larger
 *    buffer than the stream has, the old one is kept, unused, until
 *    omprt_finalize, so a HIP graph a caller captured around earlier calls
 *    stays valid however later eager calls grow the buffers.  omprt_finalize
 *    frees everything; graphs captured before it must not be replayed after
 *    it.  No memory is released from static destructors at process exit:
 *    call omprt_finalize before exiting to release it explicitly.
 */
#ifndef OMPRT_H
#define OMPRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OMPRT_OK = 0,
    OMPRT_ERR_INVALID = 1,      /* bad argument (null pointer, range, ...) */
    OMPRT_ERR_UNSUPPORTED = 2,  /* valid but not implemented (dtype/op combo) */
    OMPRT_ERR_NOMEM = 3,        /* workspace allocation failed or over limit */
    OMPRT_ERR_DEVICE = 4        /* HIP runtime error on launch/copy/capture */
} omprt_status;

typedef enum {
    OMPRT_I32 = 0, OMPRT_I64 = 1, OMPRT_F32 = 2, OMPRT_F64 = 3, OMPRT_BF16 = 4
} omprt_dtype;

/*
 * The reduction identifiers of the OpenMP reduction clause.  SUM, MAX, MIN,
 * PROD, LAND and LOR apply to every dtype; BAND, BOR and BXOR to integers
 * only (UNSUPPORTED otherwise).  Integer SUM and PROD wrap modulo 2^w;
 * LAND / LOR treat an operand as true when it is not zero (a floating NaN
 * is true) and give 0 or 1 in x's type (bf16: the bits of 1.0 or 0.0).
 * fp32 / fp64 / bf16 PROD is compensated (each factor's rounding error is
 * recovered with a fused multiply-add and carried in a second word); bf16
 * PROD, like bf16 SUM, returns the fp32 accumulator.  The batched entry
 * points take SUM, MAX and MIN only.
 */
typedef enum {
    OMPRT_SUM = 0, OMPRT_MAX = 1, OMPRT_MIN = 2, OMPRT_PROD = 3, OMPRT_BAND = 4,
    OMPRT_BOR = 5, OMPRT_BXOR = 6, OMPRT_LAND = 7, OMPRT_LOR = 8
} omprt_op;

/*
 * A static worksharing schedule:
 *   distribute dist_schedule(static[, dist_chunk]) parallel for
 *   schedule(static[, chunk])
 * over logical iterations 0..n-1 with num_teams teams of
 * threads_per_team threads.  A chunk of 0 means "no chunk size given":
 *   - dist_chunk == 0: team k executes the balanced block
 *     [k*q + min(k, r), ... + q + (k < r)) with q = n / T, r = n % T;
 *   - dist_chunk > 0: blocks [j*dc, min(n, (j+1)*dc)) go to team j mod T;
 *   - chunk == 0: inside each team block [a, b) (m = b - a) thread t
 *     executes the balanced share a + bal(m, P, t) (first m % P threads one
 *     extra iteration);
 *   - chunk > 0: chunks [a + j*c, a + min(m, (j+1)*c)) go to thread j mod P,
 *     dealt again from thread 0 in every team block.
 * Surplus teams/threads (T > n, P > m) execute nothing.
 */
typedef struct {
    int64_t n;                  /* trip count, >= 0 */
    int32_t num_teams;          /* >= 1 (0 = runtime picks, where allowed) */
    int32_t threads_per_team;   /* 1..1024 (0 = runtime picks, where allowed) */
    int64_t dist_chunk;         /* >= 0 */
    int64_t chunk;              /* >= 0 */
} omprt_sched;

/*
 * Launch configuration for reductions.  Zero fields mean "runtime picks":
 * the learned model if one is loaded (and confident), else the tuned cache,
 * else a built-in heuristic.
 */
typedef struct {
    int32_t num_teams;          /* 0, or 1..65535 */
    int32_t threads_per_team;   /* 0, or 64..1024 in steps of 64 */
    int32_t vec_bytes;          /* 0, 8 or 16: bytes per lane per load */
    int32_t unroll;             /* 0, 1, 2, 4 or 8 loads in flight per lane */
    int32_t tile_kib;           /* batched only: tile size in KiB (0, or 4..65536) */
    uint32_t flags;             /* OMPRT_CFG_* */
} omprt_config;

#define OMPRT_CFG_NO_MODEL 0x1u      /* ignore the learned model for this call */
#define OMPRT_CFG_STATIC_TILES 0x2u  /* batched: deal tiles round-robin instead of
                                        by atomic ticket */
#define OMPRT_CFG_HIST_TEAM_COPY 0x4u  /* histogram: past the LDS bin ranges, team
                                          copies in the global pool instead of
                                          atomics on hist */
#define OMPRT_CFG_HIST_DIRECT 0x8u     /* histogram: atomics on hist for any bin
                                          count (no team copy) */
#define OMPRT_CFG_HIST_PARTITION 0x20u  /* histogram: partition the keys by bin
                                          range first, then count each range in
                                          LDS (up to 8 388 608 bins) */
#define OMPRT_CFG_HIST_RANGES 0x40u     /* histogram: count the bin ranges one by
                                          one, each reading every key (up to
                                          32 ranges; beyond, atomics on hist) */
#define OMPRT_CFG_HIST_TILE_SORT 0x80u  /* histogram: sort each tile of keys by
                                          bin range into a slot of its own,
                                          then count each range's runs in LDS
                                          (up to 4 194 304 bins) */
#define OMPRT_CFG_EXACT_THREAD_MAP 0x10u /* omprt_reduce (sum / max / min): every
                                            thread reduces exactly its
                                            schedule(static) run of the team's
                                            block, instead of the team's lanes
                                            reading interleaved vectors (for
                                            comparison) */

/* One independent reduction of a batch.  x follows omprt_reduce. */
typedef struct {
    const void *d_in;
    int64_t n;
    int32_t dtype;              /* omprt_dtype */
    int32_t op;                 /* omprt_op */
    void *d_x;
} omprt_segment;

/* ----------------------------------------------------------------------- */
/* Static worksharing (host)                                               */
/* ----------------------------------------------------------------------- */

/*
 * The j-th (0-based) non-empty chunk that thread `thread` of team `team`
 * executes under schedule *s, as the half-open range [*lb, *ub) of logical
 * iterations, in execution order.  When j is at or past the thread's last
 * chunk, *lb == *ub == s->n.  *is_last is 1 when the chunk holds iteration
 * n-1 (the sequentially last iteration), else 0.  Pure host integer
 * arithmetic, O(1).  A thread's chunks do not in general form one
 * arithmetic progression (dist_chunk > 0 and chunk > 0), hence the index.
 * Defining passage: the device runtime supplies the routines the compiler
 * calls for worksharing loops (sec. 1), a lowered parallel for calling into
 * it to divide the loop's iterations (sec. 2, opening); teams are thread
 * blocks (sec. 3.1, "Global Shared Variables").  The chunk rules are the
 * static schedule of the OpenMP specification that the paper implements.
 * Errors: INVALID for NULL pointers, n < 0, num_teams < 1,
 * threads_per_team outside 1..1024, negative chunks, team/thread out of
 * range, j < 0.
 */
omprt_status omprt_for_static_bounds(const omprt_sched *s, int32_t team,
                                     int32_t thread, int64_t j, int64_t *lb,
                                     int64_t *ub, int32_t *is_last);

/* Number of non-empty chunks and of iterations thread `thread` of team
 * `team` executes under *s (the same worksharing routines, sec. 1 and
 * sec. 2).  Same errors as omprt_for_static_bounds. */
omprt_status omprt_sched_count(const omprt_sched *s, int32_t team,
                               int32_t thread, int64_t *n_chunks,
                               int64_t *n_iters);

/* ----------------------------------------------------------------------- */
/* Device work                                                             */
/* ----------------------------------------------------------------------- */

/*
 * Iteration map of schedule *s on the GPU: the thread executing iteration i
 * stores owner[i] = team * threads_per_team + thread and atomically adds 1
 * to count[i].  d_owner and d_count have s->n entries; the caller zeroes
 * d_count first (a correct map leaves every count at 1).  num_teams and
 * threads_per_team must be given (no runtime choice).  Verification
 * kernel for the schedule semantics of the worksharing routines (sec. 1,
 * sec. 2) under the team-to-thread-block mapping (sec. 3.1); the count uses
 * the device atomic add (sec. 3.1, "Atomic Operations").
 */
omprt_status omprt_static_map(const omprt_sched *s, int32_t *d_owner,
                              uint32_t *d_count, void *hip_stream);

/*
 * reduction(op:x) over d_in[0..n):  *d_x <- *d_x (op) fold(op, d_in[0..n)).
 * dtype gives d_in's element type; op any omprt_op defined for it.  *d_x
 * has the input's type, except for bf16 sums and products, whose *d_x is
 * float (the fp32 accumulator).  Integer sums wrap modulo 2^w; max/min
 * compare signed (integers) or follow IEEE maxNum / minNum (floating,
 * NaN-dropping).  fp32 and bf16 sums accumulate in
 * compensated fp32 (TwoSum per element, float-float combination); fp64 sums
 * in compensated fp64 likewise.  n == 0 leaves *d_x unchanged.  The result is deterministic for a
 * fixed (n, configuration).  Teams follow the static distribute schedule
 * (team k reduces the balanced block bal(n, T, k)); inside a team lanes read
 * interleaved vectors, which no reduction body can observe (cfg->flags
 * OMPRT_CFG_EXACT_THREAD_MAP makes every thread reduce exactly its
 * schedule(static) run instead; sum, max and min).  The cross-team
 * combine is done by the last team to finish, found with a wrap-around
 * atomic increment that leaves its counter at 0.
 * Defining passages: the region is a teams distribute parallel for with a
 * reduction clause, whose iterations the runtime divides (sec. 1, sec. 2);
 * one team is one thread block and its tree lives in team-shared memory,
 * which is uninitialised until written (sec. 3.1, "Global Shared
 * Variables", and the shared variables of the listing of the flush entry);
 * the last team is elected with the wrap-around increment inc,
 * { v = x; x = x >= e ? 0 : x + 1 } with e = T - 1 (sec. 3.1, "Atomic
 * Operations"; its AMD builtin in the declare-variant listing of sec. 3.2).
 * The flush of that listing is a device-wide fence; this library makes the
 * partials visible through tagged agent-scope atomic slot words instead, so
 * no team pays for a fence.
 * d_in needs only element alignment.  cfg may be NULL.
 * Errors: UNSUPPORTED for a dtype or op outside the enums or an op the
 * dtype does not define; INVALID for n outside 0..2^50, NULL x, NULL d_in
 * with n > 0, misaligned pointers, or cfg fields out of range; NOMEM when
 * the workspace cannot grow; DEVICE for a failed launch.
 */
omprt_status omprt_reduce(const void *d_in, int64_t n, int32_t dtype,
                          int32_t op, void *d_x, const omprt_config *cfg,
                          void *hip_stream);

/*
 * Histogram: reduction(+: hist[0:bins]) over a loop whose iteration i does
 * hist[d_keys[i]] += 1 -- an array-section reduction whose list item is
 * chosen by the data.  d_hist (bins int32, caller-initialised: its values
 * take part like x_orig) gets the counts added, modulo 2^32.  Keys outside
 * [0, bins) are not counted and set bit 4 of the stream's workspace status.
 * Each team keeps a team-shared copy of the histogram, taken with the
 * runtime's team-shared allocation, counts its balanced block of keys into
 * it with atomic adds and adds the copy into d_hist.  Up to the LDS one
 * workgroup may take (40 704 bins on gfx950's 160 KiB) the copy is in LDS;
 * up to twice that, the bins are cut into two ranges of that size, each
 * team counting the keys of one range (every key is read once per range);
 * past that the keys are first partitioned by bin range (ranges of 32 768
 * bins) into a buffer of the library's pool of 16-bit places within their
 * range, then each range's places are counted in an LDS copy of that range:
 * up to 4 194 304 bins every tile of 8192 keys is sorted by range into a
 * slot of its own (the keys read once); up to 8 388 608 bins the ranges are
 * laid out across teams (counts per range and team, a prefix sum, then the
 * scatter: the keys read twice); beyond, every key is an atomic add on
 * d_hist itself (no copy).  cfg->flags:
 * OMPRT_CFG_HIST_RANGES counts range by range up to 32 ranges;
 * OMPRT_CFG_HIST_TILE_SORT sorts tiles for any bin count up to 4 194 304;
 * OMPRT_CFG_HIST_PARTITION partitions across teams for any bin count up to
 * 8 388 608;
 * OMPRT_CFG_HIST_TEAM_COPY keeps team copies past the ranges, each a slice
 * of a global pool the library keeps per stream (team-shared allocation
 * falling back from LDS; atomics at L2); OMPRT_CFG_HIST_DIRECT takes
 * atomics on d_hist for any bin count; at most one of them.  cfg:
 * num_teams (default two per compute unit), threads_per_team (default
 * 512; the partitioned passes always take 512), unroll 1, 2 or 4 (default
 * 4).  bins 1..2^28.
 */
omprt_status omprt_histogram(const int32_t *d_keys, int64_t n, int32_t bins,
                             int32_t *d_hist, const omprt_config *cfg,
                             void *hip_stream);

/*
 * A target region in generic (non-SPMD) mode: sequential code between
 * parallel loops, run by teams whose main thread (thread 0) executes the
 * sequential code and hands each loop to its team through team-shared
 * memory while the other threads wait at the team barrier for work (the
 * device runtime's parallel-region hand-off, sec. 2.1).  The region is a
 * power iteration on diag(d_diag):
 *   repeat iters times:  w = d .* v;  s = sum w^2;  v = w / sqrt(s)
 *   *d_lambda = sqrt(s)       (the last s: the norm of D v_(iters-1))
 * d_v (n floats, device) holds the start vector and is overwritten with the
 * last normalised vector; d_diag (n floats, device) is read only;
 * *d_lambda (one float, device) is written.  s accumulates in compensated
 * fp32.  A zero vector gives s = 0 and NaN / infinity results, as the
 * arithmetic says.
 * teams: 1 = one team over the whole loop (the mode's own shape); T > 1 =
 * T co-resident teams (a cooperative launch), team k owning the balanced
 * block bal(n, T, k) of both loops and every team running the sequential
 * code on the same s, which reaches all teams by an all-gather of team
 * partials through the stream's workspace (a partial that never arrives
 * sets bit 1 of the workspace status, see omprt_workspace_status); 0 = the
 * runtime's choice: with threads 0, one team of 512 threads up to 8192
 * elements, else one team of 256 threads per 2048 elements; with threads
 * given, one team per 8 * threads elements; at most one per compute unit.  At most 512 teams and no more than fit at once
 * (OMPRT_ERR_INVALID otherwise); OMPRT_ERR_UNSUPPORTED if the device has no
 * cooperative launch.  For fixed (teams, threads) the results are
 * deterministic (the sum's rounding follows its combination order).
 * threads: 64..1024, a multiple of 64; 0 = the runtime's choice (512 for
 * one team, 256 for several).  n 1..2^32, iters >= 1;
 * d_diag and d_v must not overlap, and d_lambda lies in neither.  One
 * kernel launch on hip_stream; invalid arguments return OMPRT_ERR_INVALID
 * before anything is launched.
 */
omprt_status omprt_generic_power(const float *d_diag, float *d_v, int64_t n,
                                 int32_t iters, int32_t teams, int32_t threads,
                                 float *d_lambda, void *hip_stream);

/*
 * User-defined reduction (OpenMP's declare reduction): the reduction type,
 * its initializer, its combiner and the loop body that folds one input
 * element into a private copy are the caller's device code (C++ text), so
 *   #pragma omp declare reduction(id : omp_type : combiner) initializer(init)
 *   #pragma omp target teams distribute parallel for reduction(id : x)
 *   for (i = 0; i < n; i++) body
 * becomes one omprt_udr_declare (compiles a kernel with hiprtc for gfx950,
 * once per distinct source) and omprt_reduce_udr calls.  The runtime
 * specialises its reduction with the application's code, as the paper does
 * by linking the runtime into the application as bitcode (sec. 2.2).
 *   type_def:    defines `omp_type` (trivially copyable; acc_bytes bytes, a
 *                multiple of 4, at most 64), e.g. "struct omp_type { ... };"
 *   initializer: statements that set `omp_priv` (omp_type&) to the identity
 *   combiner:    statements that fold `omp_in` (const omp_type&) into
 *                `omp_out` (omp_type&); applied in an unspecified order, so
 *                it must be associative and commutative up to what the
 *                caller accepts
 *   body:        statements that fold the element `omp_elem` (int32_t,
 *                int64_t, float (also for bf16) or double) at position
 *                `omp_i` (int64_t) into `omp_priv`
 * The code sees the device headers' names (namespace omprt).  A source that
 * does not compile returns OMPRT_ERR_INVALID with the compiler's output in
 * omprt_last_error().  *h_handle receives a handle for omprt_reduce_udr;
 * declaring the same source and dtype again returns the same handle.
 */
typedef struct {
    const char *type_def;
    const char *initializer;
    const char *combiner;
    const char *body;
    int32_t acc_bytes;
} omprt_udr_source;

omprt_status omprt_udr_declare(const omprt_udr_source *src, int32_t dtype,
                               int32_t *h_handle);

/*
 * x <- combiner(x, r), r the reduction of d_in[0..n) (dtype as declared)
 * under the declared reduction: teams take balanced blocks, a lane folds
 * its elements into a private copy with the body in increasing position,
 * copies combine through the team tree and the last team.  d_x points to
 * one omp_type in device memory (4-byte aligned); n == 0 leaves it
 * unchanged.  cfg: num_teams and threads_per_team (others must be 0).  The
 * first call on a device loads the kernel's module there (gfx950 only).
 * Deterministic for fixed (n, configuration).
 */
omprt_status omprt_reduce_udr(int32_t handle, const void *d_in, int64_t n,
                              void *d_x, const omprt_config *cfg,
                              void *hip_stream);

/*
 * Several reduction variables of one region over the same input, e.g.
 *   reduction(+: s) reduction(max: hi) reduction(min: lo)
 * on one loop over d_in[0..n): nvars (1..3) variables with distinct ops
 * h_ops[v] among SUM, MAX, MIN and x pointers h_x[v] (host arrays of
 * device pointers; each x as for omprt_reduce).  One pass over the input
 * updates every variable; each result equals what omprt_reduce gives for
 * that op alone (same arithmetic; sums may differ in the last bits from a
 * separate launch, the accumulation order being the launch's).  cfg as
 * for omprt_reduce, except 16-byte loads, unroll 2 or 4, no learned model.
 * UNSUPPORTED for other ops; INVALID for a repeated op, nvars outside 1..3,
 * NULL or misaligned pointers.
 */
omprt_status omprt_reduce_multi(const void *d_in, int64_t n, int32_t dtype,
                                int32_t nvars, const int32_t *h_ops,
                                void *const *h_x, const omprt_config *cfg,
                                void *hip_stream);

/*
 * maxloc / minloc, the usual user-defined reduction: the largest (op
 * OMPRT_MAX) or smallest (OMPRT_MIN) value of d_in[0..n) together with its
 * position.  The pairs (*d_val, *d_idx), (d_in[0], 0), ..., (d_in[n-1],
 * n-1) are ordered by value, then by the smaller position (so a value that
 * occurs several times reports its first position, and *d_val / *d_idx take
 * part like x_orig); floating NaNs never win, -0 and +0 are equal.  On exit
 * *d_val (the input's type; bf16 bits for bf16) and *d_idx (int64) hold the
 * first pair of that order.  n == 0 leaves both unchanged.  cfg as for
 * omprt_reduce, except that loads are 16 bytes (vec_bytes 0 or 16), the
 * default unroll is 8 and the learned model is not consulted.  UNSUPPORTED for ops other than MAX / MIN.
 */
omprt_status omprt_reduce_loc(const void *d_in, int64_t n, int32_t dtype,
                              int32_t op, void *d_val, int64_t *d_idx,
                              const omprt_config *cfg, void *hip_stream);

/*
 * Array-section reduction, reduction(op: x[0:m]) over a loop of `rows`
 * iterations whose iteration i contributes d_in[i*m + j] to list item x[j]
 * (d_in row-major, rows x m):
 *     d_x[j] <- d_x[j] (op) fold(op, d_in[i*m + j] for i in [0, rows))
 * for every j in [0, m).  Each list item is a reduction variable of its own
 * (OpenMP reduction clause on an array section: a private copy per thread,
 * combined like a scalar), so element types, x's type (m entries, float for
 * bf16 sums), arithmetic and determinism are those of omprt_reduce.
 * rows == 0 or m == 0 leaves d_x unchanged.  d_in and d_x need element
 * alignment; a 16-byte aligned d_in streams in 16-byte vectors when its rows
 * (whole, or cut into column tiles) keep that alignment, otherwise one
 * element per load.  The runtime cuts the block into column tiles and row
 * periods (omprt_reduce_array_plan); teams on one tile combine through
 * tagged slots and wrap-around-increment elections, in one or two levels
 * of groups.
 * cfg (may be NULL): num_teams is the total team count aimed at (default
 * one per compute unit, two with element loads); threads_per_team 64..512 in steps of 64 (default
 * 512); unroll 1, 2, 4 or 8 loads in flight per lane (default 4 with
 * 16-byte loads, which take at most 4; 8 with element loads).  A team
 * gathers its private copies in LDS at the end: threads x unroll x elements
 * per load of them, or threads x elements per load when each load layer
 * holds whole rows of the tile; they must fit 64 KiB.  The default unroll
 * is lowered until they do; with an explicit unroll the call falls back to
 * element loads, and is INVALID if even those do not fit.  vec_bytes 0 or
 * 16 (vectors where possible) or the element size (one element per load).
 * The learned model and tuned cache are not consulted.
 * Errors: UNSUPPORTED for dtype/op out of range; INVALID for rows or m
 * negative, rows*m above 2^50, NULL or misaligned pointers, x overlapping
 * in, bad cfg fields.
 */
omprt_status omprt_reduce_array(const void *d_in, int64_t rows, int64_t m,
                                int32_t dtype, int32_t op, void *d_x,
                                const omprt_config *cfg, void *hip_stream);

/*
 * The launch omprt_reduce_array would make (host only, no device work):
 * h_out8 = {tile width W, rows per period R, column tiles, row teams per
 * tile, election groups per tile, bytes per load, threads, unroll}.
 * aligned16 says whether d_in would be 16-byte aligned.  rows, m >= 1.
 */
omprt_status omprt_reduce_array_plan(int64_t rows, int64_t m, int32_t dtype,
                                     int32_t op, int32_t aligned16,
                                     const omprt_config *cfg, int64_t *h_out8);

/*
 * count independent reductions in ONE persistent kernel launch.  h_segs is
 * a host array; each segment follows omprt_reduce's semantics.  The plan
 * (descriptor and tile tables) and a captured HIP graph of the launch are
 * cached per (stream, segment list, configuration): a repeat call with the
 * same list only replays the graph.  Segments may not alias each other's
 * outputs.  cfg's threads_per_team / unroll / vec_bytes select the tile
 * kernel; num_teams the persistent grid size (0 = one full wave of the
 * device).
 * Defining passages: each segment is one reduction region with omprt_reduce's
 * semantics; the tiles of a segment play its teams: each reduces its part
 * through the team-shared tree and the last tile, elected by the wrap-around
 * inc with e = tiles - 1, combines (sec. 3.1, "Global Shared Variables" and
 * "Atomic Operations").  Running many regions in one persistent launch is
 * this library's extension; the paper has no batched form.
 * Errors: as omprt_reduce per segment (with the segment index in the
 * message); INVALID for count < 0, NULL h_segs with count > 0, or a plan
 * built while the stream is being captured (make the call once before
 * capturing); NOMEM for the plan's tables.
 */
omprt_status omprt_reduce_batched(const omprt_segment *h_segs, int32_t count,
                                  const omprt_config *cfg, void *hip_stream);

/*
 * The same segments as omprt_reduce_batched, as one omprt_reduce launch
 * each (the plain form, for comparison).  cfg as for omprt_reduce.
 */
omprt_status omprt_reduce_each(const omprt_segment *h_segs, int32_t count,
                               const omprt_config *cfg, void *hip_stream);

/*
 * Worksharing body with a reduction, under the exact static schedule *s:
 * every iteration i is executed by the thread the schedule assigns it to,
 * and does   y[i] <- fmaf(a, x[i], y[i]);  sum += y[i]  (updated value).
 * On exit *d_sum <- *d_sum + sum (compensated fp32 as in omprt_reduce).
 * s->num_teams / threads_per_team of 0 let the runtime pick; dist_chunk and
 * chunk are honoured exactly.  x and y must not overlap.
 * Defining passages: a worksharing loop whose iterations the runtime
 * divides (sec. 1, sec. 2), with the schedule of omprt_for_static_bounds and
 * the reduction protocol of omprt_reduce (sec. 3.1).
 * Errors: INVALID for a bad schedule, NULL or misaligned pointers,
 * overlapping x and y, or more than 65535 teams.
 */
omprt_status omprt_axpy_sum(float a, const float *d_x, float *d_y,
                            float *d_sum, const omprt_sched *s,
                            const omprt_config *cfg, void *hip_stream);

/*
 * A parallel region with two worksharing loops over the same iterations,
 * the first with or without its implicit barrier (the nowait clause, whose
 * routines the device runtime provides for worksharing loops, sec. 2.1):
 *   loop 1, schedule(static, s->chunk) [nowait]:  y[i] <- fmaf(a, x[i], y[i])
 *   loop 2, schedule(static, chunk2), reduction(+: sum):  sum += y[i]
 * Both loops use s's distribute schedule (num_teams, dist_chunk), so a
 * team executes the same iterations in both and teams never wait for each
 * other.  nowait != 0 drops the team barrier between the loops; it is only
 * allowed with chunk2 == s->chunk (the same static schedule puts every
 * iteration on the same thread in both loops, so each thread reads back
 * only what it wrote), else OMPRT_ERR_INVALID.  Results equal
 * omprt_axpy_sum's: y bit for bit, *d_sum <- *d_sum + the compensated fp32
 * sum of the updated y.  s->num_teams / threads_per_team of 0 let the
 * runtime pick (as for omprt_axpy_sum); chunk2 >= 0 (0 = one block a
 * thread).  x and y must not overlap.
 */
omprt_status omprt_region_axpy_sum(float a, const float *d_x, float *d_y,
                                   float *d_sum, const omprt_sched *s,
                                   int64_t chunk2, int32_t nowait,
                                   const omprt_config *cfg, void *hip_stream);

/* ----------------------------------------------------------------------- */
/* Dynamic and guided worksharing                                          */
/* ----------------------------------------------------------------------- */

/*
 * schedule(dynamic[, c]) and schedule(guided[, c]) for the threads of a
 * team (the distribute part stays static, as *s gives it).  Each distribute
 * block of a team is handed out as a queue of chunks, one queue per block,
 * in team-shared memory; threads take chunks as they ask, so which thread
 * runs a chunk is not defined, only the chunks are (the paper lists the
 * worksharing-loop routines among what the device runtime provides, sec. 1):
 *   DYNAMIC: chunks of c iterations in order, the last one shorter;
 *   GUIDED:  the next chunk takes ceil(r / P) of the r iterations left, at
 *            least c and at most r.
 * c = s->chunk, with 0 meaning 1; P = s->threads_per_team.
 */
typedef enum { OMPRT_SCHED_DYNAMIC = 1, OMPRT_SCHED_GUIDED = 2 } omprt_sched_kind;

/*
 * The j-th chunk (0-based) of one block of m iterations under kind, as
 * offsets [*lb, *ub) from the block's start; *lb == *ub == m past the last
 * chunk.  Host arithmetic (O(j) for guided).  INVALID for a bad kind, m
 * outside 0..2^50, threads outside 1..1024, negative chunk or j, NULL
 * outputs.
 */
omprt_status omprt_queue_chunk(int32_t kind, int64_t m, int32_t threads,
                               int64_t chunk, int64_t j, int64_t *lb,
                               int64_t *ub);

/*
 * Iteration map of *s under kind on the GPU: the thread that runs iteration
 * i stores d_owner[i] = team * threads_per_team + thread and
 * d_start[i] = the first iteration of i's chunk, and adds 1 to d_count[i]
 * (the caller zeroes d_count).  tickets: chunks a thread takes per request
 * (1..64).  num_teams and threads_per_team must be given.  Guided chunk
 * bounds are computed on the host once per (block size, threads, chunk)
 * and kept on the device until omprt_finalize, or until 1024 of them exist,
 * when they are all dropped once the device is idle (the first call for a
 * block size must not be made while the stream is being captured).
 * Verification kernel for the queue semantics.
 */
omprt_status omprt_queue_map(const omprt_sched *s, int32_t kind,
                             int32_t tickets, int32_t *d_owner,
                             uint32_t *d_count, int64_t *d_start,
                             void *hip_stream);

/*
 * omprt_axpy_sum's body and sum (y[i] <- fmaf(a, x[i], y[i]); *d_sum +=
 * sum of the updated y, compensated fp32) under kind instead of a static
 * for-schedule.  s->num_teams of 0: one team per compute unit;
 * threads_per_team of 0: 512 for dynamic chunks under 16 iterations, else
 * 256 (at most 512; a guided schedule's chunk sizes follow the team size).
 * Dynamic chunks of one iteration are taken four per request.  Guided tables
 * as for omprt_queue_map.  y is bit-identical to the static schedules' result; the sum may
 * differ in its last bits (the order of accumulation depends on which
 * thread ran which chunk).
 */
omprt_status omprt_axpy_sum_queue(float a, const float *d_x, float *d_y,
                                  float *d_sum, const omprt_sched *s,
                                  int32_t kind, void *hip_stream);

/*
 * An empty target region with a trivial loop body: one launch of
 * s->num_teams teams over s->n iterations under s's static schedule whose
 * body only counts, reduction(+: iters) with one count per iteration.
 * Every thread works out its chunks, the counts go through the team tree
 * and the cross-team step like any reduction, and the last team checks
 * that the region ran exactly s->n iterations (the worksharing routines of
 * sec. 1 / sec. 2.1 plus the team-shared tree and the wrap-increment
 * election of sec. 3.1, with nothing else in the launch).  For launch
 * latency measurement and as a device-side check of the schedule
 * arithmetic.  d_iters (int64, may be NULL) receives *d_iters += the count.
 * A thread whose chunks are inconsistent, or a total other than s->n, sets
 * status bit 16 (omprt_workspace_status).  Errors: as check of *s, plus
 * INVALID for num_teams above 65535 or a misaligned d_iters.
 */
omprt_status omprt_empty_region(const omprt_sched *s, int64_t *d_iters,
                                void *hip_stream);

/* ----------------------------------------------------------------------- */
/* Device atomics                                                          */
/* ----------------------------------------------------------------------- */

/* The five atomic operations of the device runtime (paper sec. 3.1, "Atomic
 * Operations": add, max, exchange and cas as in the listing of OpenMP 5.1
 * atomics, and inc as defined in its text and target-specific listing).
 * Each returns the old value v of *X and updates *X (32-bit unsigned):
 *   ADD      { v = *X; *X = *X + E; }                  (wraps mod 2^32)
 *   INC      { v = *X; *X = (*X >= E) ? 0 : *X + 1; }
 *   MAX      { v = *X; if (*X < E) *X = E; }           (unsigned compare)
 *   EXCHANGE { v = *X; *X = E; }
 *   CAS      { v = *X; if (*X == E) *X = D; }
 * Sequentially consistent at agent scope (one GPU). */
typedef enum {
    OMPRT_ATOMIC_ADD = 0, OMPRT_ATOMIC_INC = 1, OMPRT_ATOMIC_MAX = 2,
    OMPRT_ATOMIC_EXCHANGE = 3, OMPRT_ATOMIC_CAS = 4
} omprt_atomic_op;

/*
 * n concurrent atomic operations, one per GPU thread: operation i acts on
 * d_target[d_index[i]] with operand d_e[i] (and d_d[i] for CAS; d_d may be
 * NULL otherwise) and stores the value it read in d_old[i].  Operations on
 * the same target are linearised by the hardware in an unspecified order.
 * d_index values must be < n_targets; the device checks: an operation whose
 * index is out of range is not applied, its d_old[i] receives 0xFFFFFFFF and
 * the stream's workspace status (omprt_workspace_status) becomes 2.  INVALID
 * for op out of range, n < 0, n_targets < 1 with n > 0, NULL pointers
 * (d_d may be NULL unless op is CAS).
 */
omprt_status omprt_atomic_apply(int32_t op, uint32_t *d_target, int64_t n_targets,
                                const uint32_t *d_index, const uint32_t *d_e,
                                const uint32_t *d_d, uint32_t *d_old, int64_t n,
                                void *hip_stream);

/* ----------------------------------------------------------------------- */
/* Learned launch configuration (extension; not in the paper)              */
/* ----------------------------------------------------------------------- */

/*
 * Network: F -> H1 -> H2 -> K, ReLU, fp32, softmax over K configuration
 * classes.  Parameters live in one contiguous fp32 buffer in the order
 * W1[H1][F], b1[H1], W2[H2][H1], b2[H2], W3[K][H2], b3[K] (row-major).
 */
typedef struct { int32_t F, H1, H2, K; } omprt_mlp_dims;

/* Number of fp32 parameters of a network of these dimensions. */
int64_t omprt_mlp_param_count(const omprt_mlp_dims *d);

/* Logits d_Z[B][K] of the rows d_X[B][F]. */
omprt_status omprt_mlp_forward(const omprt_mlp_dims *d, const float *d_params,
                               const float *d_X, int32_t B, float *d_Z,
                               void *hip_stream);

/*
 * Mean softmax cross-entropy of d_X[B][F] against labels d_y[B] in 0..K-1:
 * writes the loss to d_loss[0] and the gradient with respect to every
 * parameter to d_grads (same layout as d_params).  ReLU'(0) = 0.
 * B <= 65536.
 */
omprt_status omprt_mlp_loss_grad(const omprt_mlp_dims *d,
                                 const float *d_params, const float *d_X,
                                 const int32_t *d_y, int32_t B, float *d_loss,
                                 float *d_grads, void *hip_stream);

/* One Adam step (Kingma & Ba) at step number `step` >= 1 on n parameters. */
omprt_status omprt_mlp_adam(float *d_params, float *d_m, float *d_v,
                            const float *d_grads, int64_t n, int32_t step,
                            float lr, float beta1, float beta2, float eps,
                            void *hip_stream);

/*
 * The same Adam step with its step number in device memory: *d_step holds
 * the number of updates made so far (0 before the first); the step uses
 * t = *d_step + 1 and leaves *d_step = t.  Nothing depends on host values
 * that change from step to step, so a captured HIP graph of training steps
 * can be replayed.  The update equals omprt_mlp_adam's at step t bit for
 * bit.  Stream-ordered; d_step 4-byte aligned.
 */
omprt_status omprt_mlp_adam_counted(float *d_params, float *d_m, float *d_v,
                                    const float *d_grads, int64_t n, int32_t *d_step,
                                    float lr, float beta1, float beta2, float eps,
                                    void *hip_stream);

/*
 * Load (path != NULL) or unload (path == NULL) the learned picker used when
 * a reduction's cfg leaves fields at 0.  File format: text, written by the
 * package's training driver (dims, feature scaling, class table, weights).
 */
omprt_status omprt_model_load(const char *path);

/* Features of a call, as the picker sees them (16 floats, host). */
omprt_status omprt_model_features(int64_t n, int32_t dtype, int32_t op,
                                  int32_t body, int64_t chunk, float *h_f16);

/*
 * The configuration the runtime would use for a call with these
 * properties (body: 0 = plain reduction, 1 = AXPY body; chunk: the user's
 * chunk, -1 = none).  Fills *out; *source = 0 explicit, 1 learned model,
 * 2 tuned cache, 3 heuristic.
 */
omprt_status omprt_resolve_config(int64_t n, int32_t dtype, int32_t op,
                                  int32_t body, int64_t chunk,
                                  const omprt_config *cfg, omprt_config *out,
                                  int32_t *source);

/* Tuned cache entry: calls whose (dtype, op, body, floor(log2 n)) match use
 * *cfg when no model decides.  cfg == NULL removes the entry. */
omprt_status omprt_tune_set(int32_t dtype, int32_t op, int32_t body,
                            int32_t log2n, const omprt_config *cfg);

/*
 * omprt_reduce without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, kernels and
 * results as omprt_reduce, but the cross-team state (counter, epoch,
 * status, one 32-byte slot per team) lives in a fixed array of
 * 256 + 4096 * 32 bytes (128 KiB + 256 B) of static device memory that
 * each device holds until the process ends.  The call allocates nothing
 * (no hipMalloc, no hipFree, no library allocation); the array's device
 * address is looked up on the first call on each device.  Calls on one
 * device share its array: calls that overlap on one device (on different
 * streams, or concurrent host threads) race and must not be made.  The
 * array keeps the state of the last call, which is what the next call
 * needs (counter back at 0, epoch advanced).
 * Errors: those of omprt_reduce, plus INVALID when the resolved team count
 * exceeds 4096 (the array's slots); NOMEM is never returned.
 */
omprt_status omprt_reduce_noalloc(const void *d_in, int64_t n, int32_t dtype,
                                  int32_t op, void *d_x, const omprt_config *cfg,
                                  void *hip_stream);

/* ----------------------------------------------------------------------- */
/* Runtime                                                                 */
/* ----------------------------------------------------------------------- */

/* Allocate the stream's workspace for up to max_teams teams and
 * max_counters batched counters now (needed before the first call inside a
 * caller's own graph capture). */
omprt_status omprt_workspace_reserve(void *hip_stream, int32_t max_teams,
                                     int32_t max_counters);

/* Re-zero the stream's cross-team counter and status (after an aborted
 * launch).  Stream-ordered. */
omprt_status omprt_workspace_reset(void *hip_stream);

/*
 * Synchronise the stream and report its workspace status, a bit set:
 * 0 = healthy; bit 1 = a last team gave up waiting for a partial that never
 * arrived (its bounded poll expired; the result of that launch is not
 * valid -- the cross-team step publishes partials as tagged agent-scope
 * atomics and the last team polls for this launch's tag, so this only
 * happens if a participant was lost, e.g. an aborted launch); bit 2 = an
 * omprt_atomic_apply operation had an out-of-range index; bit 4 = an
 * omprt_histogram key was outside [0, bins); bit 8 = a team-shared
 * allocation found no room (its launch did nothing); bit 16 = an
 * omprt_empty_region launch found its schedule inconsistent.  The bits stay set
 * until omprt_workspace_reset (which also re-zeroes the array-reduction
 * counters).
 */
omprt_status omprt_workspace_status(void *hip_stream, int32_t *h_status);

/* Message of the last failed call on this host thread ("" if none). */
const char *omprt_last_error(void);

/* Library version string. */
const char *omprt_version(void);

/* Free every workspace, plan and graph.  Synchronises the device. */
omprt_status omprt_finalize(void);

#ifdef __cplusplus
}
#endif
#endif /* OMPRT_H */
