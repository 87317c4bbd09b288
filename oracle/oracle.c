/*
 * oracle.c -- serial CPU oracle for the data-parallel core of an OpenMP
 * device runtime (Tian, Chesterfield, Doerfert, Chapman: "Experience Report:
 * Writing A Portable GPU Runtime with OpenMP 5.1").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source, header, table or helper with
 * the HIP library; both sides only receive the same seeded input arrays.
 *
 * What it computes, and where the definition comes from:
 *
 *  - Static iteration mapping.  The paper (sec. 1) says the device runtime
 *    supplies the routines compiler-lowered worksharing loops call, and
 *    (sec. 3.1, "Global Shared Variables") that an OpenMP team is one GPU
 *    thread block.  The schedule rules themselves are OpenMP's
 *    static / dist_schedule(static) rules, which the paper relies on but
 *    does not restate.  The readings used (balanced default chunk, each
 *    distribute chunk workshared separately starting at thread 0, surplus
 *    teams/threads idle) are written out in the function comments below.
 *    The oracle enumerates the schedule literally: teams, then their
 *    distribute chunks, then threads, then their chunks, then iterations.
 *
 *  - Reductions.  A reduction(op:x) region leaves x = x_orig (op) fold(op,
 *    in[0..n)), for the OpenMP reduction identifiers + * max min & | ^ && ||.
 *    Integers wrap modulo 2^w (computed in the unsigned type of the same
 *    width); signed max/min compare signed.  Floating-point sums are formed
 *    in FP64 with Neumaier's compensated summation of the exactly widened
 *    inputs, products in FP64; floating max/min use fmax/fmin
 *    (NaN-dropping); && and || give 0 or 1.
 *
 *  - Histogram: reduction(+: hist[0:bins]) with hist[key[i]] += 1.
 *
 *  - Power iteration on a diagonal matrix (parallel loops with sequential
 *    code between them, as a generic-mode target region runs them).
 *
 *  - maxloc / minloc: the largest / smallest value with its position, ties
 *    to the smaller position (the common user-defined reduction).
 *
 *  - AXPY worksharing body: y[i] <- fmaf(a, x[i], y[i]) (one rounding), then
 *    the sum over the updated y in FP64 Neumaier.
 *
 *  - Dynamic and guided worksharing: the queue of chunks each distribute
 *    block hands out (dynamic: fixed size; guided: ceil(remaining / P), at
 *    least the chunk size).  Only the chunks are defined, not their owners.
 *
 *  - Learned-configuration extension (not in the paper): a
 *    F -> H1 -> H2 -> K ReLU multilayer perceptron with softmax
 *    cross-entropy, its analytic backward pass and one Adam step
 *    (Kingma & Ba, Algorithm 1), all in FP64.
 *
 * Everything is plain serial C with no blocking, vectorisation or
 * reordering beyond what the definitions state.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Static schedule                                                          */
/* ------------------------------------------------------------------------ */

/*
 * Balanced split of m iterations over p workers, worker t's share
 * [lo, hi).  With q = m / p and r = m % p, the first r workers get q + 1
 * iterations and the rest get q, in worker order.  This is the reading of
 * OpenMP's "schedule(static) without chunk size: approximately equal
 * chunks, at most one per thread" used throughout.
 */
void oracle_bal(int64_t m, int64_t p, int64_t t, int64_t *lo, int64_t *hi)
{
    int64_t q = m / p, r = m % p;
    int64_t start = t * q + (t < r ? t : r);
    *lo = start;
    *hi = start + q + (t < r ? 1 : 0);
}

/*
 * Enumerate the non-empty distribute chunks of team k: with dc == 0 the
 * single balanced block bal(n, T, k) (none if it is empty, i.e. surplus
 * teams when T > n); with dc > 0 the chunks
 * [j*dc, min(n, (j+1)*dc)) for j = k, k+T, k+2T, ... while j*dc < n.
 * Writes at most cap chunks; returns how many there are.
 */
static int64_t team_chunks(int64_t n, int64_t T, int64_t dc, int64_t k,
                           int64_t *lo, int64_t *hi, int64_t cap)
{
    int64_t cnt = 0;
    if (dc == 0) {
        int64_t a, b;
        oracle_bal(n, T, k, &a, &b);
        if (a == b) return 0;          /* surplus team: no iterations */
        if (cnt < cap) { lo[cnt] = a; hi[cnt] = b; }
        return 1;
    }
    for (int64_t j = k; j * dc < n; j += T) {
        int64_t a = j * dc, b = (j + 1) * dc;
        if (b > n) b = n;
        if (cnt < cap) { lo[cnt] = a; hi[cnt] = b; }
        cnt++;
    }
    return cnt;
}

/*
 * Enumerate thread t's non-empty chunks of the team chunk [a, b)
 * (m = b - a):
 * c == 0: the single block a + bal(m, P, t) (none if empty: P > m);
 * c > 0: chunks [a + j*c, a + min(m, (j+1)*c)) for j = t, t+P, ...
 * while j*c < m (round-robin, restarting at thread 0 in every team chunk).
 */
static int64_t thread_chunks(int64_t a, int64_t b, int64_t P, int64_t c,
                             int64_t t, int64_t *lo, int64_t *hi, int64_t cap)
{
    int64_t m = b - a, cnt = 0;
    if (c == 0) {
        int64_t u, v;
        oracle_bal(m, P, t, &u, &v);
        if (u == v) return 0;          /* surplus thread: no iterations */
        if (cnt < cap) { lo[cnt] = a + u; hi[cnt] = a + v; }
        return 1;
    }
    for (int64_t j = t; j * c < m; j += P) {
        int64_t u = j * c, v = (j + 1) * c;
        if (v > m) v = m;
        if (cnt < cap) { lo[cnt] = a + u; hi[cnt] = a + v; }
        cnt++;
    }
    return cnt;
}

/*
 * Materialise the whole iteration map of
 *   distribute [dist_schedule(static[, dc])] parallel for schedule(static[, c])
 * over n iterations with T teams of P threads: owner[i] = k*P + t of the
 * thread that executes iteration i, count[i] = how many times it is
 * executed.  owner[] must be pre-filled by the caller (e.g. with -1) and
 * count[] zeroed; both have n entries.  Returns 0, or -1 on bad arguments.
 */
int oracle_map(int64_t n, int64_t T, int64_t P, int64_t dc, int64_t c,
               int32_t *owner, uint32_t *count)
{
    if (n < 0 || T < 1 || P < 1 || dc < 0 || c < 0) return -1;
    for (int64_t k = 0; k < T; k++) {
        int64_t ntc = team_chunks(n, T, dc, k, NULL, NULL, 0);
        int64_t *tl = malloc(sizeof(int64_t) * (size_t)ntc);
        int64_t *th = malloc(sizeof(int64_t) * (size_t)ntc);
        team_chunks(n, T, dc, k, tl, th, ntc);
        for (int64_t jt = 0; jt < ntc; jt++) {
            for (int64_t t = 0; t < P; t++) {
                int64_t nth = thread_chunks(tl[jt], th[jt], P, c, t, NULL, NULL, 0);
                int64_t *lo = malloc(sizeof(int64_t) * (size_t)(nth ? nth : 1));
                int64_t *hi = malloc(sizeof(int64_t) * (size_t)(nth ? nth : 1));
                thread_chunks(tl[jt], th[jt], P, c, t, lo, hi, nth);
                for (int64_t q = 0; q < nth; q++)
                    for (int64_t i = lo[q]; i < hi[q]; i++) {
                        owner[i] = (int32_t)(k * P + t);
                        count[i] += 1u;
                    }
                free(lo); free(hi);
            }
        }
        free(tl); free(th);
    }
    return 0;
}

/*
 * The ordered list of chunks thread t of team k executes (across all of
 * its team's distribute chunks, in execution order).  Only chunks with at
 * least one iteration are listed.  Writes at most cap entries and returns
 * the total count.
 */
int64_t oracle_thread_chunks(int64_t n, int64_t T, int64_t P, int64_t dc,
                             int64_t c, int64_t k, int64_t t,
                             int64_t *lo, int64_t *hi, int64_t cap)
{
    int64_t total = 0;
    int64_t ntc = team_chunks(n, T, dc, k, NULL, NULL, 0);
    int64_t *tl = malloc(sizeof(int64_t) * (size_t)ntc);
    int64_t *th = malloc(sizeof(int64_t) * (size_t)ntc);
    team_chunks(n, T, dc, k, tl, th, ntc);
    for (int64_t jt = 0; jt < ntc; jt++) {
        int64_t nth = thread_chunks(tl[jt], th[jt], P, c, t, NULL, NULL, 0);
        int64_t *l = malloc(sizeof(int64_t) * (size_t)(nth ? nth : 1));
        int64_t *h = malloc(sizeof(int64_t) * (size_t)(nth ? nth : 1));
        thread_chunks(tl[jt], th[jt], P, c, t, l, h, nth);
        for (int64_t q = 0; q < nth; q++) {
            if (total < cap) { lo[total] = l[q]; hi[total] = h[q]; }
            total++;
        }
        free(l); free(h);
    }
    free(tl); free(th);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Dynamic and guided worksharing                                           */
/* ------------------------------------------------------------------------ */

/*
 * schedule(dynamic[, c]) and schedule(guided[, c]) hand a team block of m
 * iterations out as a queue of chunks, each taken by whichever thread asks
 * next, so which thread runs a chunk is not defined -- only the chunks
 * are.  (The paper lists worksharing loops among the routines the device
 * runtime provides, sec. 1; the chunk rules are OpenMP's, read as below.)
 *
 *  - dynamic: chunks of c iterations in order, the last one shorter
 *    (c == 0 means 1);
 *  - guided: the next chunk takes ceil(r / P) of the r iterations not yet
 *    handed out, but at least c (c == 0 means 1) and at most r.
 *
 * Writes the chunks of one block, as offsets [lo, hi) from its start, in
 * queue order (at most cap of them) and returns how many there are, or -1
 * for bad arguments.  kind: 0 dynamic, 1 guided.
 */
int64_t oracle_queue_chunks(int kind, int64_t m, int64_t P, int64_t c,
                            int64_t *lo, int64_t *hi, int64_t cap)
{
    if (m < 0 || P < 1 || c < 0 || (kind != 0 && kind != 1)) return -1;
    int64_t cmin = c > 0 ? c : 1;
    int64_t start = 0, cnt = 0;
    while (start < m) {
        int64_t rest = m - start;
        int64_t size = cmin;
        if (kind == 1) {
            int64_t share = (rest + P - 1) / P;   /* ceil(rest / P) */
            if (share > size) size = share;
        }
        if (size > rest) size = rest;
        if (cnt < cap) { lo[cnt] = start; hi[cnt] = start + size; }
        cnt++;
        start += size;
    }
    return cnt;
}

/*
 * distribute [dist_schedule(static[, dc])] parallel for schedule(kind[, c])
 * over n iterations with T teams of P threads: the chunks team k's queues
 * hand out, block by block (each distribute block has a queue of its own),
 * as absolute iteration ranges.  Writes at most cap chunks and returns the
 * total, or -1 for bad arguments.
 */
int64_t oracle_team_queue(int kind, int64_t n, int64_t T, int64_t P, int64_t dc,
                          int64_t c, int64_t k, int64_t *lo, int64_t *hi, int64_t cap)
{
    if (n < 0 || T < 1 || P < 1 || dc < 0 || c < 0 || k < 0 || k >= T) return -1;
    int64_t ntc = team_chunks(n, T, dc, k, NULL, NULL, 0);
    int64_t *tl = malloc(sizeof(int64_t) * (size_t)(ntc ? ntc : 1));
    int64_t *th = malloc(sizeof(int64_t) * (size_t)(ntc ? ntc : 1));
    team_chunks(n, T, dc, k, tl, th, ntc);
    int64_t total = 0;
    for (int64_t jt = 0; jt < ntc; jt++) {
        int64_t m = th[jt] - tl[jt];
        int64_t nq = oracle_queue_chunks(kind, m, P, c, NULL, NULL, 0);
        int64_t *l = malloc(sizeof(int64_t) * (size_t)(nq ? nq : 1));
        int64_t *h = malloc(sizeof(int64_t) * (size_t)(nq ? nq : 1));
        oracle_queue_chunks(kind, m, P, c, l, h, nq);
        for (int64_t q = 0; q < nq; q++) {
            if (total < cap) { lo[total] = tl[jt] + l[q]; hi[total] = tl[jt] + h[q]; }
            total++;
        }
        free(l); free(h);
    }
    free(tl); free(th);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Reductions                                                               */
/* ------------------------------------------------------------------------ */

/*
 * The reduction identifiers of the OpenMP reduction clause: + * max min on
 * every type, the bitwise & | ^ on integers, the logical && || on every
 * type (an operand counts as true when it is not zero; the result is 0 or
 * 1 in x's type).  x_orig takes part as the first operand.
 */
enum { OR_SUM = 0, OR_MAX = 1, OR_MIN = 2, OR_PROD = 3, OR_BAND = 4, OR_BOR = 5,
       OR_BXOR = 6, OR_LAND = 7, OR_LOR = 8 };

/* Integer fold in the unsigned type of the same width (sum and product
 * wrap); max/min compare signed. */
#define INT_FOLD(S, U)                                                        \
    {                                                                         \
        U acc = (U)x;                                                         \
        S m = x;                                                              \
        int flag = x != 0;                                                    \
        for (int64_t i = 0; i < n; i++) {                                     \
            U v = (U)in[i];                                                   \
            switch (op) {                                                     \
            case OR_SUM:  acc += v; break;                                    \
            case OR_PROD: acc *= v; break;                                    \
            case OR_BAND: acc &= v; break;                                    \
            case OR_BOR:  acc |= v; break;                                    \
            case OR_BXOR: acc ^= v; break;                                    \
            case OR_MAX:  if (in[i] > m) m = in[i]; break;                    \
            case OR_MIN:  if (in[i] < m) m = in[i]; break;                    \
            case OR_LAND: flag = flag && in[i] != 0; break;                   \
            case OR_LOR:  flag = flag || in[i] != 0; break;                   \
            }                                                                 \
        }                                                                     \
        if (op == OR_MAX || op == OR_MIN) return m;                           \
        if (op == OR_LAND || op == OR_LOR) return (S)flag;                    \
        return (S)acc;                                                        \
    }

int32_t oracle_reduce_i32(const int32_t *in, int64_t n, int op, int32_t x)
INT_FOLD(int32_t, uint32_t)

int64_t oracle_reduce_i64(const int64_t *in, int64_t n, int op, int64_t x)
INT_FOLD(int64_t, uint64_t)

/* Neumaier's compensated summation state (FP64). */
typedef struct { double s, c; } neum;

static void neum_add(neum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

/* bfloat16 is the upper half of an IEEE binary32: widening is exact. */
static double bf16_to_double(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

/*
 * Floating reductions.  dtype: 0 = fp32, 1 = fp64, 2 = bf16 (raw uint16).
 * sum: Neumaier FP64 over x_orig then in[0..n) in index order.
 * prod: FP64 product in index order, starting at x_orig (each step rounds
 *   once to FP64, so the result is within (n+1) 2^-53 relative of the exact
 *   product of the widened inputs, barring overflow and underflow).
 * max/min: fmax/fmin fold starting at x_orig.
 * land/lor: 0 or 1 (an operand is true when it is not zero; NaN is true).
 * Also returns sum |in[i]| (FP64 Neumaier) through abs_sum when non-NULL,
 * for the condition number kappa = sum|x_i| / |sum x_i|.
 */
double oracle_reduce_fp(const void *in, int64_t n, int dtype, int op,
                        double x, double *abs_sum)
{
    neum acc = { x, 0.0 }, aacc = { 0.0, 0.0 };
    double m = x, p = x;
    int flag = x != 0.0;
    for (int64_t i = 0; i < n; i++) {
        double v;
        if (dtype == 0) v = (double)((const float *)in)[i];
        else if (dtype == 1) v = ((const double *)in)[i];
        else v = bf16_to_double(((const uint16_t *)in)[i]);
        if (op == OR_SUM) neum_add(&acc, v);
        else if (op == OR_MAX) m = fmax(m, v);
        else if (op == OR_MIN) m = fmin(m, v);
        else if (op == OR_PROD) p *= v;
        else if (op == OR_LAND) flag = flag && v != 0.0;
        else if (op == OR_LOR) flag = flag || v != 0.0;
        if (abs_sum) neum_add(&aacc, fabs(v));
    }
    if (abs_sum) *abs_sum = aacc.s + aacc.c;
    if (op == OR_SUM) return acc.s + acc.c;
    if (op == OR_PROD) return p;
    if (op == OR_LAND || op == OR_LOR) return (double)flag;
    return m;
}

/*
 * The same folds at several prefix lengths in one pass: out[k] is what
 * oracle_reduce_i32 / oracle_reduce_i64 (dtype 0 / 1) or oracle_reduce_fp
 * (dtype 2 fp32, 3 fp64, 4 bf16 raw) would return for in[0..lens[k]) with
 * the same op (sum, max or min) and x.  lens must be ascending; the fold runs
 * over in[0..lens[nlens-1]) in index order and its running state is read out
 * as each length is passed (integer results are returned as int64, floating
 * ones as double).  Returns 0, or -1 for lengths that are not ascending or an
 * op other than sum / max / min.
 */
int oracle_fold_prefixes(const void *in, int dtype, int op, double x_fp, int64_t x_int,
                         const int64_t *lens, int64_t nlens, int64_t *out_int,
                         double *out_fp)
{
    if (op != OR_SUM && op != OR_MAX && op != OR_MIN) return -1;
    for (int64_t k = 1; k < nlens; k++)
        if (lens[k] < lens[k - 1]) return -1;
    uint64_t uacc = (uint64_t)x_int;
    int64_t im = x_int;
    neum acc = { x_fp, 0.0 };
    double m = x_fp;
    int64_t i = 0;
    for (int64_t k = 0; k < nlens; k++) {
        for (; i < lens[k]; i++) {
            if (dtype == 0 || dtype == 1) {
                int64_t v = dtype == 0 ? (int64_t)((const int32_t *)in)[i]
                                       : ((const int64_t *)in)[i];
                if (op == OR_SUM) uacc += (uint64_t)v;
                else if (op == OR_MAX && v > im) im = v;
                else if (op == OR_MIN && v < im) im = v;
            } else {
                double v;
                if (dtype == 2) v = (double)((const float *)in)[i];
                else if (dtype == 3) v = ((const double *)in)[i];
                else v = bf16_to_double(((const uint16_t *)in)[i]);
                if (op == OR_SUM) neum_add(&acc, v);
                else if (op == OR_MAX) m = fmax(m, v);
                else m = fmin(m, v);
            }
        }
        if (dtype == 0) {   /* wrap in 32 bits */
            out_int[k] = op == OR_SUM ? (int64_t)(int32_t)(uint32_t)uacc : im;
        } else if (dtype == 1) {
            out_int[k] = op == OR_SUM ? (int64_t)uacc : im;
        } else {
            out_fp[k] = op == OR_SUM ? acc.s + acc.c : m;
        }
    }
    return 0;
}

/*
 * maxloc / minloc, the usual user-defined reduction (a value with its
 * position): the pairs (x_val, x_idx), (in[0], 0), ..., (in[n-1], n-1) are
 * folded with "keep the larger (op 1) or smaller (op 2) value; on equal
 * values keep the smaller position".  That order is total, so the result
 * does not depend on the fold order.  Floating NaNs never win (as with
 * fmax/fmin), a NaN x_val loses to any element; -0 and +0 are equal.
 * dtype: 0 int32, 1 int64, 2 fp32, 3 fp64, 4 bf16 (raw uint16).  Values are
 * compared as int64 (integers) or as FP64 (floating, exactly widened).  The
 * winning value is returned through *v_int (integers) or *v_fp (floating)
 * and its position through *pos.
 */
static double loc_value_fp(const void *in, int dtype, int64_t i)
{
    if (dtype == 2) return (double)((const float *)in)[i];
    if (dtype == 3) return ((const double *)in)[i];
    return bf16_to_double(((const uint16_t *)in)[i]);
}

void oracle_reduce_loc(const void *in, int64_t n, int dtype, int op,
                       int64_t x_int, double x_fp, int64_t x_idx,
                       int64_t *v_int, double *v_fp, int64_t *pos)
{
    int64_t bi = x_int, bpos = x_idx;
    double bf = x_fp;
    for (int64_t i = 0; i < n; i++) {
        if (dtype == 0 || dtype == 1) {
            int64_t v = dtype == 0 ? (int64_t)((const int32_t *)in)[i] : ((const int64_t *)in)[i];
            int better = op == OR_MAX ? v > bi : v < bi;
            if (better || (v == bi && i < bpos)) { bi = v; bpos = i; }
        } else {
            double v = loc_value_fp(in, dtype, i);
            if (isnan(v)) continue;
            int better = isnan(bf) || (op == OR_MAX ? v > bf : v < bf);
            if (better || (v == bf && i < bpos)) { bf = v; bpos = i; }
        }
    }
    *v_int = bi;
    *v_fp = bf;
    *pos = bpos;
}

/*
 * Histogram: reduction(+: hist[0:bins]) over a loop whose iteration i does
 * hist[key[i]] += 1 -- an array-section reduction whose list item is chosen
 * by the data.  Counts wrap modulo 2^32 (int32 list items).  Keys outside
 * [0, bins) are not counted; returns how many there were.
 */
int64_t oracle_histogram(const int32_t *keys, int64_t n, int32_t bins, int32_t *hist)
{
    int64_t skipped = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t k = keys[i];
        if (k < 0 || k >= bins) { skipped++; continue; }
        hist[k] = (int32_t)((uint32_t)hist[k] + 1u);
    }
    return skipped;
}

/*
 * Power iteration on a diagonal matrix, the generic-mode region's workload
 * (sequential code between parallel loops): iters times
 *     w[i] = d[i] * v[i];  s = sum w[i]^2;  v[i] = w[i] / sqrt(s)
 * in FP64, v updated in place; *lambda = sqrt(s) of the last iteration
 * (the norm of D v, the dominant |d| once v has converged).  iters >= 1.
 */
void oracle_power_iteration(const double *d, double *v, int64_t n, int32_t iters,
                            double *lambda)
{
    double s = 0.0;
    for (int32_t k = 0; k < iters; k++) {
        neum acc = { 0.0, 0.0 };
        for (int64_t i = 0; i < n; i++) {
            v[i] = d[i] * v[i];
            neum_add(&acc, v[i] * v[i]);
        }
        s = acc.s + acc.c;
        double r = 1.0 / sqrt(s);
        for (int64_t i = 0; i < n; i++) v[i] = v[i] * r;
    }
    *lambda = sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* AXPY worksharing body                                                    */
/* ------------------------------------------------------------------------ */

/*
 * y[i] <- fmaf(a, x[i], y[i]) for i in [0, n) (updated in place), then the
 * FP64 Neumaier sum of the updated y, starting from s_orig.
 */
double oracle_axpy_sum(float a, const float *x, float *y, int64_t n,
                       double s_orig)
{
    neum acc = { s_orig, 0.0 };
    for (int64_t i = 0; i < n; i++) {
        y[i] = fmaf(a, x[i], y[i]);
        neum_add(&acc, (double)y[i]);
    }
    return acc.s + acc.c;
}

/*
 * The AXPY body at several prefix lengths in one pass: y[i] <- fmaf(a, x[i],
 * y[i]) for i < lens[nlens-1] (in place), and out[k] = the FP64 Neumaier sum
 * of the updated y[0..lens[k]) starting from s_orig -- what oracle_axpy_sum
 * returns over that prefix.  lens ascending; returns 0, or -1 otherwise.
 */
int oracle_axpy_prefix_sums(float a, const float *x, float *y, double s_orig,
                            const int64_t *lens, int64_t nlens, double *out)
{
    for (int64_t k = 1; k < nlens; k++)
        if (lens[k] < lens[k - 1]) return -1;
    neum acc = { s_orig, 0.0 };
    int64_t i = 0;
    for (int64_t k = 0; k < nlens; k++) {
        for (; i < lens[k]; i++) {
            y[i] = fmaf(a, x[i], y[i]);
            neum_add(&acc, (double)y[i]);
        }
        out[k] = acc.s + acc.c;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* MLP cost model (FP64)                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Forward and backward of z = W3 relu(W2 relu(W1 f + b1) + b2) + b3 with
 * mean softmax cross-entropy against integer labels, for a batch of B rows.
 * Layouts (row-major): X[B][F], W1[H1][F], W2[H2][H1], W3[K][H2].
 * Outputs: *loss, logits Z[B][K] (may be NULL) and, when g* are non-NULL,
 * the gradients of the mean loss with respect to every parameter.
 * ReLU'(0) is taken as 0.
 */
double oracle_mlp_loss_grad(const double *X, const int32_t *y, int64_t B,
                            int64_t F, int64_t H1, int64_t H2, int64_t K,
                            const double *W1, const double *b1,
                            const double *W2, const double *b2,
                            const double *W3, const double *b3,
                            double *Z, double *gW1, double *gb1,
                            double *gW2, double *gb2, double *gW3,
                            double *gb3)
{
    double *a1 = calloc((size_t)(B * H1), sizeof(double));
    double *a2 = calloc((size_t)(B * H2), sizeof(double));
    double *z = calloc((size_t)(B * K), sizeof(double));
    double *dz = calloc((size_t)(B * K), sizeof(double));
    double *d2 = calloc((size_t)(B * H2), sizeof(double));
    double *d1 = calloc((size_t)(B * H1), sizeof(double));
    double loss = 0.0;

    for (int64_t r = 0; r < B; r++) {
        for (int64_t j = 0; j < H1; j++) {
            double s = b1[j];
            for (int64_t i = 0; i < F; i++) s += W1[j * F + i] * X[r * F + i];
            a1[r * H1 + j] = s > 0.0 ? s : 0.0;
        }
        for (int64_t j = 0; j < H2; j++) {
            double s = b2[j];
            for (int64_t i = 0; i < H1; i++) s += W2[j * H1 + i] * a1[r * H1 + i];
            a2[r * H2 + j] = s > 0.0 ? s : 0.0;
        }
        for (int64_t j = 0; j < K; j++) {
            double s = b3[j];
            for (int64_t i = 0; i < H2; i++) s += W3[j * H2 + i] * a2[r * H2 + i];
            z[r * K + j] = s;
        }
        /* softmax with the maximum subtracted, then -log p[y] */
        double mx = z[r * K];
        for (int64_t j = 1; j < K; j++) if (z[r * K + j] > mx) mx = z[r * K + j];
        double den = 0.0;
        for (int64_t j = 0; j < K; j++) den += exp(z[r * K + j] - mx);
        loss += -((z[r * K + y[r]] - mx) - log(den));
        for (int64_t j = 0; j < K; j++) {
            double p = exp(z[r * K + j] - mx) / den;
            dz[r * K + j] = (p - (j == y[r] ? 1.0 : 0.0)) / (double)B;
        }
    }
    loss /= (double)B;
    if (Z) memcpy(Z, z, sizeof(double) * (size_t)(B * K));

    if (gW1) {
        memset(gW3, 0, sizeof(double) * (size_t)(K * H2));
        memset(gb3, 0, sizeof(double) * (size_t)K);
        memset(gW2, 0, sizeof(double) * (size_t)(H2 * H1));
        memset(gb2, 0, sizeof(double) * (size_t)H2);
        memset(gW1, 0, sizeof(double) * (size_t)(H1 * F));
        memset(gb1, 0, sizeof(double) * (size_t)H1);
        for (int64_t r = 0; r < B; r++) {
            for (int64_t j = 0; j < K; j++) {
                gb3[j] += dz[r * K + j];
                for (int64_t i = 0; i < H2; i++)
                    gW3[j * H2 + i] += dz[r * K + j] * a2[r * H2 + i];
            }
            for (int64_t i = 0; i < H2; i++) {
                double s = 0.0;
                for (int64_t j = 0; j < K; j++) s += dz[r * K + j] * W3[j * H2 + i];
                d2[r * H2 + i] = a2[r * H2 + i] > 0.0 ? s : 0.0;
            }
            for (int64_t j = 0; j < H2; j++) {
                gb2[j] += d2[r * H2 + j];
                for (int64_t i = 0; i < H1; i++)
                    gW2[j * H1 + i] += d2[r * H2 + j] * a1[r * H1 + i];
            }
            for (int64_t i = 0; i < H1; i++) {
                double s = 0.0;
                for (int64_t j = 0; j < H2; j++) s += d2[r * H2 + j] * W2[j * H1 + i];
                d1[r * H1 + i] = a1[r * H1 + i] > 0.0 ? s : 0.0;
            }
            for (int64_t j = 0; j < H1; j++) {
                gb1[j] += d1[r * H1 + j];
                for (int64_t i = 0; i < F; i++)
                    gW1[j * F + i] += d1[r * H1 + j] * X[r * F + i];
            }
        }
    }
    free(a1); free(a2); free(z); free(dz); free(d2); free(d1);
    return loss;
}

/*
 * One Adam step (Kingma & Ba, Algorithm 1) on n parameters at step number
 * t >= 1:  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *          w <- w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
void oracle_adam(double *w, double *m, double *v, const double *g, int64_t n,
                 int64_t t, double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; i++) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Device atomics                                                           */
/* ------------------------------------------------------------------------ */

/*
 * The runtime's five atomic operations on 32-bit unsigned words, applied
 * one after another in index order (one valid linearisation of concurrent
 * execution).  Paper sec. 3.1 defines them: add { v = x; x += e; },
 * max { v = x; if (x < e) x = e; } (unsigned), exchange { v = x; x = e; },
 * cas { v = x; if (x == e) x = d; }, and inc { v = x; x = x >= e ? 0 : x+1; };
 * each returns v.  op: 0 add, 1 inc, 2 max, 3 exchange, 4 cas.  An index at
 * or beyond n_targets is skipped with old = 0xFFFFFFFF.  Returns the number
 * of skipped operations.
 */
int64_t oracle_atomic_serial(int op, uint32_t *target, int64_t n_targets,
                             const uint32_t *index, const uint32_t *e,
                             const uint32_t *d, uint32_t *old, int64_t n)
{
    int64_t skipped = 0;
    for (int64_t i = 0; i < n; i++) {
        if ((int64_t)index[i] >= n_targets) {
            old[i] = 0xFFFFFFFFu;
            skipped++;
            continue;
        }
        uint32_t *x = &target[index[i]];
        uint32_t v = *x;
        switch (op) {
        case 0: *x = v + e[i]; break;
        case 1: *x = (v >= e[i]) ? 0u : v + 1u; break;
        case 2: if (v < e[i]) *x = e[i]; break;
        case 3: *x = e[i]; break;
        case 4: if (v == e[i]) *x = d[i]; break;
        }
        old[i] = v;
    }
    return skipped;
}
