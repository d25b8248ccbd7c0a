/*
 * ac_split.c -- the paper's own parallel design on the host CPU: the
 * pattern list is cut into N contiguous slices, and each of N POSIX
 * threads builds the goto/failure/output machine of its slice and then
 * reads the whole text with it (section IV.A, second design; Fig. 3).  The
 * paper times the whole run (machine construction and matching) and reports
 * the speed-up of N threads over one (abstract; section V, Figs. 4-5).
 *
 * TEST INFRASTRUCTURE AND CPU BASELINE ONLY.  It reuses the oracle's plain
 * machine (ac_oracle.c) for every slice, so its matches are the oracle's by
 * construction; the tests check that the union of the slices' matches is
 * the single machine's set (partition invariance of the second design).  The
 * product library never calls it.
 *
 * Slices hold consecutive patterns and differ in size by at most one
 * pattern.  Pattern ids stay global: slice t reports id first_t + i for its
 * i-th pattern.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef struct oracle_machine oracle_machine;
int oracle_build(const uint8_t *sym, const uint64_t *off, uint32_t n_patterns, uint32_t sigma,
                 oracle_machine **out);
void oracle_free(oracle_machine *m);
int64_t oracle_scan(const oracle_machine *m, const uint8_t *text, uint64_t n, uint32_t *pid,
                    uint32_t *end, uint64_t cap);

#define SPLIT_E_INVALID (-1)
#define SPLIT_E_NOMEM (-5)
#define SPLIT_E_THREAD (-9)

typedef struct {
    /* inputs */
    const uint8_t *sym;
    const uint64_t *off;  /* rebased offsets of this slice (count + 1)   */
    uint32_t count;       /* patterns in the slice                       */
    uint32_t first;       /* global id of its first pattern              */
    uint32_t sigma;
    const uint8_t *text;
    uint64_t n;
    uint32_t *pid, *end;  /* this slice's output area (cap records)     */
    uint64_t cap;
    int build;            /* 1: build the machine, then scan; 0: scan only */
    /* state and results */
    oracle_machine *m;
    int64_t total;
    int rc;
    double build_s, scan_s;
} slice_job;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void *slice_main(void *arg) {
    slice_job *j = (slice_job *)arg;
    double t0 = now_s();
    if (j->build) {
        j->rc = j->count ? oracle_build(j->sym, j->off, j->count, j->sigma, &j->m) : 0;
        if (j->rc) return NULL;
    }
    double t1 = now_s();
    j->total = j->m ? oracle_scan(j->m, j->text, j->n, j->pid, j->end, j->cap) : 0;
    if (j->total < 0) {
        j->rc = (int)j->total;
        return NULL;
    }
    /* the slice's ids are local to it: make them global */
    const uint64_t w = (uint64_t)j->total < j->cap ? (uint64_t)j->total : j->cap;
    for (uint64_t k = 0; k < w; ++k) j->pid[k] += j->first;
    double t2 = now_s();
    j->build_s = t1 - t0;
    j->scan_s = t2 - t1;
    return NULL;
}

static int run_threads(slice_job *jobs, uint32_t parts, double *wall_s) {
    pthread_t *th = (pthread_t *)calloc(parts, sizeof(pthread_t));
    if (!th) return SPLIT_E_NOMEM;
    int rc = 0;
    uint32_t started = 0;
    const double t0 = now_s();
    for (; started < parts; ++started)
        if (pthread_create(&th[started], NULL, slice_main, &jobs[started]) != 0) {
            rc = SPLIT_E_THREAD;
            break;
        }
    for (uint32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
    *wall_s = now_s() - t0;
    free(th);
    for (uint32_t t = 0; t < parts && !rc; ++t) rc = jobs[t].rc;
    return rc;
}

/* split_run: N = parts threads, each building its slice's machine and then
 * scanning the whole text, timed as one run (the paper's measurement), then
 * the same machines scanning again, timed alone.
 *   sym, off, n_patterns  patterns in CSR form (as for oracle_build)
 *   text, n               codes < sigma
 *   pid, end, cap         per-slice output areas: slice t writes at most cap
 *                         records at pid + t*cap, end + t*cap, in (end, id)
 *                         order within the slice; NULL with cap 0 counts only
 *   counts                parts entries: matches found by each slice
 *   wall_build_scan_s     wall time of the first run (build + scan)
 *   wall_scan_s           wall time of the second run (scan only)
 *   build_s, scan_s       parts entries each (may be NULL): per-thread times
 *                         of the first run
 * Returns 0 or a negative oracle/split error code. */
int split_run(const uint8_t *sym, const uint64_t *off, uint32_t n_patterns, uint32_t sigma,
              const uint8_t *text, uint64_t n, uint32_t parts, uint32_t *pid, uint32_t *end,
              uint64_t cap, uint64_t *counts, double *wall_build_scan_s, double *wall_scan_s,
              double *build_s, double *scan_s) {
    if (!sym || !off || !n_patterns || !parts || parts > n_patterns || (n && !text) ||
        (cap && (!pid || !end)) || !counts || !wall_build_scan_s || !wall_scan_s)
        return SPLIT_E_INVALID;
    slice_job *jobs = (slice_job *)calloc(parts, sizeof(slice_job));
    uint64_t *offs = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n_patterns + parts));
    if (!jobs || !offs) {
        free(jobs);
        free(offs);
        return SPLIT_E_NOMEM;
    }
    uint64_t *o = offs;
    for (uint32_t t = 0; t < parts; ++t) {
        const uint32_t a = (uint32_t)((uint64_t)n_patterns * t / parts);
        const uint32_t b = (uint32_t)((uint64_t)n_patterns * (t + 1) / parts);
        for (uint32_t i = a; i <= b; ++i) o[i - a] = off[i] - off[a];
        slice_job *j = &jobs[t];
        j->sym = sym + off[a];
        j->off = o;
        j->count = b - a;
        j->first = a;
        j->sigma = sigma;
        j->text = text;
        j->n = n;
        j->pid = cap ? pid + (uint64_t)t * cap : NULL;
        j->end = cap ? end + (uint64_t)t * cap : NULL;
        j->cap = cap;
        j->build = 1;
        o += (b - a) + 1;
    }
    int rc = run_threads(jobs, parts, wall_build_scan_s);
    if (!rc) {
        for (uint32_t t = 0; t < parts; ++t) {
            counts[t] = (uint64_t)jobs[t].total;
            if (build_s) build_s[t] = jobs[t].build_s;
            if (scan_s) scan_s[t] = jobs[t].scan_s;
            jobs[t].build = 0;
        }
        rc = run_threads(jobs, parts, wall_scan_s);
    }
    for (uint32_t t = 0; t < parts; ++t) oracle_free(jobs[t].m);
    free(jobs);
    free(offs);
    return rc;
}
