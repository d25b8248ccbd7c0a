/*
 * ac.h -- Aho-Corasick multi-pattern matching on MI355X (gfx950): C ABI.
 *
 * The paper (section III.A) splits Aho-Corasick into two stages: building a
 * string-matching machine from the keywords, then reading the input string
 * once with that machine.  Section IV.B describes the library interface the
 * authors used: an array of pattern strings and one input string in, the
 * matched pattern and its position in the input out.  This header exposes
 * the same two stages:
 *
 *   ac_build      stage 1, on the host: keyword trie (goto function),
 *                 breadth-first failure links and output sets, compiled into
 *                 a dense transition table (goto completed through failure
 *                 links) plus output-set offsets, then copied to the GPU.
 *   ac_scan       stage 2, on the GPU: every (pattern id, end position)
 *                 occurrence in a device-resident text, written in
 *                 (end position, pattern id) order.
 *   ac_scan_batch many independent (text, dictionary) instances in one
 *                 sequence of persistent launches.
 *   ac_encode     letters -> symbol codes, or DNA -> 2 bits per base.
 *
 * Conventions:
 *   - Symbols are codes 0 .. sigma-1.  Pattern i (0-based, input order) is
 *     symbols[offsets[i] .. offsets[i+1]); patterns may repeat and each copy
 *     is reported under its own id.
 *   - A match is (pattern_id, end_pos) with end_pos the 0-based index of the
 *     pattern's last symbol in the text.
 *   - Text formats: AC_TEXT_U8 holds one code per byte; AC_TEXT_2BIT (sigma
 *     must be 4) holds four codes per byte, base i in byte i/4 at bits
 *     2*(i%4) and 2*(i%4)+1 (least significant first).
 *   - Device pointers are plain HIP device addresses (hipMalloc or a torch
 *     tensor's data pointer); host pointers are ordinary memory.  A stream
 *     argument is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every function returns AC_OK (0) or a negative AC_E_* code and never
 *     throws.  Arguments are validated on the host before anything is
 *     enqueued; on an error nothing is enqueued.  Launch errors map to
 *     AC_E_HIP.
 *   - Thread safety: a dictionary is read-only after ac_build; scans with
 *     the same dictionary may run concurrently on different streams.
 */
#ifndef AC_H
#define AC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AC_OK 0
#define AC_E_INVALID (-1)        /* null pointer, bad enum value or size     */
#define AC_E_EMPTY_PATTERN (-2)  /* a pattern of length 0                    */
#define AC_E_SYMBOL (-3)         /* a pattern symbol >= sigma                */
#define AC_E_TOO_LARGE (-4)      /* text >= 2^32 symbols, table >= 2^32 B    */
#define AC_E_NOMEM (-5)          /* host or device allocation failed         */
#define AC_E_OVERFLOW (-6)       /* workspace smaller than required          */
#define AC_E_HIP (-7)            /* a HIP runtime call or launch failed      */
#define AC_E_NO_DEVICE (-8)      /* dictionary was built without GPU tables  */
#define AC_E_TIMEOUT (-9)        /* a wait ended before its request finished */

#define AC_TEXT_U8 0
#define AC_TEXT_2BIT 1

#define AC_ALPHA_DNA 0      /* A C G T -> 0 1 2 3 (either case)           */
#define AC_ALPHA_PROTEIN 1  /* A C D E F G H I K L M N P Q R S T V W Y -> 0..19 */

#define AC_PLACE_AUTO 0     /* library chooses                              */
#define AC_PLACE_LDS 1      /* whole table in LDS (must fit)                */
#define AC_PLACE_GLOBAL 2   /* table read through L1/L2 from HBM            */
#define AC_PLACE_HYBRID 3   /* most visited rows in LDS as 16-bit ids, rest global */
#define AC_PLACE_LDS2 4     /* DNA in 2-bit text only: transitions over two
                             * symbols at once (states x 16 entries) in LDS,
                             * one lookup per two bases; needs states * 64
                             * bytes of LDS, else falls back to AC_PLACE_LDS */
#define AC_PLACE_LDS16 5    /* whole table in LDS as 16-bit state ids (sigma *
                             * 2 bytes per row; dictionaries of fewer than
                             * 65,535 states): the default when the 32-bit
                             * table does not fit LDS but this one does; a
                             * request that does not fit falls back to
                             * AC_PLACE_HYBRID */

#define AC_BUILD_HOST_ONLY 1u /* compile tables on the host only (no GPU)   */
#define AC_BUILD_SERIAL 2u    /* compile on one host thread (default: up to 16
                               * threads, level by level); same tables      */

/* Work units of the scan: a segment is AC_SEGMENT text symbols; segments
 * with at least AC_DENSE_SEGMENT_MATCHES matches are written by a whole
 * wavefront each (the AC_K_EMIT_DENSE kernel), the others by four lanes. */
#define AC_SEGMENT 64
#define AC_DENSE_SEGMENT_MATCHES 256

typedef struct ac_dict ac_dict;
typedef struct ac_batch ac_batch;

/* One occurrence: 8 bytes. */
typedef struct {
    uint32_t pattern_id;
    uint32_t end_pos;
} ac_match;

typedef struct {
    uint32_t sigma;      /* alphabet size, 2..256                            */
    uint32_t placement;  /* AC_PLACE_* default for scans with this dict      */
    uint32_t flags;      /* AC_BUILD_HOST_ONLY | AC_BUILD_SERIAL, or 0       */
    uint32_t hot_states; /* rows kept in LDS by AC_PLACE_HYBRID; 0 = fill LDS */
} ac_build_opts;

typedef struct {
    uint32_t states;             /* automaton states (root = 0)            */
    uint32_t patterns;
    uint32_t sigma;
    uint32_t min_len, max_len;   /* shortest / longest pattern             */
    uint32_t first_output_state; /* states >= this have a non-empty output */
    uint32_t max_output;         /* largest output set                     */
    uint32_t placement;          /* default placement chosen by ac_build   */
    uint32_t hot_states;         /* rows in LDS (16-bit) for AC_PLACE_HYBRID */
    uint32_t has_device;         /* 1 if the GPU tables exist              */
    uint64_t output_entries;     /* sum of output-set sizes                */
    uint64_t table_bytes;        /* dense table, bytes                     */
    double build_ms;             /* host time of ac_build, tables only     */
} ac_dict_info;

/* Launch shape of a scan.  Zero fields take the library's choice. */
typedef struct {
    uint32_t chunk;         /* text symbols per chunk: multiple of 64, <= 2048 */
    uint32_t block_threads; /* 64..1024, multiple of 64                      */
    uint32_t placement;     /* AC_PLACE_*; AUTO = the dictionary's default   */
    uint32_t blocks_per_cu; /* persistent blocks per compute unit            */
    uint32_t chains;        /* chunks walked at once by one lane: 1, 2 or 4  */
} ac_tune;

/* ---------------------------------------------------------------- stage 1
 * ac_build: compile patterns into a dictionary (section III.A, Figure 1:
 * goto function, failure function, output function).
 *   symbols, offsets  host CSR list of n_patterns >= 1 patterns; offsets has
 *                     n_patterns + 1 entries, offsets[0] = 0.  Copied; the
 *                     caller may free them on return.
 *   opts              may be NULL only for sigma = 4 defaults.
 *   out               receives the dictionary; release with ac_destroy.
 * Errors: AC_E_INVALID, AC_E_EMPTY_PATTERN, AC_E_SYMBOL, AC_E_TOO_LARGE
 * (more than 2^27 states or a table of 2^32 bytes or more), AC_E_NOMEM,
 * AC_E_HIP (device upload failed). */
int ac_build(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
             const ac_build_opts *opts, ac_dict **out);

/* Release a dictionary built by stage 1 (section III.A): host and device
 * memory.  NULL is ignored.  The caller must have synchronised every stream
 * that uses it. */
void ac_destroy(ac_dict *dict);

int ac_dict_get_info(const ac_dict *dict, ac_dict_info *info);

/* Host copies of the compiled stage-1 tables (section III.A, Figures 1-2:
 * the goto function completed through the failure function, and the output
 * function), for inspection and CPU checks:
 *   delta    states*sigma entries: delta[s*sigma + a] = next state of s on
 *            symbol a (renumbered ids; root = 0).
 *   out_off  (states - first_output_state + 1) offsets into out_ids for the
 *            output set of state first_output_state + k.
 *   out_ids  output_entries pattern ids, each set sorted ascending.
 *   depth    states entries: length of the prefix spelled by each state.
 * Any pointer may be NULL to skip that table. */
int ac_debug_export(const ac_dict *dict, uint32_t *delta, uint32_t *out_off,
                    uint32_t *out_ids, uint32_t *depth);

/* ---------------------------------------------------------------- encoding
 * ac_encode: the input string of the matching stage (section III.A, read
 * from a file of nucleotide or amino-acid letters in section IV.B) turned
 * into symbol codes on the GPU.
 * d_ascii (n letters, device) -> d_out (device) as AC_TEXT_U8
 * codes (n bytes) or, for AC_ALPHA_DNA only, AC_TEXT_2BIT ((n+3)/4 bytes,
 * unused bits of the last byte zero).  Letters outside the alphabet are
 * encoded as code 0 and counted into *d_invalid (device uint64, may be NULL;
 * it is overwritten, not accumulated).  Stream-ordered. */
int ac_encode(const uint8_t *d_ascii, uint64_t n, uint32_t alphabet, uint32_t fmt,
              void *d_out, uint64_t *d_invalid, void *stream);

/* ---------------------------------------------------------------- stage 2
 * ac_scan: all occurrences of the dictionary's patterns in a device text
 * (section III.A, stage 2: one pass over the input).
 *   d_text      device text of n symbols in format fmt (n < 2^32).  Codes
 *               >= sigma give unspecified matches but never an access
 *               outside the dictionary's tables.
 *   d_out       device array of capacity ac_match slots.  The first
 *               min(total, capacity) matches in (end_pos, pattern_id) order
 *               are written; slots beyond are untouched.
 *   d_count     device uint64: receives the total number of matches, which
 *               may exceed capacity (then re-run with a larger d_out).
 *   tune        NULL = library choice.
 *   d_workspace device scratch of workspace_bytes (see
 *               ac_scan_workspace_size), or NULL to let the library take it
 *               from HIP's stream-ordered allocator for this call.
 *   stream      hipStream_t as void*.
 * Returns after enqueueing; results are valid once the stream reaches this
 * point.  Concurrent calls must not share a workspace. */
int ac_scan_workspace_size(const ac_dict *dict, uint64_t n, uint32_t fmt,
                           const ac_tune *tune, uint64_t *bytes);
int ac_scan(const ac_dict *dict, const void *d_text, uint64_t n, uint32_t fmt,
            ac_match *d_out, uint64_t capacity, uint64_t *d_count,
            const ac_tune *tune, void *d_workspace, uint64_t workspace_bytes,
            void *stream);

/* ac_scan_noalloc: ac_scan for callers that cannot allocate memory (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, results and errors as for ac_scan, without a
 * workspace argument: the workspace is a device array of
 * AC_NOALLOC_MAX_WORKSPACE bytes inside the library, one per device, held
 * from the library's load until the process ends.  The call allocates no
 * memory (no hipMalloc, no stream-ordered allocation) and enqueues kernels
 * only.  AC_E_TOO_LARGE when ac_scan_workspace_size(dict, n, fmt, tune)
 * exceeds AC_NOALLOC_MAX_WORKSPACE (about 60 M symbols at the default launch
 * shape); AC_E_INVALID for a partitioned dictionary (its scan allocates).
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (several streams or
 * host threads) race and must be serialised by the caller. */
#define AC_NOALLOC_MAX_WORKSPACE (64ull << 20)
int ac_scan_noalloc(const ac_dict *dict, const void *d_text, uint64_t n, uint32_t fmt,
                    ac_match *d_out, uint64_t capacity, uint64_t *d_count, const ac_tune *tune,
                    void *stream);

/* ---------------------------------------------------------------- variants
 * ac_build_partitioned: the paper's second design (section IV.A, Figure 3):
 * the pattern list is split into `parts` contiguous slices of about equal
 * length, and each slice is compiled into its own machine; parts = 0 picks
 * the fewest slices whose tables all fit LDS (as 16-bit rows).  Pattern ids
 * stay global (slice i reports ids from its first pattern's index).  The
 * result is used with ac_scan like any dictionary: every machine scans the
 * whole text (one batched launch sequence), and the slices' matches are
 * merged into (end_pos, pattern_id) order by a stable radix sort on end
 * position.  Such a scan synchronises its stream once to size temporary
 * buffers, takes them from HIP's stream-ordered allocator, and ignores
 * d_workspace (ac_scan_workspace_size, ac_debug_export and the batch entry
 * points reject a partitioned dictionary: AC_E_INVALID).  Errors as for
 * ac_build. */
int ac_build_partitioned(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
                         const ac_build_opts *opts, uint32_t parts, ac_dict **out);
/* Number of slices of a partitioned dictionary (0 for an ordinary one) and,
 * if first_ids is not NULL, the first pattern id of each (parts entries). */
int ac_dict_parts(const ac_dict *dict, uint32_t *parts, uint32_t *first_ids);

/* ac_scan_pfac: the failure-less form of stage 2 (related work, section
 * II): one thread per text position walks the trie (goto function only)
 * from the root along the text until an edge is missing and reports the
 * patterns ending exactly at each state it enters, so every occurrence is
 * found from its start; up to max_len lookups per position instead of one.
 * Arguments and results as for ac_scan (the same set, in (end_pos,
 * pattern_id) order after a radix sort); n < 2^31.  Synchronises the stream
 * once to size temporary buffers, which come from HIP's stream-ordered
 * allocator.  AC_E_TOO_LARGE if the table has 2^31 bytes or more. */
int ac_scan_pfac(const ac_dict *dict, const void *d_text, uint64_t n, uint32_t fmt,
                 ac_match *d_out, uint64_t capacity, uint64_t *d_count, void *stream);

/* ac_sort_matches: put match records (section IV.B: each occurrence is a
 * matched pattern and its position) into the canonical order of this
 * library: sort n device records in place into (end_pos,
 * pattern_id) order -- the order ac_scan writes -- by a radix sort over the
 * low end_bits bits of end_pos (0 = 32) and all of pattern_id.  With
 * AC_SORT_BY_END only end_pos is sorted on, stably: enough when records with
 * equal end_pos are already in id order.  n < 2^31.  d_workspace of
 * ac_sort_workspace_size(n) bytes, or NULL to take it from HIP's
 * stream-ordered allocator.  Stream-ordered. */
#define AC_SORT_BY_END 1u
int ac_sort_workspace_size(uint64_t n, uint64_t *bytes);
int ac_sort_matches(ac_match *d_matches, uint64_t n, uint32_t flags, uint32_t end_bits,
                    void *d_workspace, uint64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- batches
 * Many independent matching jobs at once (section IV.A: the work is split
 * into independent scans run in parallel; here each job is its own
 * (dictionary, text) pair).  One instance of a batch: its own dictionary,
 * text, output and count, with the meaning of the same-named ac_scan
 * arguments. */
typedef struct {
    const ac_dict *dict;
    const void *d_text;
    uint64_t n;
    uint32_t fmt;
    uint32_t reserved;
    ac_match *d_out;
    uint64_t capacity;
    uint64_t *d_count;
} ac_batch_item;

/* ac_batch_create (section IV.A, as above): plan a batch once (work list
 * of (instance, chunk range) tiles grouped by instance, descriptors uploaded
 * to the device, workspace allocated) so that ac_batch_run only launches
 * kernels: it can be replayed and captured in a hipGraph.  The items'
 * buffers must stay valid for the life of the plan; the plan owns its
 * descriptor and workspace memory.  Errors as for ac_scan (checked for every
 * item), AC_E_NOMEM. */
int ac_batch_create(const ac_batch_item *items, uint32_t n_items, const ac_tune *tune,
                    ac_batch **out);
/* ac_batch_run: enqueue the planned scans on `stream` (section IV.A, as
 * above); results as for ac_scan, per item.  Runs of one plan must not
 * overlap (they share its workspace).  AC_E_INVALID for a NULL plan. */
int ac_batch_run(ac_batch *batch, void *stream);
/* Release a plan; NULL is ignored.  Its runs must have completed. */
void ac_batch_destroy(ac_batch *batch);

/* ac_scan_batch (section IV.A, as above): plan + run in one call.  The
 * batch's device memory (descriptors and workspace,
 * ac_scan_batch_workspace_size bytes) is d_workspace when it is not NULL
 * (AC_E_OVERFLOW if workspace_bytes is smaller), else it comes from HIP's
 * stream-ordered allocator and is released when the stream reaches the end
 * of the batch.  Errors as for ac_scan, checked for every item before
 * anything is enqueued.  Concurrent calls must not share a workspace. */
int ac_scan_batch_workspace_size(const ac_batch_item *items, uint32_t n_items,
                                 const ac_tune *tune, uint64_t *bytes);
int ac_scan_batch(const ac_batch_item *items, uint32_t n_items, const ac_tune *tune,
                  void *d_workspace, uint64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- serving
 * A continuous-batching server over device-resident dictionaries: many
 * independent scans (section IV.A) submitted at any time, grouped into
 * batches that run on several streams while further requests are admitted.
 * Requests are DNA letters (ACGT, either case) against one of the server's
 * dictionaries; each request's matches equal those of ac_scan on its text
 * alone, in (end_pos, pattern_id) order.
 *
 * Threads: ac_server_submit queues a request and returns at once (waiting
 * only while the pinned staging ring is full); copier threads stage the
 * letters; a worker admits staged requests while device memory (the budget)
 * and a free in-flight slot allow, runs each batch (one copy of its letters,
 * ac_encode, ac_scan_batch, copies of counts and matches back) and hands the
 * matches to per-request host buffers.  Device memory counted per request:
 * letters, packed text, reserved matches, count and an upper bound of its
 * share of the batch workspace.  Matches are reserved from a running
 * estimate of each dictionary's matches per base; a request whose matches
 * overflow its reservation is scanned again, alone, exactly sized.  A
 * request that can never fit the budget is refused (AC_E_NOMEM from
 * ac_server_wait); letters outside ACGTacgt give AC_E_SYMBOL.  After a HIP
 * failure every unfinished request gets AC_E_HIP and submits are refused. */
typedef struct ac_server ac_server;

typedef struct {
    uint64_t budget_bytes;  /* device memory for requests; 0 = 90% of the free memory
                               (always capped at that) */
    uint64_t staging_bytes; /* pinned staging ring for letters; 0 = 256 MiB (a longer
                               request gets a pinned buffer of its own) */
    uint32_t max_batch;     /* requests per batch; 0 = 256 (at most 4096) */
    uint32_t streams;       /* batches in flight; 0 = 4 (at most 16) */
    uint32_t copy_threads;  /* threads staging letters; 0 = 8 (at most 64) */
    uint32_t max_wait_us;   /* while batches are in flight, a batch that could grow
                               waits up to this long for requests being staged */
    uint32_t fail_batch;    /* fault injection for tests: the k-th batch's device
                               allocation is reported failed (0 = never) */
    uint32_t reserved;
    double margin;          /* reserved matches = margin * (mean + 2 sqrt(mean)) + 64;
                               negative = 2.0 */
    ac_tune tune;           /* launch shape of the batches (zeros: library choice) */
} ac_server_opts;

typedef struct {
    uint64_t requests;      /* finished successfully */
    uint64_t bases, matches, batches, reruns;
    uint64_t overlapped;    /* batches launched while another was in flight */
    uint64_t peak_bytes;    /* largest device memory counted at once */
    uint64_t budget_bytes;
    double wall_s;          /* first submit to last completion */
    int32_t failed;         /* AC_OK, or the HIP failure that stopped the server */
    int32_t reserved;
} ac_server_counters;

/* Create a server over n_dicts dictionaries (sigma 4, with device tables;
 * they must outlive the server).  Starts its threads. */
int ac_server_create(ac_dict *const *dicts, uint32_t n_dicts, const ac_server_opts *opts,
                     ac_server **out);
/* Queue n letters (host memory; they must stay valid until ac_server_wait
 * has returned for this request) against dictionary dict_id; *ticket names
 * the request.  AC_E_INVALID after ac_server_destroy has begun. */
int ac_server_submit(ac_server *server, const uint8_t *letters, uint64_t n, uint32_t dict_id,
                     uint64_t *ticket);
/* Wait for a request (timeout_us < 0: without limit; AC_E_TIMEOUT when it
 * expires).  On AC_OK, *matches (host memory owned by the server) holds
 * *count matches until ac_server_release; *latency_s (may be NULL) is the
 * time from submit to completion.  A failed request returns its code. */
int ac_server_wait(ac_server *server, uint64_t ticket, int64_t timeout_us,
                   const ac_match **matches, uint64_t *count, double *latency_s);
/* Device bytes a request of n letters for dictionary dict_id would be
 * counted against the budget now (it depends on the running estimate of
 * matches per base). */
int ac_server_request_charge(ac_server *server, uint64_t n, uint32_t dict_id, uint64_t *bytes);
/* Free a finished request's results (AC_E_INVALID while it is pending). */
int ac_server_release(ac_server *server, uint64_t ticket);
/* Counters, and up to max_latencies latencies (seconds, completion order). */
int ac_server_stats(ac_server *server, ac_server_counters *stats, double *latencies,
                    uint64_t max_latencies);
/* Finish every queued request, stop the threads, free the server; returns
 * stats.failed.  NULL is ignored. */
int ac_server_destroy(ac_server *server);

/* ---------------------------------------------------------------- timing
 * Kernel timing for measurement.  While enabled, every call above records a
 * pair of hipEvents on its stream around each timed kernel it launches (do
 * not enable it while a stream is being captured into a graph).  on: 0 off,
 * AC_TIMING_ALL every kind, or AC_TIMING_KIND(k) bits for chosen kinds only
 * (each event pair adds a little time to the stream, so a measurement of
 * the whole sequence can time just the kernel it needs).  ac_timing_read
 * waits for the recorded events, adds their elapsed times to per-kind totals
 * and returns them: ms[k] and launches[k] for k < AC_K_KINDS (arrays of
 * AC_K_KINDS entries, either may be NULL); reset != 0 clears the totals. */
#define AC_TIMING_ALL 1
#define AC_TIMING_KIND(k) (2 << (k))
#define AC_K_ENCODE 0   /* ac_encode                                   */
#define AC_K_COUNT 1    /* pass 1: walk chunks, count matches per segment */
#define AC_K_OFFSETS 2  /* prefix sums over tiles                         */
#define AC_K_SCATTER 3  /* work list of segments with matches             */
#define AC_K_EMIT 4     /* pass 2, sparse segments: one lane each          */
#define AC_K_TOTALS 5   /* per-instance totals (batches)                 */
#define AC_K_EMIT_DENSE 6 /* pass 2, dense segments: one wave each       */
#define AC_K_PFAC 7     /* failure-less scan (count and write passes)     */
#define AC_K_SORT 8     /* radix sort of match records                    */
#define AC_K_KINDS 9
int ac_timing_enable(int on);
int ac_timing_read(double *ms, uint64_t *launches, int reset);

/* ---------------------------------------------------------------- misc */
const char *ac_status_str(int status);

/* Device properties the launch heuristics use (compute units, LDS bytes per
 * block).  Returns AC_E_HIP when no GPU is visible. */
int ac_device_info(uint32_t *compute_units, uint32_t *lds_bytes_per_block);

#ifdef __cplusplus
}
#endif
#endif /* AC_H */
