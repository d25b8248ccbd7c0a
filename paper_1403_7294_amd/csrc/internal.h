// Internal declarations shared by the host automaton compiler
// (automaton.cpp), the C-ABI entry points (api.cpp) and the GPU code
// (scan.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/ac.h"

namespace acx {

// Host form of a compiled dictionary.
//
// States are renumbered so that the root is 0, states whose output set is
// empty come first, most likely to be visited first (which is what the
// LDS-resident "hot" prefix of the table wants), and states with a non-empty
// output set come last: "state >= first_output" is then the whole match test
// of the scan.
struct HostTables {
    uint32_t sigma = 0;
    uint32_t states = 0;
    uint32_t patterns = 0;
    uint32_t min_len = 0, max_len = 0;
    uint32_t first_output = 0;
    uint32_t max_output = 0;
    std::vector<uint32_t> delta;    // states*sigma, next-state ids
    std::vector<uint32_t> out_off;  // states-first_output+1
    std::vector<uint32_t> out_ids;  // concatenated output sets, ids ascending
    std::vector<uint32_t> depth;    // prefix length spelled by each state
    // goto function alone (the trie), for the failure-less kernel:
    // states*sigma child ids, 0 = no edge (the root is nobody's child), and
    // the patterns ending exactly at each state (CSR over all states)
    std::vector<uint32_t> go;
    std::vector<uint32_t> own_off;  // states+1
    std::vector<uint32_t> own_ids;  // patterns, ids ascending per state
};

// Stage 1 of the method on the host: trie, failure links, completed
// transitions, output sets, renumbering, on `threads` host threads (0: up to
// 16).  The tables do not depend on the thread count.  Returns an AC_* status.
int compile_automaton(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
                      uint32_t sigma, HostTables *out, uint32_t threads = 0);

// Exact division of a row byte offset (state * sigma * 4) by sigma * 4:
// state = (offset >> tz) * inv (mod 2^32), with sigma*4 = 2^tz * odd and
// inv the inverse of odd modulo 2^32.
struct RowDiv {
    uint32_t tz = 0;
    uint32_t inv = 1;
};
RowDiv make_row_div(uint32_t sigma);

// Allocation-failure injection for tests: with AC_TEST_FAIL_ALLOC=<n> in the
// environment, the n-th allocation the library checks (counted from 1 over
// the life of the process) is reported as failed, and the caller takes the
// same path as for a real failure (AC_E_NOMEM, everything released).
// Without the variable it is always false.
bool test_alloc_fails();

}  // namespace acx

struct ihipStream_t;

// The opaque dictionary handle.
struct ac_dict {
    acx::HostTables host;
    uint32_t placement = AC_PLACE_AUTO;  // default for scans
    uint32_t hot_states = 0;             // LDS rows for hybrid placement
    double build_ms = 0.0;
    // device copies (null when built host-only)
    int device = -1;
    uint32_t *d_delta = nullptr;    // states*sigma row byte offsets
    uint32_t *d_out_off = nullptr;
    uint32_t *d_out_ids = nullptr;
    uint32_t *d_out_size = nullptr;  // |out(s)| per output state
    uint32_t *d_delta_sz = nullptr;  // sigma 4: row offset | |out(target)| << 24 (count walk)
    uint16_t *d_hot16 = nullptr;  // first hot16_rows rows as 16-bit ids (0xFFFF: see table)
    uint16_t *d_hot16c = nullptr;  // the same, output targets also 0xFFFF (count-table walk)
    uint32_t hot16_rows = 0;
    // the whole table as 16-bit state ids (states < 65,535 and the table
    // fits LDS), for AC_PLACE_LDS16
    uint16_t *d_tab16 = nullptr;
    uint32_t tab16_bytes = 0;
    // sigma 4 only, when it fits LDS: transitions over two symbols,
    // states x 16 entries; entry = next row offset (next * 64), bit 31 set
    // when the state after the first symbol has an output set
    uint32_t *d_delta2 = nullptr;
    uint32_t delta2_bytes = 0;
    // failure-less kernel tables: goto entries as row offsets of the child
    // (0 = no edge), bit 31 set when the child has patterns of its own
    uint32_t *d_go = nullptr;
    uint32_t *d_own_off = nullptr;
    uint32_t *d_own_ids = nullptr;
    // a partitioned dictionary (pattern slices, each its own machine) holds
    // no tables itself; part i reports pattern ids from part_base[i]
    std::vector<ac_dict *> parts;
    std::vector<uint32_t> part_base;
    uint64_t table_bytes = 0;
};

namespace acx {
// Device-side upload / release (scan.hip).
int upload_dict(ac_dict *d);
void release_dict(ac_dict *d);
// Largest dynamic LDS allocation one block may use, and compute units.
int device_limits(uint32_t *cus, uint32_t *lds_bytes);
// Radix sort of match records into (end, id) order (sort.hip).
uint64_t sort_workspace_bytes(uint64_t n);
int sort_matches(ac_match *d, uint64_t n, uint32_t flags, uint32_t end_bits, void *ws,
                 uint64_t ws_bytes, ihipStream_t *st);
int exclusive_sum_u64(const unsigned long long *in, unsigned long long *out, uint64_t n,
                      ihipStream_t *st);
// Scan with a partitioned dictionary (scan.hip).
int scan_partitioned(const ac_dict *d, const void *text, uint64_t n, uint32_t fmt, ac_match *out,
                     uint64_t cap, uint64_t *count, const ac_tune *tune, ihipStream_t *st);
}  // namespace acx
