// GPU stage of Aho-Corasick for gfx950 (MI355X): the single-pass scan of the
// paper's section III.A, run as many independent passes over text chunks.
//
// Decomposition (the paper's section IV.A, first design, made exact): lane j
// owns the end positions [j*C, (j+1)*C) of the text.  It starts at the root
// max_len-1 symbols (rounded up to a whole 32-bit text word) before j*C, so
// that from j*C on its state equals the state a single pass from the start
// of the text would hold: after any text prefix the machine is in the
// longest suffix of that prefix that is a trie prefix, and no trie prefix is
// longer than max_len.  Every match is therefore reported by exactly one lane.
//
// A scan is a short sequence of launches on the caller's stream:
//   k_count      every lane walks its chunk once, one table lookup per
//                symbol, and counts the matches ending in each 64-symbol
//                segment (sum of the output-set sizes of the states entered).
//                For each segment with matches it stores the count and the
//                states entering its four 16-symbol quarters; per chunk it
//                stores the total and a segment bit mask.
//   k_tile_scan  one block: exclusive offsets of the per-tile totals.
//   k_scatter    the work list: every segment with matches, with its
//                quarter states and its first output slot, in text order;
//                segments with many matches are listed after the others.
//   k_emit       sparse segments: four lanes per segment re-walk its quarters
//                from the stored states and write each match at its slot.
//   k_emit_dense dense segments: one wave per segment, writes coalesced.
// Matches therefore come out in (end position, pattern id) order with no
// sort, and a too-small output buffer still receives the first matches.
//
// The transition table holds row byte offsets (state * sigma * 4); it lives
// in LDS when it fits, in HBM behind the L1/L2 caches otherwise, or split
// with the first (most visited, shallowest) rows in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace acx {

constexpr uint32_t kSeg = AC_SEGMENT;     // symbols per segment
constexpr uint32_t kQuarter = kSeg / 4;   // symbols per quarter segment
// Output events of a segment kept by the count pass (at most 4): output
// set index << 6 | position in the segment; unused slots kEvNone, and
// kEvMany in the first slot when the segment has more (or an index that
// does not fit 26 bits).
constexpr uint32_t kEvSlots = 4;
constexpr uint32_t kEvNone = 0xFFFFFFFFu;
constexpr uint32_t kEvMany = 0xFFFFFFFEu;
constexpr uint32_t kEvMaxSet = (1u << 26) - 2;
constexpr uint32_t kMaxChunk = 2048;      // 32 segments: one bit each in a chunk mask
constexpr uint32_t kDenseMatches = AC_DENSE_SEGMENT_MATCHES;  // listed last, one wave each
constexpr uint32_t kLdsPad = 1024;        // zero bytes after an LDS table (u8 codes >= sigma)
constexpr uint32_t kMaxCountThreads = 1024;

// Per-instance parameters of a scan, shared by host and device.
struct Inst {
    const uint32_t *delta;  // row byte offsets: delta[s*sigma+a] = next*sigma*4
    const uint32_t *out_off;
    const uint32_t *out_ids;
    const uint32_t *out_size;  // |out(s)| per output state (count pass)
    const uint32_t *delta_sz;  // sigma 4: count table (row offset | |out(target)| << 24)
    uint32_t n_ids;            // entries of out_ids
    const uint16_t *hot16;   // 16-bit rows for the hybrid placement
    const uint16_t *hot16c;  // the same with every output target escaped (count-table walk)
    const uint16_t *tab16;   // the whole table as 16-bit ids (lds_all == 2)
    const uint8_t *text;
    ac_match *out;
    unsigned long long *count;
    uint64_t capacity;
    uint32_t n;            // text symbols
    uint32_t text_bytes4;  // text bytes rounded up to a multiple of 4
    uint32_t table_bytes;
    uint32_t fo_bytes;     // row offset of the first state with output
    uint32_t fo_state;     // its state number
    uint32_t hot_bytes;    // LDS: table bytes; hybrid: first row offset not in LDS; else 0
    uint32_t lds_all;      // 1: whole table in LDS (with zero pad); 2: as 16-bit ids
    uint32_t lds_bytes;    // bytes the count kernel copies into LDS
    uint32_t n_chunks;
    uint32_t chunk_base;   // first chunk of this instance in the chunk arrays
    uint32_t seg_base;     // its first segment in the segment arrays
    uint32_t chunk;        // symbols per chunk (a multiple of the segment)
    uint32_t warm;         // text words walked before a chunk (max_len - 1 symbols, rounded up)
    uint32_t first_tile;   // first tile of this instance
    uint32_t n_tiles;
    uint32_t div_tz, div_inv;
    uint32_t sigma;
    const uint32_t *delta2;  // two-symbol transitions (stride2 only)
    uint32_t stride2;        // 1: the count pass walks two symbols per lookup from LDS
    uint32_t fo2_bytes;      // first output row offset in the two-symbol table
    uint32_t walk_sz;        // 1: the emit walks read the count table (masked), which the
                             // count pass has just pulled into L2, instead of delta
};

struct TileDesc {
    uint32_t inst;
    uint32_t first;  // first chunk (instance-local)
    uint32_t count;  // chunks in this tile
    uint32_t pad;
};

// ------------------------------------------------------------------ count

struct ChunkOut {
    uint32_t m;      // matches ending in the chunk
    uint32_t mask;   // segments with matches
    uint32_t dense;  // of which with >= kDenseMatches matches
};

// Per-lane geometry of one chain (one chunk).
struct ChainIn {
    uint32_t j;     // chunk (instance-local)
    uint32_t lim;   // symbols of the chunk inside the text (0: no chunk)
    uint32_t seg0;  // first segment in the segment arrays
};

// Walk CH chunks at once (independent lookup chains that keep more loads in
// flight per lane) and count the matches ending in each 64-symbol segment.
// A word is walked with one lookup per symbol plus a running max; only a
// word that reaches an output state adds output-set sizes (rare).  For each
// segment with matches the entry state and the count are stored.
template <int FMT, int PLACE, int CH, bool ROW16 = false>
__device__ __forceinline__ void walk_count(const UTable<PLACE, ROW16> &tab, const UText &txt,
                                           const uint32_t *__restrict__ out_size,
                                           uint32_t out_size_bytes, uint32_t fo,
                                           uint32_t fo_state, uint32_t tz, uint32_t inv,
                                           uint32_t chunk, uint32_t warm, const ChainIn (&in)[CH],
                                           u32x4 *__restrict__ seg_state,
                                           uint32_t *__restrict__ seg_m, ChunkOut (&r)[CH]) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    constexpr uint32_t WPS = kSeg / SPW;  // text words per segment
    const uint32_t wpc = chunk / SPW, spc = chunk / kSeg;
    const rsrc_t sizes = make_rsrc(out_size, out_size_bytes);
    uint32_t s[CH], w0[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        w0[c] = in[c].j * wpc;
        s[c] = 0;
        r[c] = ChunkOut{0, 0, 0};
    }
    // warm-up, chains interleaved
    for (uint32_t i = 0; i < warm; ++i) {
        uint32_t x[CH];
        bool live[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int w = (int)w0[c] - (int)warm + (int)i;
            x[c] = txt.word(w);
            live[c] = w >= 0;
        }
#pragma unroll
        for (uint32_t k = 0; k < SPW; ++k) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const uint32_t ns = tab(s[c] + sym_bytes<FMT>(x[c], k));
                s[c] = live[c] ? ns : s[c];
            }
        }
    }
    // text vectors (4 words) in flight ahead of the walk: 128 bases of
    // 2-bit text, 64 byte symbols
    constexpr uint32_t PD = FMT == AC_TEXT_2BIT ? 2 : 4;
    u32x4 nx[CH][PD];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (uint32_t p = 0; p < PD; ++p)
            nx[c][p] = 4 * p < wpc ? txt.vec_once(w0[c] + 4 * p) : u32x4{0, 0, 0, 0};
    for (uint32_t g = 0; g < spc; ++g) {
        uint32_t qs[CH][4], sm[CH], ev[CH][kEvSlots], ne[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            sm[c] = 0;
            ne[c] = 0;
#pragma unroll
            for (uint32_t e = 0; e < kEvSlots; ++e) ev[c][e] = kEvNone;
        }
#pragma unroll
        for (uint32_t v = 0; v < WPS; v += 4) {
            u32x4 x4[CH];
            const uint32_t wn = g * WPS + v + 4 * PD;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                x4[c] = nx[c][0];
#pragma unroll
                for (uint32_t p = 0; p + 1 < PD; ++p) nx[c][p] = nx[c][p + 1];
                if (wn < wpc) nx[c][PD - 1] = txt.vec_once(w0[c] + wn);
            }
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
                uint32_t st[CH][SPW];
                uint32_t acc[CH];
                // the state on entry to each quarter segment
                if (((v + q) * SPW) % kQuarter == 0) {
#pragma unroll
                    for (int c = 0; c < CH; ++c) qs[c][(v + q) * SPW / kQuarter] = s[c];
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) acc[c] = 0;
#pragma unroll
                for (uint32_t k = 0; k < SPW; ++k) {
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        s[c] = tab(s[c] + sym_bytes<FMT>(x4[c][q], k));
                        st[c][k] = s[c];
                        acc[c] = acc[c] > s[c] ? acc[c] : s[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (acc[c] >= fo) {
                        // some state of this word has an output set: add the
                        // set sizes.  The offset loads of all positions are
                        // issued before the first is used, so the word costs
                        // one memory latency, not one per output state.
                        const uint32_t p0 = (g * WPS + v + q) * SPW;
                        // one output state over the whole word (the inside
                        // of a dense run): one size load, no events kept
                        bool same = p0 + SPW <= in[c].lim;
#pragma unroll
                        for (uint32_t k = 1; k < SPW; ++k) same = same && st[c][k] == st[c][0];
                        if (same) {
                            const uint32_t o0 = row_state_f<FMT>(st[c][0], tz, inv) - fo_state;
                            sm[c] += SPW * buf_load(sizes, o0 * 4u);
                            ne[c] = kEvSlots + 1;
                            continue;
                        }
                        if constexpr (PLACE == PL_LDS || PLACE == PL_LDS16) {
                            // small tables: one position at a time (fewer
                            // registers; the lookups are cheap)
#pragma unroll
                            for (uint32_t k = 0; k < SPW; ++k) {
                                if (st[c][k] >= fo && p0 + k < in[c].lim) {
                                    const uint32_t o =
                                        row_state_f<FMT>(st[c][k], tz, inv) - fo_state;
                                    sm[c] += buf_load(sizes, o * 4u);
                                    const uint32_t e =
                                        o <= kEvMaxSet ? o << 6 | ((v + q) * SPW + k) : kEvMany;
#pragma unroll
                                    for (uint32_t u = 0; u < kEvSlots; ++u)
                                        ev[c][u] = ne[c] == u ? e : ev[c][u];
                                    ne[c] = e == kEvMany ? kEvSlots + 1 : ne[c] + 1;
                                }
                            }
                            continue;
                        }
                        uint32_t o[SPW], sz[SPW];
#pragma unroll
                        for (uint32_t k = 0; k < SPW; ++k) {
                            const bool hit = st[c][k] >= fo && p0 + k < in[c].lim;
                            o[k] = hit ? row_state_f<FMT>(st[c][k], tz, inv) - fo_state : kEvNone;
                            // out of range for positions without output: no
                            // memory access, value 0
                            sz[k] = buf_load(sizes, hit ? o[k] * 4u : 0xFFFFFFF0u);
                        }
#pragma unroll
                        for (uint32_t k = 0; k < SPW; ++k) {
                            sm[c] += sz[k];
                            if (o[k] != kEvNone) {
                                const uint32_t e = o[k] <= kEvMaxSet
                                                       ? o[k] << 6 | ((v + q) * SPW + k)
                                                       : kEvMany;
#pragma unroll
                                for (uint32_t u = 0; u < kEvSlots; ++u)
                                    ev[c][u] = ne[c] == u ? e : ev[c][u];
                                ne[c] = e == kEvMany ? kEvSlots + 1 : ne[c] + 1;
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (sm[c]) {
                r[c].mask |= 1u << g;
                u32x4 *rec = seg_state + 2 * (in[c].seg0 + g);
                rec[0] = u32x4{qs[c][0], qs[c][1], qs[c][2], qs[c][3]};
                rec[1] = ne[c] <= kEvSlots ? u32x4{ev[c][0], ev[c][1], ev[c][2], ev[c][3]}
                                           : u32x4{kEvMany, kEvNone, kEvNone, kEvNone};
                seg_m[in[c].seg0 + g] = sm[c];
                r[c].dense += sm[c] >= kDenseMatches;
            }
            r[c].m += sm[c];
        }
    }
}

// Count table for 2-bit text (sigma 4, 16-byte rows).  Its 32-bit entries
// are the target's row offset (below 2^24) with |out(target)| in the top
// byte, so the walk counts matches as it goes.  The 16-bit rows in LDS hold
// the ids of output-free targets; 0xFFFF (an output state, or an id past 16
// bits) means "read the 32-bit entry".  A lane on a row in LDS gives the
// global load an offset past the buffer's end (value 0, no memory access);
// a lane on any other row reads the LDS zero word just past the 16-bit rows
// (byte hot / 2).  The next entry is then (h << 4) | v for every lane.
constexpr uint32_t kRowBits = 0x00FFFFFFu;  // row offset part of a count-table entry

// The table the emit kernels walk: the count table, masked to row offsets,
// when the count pass walked it (it is then in L2, while delta is not),
// else delta.
struct MTable {
    rsrc_t g;
    uint32_t mask;
    __device__ __forceinline__ uint32_t operator()(uint32_t a) const { return buf_load(g, a) & mask; }
};
__device__ __forceinline__ MTable emit_table(const uint32_t *delta, const uint32_t *delta_sz,
                                             uint32_t walk_sz, uint32_t bytes) {
    return walk_sz ? MTable{make_rsrc(delta_sz, bytes), kRowBits}
                   : MTable{make_rsrc(delta, bytes), 0xFFFFFFFFu};
}

struct HotTable16 {
    rsrc_t g;      // count table
    rsrc_t gc;     // the same from the first row not in LDS on
    uint32_t hot;  // first row offset not in LDS
    // One lookup for each of CH independent chains: every chain's global
    // and LDS reads are issued before any result is used, and the rare
    // escape is tested once for all chains, so the chains' latencies
    // overlap inside the wave.  The cold rows are addressed from `hot` on:
    // a lane on a row in LDS gives an offset that wraps past the end of
    // that range, so its load returns 0 with no memory access and the
    // step needs no select.
    template <int CH>
    __device__ __forceinline__ void step(const uint32_t (&a)[CH], uint32_t (&r)[CH]) const {
        // the 16-bit rows start at LDS address 0 (the count kernel has no
        // static LDS; the host checks that before choosing this walk)
        typedef __attribute__((address_space(3))) uint16_t lds_u16;
        uint32_t v[CH], h[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) v[c] = buf_load(gc, a[c] - hot);
#pragma unroll
        for (int c = 0; c < CH; ++c) h[c] = *(const lds_u16 *)(uintptr_t)(min(a[c], hot) >> 1);
        bool esc = false;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            r[c] = h[c] << 4 | v[c];
            esc = esc || h[c] > 0xFFFEu;
        }
        if (esc) {
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (h[c] > 0xFFFEu) r[c] = buf_load(g, a[c]);
        }
    }
};

// The count walk for 2-bit text against a HotTable16.  Rows are 16-byte
// aligned, so a symbol's column is OR-ed into the row offset, and every
// step adds the entered state's output-set size from the entry's top byte:
// no per-word output test and no re-read of sizes.  Positions past the
// chunk's text (only in the text's last word) are walked by a variant that
// drops their counts.  One output event is kept per segment: a running max
// of (entry | position in the word) lands on an output state whenever the
// word has one (only those entries have a nonzero top byte), and a segment
// whose count equals that state's set size has exactly one position with
// output -- the common case for segments with few matches.  Other segments
// are marked as having many events (the emit pass walks their quarters).
template <int CH>
__device__ __forceinline__ void walk_count_h16(const HotTable16 &tab, const UText &txt,
                                               uint32_t fo, uint32_t chunk, uint32_t warm,
                                               const ChainIn (&in)[CH],
                                               u32x4 *__restrict__ seg_state,
                                               uint32_t *__restrict__ seg_m, ChunkOut (&r)[CH]) {
    constexpr uint32_t SPW = 16;          // bases per text word
    constexpr uint32_t WPS = kSeg / SPW;  // words per segment (one per quarter)
    static_assert(WPS == 4 && kQuarter == SPW, "a quarter segment is one text word");
    const uint32_t wpc = chunk / SPW, spc = chunk / kSeg;
    uint32_t s[CH], w0[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        w0[c] = in[c].j * wpc;
        s[c] = 0;
        r[c] = ChunkOut{0, 0, 0};
    }
    // Text comes in batches: the warm-up words and each group of four
    // segments (256 bases) are loaded together, so the walk waits for text
    // once per group -- on gfx9 the wait for a table lookup also waits for
    // every older load, so a load per segment would stall once per segment.
    constexpr uint32_t G = 4;
    u32x4 ct[CH][G];
    auto load_group = [&](uint32_t g0) {
#pragma unroll
        for (int c = 0; c < CH; ++c)
#pragma unroll
            for (uint32_t p = 0; p < G; ++p)
                ct[c][p] = g0 + p < spc ? txt.vec_once(w0[c] + WPS * (g0 + p)) : u32x4{0, 0, 0, 0};
    };
    auto warm_word = [&](uint32_t x[CH], const bool live[CH]) {
#pragma unroll
        for (uint32_t k = 0; k < SPW; ++k) {
            uint32_t a[CH], ns[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) a[c] = __builtin_amdgcn_ubfe(x[c], 2 * k, 2) << 2 | s[c];
            tab.step<CH>(a, ns);
#pragma unroll
            for (int c = 0; c < CH; ++c) s[c] = live[c] ? ns[c] & kRowBits : s[c];
        }
    };
    if (warm <= 2) {
        // (patterns of up to 33 bases) the warm-up words with the first group
        uint32_t wx[CH][2];
#pragma unroll
        for (int c = 0; c < CH; ++c)
#pragma unroll
            for (uint32_t i = 0; i < 2; ++i)
                wx[c][i] = i < warm ? txt.word((int)w0[c] - (int)warm + (int)i) : 0u;
        load_group(0);
        for (uint32_t i = 0; i < warm; ++i) {
            uint32_t x[CH];
            bool live[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                x[c] = i == 0 ? wx[c][0] : wx[c][1];
                live[c] = (int)w0[c] - (int)warm + (int)i >= 0;
            }
            warm_word(x, live);
        }
    } else {
        for (uint32_t i = 0; i < warm; ++i) {
            uint32_t x[CH];
            bool live[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int w = (int)w0[c] - (int)warm + (int)i;
                x[c] = txt.word(w);
                live[c] = w >= 0;
            }
            warm_word(x, live);
        }
        load_group(0);
    }
    for (uint32_t g = 0; g < spc; ++g) {
        const uint32_t gi = g % G;
        if (gi == 0 && g > 0) load_group(g);
        uint32_t qs[CH][4], sm[CH], he[CH], hq[CH];
        u32x4 x4[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            sm[c] = 0;
            he[c] = 0;  // an output entry | its position in the word (0: none yet)
            hq[c] = 0;  // the word it was seen in
            x4[c] = gi == 0 ? ct[c][0] : gi == 1 ? ct[c][1] : gi == 2 ? ct[c][2] : ct[c][3];
        }
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t p0 = (g * WPS + q) * SPW;
            bool part = false;
            uint32_t hw[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                qs[c][q] = s[c];
                hw[c] = 0;
                part = part || (in[c].lim != 0 && p0 + SPW > in[c].lim);
            }
            if (!part) {
#pragma unroll
                for (uint32_t k = 0; k < SPW; ++k) {
                    uint32_t a[CH], ns[CH];
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        a[c] = __builtin_amdgcn_ubfe(x4[c][q], 2 * k, 2) << 2 | s[c];
                    tab.step<CH>(a, ns);
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        sm[c] += ns[c] >> 24;
                        hw[c] = max(hw[c], ns[c] | k);
                        s[c] = ns[c] & kRowBits;
                    }
                }
            } else {
                // the text ends inside (or before) this word
#pragma unroll
                for (uint32_t k = 0; k < SPW; ++k) {
                    uint32_t a[CH], ns[CH];
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        a[c] = __builtin_amdgcn_ubfe(x4[c][q], 2 * k, 2) << 2 | s[c];
                    tab.step<CH>(a, ns);
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const bool ok = p0 + k < in[c].lim;
                        sm[c] += ok ? ns[c] >> 24 : 0u;
                        hw[c] = ok ? max(hw[c], ns[c] | k) : hw[c];
                        s[c] = ns[c] & kRowBits;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const bool hit = hw[c] > kRowBits;
                he[c] = hit ? hw[c] : he[c];
                hq[c] = hit ? q : hq[c];
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (in[c].lim == 0) sm[c] = 0;  // a lane past the tile's last chunk
            if (sm[c]) {
                r[c].mask |= 1u << g;
                u32x4 *rec = seg_state + 2 * (in[c].seg0 + g);
                rec[0] = u32x4{qs[c][0], qs[c][1], qs[c][2], qs[c][3]};
                // one position with output: its event (set index, position)
                const bool one = sm[c] == he[c] >> 24;
                const uint32_t o = (((he[c] & kRowBits) >> 4) - (fo >> 4));
                rec[1] = u32x4{one && o <= kEvMaxSet ? o << 6 | hq[c] * SPW | (he[c] & 15u)
                                                     : kEvMany,
                               kEvNone, kEvNone, kEvNone};
                seg_m[in[c].seg0 + g] = sm[c];
                r[c].dense += sm[c] >= kDenseMatches;
            }
            r[c].m += sm[c];
        }
    }
}

// The same walk over 2-bit DNA with the two-symbol table in LDS: one lookup
// per two bases.  An entry is the row offset of the state after both
// symbols (state * 64) with bit 31 set when the state after the first symbol
// has an output set, so a running max over the entries of a word exceeds the
// first output row offset exactly when some state entered in the word has
// an output set.  For such a word the states after the first symbol of the
// flagged pairs are read from the single-symbol table (all at once), then
// the output-set sizes of every state entered.  Quarter
// states are stored as single-symbol row offsets, which the emit kernels
// read.
template <int CH>
__device__ __forceinline__ void walk_count2(rsrc_t g1, const UText &txt,
                                            const uint32_t *__restrict__ out_size,
                                            uint32_t out_size_bytes, uint32_t fo1,
                                            uint32_t fo2, uint32_t fo_state, uint32_t tz,
                                            uint32_t inv, uint32_t chunk, uint32_t warm,
                                            const ChainIn (&in)[CH], u32x4 *__restrict__ seg_state,
                                            uint32_t *__restrict__ seg_m, ChunkOut (&r)[CH]) {
    constexpr uint32_t SPW = 16;          // bases per text word
    constexpr uint32_t WPS = kSeg / SPW;  // words per segment (4)
    constexpr uint32_t kMask = 0x7FFFFFFFu;
    const uint32_t wpc = chunk / SPW, spc = chunk / kSeg;
    const rsrc_t sizes = make_rsrc(out_size, out_size_bytes);
    uint32_t s[CH], w0[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        w0[c] = in[c].j * wpc;
        s[c] = 0;
        r[c] = ChunkOut{0, 0, 0};
    }
    for (uint32_t i = 0; i < warm; ++i) {
        uint32_t x[CH];
        bool live[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int w = (int)w0[c] - (int)warm + (int)i;
            x[c] = txt.word(w);
            live[c] = w >= 0;
        }
#pragma unroll
        for (uint32_t k = 0; k < SPW / 2; ++k) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const uint32_t ns = lds_load(s[c] + ((x[c] >> (4 * k)) & 15u) * 4u) & kMask;
                s[c] = live[c] ? ns : s[c];
            }
        }
    }
    constexpr uint32_t PD = 2;  // segments of text in flight ahead of the walk
    u32x4 nx[CH][PD];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (uint32_t p = 0; p < PD; ++p)
            nx[c][p] = 4 * p < wpc ? txt.vec_once(w0[c] + 4 * p) : u32x4{0, 0, 0, 0};
    for (uint32_t g = 0; g < spc; ++g) {
        uint32_t qs[CH][4], sm[CH], ev[CH][kEvSlots], ne[CH];
        u32x4 x4[CH];
        const uint32_t wn = g * WPS + 4 * PD;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            sm[c] = 0;
            ne[c] = 0;
#pragma unroll
            for (uint32_t e = 0; e < kEvSlots; ++e) ev[c][e] = kEvNone;
            x4[c] = nx[c][0];
#pragma unroll
            for (uint32_t p = 0; p + 1 < PD; ++p) nx[c][p] = nx[c][p + 1];
            if (wn < wpc) nx[c][PD - 1] = txt.vec_once(w0[c] + wn);
        }
#pragma unroll
        for (uint32_t q = 0; q < WPS; ++q) {
            uint32_t acc[CH], s_in[CH], pe[CH][SPW / 2];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                s_in[c] = s[c];
                qs[c][q] = s[c] >> 2;  // single-symbol row offset
                acc[c] = 0;
            }
#pragma unroll
            for (uint32_t k = 0; k < SPW / 2; ++k) {
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const uint32_t e = lds_load(s[c] + ((x4[c][q] >> (4 * k)) & 15u) * 4u);
                    pe[c][k] = e;
                    acc[c] = acc[c] > e ? acc[c] : e;
                    s[c] = e & kMask;
                }
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                if (acc[c] >= fo2) {
                    // single-symbol states of the word: the state after each
                    // pair is known; the one after the first symbol of a
                    // flagged pair is read from the single-symbol table, all
                    // such reads issued together
                    const uint32_t p0 = (g * WPS + q) * SPW;
                    uint32_t t1[SPW];
#pragma unroll
                    for (uint32_t k = 0; k < SPW / 2; ++k) {
                        const uint32_t prev = (k ? pe[c][k - 1] & kMask : s_in[c]) >> 2;
                        const uint32_t a1 = (x4[c][q] >> (4 * k)) & 3u;
                        t1[2 * k] = (pe[c][k] & ~kMask) ? buf_load(g1, prev + a1 * 4u) : 0u;
                        t1[2 * k + 1] = (pe[c][k] & kMask) >> 2;
                    }
                    uint32_t o[SPW], sz[SPW];
#pragma unroll
                    for (uint32_t k = 0; k < SPW; ++k) {
                        const bool hit = t1[k] >= fo1 && p0 + k < in[c].lim;
                        o[k] = hit ? (t1[k] >> 4) - fo_state : kEvNone;
                        sz[k] = buf_load(sizes, hit ? o[k] * 4u : 0xFFFFFFF0u);
                    }
#pragma unroll
                    for (uint32_t k = 0; k < SPW; ++k) {
                        sm[c] += sz[k];
                        if (o[k] != kEvNone) {
                            const uint32_t e = o[k] <= kEvMaxSet ? o[k] << 6 | (q * SPW + k)
                                                                 : kEvMany;
#pragma unroll
                            for (uint32_t u = 0; u < kEvSlots; ++u)
                                ev[c][u] = ne[c] == u ? e : ev[c][u];
                            ne[c] = e == kEvMany ? kEvSlots + 1 : ne[c] + 1;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (sm[c]) {
                r[c].mask |= 1u << g;
                u32x4 *rec = seg_state + 2 * (in[c].seg0 + g);
                rec[0] = u32x4{qs[c][0], qs[c][1], qs[c][2], qs[c][3]};
                rec[1] = ne[c] <= kEvSlots ? u32x4{ev[c][0], ev[c][1], ev[c][2], ev[c][3]}
                                           : u32x4{kEvMany, kEvNone, kEvNone, kEvNone};
                seg_m[in[c].seg0 + g] = sm[c];
                r[c].dense += sm[c] >= kDenseMatches;
            }
            r[c].m += sm[c];
        }
    }
}

// Copy the LDS part of a table (zero-filled past the table's end).  Each
// thread has 16 dword loads in flight before its first LDS write, so a
// 160 KB table takes a few memory latencies rather than one per 4 KB.
__device__ __forceinline__ void load_lds_table(rsrc_t g, uint32_t bytes, uint32_t lds_off = 0) {
    extern __shared__ uint32_t dyn_smem[];
    constexpr uint32_t U = 4;
    const uint32_t step = blockDim.x * 16u;
    for (uint32_t base = threadIdx.x * 16u; base < bytes; base += U * step) {
        uint32_t v[U][4];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) v[u][i] = buf_load(g, base + u * step + 4u * i);
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) {
                const uint32_t o = base + u * step + 4u * i;
                if (o < bytes) ((lds_u32 *)dyn_smem)[(lds_off + o) >> 2] = v[u][i];
            }
    }
}

// Persistent count kernel.  Block b takes a contiguous range of tiles; a
// tile is CH * blockDim.x consecutive chunks of one instance: lane t walks
// chunks first + t * CH + c for c < CH.
// MODE selects the placements the kernel is compiled for: kCountAny (all,
// chosen per instance), kCountLds (whole table in LDS) or kCountHybrid (hot
// rows in LDS, the rest from L2).  Without the other placements' code a
// kernel needs fewer registers: more waves or more chains per lane fit.
constexpr int kCountAny = 0, kCountLds = 1, kCountHybrid = 2;
template <int FMT, bool BATCH, int CH, int MODE = kCountAny>
__global__ __launch_bounds__(kMaxCountThreads) void k_count(
    Inst single, const Inst *__restrict__ insts, const TileDesc *__restrict__ tiles,
    uint32_t t_base, uint32_t n_tiles, uint32_t red_off,
    uint32_t *__restrict__ cnt,
    uint32_t *__restrict__ mask, u32x4 *__restrict__ seg_state, uint32_t *__restrict__ seg_m,
    unsigned long long *__restrict__ tile_m, uint32_t *__restrict__ tile_zs,
    uint32_t *__restrict__ tile_zd) {
    // block reduction slots after the LDS table (the kernel has no static
    // LDS, so the table starts at LDS address 0)
    extern __shared__ uint32_t dyn_smem[];
    typedef __attribute__((address_space(3))) unsigned long long lds_u64;
    lds_u64 *red_a = (lds_u64 *)((lds_u8 *)(lds_u32 *)dyn_smem + red_off);
    lds_u32 *red_b = (lds_u32 *)((lds_u8 *)(lds_u32 *)dyn_smem + red_off + 128u);
    lds_u32 *red_c = red_b + 16;
    // this launch covers tiles t_base .. t_base + n_tiles - 1
    const uint32_t t0 = t_base + (uint32_t)(((uint64_t)n_tiles * blockIdx.x) / gridDim.x);
    const uint32_t t1 = t_base + (uint32_t)(((uint64_t)n_tiles * (blockIdx.x + 1)) / gridDim.x);
    int cur = -1;
    for (uint32_t t = t0; t < t1; ++t) {
        uint32_t inst = 0, first, count;
        if constexpr (BATCH) {
            const TileDesc td = tiles[t];
            inst = uniform(td.inst);
            first = uniform(td.first);
            count = uniform(td.count);
        } else {
            first = t * blockDim.x * CH;
            count = min(blockDim.x * CH, single.n_chunks - first);
        }
        const Inst &I = BATCH ? insts[inst] : single;
        const uint32_t table_bytes = uniform(I.table_bytes);
        const uint32_t hot = uniform(I.hot_bytes);
        const uint32_t lds_all = uniform(I.lds_all);
        const uint32_t row = uniform(I.sigma) * 4u;
        const rsrc_t gtab = make_rsrc(uniform(I.delta), table_bytes);
        if ((int)inst != cur) {
            if (hot) {
                const uint32_t lb = uniform(I.lds_bytes);
                __syncthreads();
                if (uniform(I.stride2))
                    load_lds_table(make_rsrc(uniform(I.delta2), lb), lb);
                else if (lds_all == 2)
                    load_lds_table(make_rsrc(uniform(I.tab16), table_bytes >> 1), lb);
                else if (lds_all)
                    load_lds_table(gtab, lb);
                else  // 16-bit rows, then zeros up to lb
                    load_lds_table(make_rsrc(MODE == kCountHybrid && FMT == AC_TEXT_2BIT
                                                 ? uniform(I.hot16c)
                                                 : uniform(I.hot16),
                                             ((hot >> 1) + 3u) & ~3u),
                                   lb);
                __syncthreads();
            }
            cur = (int)inst;
        }
        const uint32_t n = uniform(I.n);
        const uint32_t tb4 = uniform(I.text_bytes4);
        const UText txt{make_rsrc(uniform(I.text), tb4), tb4};
        const uint32_t *out_size = uniform(I.out_size);
        const uint32_t fo = uniform(I.fo_bytes), fos = uniform(I.fo_state);
        // bytes of the output-set sizes (one entry per output state)
        const uint32_t size_bytes = (uniform(I.table_bytes) / row - fos) * 4u;
        const uint32_t tz = uniform(I.div_tz), inv = uniform(I.div_inv);
        const uint32_t cbase = uniform(I.chunk_base);
        const uint32_t chunk = uniform(I.chunk), warm = uniform(I.warm);
        const uint32_t spc = chunk / kSeg, sbase = uniform(I.seg_base);
        ChainIn in[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const uint32_t k = threadIdx.x * CH + c;
            const bool valid = k < count;
            in[c].j = valid ? first + k : first;
            const uint64_t begin = (uint64_t)in[c].j * chunk;
            in[c].lim = valid ? (uint32_t)min<uint64_t>(chunk, n - begin) : 0u;
            in[c].seg0 = sbase + in[c].j * spc;
        }
        ChunkOut co[CH];
        bool done = false;
        if constexpr (MODE == kCountLds) {
            if (lds_all == 2)
                walk_count<FMT, PL_LDS16, CH, FMT == AC_TEXT_2BIT>(
                    UTable<PL_LDS16, FMT == AC_TEXT_2BIT>{gtab, hot, row}, txt, out_size,
                    size_bytes, fo, fos, tz, inv, chunk, warm, in, seg_state, seg_m, co);
            else
                walk_count<FMT, PL_LDS, CH>(UTable<PL_LDS>{gtab, hot, row}, txt, out_size,
                                            size_bytes, fo, fos, tz, inv, chunk, warm, in,
                                            seg_state, seg_m, co);
            done = true;
        } else if constexpr (MODE == kCountHybrid) {
            if constexpr (FMT == AC_TEXT_2BIT)
                walk_count_h16<CH>(HotTable16{make_rsrc(uniform(I.delta_sz), table_bytes),
                                           make_rsrc((const uint8_t *)uniform(I.delta_sz) + hot,
                                                     table_bytes - hot),
                                           hot},
                                   txt, fo, chunk, warm, in, seg_state, seg_m, co);
            else
                walk_count<FMT, PL_HYBRID, CH>(UTable<PL_HYBRID>{gtab, hot, row}, txt, out_size,
                                               size_bytes, fo, fos, tz, inv, chunk, warm, in,
                                               seg_state, seg_m, co);
            done = true;
        } else if constexpr (FMT == AC_TEXT_2BIT) {
            if (uniform(I.stride2)) {
                walk_count2<CH>(gtab, txt, out_size, size_bytes, fo, uniform(I.fo2_bytes), fos, tz,
                                inv, chunk, warm, in, seg_state, seg_m, co);
                done = true;
            }
        }
        if (done) {
        } else if (lds_all == 2) {
            walk_count<FMT, PL_LDS16, CH, FMT == AC_TEXT_2BIT>(
                UTable<PL_LDS16, FMT == AC_TEXT_2BIT>{gtab, hot, row}, txt, out_size, size_bytes,
                fo, fos, tz, inv, chunk, warm, in, seg_state, seg_m, co);
        } else if (lds_all) {
            walk_count<FMT, PL_LDS, CH>(UTable<PL_LDS>{gtab, hot, row}, txt, out_size, size_bytes,
                                        fo, fos, tz, inv, chunk, warm, in, seg_state, seg_m, co);
        } else if (hot == 0) {
            walk_count<FMT, PL_GLOBAL, CH>(UTable<PL_GLOBAL>{gtab, 0, row}, txt, out_size,
                                           size_bytes, fo, fos, tz, inv, chunk, warm, in,
                                           seg_state, seg_m, co);
        } else {
            // 2-bit text means sigma 4: a row is 16 bytes, an id becomes a
            // row offset by a shift
            walk_count<FMT, PL_HYBRID, CH, FMT == AC_TEXT_2BIT>(
                UTable<PL_HYBRID, FMT == AC_TEXT_2BIT>{gtab, hot, row}, txt, out_size, size_bytes,
                fo, fos, tz, inv, chunk, warm, in, seg_state, seg_m, co);
        }
        unsigned long long m = 0;
        uint32_t zs = 0, zd = 0;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (threadIdx.x * CH + c < count) {
                cnt[cbase + in[c].j] = co[c].m;
                mask[cbase + in[c].j] = co[c].mask;
            }
            m += co[c].m;
            zs += __builtin_popcount(co[c].mask) - co[c].dense;
            zd += co[c].dense;
        }
        // tile totals: matches, sparse and dense segments
        const unsigned long long wa = wave_sum_u64(m);
        const uint32_t wb = wave_sum_u32(zs), wc = wave_sum_u32(zd);
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) {
            red_a[wid] = wa;
            red_b[wid] = wb;
            red_c[wid] = wc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long a = 0;
            uint32_t b = 0, d = 0;
            for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
                a += red_a[w];
                b += red_b[w];
                d += red_c[w];
            }
            tile_m[t] = a;
            tile_zs[t] = b;
            tile_zd[t] = d;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ offsets

// One block: exclusive offsets of the tile totals.  totals[0] = matches,
// totals[1] = sparse segments, totals[2] = dense segments; entry n of each
// offset array holds the grand total.
__global__ __launch_bounds__(1024) void k_tile_scan(
    const unsigned long long *__restrict__ tile_m, const uint32_t *__restrict__ tile_zs,
    const uint32_t *__restrict__ tile_zd, uint32_t n, unsigned long long *tile_moff,
    uint32_t *tile_zsoff, uint32_t *tile_zdoff, unsigned long long *totals,
    unsigned long long *single_count) {
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t b = min(n, threadIdx.x * per), e = min(n, b + per);
    Scan3 v = {0, 0, 0};
    for (uint32_t i = b; i < e; ++i) {
        v.a += tile_m[i];
        v.b += tile_zs[i];
        v.c += tile_zd[i];
    }
    Scan3 ex, tot;
    block_excl_scan3(v, &ex, &tot);
    for (uint32_t i = b; i < e; ++i) {
        tile_moff[i] = ex.a;
        tile_zsoff[i] = ex.b;
        tile_zdoff[i] = ex.c;
        ex.a += tile_m[i];
        ex.b += tile_zs[i];
        ex.c += tile_zd[i];
    }
    if (threadIdx.x == 0) {
        tile_moff[n] = tot.a;
        tile_zsoff[n] = tot.b;
        tile_zdoff[n] = tot.c;
        totals[0] = tot.a;
        totals[1] = tot.b;
        totals[2] = tot.c;
        if (single_count) *single_count = tot.a;
    }
}

// One block per tile: append every segment with matches to the work list,
// with its entry state and the offset of its first match (relative to its
// instance's output).  Sparse segments fill the list from the front in text
// order, dense ones follow all sparse ones, also in text order.  Thread t
// handles the tile's chunks t * per .. t * per + per - 1.
template <bool BATCH>
__global__ __launch_bounds__(kMaxCountThreads) void k_scatter(
    Inst single, const Inst *__restrict__ insts, const TileDesc *__restrict__ tiles,
    uint32_t per, const uint32_t *__restrict__ cnt,
    const uint32_t *__restrict__ mask, const u32x4 *__restrict__ seg_state,
    const uint32_t *__restrict__ seg_m, const unsigned long long *__restrict__ tile_moff,
    const uint32_t *__restrict__ tile_zsoff, const uint32_t *__restrict__ tile_zdoff,
    const unsigned long long *__restrict__ totals, uint32_t *__restrict__ list_seg,
    u32x4 *__restrict__ list_state, unsigned long long *__restrict__ list_moff,
    uint32_t *__restrict__ list_inst) {
    const uint32_t t = blockIdx.x;
    uint32_t inst = 0, first, count, cbase = 0;
    unsigned long long base_off = 0;
    if constexpr (BATCH) {
        const TileDesc td = tiles[t];
        inst = td.inst;
        first = td.first;
        count = td.count;
        cbase = insts[inst].chunk_base;
        base_off = tile_moff[insts[inst].first_tile];
    } else {
        first = t * blockDim.x * per;
        count = min(blockDim.x * per, single.n_chunks - first);
    }
    const Inst &I = BATCH ? insts[inst] : single;
    const uint32_t spc = I.chunk / kSeg, sbase = I.seg_base;
    const uint32_t k0 = threadIdx.x * per;
    const uint32_t k1 = min(k0 + per, count);
    unsigned long long m = 0;
    uint32_t zs = 0, zd = 0;
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t g = cbase + first + k;
        m += cnt[g];
        const uint32_t mk = mask[g];
        uint32_t d = 0;
        const uint32_t s0 = sbase + (first + k) * spc;
        for (uint32_t b = mk; b; b &= b - 1) d += seg_m[s0 + __builtin_ctz(b)] >= kDenseMatches;
        zd += d;
        zs += __builtin_popcount(mk) - d;
    }
    Scan3 ex, tot;
    block_excl_scan3(Scan3{m, zs, zd}, &ex, &tot);
    const uint32_t n_sparse = (uint32_t)totals[1];
    uint32_t ks = tile_zsoff[t] + ex.b;
    uint32_t kd = n_sparse + tile_zdoff[t] + ex.c;
    unsigned long long off = tile_moff[t] + ex.a - base_off;
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t j = first + k;
        const uint32_t g = cbase + j;
        for (uint32_t b = mask[g]; b; b &= b - 1) {
            const uint32_t i = __builtin_ctz(b);
            const uint32_t gs = sbase + j * spc + i;
            const uint32_t sm = seg_m[gs];
            const uint32_t kk = sm >= kDenseMatches ? kd++ : ks++;
            list_seg[kk] = j * spc + i;
            list_state[kk] = seg_state[2 * gs];
            list_moff[kk] = off;
            if constexpr (BATCH) list_inst[kk] = inst;
            off += sm;
        }
    }
}

__global__ void k_inst_totals(const Inst *__restrict__ insts, uint32_t n_inst,
                              const unsigned long long *__restrict__ tile_moff) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const Inst &I = insts[i];
    *I.count = tile_moff[I.first_tile + I.n_tiles] - tile_moff[I.first_tile];
}

__global__ void k_fill_u64(unsigned long long *p, uint32_t n, unsigned long long v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ emit

// Write the output set ids[a .. a+len) of a state entered at end position e
// into out[off ..], skipping slots >= cap.  Ids are fetched 16 at a time so
// that one memory latency covers 16 matches.
__device__ __forceinline__ void write_set(ac_match *__restrict__ out, unsigned long long off,
                                          unsigned long long cap,
                                          const uint32_t *__restrict__ ids, uint32_t a,
                                          uint32_t len, uint32_t e) {
    constexpr uint32_t B = 16;
    for (uint32_t i = 0; i < len; i += B) {
        uint32_t v[B];
#pragma unroll
        for (uint32_t u = 0; u < B; ++u) v[u] = (i + u < len) ? ids[a + i + u] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < B; ++u) {
            const unsigned long long d = off + i + u;
            if (i + u < len && d < cap) {
                ac_match m;
                m.pattern_id = v[u];
                m.end_pos = e;
                out[d] = m;
            }
        }
    }
}

// One listed sparse segment, four lanes (lane q = quarter q; `act` false on
// lanes past the list, which still take part in the shuffles).  With up to
// four kept events lane q writes event q; otherwise lane q walks quarter q
// (16 symbols) from the state the count pass stored for it, so a segment
// costs 16 dependent lookups instead of 64.  A walking lane records its
// output events (state, position) in LDS during the walk -- at most one per
// position, so 16 slots always suffice -- and writes after the walk: on gfx9
// a wave's wait for a load also waits for its earlier stores, so a store
// inside the lookup chain would stall every later step.  The four lanes are
// adjacent in the wave; the offset of each quarter's first match is an
// exclusive sum of the quarters' match counts over them.  Within a quarter,
// events are written in position order and each output set in id order,
// which is the (end, id) order.
constexpr uint32_t kEmitThreads = 256;

template <int FMT, bool BATCH>
__device__ __forceinline__ void emit_group(const Inst &single, const Inst *__restrict__ insts,
                                           const uint32_t *__restrict__ list_seg,
                                           const u32x4 *__restrict__ list_state,
                                           const unsigned long long *__restrict__ list_moff,
                                           const uint32_t *__restrict__ list_inst,
                                           const u32x4 *__restrict__ seg_rec, bool act,
                                           uint32_t idx, uint32_t q, uint32_t tid,
                                           uint32_t (*ev_set)[kEmitThreads],
                                           uint8_t (*ev_pos)[kEmitThreads]) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    constexpr uint32_t WPS = kSeg / SPW;
    constexpr uint32_t WPQ = kQuarter / SPW;  // text words per quarter
    uint32_t ne = 0, matches = 0;
    uint32_t e0 = 0;
    unsigned long long off0 = 0;
    if (act) {
        const uint32_t inst = BATCH ? list_inst[idx] : 0u;
        const Inst &I = BATCH ? insts[inst] : single;
        const uint32_t seg = list_seg[idx];
        const u32x4 qs = list_state[idx];
        off0 = list_moff[idx];
        e0 = seg * kSeg;
        const uint32_t lim = min(kSeg, I.n - e0);
        const uint32_t fo = I.fo_bytes, fos = I.fo_state, tz = I.div_tz, inv = I.div_inv;
        const uint32_t *out_off = I.out_off;
        const u32x4 evs = seg_rec[2 * (I.seg_base + seg) + 1];
        auto walk = [&](const auto &tab, const auto &txt) {
            uint32_t st = q == 0 ? qs.x : q == 1 ? qs.y : q == 2 ? qs.z : qs.w;
#pragma unroll
            for (uint32_t w = 0; w < WPQ; ++w) {
                const uint32_t x = txt.word((int)(seg * WPS + q * WPQ + w));
#pragma unroll
                for (uint32_t k = 0; k < SPW; ++k) {
                    st = tab(st + sym_bytes<FMT>(x, k));
                    const uint32_t p = q * kQuarter + w * SPW + k;
                    if (st >= fo && p < lim) {
                        ev_set[ne][tid] = row_state(st, tz, inv) - fos;
                        ev_pos[ne][tid] = (uint8_t)p;
                        ++ne;
                    }
                }
            }
        };
        if (evs.x != kEvMany) {
            // the count pass's events: event q for lane q
            const uint32_t e = q == 0 ? evs.x : q == 1 ? evs.y : q == 2 ? evs.z : evs.w;
            if (e != kEvNone) {
                ev_set[0][tid] = e >> 6;
                ev_pos[0][tid] = (uint8_t)(e & 63u);
                ne = 1;
            }
        } else if constexpr (BATCH) {
            walk(LTable{I.delta, I.table_bytes}, LText{(const uint32_t *)I.text, I.text_bytes4});
        } else {
            walk(emit_table(single.delta, single.delta_sz, single.walk_sz, single.table_bytes),
                 UText{make_rsrc(single.text, single.text_bytes4), single.text_bytes4});
        }
        for (uint32_t j = 0; j < ne; ++j) {
            const uint32_t o = ev_set[j][tid];
            matches += out_off[o + 1] - out_off[o];
        }
    }
    // exclusive sum over the quarters before this one
    const uint32_t m1 = __shfl_up(matches, 1, 64);
    const uint32_t m2 = __shfl_up(matches, 2, 64);
    const uint32_t m3 = __shfl_up(matches, 3, 64);
    const uint32_t before = (q >= 1 ? m1 : 0u) + (q >= 2 ? m2 : 0u) + (q >= 3 ? m3 : 0u);
    if (act && ne) {
        const Inst &I = BATCH ? insts[list_inst[idx]] : single;
        const uint32_t *out_off = I.out_off;
        unsigned long long off = off0 + before;
        for (uint32_t j = 0; j < ne; ++j) {
            const uint32_t o = ev_set[j][tid];
            const uint32_t a = out_off[o], len = out_off[o + 1] - a;
            write_set(I.out, off, I.capacity, I.out_ids, a, len, e0 + ev_pos[j][tid]);
            off += len;
        }
    }
}

// Sparse part of the work list.  A single scan gives each listed segment one
// lane first: when the count pass kept a single output event for it (the
// common case), the lane writes that set itself and no text is read; the
// wave then takes its other segments four lanes each (emit_group).  A batch
// (whose count walk keeps up to four events, so that multi-event segments
// are common) gives every segment four lanes from the start.
template <int FMT, bool BATCH>
__global__ __launch_bounds__(kEmitThreads) void k_emit(
    Inst single, const Inst *__restrict__ insts, const uint32_t *__restrict__ list_seg,
    const u32x4 *__restrict__ list_state, const unsigned long long *__restrict__ list_moff,
    const uint32_t *__restrict__ list_inst, const unsigned long long *__restrict__ totals,
    const u32x4 *__restrict__ seg_rec) {
    __shared__ uint32_t ev_set[kQuarter][kEmitThreads];
    __shared__ uint8_t ev_pos[kQuarter][kEmitThreads];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, wbase = tid - lane;
    const uint32_t q = lane & 3;
    const uint32_t items = (uint32_t)totals[1];
    // the loop bounds are uniform over the wave, so every lane of a group
    // takes part in the group's shuffles
    if constexpr (BATCH) {
        for (uint32_t base = blockIdx.x * blockDim.x + wbase; base < 4u * items;
             base += gridDim.x * blockDim.x) {
            const uint32_t li = base + lane;
            emit_group<FMT, BATCH>(single, insts, list_seg, list_state, list_moff, list_inst,
                                   seg_rec, li < 4u * items, li >> 2, q, tid, ev_set, ev_pos);
        }
    } else {
        __shared__ uint32_t group_lane[kEmitThreads];  // per wave: lane of its r-th group segment
        for (uint32_t base = blockIdx.x * blockDim.x + wbase; base < items;
             base += gridDim.x * blockDim.x) {
            const uint32_t li = base + lane;
            bool group = false;
            if (li < items) {
                const uint32_t seg = list_seg[li];
                const u32x4 evs = seg_rec[2 * (single.seg_base + seg) + 1];
                if (evs.x == kEvMany || evs.y != kEvNone) {
                    group = true;
                } else if (evs.x != kEvNone) {
                    const uint32_t a = single.out_off[evs.x >> 6];
                    const uint32_t len = single.out_off[(evs.x >> 6) + 1] - a;
                    write_set(single.out, list_moff[li], single.capacity, single.out_ids, a, len,
                              seg * kSeg + (evs.x & 63u));
                }
            }
            const uint64_t gm = __ballot(group);
            if (group) group_lane[wbase + __builtin_popcountll(gm & ((1ull << lane) - 1))] = lane;
            wave_sync();
            const uint32_t n_group = (uint32_t)__builtin_popcountll(gm);
            for (uint32_t r0 = 0; r0 < n_group; r0 += 16) {
                const uint32_t r = r0 + (lane >> 2);
                const bool act = r < n_group;
                emit_group<FMT, BATCH>(single, insts, list_seg, list_state, list_moff, list_inst,
                                       seg_rec, act, act ? base + group_lane[wbase + r] : 0u, q,
                                       tid, ev_set, ev_pos);
            }
            // every lane has read this round's entries before the next round
            // writes them
            wave_sync();
        }
    }
}

// Dense part of the work list.  A wave takes kDenseBatch listed segments at
// once.  For each of them, four groups of 16 lanes walk the segment's four
// quarters from the states the count pass stored (16 dependent lookups per
// quarter); the segments' walks are independent chains, interleaved, so one
// walk latency serves the whole batch.  Lane k of group g keeps the state
// entered at position 16 g + k.  Only then are the batch's records written:
// on gfx9 a wave's wait for a load also waits for its earlier stores, so
// walking between the stores of consecutive segments would pay the store
// drain and the walk latency per segment.
//
// A segment's positions are written as runs of equal states (a poly-A run
// is one long run of the deepest all-A state): a run of r positions whose
// set has L ids is r * L consecutive slots, item t of the run being id
// t % L at end position first + t / L.  The wave writes the run
// item-parallel, lane i taking items i, i + 64, ... (with a trip count
// uniform over the wave, so no lane is inactive during a shuffle), so every
// store instruction covers 64 consecutive 8-byte slots; the run's ids sit in
// two registers per lane and are picked with a wave shuffle (an LDS-path
// operation, which does not wait for the wave's stores the way a memory
// load would).  Sets longer than 128 ids take a slower path that loads them
// per position.
constexpr uint32_t kDenseThreads = 256;
constexpr uint32_t kDenseBatch = 4;

// Records of one dense segment.  Lane l holds `mine`, the state entered at
// position l, and (a, len), where its output set starts in the id array
// and its size (len 0: no output, or past the text).
__device__ __forceinline__ void dense_runs(uint32_t mine, uint32_t a, uint32_t len,
                                           uint32_t lane, uint32_t e0, unsigned long long off0,
                                           unsigned long long cap,
                                           const uint32_t *__restrict__ ids,
                                           ac_match *__restrict__ out) {
    const bool has = len != 0;
    const uint32_t excl = wave_incl_scan(len) - len;
    // runs: a run starts at an output position whose predecessor is in a
    // different state or has no output; it ends before the next start or
    // the next position without output
    const uint32_t prev = __shfl_up(mine, 1, 64);
    const bool prev_has = __shfl_up((uint32_t)has, 1, 64) != 0;
    const bool start = has && (lane == 0 || !prev_has || prev != mine);
    uint64_t starts = __ballot(start);
    const uint64_t stops = __ballot(start || !has);
    while (starts) {
        const uint32_t k = (uint32_t)__builtin_ctzll(starts);
        starts &= starts - 1;
        const uint64_t after = stops & ~((2ull << k) - 1ull);  // bits above k
        const uint32_t kend = after ? (uint32_t)__builtin_ctzll(after) : 64u;
        const uint32_t r = kend - k;
        const uint32_t L = __builtin_amdgcn_readlane(len, k);
        const uint32_t ka = __builtin_amdgcn_readlane(a, k);
        const unsigned long long ko = off0 + __builtin_amdgcn_readlane(excl, k);
        if (ko >= cap) break;
        const uint32_t T = r * L;
        const uint32_t e = e0 + k;
        if (L <= 128) {
            uint32_t v0 = 0, v1 = 0;
            if (L <= 16) {
                // wave-uniform reads through the scalar cache: they do not
                // wait for this wave's earlier stores as a vector load would
                // (indices past the set repeat its last id: never read past
                // the array)
#pragma unroll
                for (uint32_t j = 0; j < 16; ++j) {
                    const uint32_t x = ids[ka + min(j, L - 1)];
                    v0 = lane == j ? x : v0;
                }
            } else {
                v0 = lane < L ? ids[ka + lane] : 0u;
                v1 = lane + 64 < L ? ids[ka + 64 + lane] : 0u;
            }
            // item t = lane + 64 u of the run is id t % L at position t / L;
            // a step of 64 items moves the id index by dj and the position
            // by di (64 = di * L + dj), plus one when the index wraps.  The
            // index is kept as a byte address for the shuffle.
            const uint32_t di = 64u / L, dj4 = (64u - di * L) * 4u, L4 = L * 4u;
            uint32_t i = lane / L;
            uint32_t ja = (lane - i * L) * 4u;
            // items below lim fit the output (the capacity may cut the run)
            const uint32_t lim = (uint32_t)min<unsigned long long>(T, cap - ko);
            ac_match *const run = out + ko;
            // uniform trip count: every lane takes part in each shuffle
            for (uint32_t base = 0; base < T; base += 64) {
                const uint32_t x0 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)ja, (int)v0);
                uint32_t id = x0;
                if (L > 64) {
                    const uint32_t x1 =
                        (uint32_t)__builtin_amdgcn_ds_bpermute((int)(ja & 255u), (int)v1);
                    id = ja < 256u ? x0 : x1;
                }
                if (base + lane < lim) {
                    ac_match m;
                    m.pattern_id = id;
                    m.end_pos = e + i;
                    run[base + lane] = m;
                }
                ja += dj4;
                i += di;
                if (ja >= L4) {
                    ja -= L4;
                    ++i;
                }
            }
        } else {
            for (uint32_t i = 0; i < r; ++i) {
                for (uint32_t j = lane; j < L; j += 64) {
                    const unsigned long long d = ko + (unsigned long long)i * L + j;
                    if (d < cap) {
                        ac_match m;
                        m.pattern_id = ids[ka + j];
                        m.end_pos = e + i;
                        out[d] = m;
                    }
                }
            }
        }
    }
}

// ids1 / out1: a single scan's id array and output, as separate kernel
// arguments so that the compiler knows the stores never touch the ids and
// reads a run's ids through the scalar cache (batches use each instance's).
template <int FMT, bool BATCH>
__global__ __launch_bounds__(kDenseThreads) void k_emit_dense(
    Inst single, const Inst *__restrict__ insts, const uint32_t *__restrict__ list_seg,
    const u32x4 *__restrict__ list_state, const unsigned long long *__restrict__ list_moff,
    const uint32_t *__restrict__ list_inst, const unsigned long long *__restrict__ totals,
    const uint32_t *__restrict__ ids1, ac_match *__restrict__ out1) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    constexpr uint32_t WPS = kSeg / SPW;
    constexpr uint32_t WPQ = kQuarter / SPW;  // text words per quarter
    constexpr uint32_t B = kDenseBatch;
    const uint32_t n_sparse = (uint32_t)totals[1];
    const uint32_t n_dense = (uint32_t)totals[2];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gq = lane / kQuarter;  // the quarter this lane's group walks
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t w = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * B; w < n_dense;
         w += waves * B) {
        uint32_t idx[B], seg[B], s[B], mine[B];
        MTable tab[B];
        UText txt[B];
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
            // past the list's end a slot walks the batch's first segment again
            // and writes nothing
            idx[b] = n_sparse + (w + b < n_dense ? w + b : w);
            const Inst &I = BATCH ? insts[uniform(list_inst[idx[b]])] : single;
            seg[b] = uniform(list_seg[idx[b]]);
            const u32x4 qs = list_state[idx[b]];
            s[b] = gq == 0 ? uniform(qs.x) : gq == 1 ? uniform(qs.y) : gq == 2 ? uniform(qs.z)
                                                                    : uniform(qs.w);
            mine[b] = 0;
            const uint32_t tb4 = uniform(I.text_bytes4);
            tab[b] = emit_table(uniform(I.delta), uniform(I.delta_sz), uniform(I.walk_sz),
                                uniform(I.table_bytes));
            txt[b] = UText{make_rsrc(uniform(I.text), tb4), tb4};
        }
#pragma unroll
        for (uint32_t wq = 0; wq < WPQ; ++wq) {
            uint32_t x[B];
#pragma unroll
            for (uint32_t b = 0; b < B; ++b) x[b] = txt[b].word((int)(seg[b] * WPS + gq * WPQ + wq));
#pragma unroll
            for (uint32_t k = 0; k < SPW; ++k) {
#pragma unroll
                for (uint32_t b = 0; b < B; ++b) {
                    s[b] = tab[b](s[b] + sym_bytes<FMT>(x[b], k));
                    if (lane % kQuarter == wq * SPW + k) mine[b] = s[b];
                }
            }
        }
        // where each position's output set starts and its size, for the
        // whole batch before the first store
        uint32_t a[B], len[B];
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
            const Inst &I = BATCH ? insts[uniform(list_inst[idx[b]])] : single;
            const uint32_t e0 = seg[b] * kSeg;
            const bool has = mine[b] >= uniform(I.fo_bytes) && lane < uniform(I.n) - e0;
            const uint32_t o = has ? row_state(mine[b], uniform(I.div_tz), uniform(I.div_inv)) -
                                         uniform(I.fo_state)
                                   : 0u;
            const uint32_t *out_off = uniform(I.out_off);
            a[b] = has ? out_off[o] : 0u;
            len[b] = has ? out_off[o + 1] : 0u;
        }
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
            if (w + b >= n_dense) break;
            const Inst &I = BATCH ? insts[uniform(list_inst[idx[b]])] : single;
            const unsigned long long off0 = uniform(list_moff[idx[b]]);
            const unsigned long long cap = uniform(I.capacity);
            if (off0 >= cap) continue;
            dense_runs(mine[b], a[b], len[b] - a[b], lane, seg[b] * kSeg, off0, cap,
                       BATCH ? uniform(I.out_ids) : ids1, BATCH ? uniform(I.out) : out1);
        }
    }
}

// Dense emit of a single scan whose output-set tables fit LDS (set offsets,
// then ids): each block copies them into LDS once, and a run then reads its
// ids with LDS loads -- which, unlike memory loads, do not wait for the
// wave's earlier stores -- with no per-run shuffle setup, for sets of any
// size.  Walks, batching and the order of the records are those of
// k_emit_dense.
constexpr uint32_t kDenseLdsThreads = 1024;

__device__ __forceinline__ void dense_runs_lds(uint32_t mine, uint32_t a, uint32_t len,
                                               uint32_t lane, uint32_t e0,
                                               unsigned long long off0, unsigned long long cap,
                                               uint32_t ids_lds, ac_match *__restrict__ out) {
    const bool has = len != 0;
    const uint32_t excl = wave_incl_scan(len) - len;
    const uint32_t prev = __shfl_up(mine, 1, 64);
    const bool prev_has = __shfl_up((uint32_t)has, 1, 64) != 0;
    const bool start = has && (lane == 0 || !prev_has || prev != mine);
    uint64_t starts = __ballot(start);
    const uint64_t stops = __ballot(start || !has);
    while (starts) {
        const uint32_t k = (uint32_t)__builtin_ctzll(starts);
        starts &= starts - 1;
        const uint64_t after = stops & ~((2ull << k) - 1ull);  // bits above k
        const uint32_t kend = after ? (uint32_t)__builtin_ctzll(after) : 64u;
        const uint32_t r = kend - k;
        const uint32_t L = __builtin_amdgcn_readlane(len, k);
        const uint32_t ka = __builtin_amdgcn_readlane(a, k);
        const unsigned long long ko = off0 + __builtin_amdgcn_readlane(excl, k);
        if (ko >= cap) break;
        const uint32_t T = r * L;
        const uint32_t e = e0 + k;
        // item t = lane + 64 u is id t % L at position t / L; a step of 64
        // items moves the id by dj and the position by di, plus one when
        // the id index wraps.  The id is kept as its LDS byte address.
        const uint32_t di = 64u / L, dj4 = (64u - di * L) * 4u;
        uint32_t i = lane / L;
        const uint32_t lo = ids_lds + ka * 4u, hi = lo + L * 4u;
        uint32_t ja = lo + (lane - i * L) * 4u;
        // items below lim fit the output (the capacity may cut the run);
        // whole steps of 64 first, unchecked, then the partial one
        const uint32_t lim = (uint32_t)min<unsigned long long>(T, cap - ko);
        ac_match *run = out + ko + lane;
        uint32_t base = 0;
        auto step = [&]() {
            ja += dj4;
            i += di;
            if (ja >= hi) {
                ja -= L * 4u;
                ++i;
            }
        };
        // four steps at a time: their LDS reads are in flight together
        for (; base + 256 <= lim; base += 256) {
            uint32_t id[4], pos[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                id[u] = lds_load(ja);
                pos[u] = e + i;
                step();
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ac_match m;
                m.pattern_id = id[u];
                m.end_pos = pos[u];
                run[64 * u] = m;
            }
            run += 256;
        }
        for (; base + 64 <= lim; base += 64) {
            ac_match m;
            m.pattern_id = lds_load(ja);
            m.end_pos = e + i;
            *run = m;
            run += 64;
            step();
        }
        if (base + lane < lim) {
            ac_match m;
            m.pattern_id = lds_load(ja);
            m.end_pos = e + i;
            *run = m;
        }
    }
}

template <int FMT>
__global__ __launch_bounds__(kDenseLdsThreads) void k_emit_dense_lds(
    Inst I, const uint32_t *__restrict__ list_seg, const u32x4 *__restrict__ list_state,
    const unsigned long long *__restrict__ list_moff, const unsigned long long *__restrict__ totals,
    uint32_t off_bytes, uint32_t ids_bytes, ac_match *__restrict__ out) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    constexpr uint32_t WPS = kSeg / SPW;
    constexpr uint32_t WPQ = kQuarter / SPW;
    constexpr uint32_t B = kDenseBatch;
    const uint32_t n_sparse = (uint32_t)totals[1];
    const uint32_t n_dense = (uint32_t)totals[2];
    // set offsets at LDS 0, ids after them
    const uint32_t ids_lds = (off_bytes + 15u) & ~15u;
    load_lds_table(make_rsrc(uniform(I.out_off), off_bytes), off_bytes);
    load_lds_table(make_rsrc(uniform(I.out_ids), ids_bytes), ids_bytes, ids_lds);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gq = lane / kQuarter;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const MTable tab = emit_table(uniform(I.delta), uniform(I.delta_sz), uniform(I.walk_sz),
                                  uniform(I.table_bytes));
    const uint32_t tb4 = uniform(I.text_bytes4);
    const UText txt{make_rsrc(uniform(I.text), tb4), tb4};
    const uint32_t fo = uniform(I.fo_bytes), fos = uniform(I.fo_state);
    const uint32_t tz = uniform(I.div_tz), inv = uniform(I.div_inv);
    const uint32_t n = uniform(I.n);
    const unsigned long long cap = uniform(I.capacity);
    for (uint32_t w = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * B; w < n_dense;
         w += waves * B) {
        uint32_t idx[B], seg[B], s[B], mine[B];
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
            idx[b] = n_sparse + (w + b < n_dense ? w + b : w);
            seg[b] = uniform(list_seg[idx[b]]);
            const u32x4 qs = list_state[idx[b]];
            s[b] = gq == 0 ? uniform(qs.x) : gq == 1 ? uniform(qs.y) : gq == 2 ? uniform(qs.z)
                                                                    : uniform(qs.w);
            mine[b] = 0;
        }
#pragma unroll
        for (uint32_t wq = 0; wq < WPQ; ++wq) {
            uint32_t x[B];
#pragma unroll
            for (uint32_t b = 0; b < B; ++b) x[b] = txt.word((int)(seg[b] * WPS + gq * WPQ + wq));
#pragma unroll
            for (uint32_t k = 0; k < SPW; ++k) {
#pragma unroll
                for (uint32_t b = 0; b < B; ++b) {
                    s[b] = tab(s[b] + sym_bytes<FMT>(x[b], k));
                    if (lane % kQuarter == wq * SPW + k) mine[b] = s[b];
                }
            }
        }
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
            if (w + b >= n_dense) break;
            const unsigned long long off0 = uniform(list_moff[idx[b]]);
            if (off0 >= cap) continue;
            const uint32_t e0 = seg[b] * kSeg;
            const bool has = mine[b] >= fo && lane < n - e0;
            const uint32_t o = has ? row_state(mine[b], tz, inv) - fos : 0u;
            const uint32_t a = has ? lds_load(o * 4u) : 0u;
            const uint32_t len = has ? lds_load(o * 4u + 4u) - a : 0u;
            dense_runs_lds(mine[b], a, len, lane, e0, off0, cap, ids_lds, out);
        }
    }
}

// ------------------------------------------------------------------ encode

// Letters -> codes.  DNA uses the bit identity code = ((ch>>1) ^ (ch>>2)) & 3
// for A C G T a c g t (0 1 2 3); protein letters index a 26-entry table by
// (ch | 0x20) - 'a' (0xFF = not an amino-acid letter).  Each thread handles
// 16 letters.
__constant__ uint8_t c_protein_lut[32] = {
    0,    0xFF, 1,    2,    3,    4,    5,    6,    7,    0xFF, 8,    9,    10,   11,   0xFF, 12,
    13,   14,   15,   16,   0xFF, 17,   18,   0xFF, 19,   0xFF, 0xFF, 0xFF, 0xFF, 0xFF, 0xFF, 0xFF};

__device__ __forceinline__ uint32_t protein_code(uint32_t ch) {
    const uint32_t i = (ch | 0x20u) - (uint32_t)'a';
    return i < 26u ? c_protein_lut[i] : 0xFFu;
}

__device__ __forceinline__ bool dna_ok(uint32_t ch) {
    const uint32_t l = ch | 0x20u;
    return l == 'a' || l == 'c' || l == 'g' || l == 't';
}

template <int ALPHA, int FMT>
__global__ __launch_bounds__(256) void k_encode(const uint8_t *__restrict__ in, uint64_t n,
                                                uint8_t *__restrict__ out,
                                                unsigned long long *invalid) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t p = g * 16;
    uint32_t bad = 0;
    if (p < n) {
        uint8_t ch[16];
        if (p + 16 <= n && (((uintptr_t)(in + p)) & 15) == 0) {
            const u32x4 v = *(const u32x4 *)(in + p);
#pragma unroll
            for (int i = 0; i < 16; ++i) ch[i] = (uint8_t)(v[i >> 2] >> (8 * (i & 3)));
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) ch[i] = (p + i < n) ? in[p + i] : (uint8_t)'A';
        }
        uint8_t code[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint32_t c = ch[i];
            if constexpr (ALPHA == AC_ALPHA_DNA) {
                const bool ok = dna_ok(c);
                bad += !ok && (p + i < n);
                code[i] = ok ? (uint8_t)(((c >> 1) ^ (c >> 2)) & 3u) : 0;
            } else {
                const uint32_t v = protein_code(c);
                const bool ok = v != 0xFFu;
                bad += !ok && (p + i < n);
                code[i] = ok ? (uint8_t)v : 0;
            }
            if (p + i >= n) code[i] = 0;
        }
        if constexpr (FMT == AC_TEXT_2BIT) {
            uint32_t w = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) w |= (uint32_t)code[i] << (2 * i);
            const uint64_t ob = p / 4;             // output byte
            const uint64_t nb = (n + 3) / 4;       // output bytes in total
            if (ob + 4 <= nb && (((uintptr_t)(out + ob)) & 3) == 0) {
                *(uint32_t *)(out + ob) = w;
            } else {
                for (int i = 0; i < 4; ++i)
                    if (ob + i < nb) out[ob + i] = (uint8_t)(w >> (8 * i));
            }
        } else {
            if (p + 16 <= n && (((uintptr_t)(out + p)) & 15) == 0) {
                u32x4 v;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    v[q] = (uint32_t)code[4 * q] | ((uint32_t)code[4 * q + 1] << 8) |
                           ((uint32_t)code[4 * q + 2] << 16) | ((uint32_t)code[4 * q + 3] << 24);
                *(u32x4 *)(out + p) = v;
            } else {
                for (int i = 0; i < 16; ++i)
                    if (p + i < n) out[p + i] = code[i];
            }
        }
    }
    if (invalid) {
        const uint32_t b = wave_sum_u32(bad);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(invalid, (unsigned long long)b);
    }
}

// DNA letters -> 2-bit codes, 64 letters per thread.  A wave covers 4096
// letters: load q of lane i reads the 16 letters at wave base + 1024 q + 16 i
// (four fully coalesced 1 KB loads per wave, non-temporal), and each 16
// letters become one 32-bit store.  Four letters are handled per 32-bit
// word at once: code = ((ch>>1) ^ (ch>>2)) & 3 in every byte, then the four
// 2-bit fields are gathered into one byte.  A byte is valid when (ch | 0x20)
// is one of a c g t, which is the case exactly when it equals the lowercase
// letter of its own code ('A' 'C' 'G' 'T' and their lowercase forms map to
// codes 0 1 2 3, and (ch | 0x20) = letter leaves only those two forms).  One
// byte permute looks the four letters up at once, and the exact per-byte
// zero test z(v) = ~(((v & 0x7F..) + 0x7F..) | v) & 0x80.., which has no
// carries between bytes, compares them.  The kernel is bound by its integer
// work, so one lookup and one test per word in place of four tests matter.
// The last partial wave (and unaligned buffers) take byte loads and stores,
// with letters past n neither counted nor stored.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t v) {
    return ~(((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
}

// Codes of the four letters of x (bits 0-1 of each byte, invalid letters
// included) and the valid-letter mask (0x80 in each valid byte).
__device__ __forceinline__ uint32_t dna_codes4(uint32_t x, uint32_t &ok) {
    constexpr uint32_t kLetters = 0x74676361u;  // bytes 0..3: 'a' 'c' 'g' 't'
    const uint32_t t = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    // selectors 0..3 pick bytes of the table (both operands hold it)
    ok = zero_bytes((x | 0x20202020u) ^ __builtin_amdgcn_perm(kLetters, kLetters, t));
    return t;
}

__global__ __launch_bounds__(256) void k_encode_dna2(const uint8_t *__restrict__ in, uint64_t n,
                                                     uint8_t *__restrict__ out,
                                                     unsigned long long *invalid) {
    constexpr int kNonTemporal = 2;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wb = ((uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u)) * 64u;
    uint32_t bad = 0;
    const bool wfull = wb + 4096 <= n && (((uintptr_t)in) & 15) == 0 && (((uintptr_t)out) & 3) == 0;
    if (wfull) {
        const rsrc_t r = make_rsrc(in, (uint32_t)n);
        u32x4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = __builtin_amdgcn_raw_buffer_load_b128(
                r, (uint32_t)(wb + 1024u * q + 16u * lane), 0, kNonTemporal);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t packed = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                uint32_t ok;
                const uint32_t t = dna_codes4(v[q][w], ok) & (ok >> 7) * 3u;
                bad += __builtin_popcount(~ok & 0x80808080u);
                packed |= ((t | (t >> 6) | (t >> 12) | (t >> 18)) & 0xFFu) << (8 * w);
            }
            *(uint32_t *)(out + (wb + 1024u * q + 16u * lane) / 4) = packed;
        }
    } else {
        const uint64_t p = wb + 64u * lane;
        if (p < n) {
            u32x4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    uint32_t x = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint64_t i = p + 16u * q + 4u * w + k;
                        x |= (i < n ? (uint32_t)in[i] : 0u) << (8 * k);
                    }
                    v[q][w] = x;
                }
            u32x4 o;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t packed = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    uint32_t ok;
                    const uint32_t c = dna_codes4(v[q][w], ok);
                    const int64_t rem = (int64_t)n - (int64_t)(p + 16u * q + 4u * w);
                    const uint32_t live = rem >= 4 ? 0x80808080u
                                          : rem <= 0 ? 0u
                                                     : (uint32_t)((1ull << (8 * rem)) - 1u) &
                                                           0x80808080u;
                    bad += __builtin_popcount(~ok & live);
                    const uint32_t t = c & ((ok & live) >> 7) * 3u;
                    packed |= ((t | (t >> 6) | (t >> 12) | (t >> 18)) & 0xFFu) << (8 * w);
                }
                o[q] = packed;
            }
            const uint64_t ob = p / 4;
            const uint64_t nb = (n + 3) / 4;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (ob + i < nb) out[ob + i] = (uint8_t)(o[i >> 2] >> (8 * (i & 3)));
        }
    }
    if (invalid) {
        const uint32_t b = wave_sum_u32(bad);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(invalid, (unsigned long long)b);
    }
}

// ================================================================== host

#define HIP_OK(x)                          \
    do {                                   \
        if ((x) != hipSuccess) {           \
            (void)hipGetLastError();       \
            return AC_E_HIP;               \
        }                                  \
    } while (0)

struct DevProps {
    bool init = false;
    uint32_t cus = 0;
    uint32_t lds = 0;
};
static std::mutex g_props_mu;
static DevProps g_props[64];

int device_limits(uint32_t *cus, uint32_t *lds) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return AC_E_HIP;
    std::lock_guard<std::mutex> lk(g_props_mu);
    DevProps &p = g_props[dev];
    if (!p.init) {
        int v = 0;
        HIP_OK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
        p.cus = (uint32_t)v;
        int l1 = 0, l2 = 0;
        HIP_OK(hipDeviceGetAttribute(&l1, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        HIP_OK(hipDeviceGetAttribute(&l2, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
        p.lds = (uint32_t)std::max(l1, l2);
        if (p.lds > 160u * 1024u) p.lds = 160u * 1024u;
        p.init = true;
    }
    if (cus) *cus = p.cus;
    if (lds) *lds = p.lds;
    return AC_OK;
}

// Largest dynamic LDS a count block may use (the kernel's static LDS is
// below 512 bytes).
static uint32_t count_lds_limit(uint32_t lds) { return lds - 512; }

int upload_dict(ac_dict *d) {
    const HostTables &T = d->host;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    uint32_t cus = 0, lds = 0;
    int rc = device_limits(&cus, &lds);
    if (rc) return rc;
    // 16-bit copy of the hottest output-free rows for the hybrid placement
    const uint32_t hot_rows =
        std::min<uint32_t>(T.first_output, count_lds_limit(lds) / (T.sigma * 2u));
    // (+2 entries: the LDS copy reads whole 32-bit words)
    std::vector<uint16_t> hot16((size_t)std::max<uint32_t>(hot_rows, 1) * T.sigma + 2, 0);
    for (size_t i = 0; i < (size_t)hot_rows * T.sigma; ++i)
        hot16[i] = T.delta[i] < 0xFFFFu ? (uint16_t)T.delta[i] : (uint16_t)0xFFFFu;
    // for the count-table walk, transitions into output states are read from
    // the 32-bit count table (which carries the set sizes): escape them too
    std::vector<uint16_t> hot16c(hot16);
    for (size_t i = 0; i < (size_t)hot_rows * T.sigma; ++i)
        if (T.delta[i] >= T.first_output) hot16c[i] = 0xFFFFu;
    d->hot16_rows = hot_rows;
    // every row as 16-bit ids, when all ids fit 16 bits and the table fits
    // the count kernel's LDS beside its zero pad
    std::vector<uint16_t> tab16;
    const uint64_t t16 = (uint64_t)T.states * T.sigma * 2u;
    if (T.states < 0xFFFFu && t16 + kLdsPad / 2 <= count_lds_limit(lds)) {
        tab16.resize(T.delta.size() + 2, 0);  // (+2: the LDS copy reads whole words)
        for (size_t i = 0; i < T.delta.size(); ++i) tab16[i] = (uint16_t)T.delta[i];
    }
    // two-symbol table, when it fits the count kernel's LDS
    std::vector<uint32_t> d2;
    if (T.sigma == 4 && (uint64_t)T.states * 64u <= count_lds_limit(lds)) {
        d2.resize((size_t)T.states * 16);
        for (uint32_t s = 0; s < T.states; ++s)
            for (uint32_t c1 = 0; c1 < 4; ++c1) {
                const uint32_t t1 = T.delta[(size_t)s * 4 + c1];
                const uint32_t flag = t1 >= T.first_output ? 0x80000000u : 0u;
                for (uint32_t c2 = 0; c2 < 4; ++c2)
                    d2[(size_t)s * 16 + c1 + 4 * c2] = T.delta[(size_t)t1 * 4 + c2] * 64u | flag;
            }
    }
    std::vector<uint32_t> rows(T.delta.size());
    const uint32_t row = T.sigma * 4u;
    for (size_t i = 0; i < rows.size(); ++i) rows[i] = T.delta[i] * row;
    // failure-less kernel: child row offsets (bit 31: the child has its own
    // patterns); row offsets must stay below 2^31
    std::vector<uint32_t> go;
    if (rows.size() * 4 < (1ull << 31)) {
        go.resize(T.go.size());
        for (size_t i = 0; i < go.size(); ++i) {
            const uint32_t t = T.go[i];
            go[i] = t ? t * row | (T.own_off[t + 1] > T.own_off[t] ? 0x80000000u : 0u) : 0u;
        }
    }
    const size_t off_bytes = T.out_off.size() * 4;
    std::vector<uint32_t> sizes(std::max<size_t>(1, T.out_off.size() - 1), 0);
    for (size_t i = 0; i + 1 < T.out_off.size(); ++i) sizes[i] = T.out_off[i + 1] - T.out_off[i];
    // sigma 4: the count table, row offset | |out(target)| << 24, when row
    // offsets fit 24 bits and set sizes 8 bits
    std::vector<uint32_t> dsz;
    if (T.sigma == 4 && rows.size() * 4 <= kRowBits + 1ull && T.max_output <= 255) {
        dsz.resize(rows.size());
        for (size_t i = 0; i < rows.size(); ++i) {
            const uint32_t t = T.delta[i];
            const uint32_t n = t >= T.first_output ? sizes[t - T.first_output] : 0u;
            dsz[i] = rows[i] | n << 24;
        }
    }
    const size_t ids_bytes = std::max<size_t>(4, T.out_ids.size() * 4);
    if (test_alloc_fails() || hipMalloc((void **)&d->d_delta, rows.size() * 4) != hipSuccess ||
        hipMalloc((void **)&d->d_out_off, off_bytes) != hipSuccess ||
        hipMalloc((void **)&d->d_out_ids, ids_bytes) != hipSuccess ||
        hipMalloc((void **)&d->d_out_size, sizes.size() * 4) != hipSuccess ||
        hipMalloc((void **)&d->d_hot16, hot16.size() * 2) != hipSuccess ||
        hipMalloc((void **)&d->d_hot16c, hot16c.size() * 2) != hipSuccess ||
        (!dsz.empty() && hipMalloc((void **)&d->d_delta_sz, dsz.size() * 4) != hipSuccess) ||
        (!tab16.empty() && hipMalloc((void **)&d->d_tab16, tab16.size() * 2) != hipSuccess) ||
        (!d2.empty() && hipMalloc((void **)&d->d_delta2, d2.size() * 4) != hipSuccess) ||
        (!go.empty() && (hipMalloc((void **)&d->d_go, go.size() * 4) != hipSuccess ||
                         hipMalloc((void **)&d->d_own_off, T.own_off.size() * 4) != hipSuccess ||
                         hipMalloc((void **)&d->d_own_ids, T.own_ids.size() * 4) != hipSuccess))) {
        (void)hipGetLastError();
        release_dict(d);
        return AC_E_NOMEM;
    }
    if (hipMemcpy(d->d_delta, rows.data(), rows.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_out_off, T.out_off.data(), off_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_out_size, sizes.data(), sizes.size() * 4, hipMemcpyHostToDevice) !=
            hipSuccess ||
        (!T.out_ids.empty() &&
         hipMemcpy(d->d_out_ids, T.out_ids.data(), T.out_ids.size() * 4, hipMemcpyHostToDevice) !=
             hipSuccess) ||
        hipMemcpy(d->d_hot16, hot16.data(), hot16.size() * 2, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(d->d_hot16c, hot16c.data(), hot16c.size() * 2, hipMemcpyHostToDevice) !=
            hipSuccess ||
        (!dsz.empty() &&
         hipMemcpy(d->d_delta_sz, dsz.data(), dsz.size() * 4, hipMemcpyHostToDevice) !=
             hipSuccess) ||
        (!d2.empty() &&
         hipMemcpy(d->d_delta2, d2.data(), d2.size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        (!tab16.empty() && hipMemcpy(d->d_tab16, tab16.data(), tab16.size() * 2,
                                     hipMemcpyHostToDevice) != hipSuccess) ||
        (!go.empty() &&
         (hipMemcpy(d->d_go, go.data(), go.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d->d_own_off, T.own_off.data(), T.own_off.size() * 4,
                    hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d->d_own_ids, T.own_ids.data(), T.own_ids.size() * 4,
                    hipMemcpyHostToDevice) != hipSuccess))) {
        (void)hipGetLastError();
        release_dict(d);
        return AC_E_HIP;
    }
    d->delta2_bytes = (uint32_t)(d2.size() * 4);
    d->tab16_bytes = tab16.empty() ? 0u : (uint32_t)t16;
    d->device = dev;
    return AC_OK;
}

void release_dict(ac_dict *d) {
    if (d->d_delta) (void)hipFree(d->d_delta);
    if (d->d_out_off) (void)hipFree(d->d_out_off);
    if (d->d_out_ids) (void)hipFree(d->d_out_ids);
    if (d->d_out_size) (void)hipFree(d->d_out_size);
    d->d_out_size = nullptr;
    if (d->d_hot16) (void)hipFree(d->d_hot16);
    if (d->d_hot16c) (void)hipFree(d->d_hot16c);
    d->d_hot16c = nullptr;
    if (d->d_tab16) (void)hipFree(d->d_tab16);
    d->d_tab16 = nullptr;
    d->tab16_bytes = 0;
    if (d->d_delta_sz) (void)hipFree(d->d_delta_sz);
    d->d_delta_sz = nullptr;
    if (d->d_delta2) (void)hipFree(d->d_delta2);
    if (d->d_go) (void)hipFree(d->d_go);
    if (d->d_own_off) (void)hipFree(d->d_own_off);
    if (d->d_own_ids) (void)hipFree(d->d_own_ids);
    d->d_delta = d->d_out_off = d->d_out_ids = d->d_delta2 = nullptr;
    d->d_go = d->d_own_off = d->d_own_ids = nullptr;
    d->d_hot16 = nullptr;
    d->delta2_bytes = 0;
    (void)hipGetLastError();
}

// ---------------------------------------------------------- kernel timing

struct TimedPair {
    int kind;
    hipEvent_t a, b;
};
static std::mutex g_tm_mu;
static uint32_t g_tm_mask = 0;  // bit k: time kernels of kind k
static std::vector<TimedPair> g_tm_pending;
static std::vector<hipEvent_t> g_tm_free;
static double g_tm_ms[AC_K_KINDS];
static uint64_t g_tm_n[AC_K_KINDS];

static hipEvent_t tm_event() {
    if (!g_tm_free.empty()) {
        hipEvent_t e = g_tm_free.back();
        g_tm_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Records an event pair around one kernel launch when timing is enabled.
struct KTimer {
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr;
    KTimer(int k, hipStream_t s) : kind(k), st(s) {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        if (!(g_tm_mask >> kind & 1u)) return;
        a = tm_event();
        if (a) (void)hipEventRecord(a, st);
    }
    ~KTimer() {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_tm_mu);
        hipEvent_t b = tm_event();
        if (!b) return;
        (void)hipEventRecord(b, st);
        g_tm_pending.push_back({kind, a, b});
    }
};

// ---------------------------------------------------------- launch geometry

static uint32_t spw_of(uint32_t fmt) { return fmt == AC_TEXT_2BIT ? 16u : 4u; }

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct Geom {
    uint32_t chunk = 0, threads = 0, warm = 0, grid_count = 0, chains = 1;
    uint32_t grid_emit = 0, grid_dense = 0;  // bounded by the largest possible work list
    uint32_t lds_bytes = 0;  // dynamic LDS of k_count
    uint64_t n_chunks = 0, n_tiles = 0, segs = 0;
    // a batch without a requested chunk size gives an instance too short to
    // fill one tile shorter chunks, so that more lanes share its text and
    // its tile's walk ends sooner
    bool adapt = false;
    uint64_t n_segs() const { return segs; }
    uint32_t chunk_of(uint64_t n) const {
        if (!adapt) return chunk;
        const uint64_t per_tile = (uint64_t)threads * chains;
        const uint64_t want = ((n + per_tile - 1) / per_tile + kSeg - 1) / kSeg * kSeg;
        return (uint32_t)std::max<uint64_t>(kSeg, std::min<uint64_t>(chunk, want));
    }
};

struct Workspace {
    uint32_t *cnt, *mask;                 // per chunk
    u32x4 *seg_state;                     // per segment: quarter states, then events
    uint32_t *seg_m;                      // per segment: matches (written where > 0)
    unsigned long long *tile_m;           // per tile
    uint32_t *tile_zs, *tile_zd;
    unsigned long long *tile_moff;        // per tile, + grand total
    uint32_t *tile_zsoff, *tile_zdoff;
    unsigned long long *totals;           // matches, sparse segments, dense segments
    uint32_t *list_seg, *list_inst;       // work list of segments
    u32x4 *list_state;
    unsigned long long *list_moff;
};

static uint64_t ws_layout(const Geom &g, bool batch, char *base, Workspace *w) {
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        char *p = base ? base + o : nullptr;
        o += align256(std::max<uint64_t>(bytes, 8));
        return p;
    };
    const uint64_t C = g.n_chunks, T = g.n_tiles, S = g.n_segs();
    Workspace t;
    t.cnt = (uint32_t *)take(4 * C);
    t.mask = (uint32_t *)take(4 * C);
    t.seg_state = (u32x4 *)take(32 * S);
    t.seg_m = (uint32_t *)take(4 * S);
    t.tile_m = (unsigned long long *)take(8 * T);
    t.tile_zs = (uint32_t *)take(4 * T);
    t.tile_zd = (uint32_t *)take(4 * T);
    t.tile_moff = (unsigned long long *)take(8 * (T + 1));
    t.tile_zsoff = (uint32_t *)take(4 * (T + 1));
    t.tile_zdoff = (uint32_t *)take(4 * (T + 1));
    t.totals = (unsigned long long *)take(32);
    t.list_seg = (uint32_t *)take(4 * S);
    t.list_state = (u32x4 *)take(16 * S);
    t.list_inst = batch ? (uint32_t *)take(4 * S) : nullptr;
    t.list_moff = (unsigned long long *)take(8 * S);
    if (w) *w = t;
    return o;
}

// Placement of one dictionary's table for the count kernel: the LDS bytes
// it copies, the hot bound of the table accessors and whether the whole
// table is in LDS.
struct Placement {
    uint32_t hot = 0;        // see Inst::hot_bytes
    uint32_t lds_all = 0;
    uint32_t lds_bytes = 0;  // dynamic LDS the count kernel needs
    uint32_t stride2 = 0;    // two-symbol table in LDS
};

static Placement choose_placement(const ac_dict *d, uint32_t requested, uint32_t lds_limit,
                                  uint32_t fmt) {
    Placement pl;
    const uint32_t tb = (uint32_t)d->table_bytes;
    const uint32_t sigma = d->host.sigma;
    uint32_t p = requested ? requested : d->placement;
    const bool fits = tb + kLdsPad <= lds_limit;
    const bool two = fmt == AC_TEXT_2BIT && d->d_delta2 && d->delta2_bytes <= lds_limit;
    if (p == AC_PLACE_LDS2) {
        if (two) {
            pl.stride2 = 1;
            pl.lds_all = 1;
            pl.hot = d->delta2_bytes;
            pl.lds_bytes = d->delta2_bytes;
            return pl;
        }
        p = AC_PLACE_LDS;
    }
    const bool fits16 = d->d_tab16 && d->tab16_bytes + kLdsPad / 2 <= lds_limit;
    if (p == AC_PLACE_AUTO) p = fits ? AC_PLACE_LDS : fits16 ? AC_PLACE_LDS16 : AC_PLACE_HYBRID;
    if (p == AC_PLACE_LDS && !fits) p = AC_PLACE_HYBRID;
    if (p == AC_PLACE_LDS16 && !fits16) p = AC_PLACE_HYBRID;
    if (p == AC_PLACE_LDS16) {
        // 16-bit ids of every row, then zeros
        pl.hot = tb;
        pl.lds_all = 2;
        pl.lds_bytes = ((d->tab16_bytes + 3u) & ~3u) + kLdsPad / 2;
        return pl;
    }
    if (p == AC_PLACE_HYBRID && d->hot16_rows == 0) p = AC_PLACE_GLOBAL;
    if (p == AC_PLACE_LDS) {
        pl.hot = tb;
        pl.lds_all = 1;
        pl.lds_bytes = tb + kLdsPad;
    } else if (p == AC_PLACE_HYBRID) {
        // the 16-bit rows, then one zero word (read by lanes on other rows)
        uint32_t rows = std::min<uint32_t>(d->hot16_rows, (lds_limit - 8u) / (sigma * 2u));
        if (d->hot_states) rows = std::min(rows, d->hot_states);
        pl.hot = rows * sigma * 4u;
        pl.lds_bytes = ((rows * sigma * 2u + 3u) & ~3u) + 4u;
        if (rows == 0) pl = Placement{};
    }
    return pl;
}

static int resolve_geom(const ac_dict *const *dicts, const uint64_t *ns, uint32_t n_inst,
                        uint32_t fmt, const ac_tune *tune, Geom *g) {
    uint32_t cus = 0, lds = 0;
    int rc = device_limits(&cus, &lds);
    if (rc != AC_OK) return rc;
    const uint32_t lds_limit = count_lds_limit(lds);
    uint32_t max_len = 1, max_out = 1;
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        max_len = std::max(max_len, dicts[i]->host.max_len);
        max_out = std::max(max_out, dicts[i]->host.max_output);
        total += ns[i];
    }
    // per-chunk match counts are 32-bit
    if ((uint64_t)kSeg * max_out >= (1ull << 32)) return AC_E_TOO_LARGE;
    uint32_t max_chunk = kMaxChunk;
    while ((uint64_t)max_chunk * max_out >= (1ull << 32)) max_chunk /= 2;
    const uint32_t spw = spw_of(fmt);
    g->warm = (max_len - 1 + spw - 1) / spw;
    g->threads = (tune && tune->block_threads) ? tune->block_threads : 1024u;
    if (g->threads < 64 || g->threads > kMaxCountThreads || g->threads % 64) return AC_E_INVALID;
    // chains per lane: one by default; a single 2-bit scan in the hybrid
    // placement walks two at once (its walk keeps few registers, and two
    // independent chains overlap their L2 latencies)
    g->chains = 1;
    if (tune && tune->chains) {
        g->chains = tune->chains;
    } else if (n_inst == 1 && fmt == AC_TEXT_2BIT && dicts[0]->d_delta_sz) {
        const Placement pl =
            choose_placement(dicts[0], tune ? tune->placement : 0, lds_limit, fmt);
        if (pl.hot && !pl.lds_all && !pl.stride2) g->chains = 2;
    }
    if (g->chains != 1 && g->chains != 2 && g->chains != 4) return AC_E_INVALID;
    const uint32_t per_tile = g->threads * g->chains;  // chunks per tile
    uint32_t chunk = tune ? tune->chunk : 0;
    if (chunk && (chunk % kSeg || chunk > kMaxChunk)) return AC_E_INVALID;
    if (chunk > max_chunk) return AC_E_TOO_LARGE;
    // LDS need of the count kernel
    uint32_t lds_bytes = 0;
    const uint32_t req = tune ? tune->placement : 0;
    if (req > AC_PLACE_LDS16) return AC_E_INVALID;
    for (uint32_t i = 0; i < n_inst; ++i)
        lds_bytes = std::max(lds_bytes, choose_placement(dicts[i], req, lds_limit, fmt).lds_bytes);
    g->lds_bytes = lds_bytes;
    uint32_t bpc = (tune && tune->blocks_per_cu) ? tune->blocks_per_cu
                                                  : std::max(1u, 2048u / g->threads);
    if (lds_bytes) bpc = std::max(1u, std::min(bpc, (lds + 0u) / (lds_bytes + 512u)));
    const uint64_t slots = (uint64_t)cus * bpc;
    if (!chunk) {
        // short chunks keep more lanes busy; 256 DNA bases (64 bytes packed)
        // or 64 letters balance that against the warm-up before each chunk
        chunk = std::min<uint32_t>(fmt == AC_TEXT_2BIT ? 256 : 64, max_chunk);
        while (chunk > kSeg && (total / chunk) / per_tile < slots) chunk /= 2;
    }
    g->chunk = chunk;
    g->adapt = n_inst > 1 && !(tune && tune->chunk);
    g->n_chunks = 0;
    g->n_tiles = 0;
    g->segs = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const uint32_t ci = g->chunk_of(ns[i]);
        const uint64_t c = (ns[i] + ci - 1) / ci;
        g->n_chunks += c;
        g->n_tiles += (c + per_tile - 1) / per_tile;
        g->segs += c * (ci / kSeg);
    }
    if (g->n_chunks >= (1ull << 31) || g->n_tiles >= (1ull << 31)) return AC_E_TOO_LARGE;
    g->grid_count = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g->n_tiles, slots));
    // persistent emit grids, no larger than the work list can ever need
    const uint64_t segs = g->n_segs();
    g->grid_emit = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)cus * 8, (4 * segs + kEmitThreads - 1) / kEmitThreads));
    g->grid_dense = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)cus * 8, (segs + kDenseThreads / 64 - 1) / (kDenseThreads / 64)));
    return AC_OK;
}

static void fill_inst(const ac_dict *d, const void *text, uint64_t n, uint32_t fmt, ac_match *out,
                      uint64_t cap, uint64_t *count, uint32_t req_place, uint32_t lds_limit,
                      Inst *I) {
    memset(I, 0, sizeof(*I));
    I->delta = d->d_delta;
    I->out_off = d->d_out_off;
    I->out_ids = d->d_out_ids;
    I->out_size = d->d_out_size;
    I->delta_sz = d->d_delta_sz;
    I->n_ids = (uint32_t)d->host.out_ids.size();
    I->text = (const uint8_t *)text;
    I->out = out;
    I->count = (unsigned long long *)count;
    I->capacity = cap;
    I->n = (uint32_t)n;
    const uint64_t bytes = fmt == AC_TEXT_2BIT ? (n + 3) / 4 : n;
    I->text_bytes4 = (uint32_t)((bytes + 3) & ~uint64_t(3));
    I->table_bytes = (uint32_t)d->table_bytes;
    I->fo_state = d->host.first_output;
    I->fo_bytes = d->host.first_output * d->host.sigma * 4u;
    const Placement pl = choose_placement(d, req_place, lds_limit, fmt);
    I->stride2 = pl.stride2;
    I->delta2 = d->d_delta2;
    I->fo2_bytes = d->host.first_output * 64u;
    I->hot_bytes = pl.hot;
    I->lds_all = pl.lds_all;
    I->lds_bytes = pl.lds_bytes;
    I->hot16 = d->d_hot16;
    I->hot16c = d->d_hot16c;
    I->tab16 = d->d_tab16;
    const RowDiv rd = make_row_div(d->host.sigma);
    I->div_tz = rd.tz;
    I->div_inv = rd.inv;
    I->sigma = d->host.sigma;
}

template <typename K>
static int allow_lds(K kernel, uint32_t bytes) {
    if (bytes > 64 * 1024)
        HIP_OK(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes));
    return AC_OK;
}

// Blocks of a persistent grid: no more than the device keeps resident at
// once.  A block that could start only after others finish would run its
// share of the work as a second, partial round.
template <typename K>
static uint32_t resident_grid(K kernel, uint32_t threads, uint32_t want, uint32_t dyn_lds = 0) {
    static std::mutex mu;
    static std::map<std::pair<const void *, uint32_t>, int> per_cu;
    const std::pair<const void *, uint32_t> key((const void *)kernel, dyn_lds);
    int n = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = per_cu.find(key);
        if (it != per_cu.end()) n = it->second;
    }
    if (n == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)kernel, (int)threads,
                                                         dyn_lds) != hipSuccess ||
            n <= 0) {
            (void)hipGetLastError();
            n = 1;
        }
        std::lock_guard<std::mutex> lk(mu);
        per_cu[key] = n;
    }
    uint32_t cus = 1;
    if (device_limits(&cus, nullptr) != AC_OK) cus = 1;
    return std::max<uint32_t>(1, std::min<uint64_t>(want, (uint64_t)cus * (uint32_t)n));
}

static const uint64_t kMaxText = (1ull << 32) - 256;

static int validate_text(const ac_dict *d, const void *text, uint64_t n, uint32_t fmt) {
    if (fmt != AC_TEXT_U8 && fmt != AC_TEXT_2BIT) return AC_E_INVALID;
    if (fmt == AC_TEXT_2BIT && d->host.sigma != 4) return AC_E_INVALID;
    if (n >= kMaxText) return AC_E_TOO_LARGE;
    if (n && !text) return AC_E_INVALID;
    return AC_OK;
}

template <int FMT, bool BATCH, int CH>
static int launch_count_ch(const Geom &g, const Inst &I, const Inst *insts,
                           const TileDesc *tiles, const Workspace &w, int mode,
                           uint32_t t_base, uint32_t n_tiles, hipStream_t st) {
    if (n_tiles == 0) return AC_OK;
    auto kc = k_count<FMT, BATCH, CH, kCountAny>;
    if (mode == kCountLds) kc = k_count<FMT, BATCH, CH, kCountLds>;
    // the hybrid-only kernel serves single scans (a batch mixes placements)
    if constexpr (!BATCH)
        if (mode == kCountHybrid) {
            kc = k_count<FMT, BATCH, CH, kCountHybrid>;
            // its 2-bit walk addresses the LDS rows from address 0: no static LDS
            hipFuncAttributes fa;
            if (hipFuncGetAttributes(&fa, (const void *)kc) != hipSuccess || fa.sharedSizeBytes)
                return AC_E_HIP;
        }
    // the table, then the block reduction slots (16 u64 + 32 u32)
    const uint32_t red_off = (g.lds_bytes + 7u) & ~7u;
    const uint32_t dyn = red_off + 256u;
    int rc = allow_lds(kc, dyn);
    if (rc) return rc;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(n_tiles, g.grid_count);
    KTimer tm(AC_K_COUNT, st);
    hipLaunchKernelGGL(kc, dim3(grid), dim3(g.threads), dyn, st, I, insts, tiles, t_base,
                       n_tiles, red_off, w.cnt, w.mask, w.seg_state, w.seg_m, w.tile_m,
                       w.tile_zs, w.tile_zd);
    return AC_OK;
}

template <int FMT, bool BATCH>
static int launch_count(const Geom &g, const Inst &I, const Inst *insts, const TileDesc *tiles,
                        const Workspace &w, int mode, uint32_t t_base, uint32_t n_tiles,
                        hipStream_t st) {
    switch (g.chains) {
        case 1:
            return launch_count_ch<FMT, BATCH, 1>(g, I, insts, tiles, w, mode, t_base, n_tiles,
                                                  st);
        case 2:
            return launch_count_ch<FMT, BATCH, 2>(g, I, insts, tiles, w, mode, t_base, n_tiles,
                                                  st);
        default:
            return launch_count_ch<FMT, BATCH, 4>(g, I, insts, tiles, w, mode, t_base, n_tiles,
                                                  st);
    }
}

template <int FMT>
static int launch_single(const Geom &g, const Inst &I, const Workspace &w, hipStream_t st) {
    const uint32_t T = (uint32_t)g.n_tiles;
    // the 2-bit hybrid walk reads the count table (built when it fits 24-bit
    // row offsets and 8-bit set sizes)
    const bool hyb_ok = FMT != AC_TEXT_2BIT || I.delta_sz;
    const int mode = I.stride2              ? kCountAny
                     : I.lds_all            ? kCountLds
                     : I.hot_bytes && hyb_ok ? kCountHybrid
                                            : kCountAny;
    int rc = launch_count<FMT, false>(g, I, nullptr, nullptr, w, mode, 0, T, st);
    if (rc) return rc;
    // the emit walks follow the table the count pass read
    Inst E = I;
    E.walk_sz = mode == kCountHybrid && FMT == AC_TEXT_2BIT && I.delta_sz ? 1u : 0u;
    {
        KTimer tm(AC_K_OFFSETS, st);
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, w.tile_m, w.tile_zs,
                           w.tile_zd, T, w.tile_moff, w.tile_zsoff, w.tile_zdoff, w.totals,
                           I.count);
    }
    {
        KTimer tm(AC_K_SCATTER, st);
        hipLaunchKernelGGL(k_scatter<false>, dim3(T), dim3(g.threads), 0, st, I, nullptr, nullptr,
                           g.chains, w.cnt, w.mask, w.seg_state, w.seg_m, w.tile_moff,
                           w.tile_zsoff, w.tile_zdoff, w.totals, w.list_seg, w.list_state,
                           w.list_moff, nullptr);
    }
    {
        KTimer tm(AC_K_EMIT, st);
        hipLaunchKernelGGL((k_emit<FMT, false>),
                           dim3(resident_grid(k_emit<FMT, false>, kEmitThreads, g.grid_emit)),
                           dim3(kEmitThreads), 0, st, E,
                           nullptr, w.list_seg, w.list_state, w.list_moff, nullptr, w.totals,
                           w.seg_state);
    }
    // output-set tables for the staged dense emit: offsets (n_out + 1),
    // then ids, both in LDS
    const uint32_t n_out = (I.table_bytes - I.fo_bytes) / (I.sigma * 4u);
    const uint64_t off_bytes = 4ull * (n_out + 1), ids_bytes = 4ull * I.n_ids;
    uint32_t lds = 0;
    if (device_limits(nullptr, &lds) != AC_OK) lds = 0;
    if (((off_bytes + 15) & ~15ull) + ids_bytes + 1024 <= lds) {  // (+ the kernel's static LDS)
        KTimer tm(AC_K_EMIT_DENSE, st);
        const uint32_t dyn = (uint32_t)(((off_bytes + 15) & ~15ull) + ids_bytes);
        int rc2 = allow_lds(k_emit_dense_lds<FMT>, dyn);
        if (rc2) return rc2;
        hipLaunchKernelGGL((k_emit_dense_lds<FMT>),
                           dim3(resident_grid(k_emit_dense_lds<FMT>, kDenseLdsThreads,
                                              g.grid_dense, dyn)),
                           dim3(kDenseLdsThreads), dyn, st, E, w.list_seg, w.list_state,
                           w.list_moff, w.totals, (uint32_t)off_bytes, (uint32_t)ids_bytes,
                           I.out);
    } else {
        KTimer tm(AC_K_EMIT_DENSE, st);
        hipLaunchKernelGGL((k_emit_dense<FMT, false>),
                           dim3(resident_grid(k_emit_dense<FMT, false>, kDenseThreads,
                                              g.grid_dense)),
                           dim3(kDenseThreads), 0,
                           st, E, nullptr, w.list_seg, w.list_state, w.list_moff, nullptr,
                           w.totals, I.out_ids, I.out);
    }
    HIP_OK(hipGetLastError());
    return AC_OK;
}

// Workspace of ac_scan_noalloc: the scratch memory of one scan, kept in a
// file-scope device array so that a scan can run where allocating is not
// allowed.  Each device that loads the library holds its own copy until the
// process ends.  In host code the array's name is a host-side stand-in, not a
// device address: the device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels.
constexpr uint64_t kScratchBytes = AC_NOALLOC_MAX_WORKSPACE;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void *g_scratch[64];

static int scratch_address(void **p) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return AC_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *q = nullptr;
        HIP_OK(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
        if (!q) return AC_E_HIP;
        g_scratch[dev] = q;
    }
    *p = g_scratch[dev];
    return AC_OK;
}

}  // namespace acx

using namespace acx;

extern "C" {

int ac_device_info(uint32_t *compute_units, uint32_t *lds_bytes_per_block) {
    return device_limits(compute_units, lds_bytes_per_block);
}

int ac_timing_enable(int on) {
    const uint32_t all = (1u << AC_K_KINDS) - 1u;
    if (on < 0 || (on != AC_TIMING_ALL && ((uint32_t)on >> 1) & ~all)) return AC_E_INVALID;
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm_mask = on == AC_TIMING_ALL ? all : (uint32_t)on >> 1;
    return AC_OK;
}

int ac_timing_read(double *ms, uint64_t *launches, int reset) {
    std::vector<TimedPair> pend;
    {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        pend.swap(g_tm_pending);
    }
    int rc = AC_OK;
    double add[AC_K_KINDS] = {0};
    uint64_t cnt[AC_K_KINDS] = {0};
    for (const TimedPair &p : pend) {
        float t = 0.f;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&t, p.a, p.b) != hipSuccess) {
            (void)hipGetLastError();
            rc = AC_E_HIP;
        } else {
            add[p.kind] += t;
            cnt[p.kind] += 1;
        }
    }
    std::lock_guard<std::mutex> lk(g_tm_mu);
    for (const TimedPair &p : pend) {
        g_tm_free.push_back(p.a);
        g_tm_free.push_back(p.b);
    }
    for (int k = 0; k < AC_K_KINDS; ++k) {
        g_tm_ms[k] += add[k];
        g_tm_n[k] += cnt[k];
        if (ms) ms[k] = g_tm_ms[k];
        if (launches) launches[k] = g_tm_n[k];
        if (reset) {
            g_tm_ms[k] = 0;
            g_tm_n[k] = 0;
        }
    }
    return rc;
}

int ac_scan_workspace_size(const ac_dict *d, uint64_t n, uint32_t fmt, const ac_tune *tune,
                           uint64_t *bytes) {
    if (!d || !bytes || !d->parts.empty()) return AC_E_INVALID;
    int rc = validate_text(d, (const void *)1, n, fmt);
    if (rc) return rc;
    Geom g;
    rc = resolve_geom(&d, &n, 1, fmt, tune, &g);
    if (rc) return rc;
    *bytes = ws_layout(g, false, nullptr, nullptr);
    return AC_OK;
}

int ac_scan(const ac_dict *d, const void *d_text, uint64_t n, uint32_t fmt, ac_match *d_out,
            uint64_t capacity, uint64_t *d_count, const ac_tune *tune, void *d_workspace,
            uint64_t workspace_bytes, void *stream) {
    if (!d || !d_count) return AC_E_INVALID;
    if (capacity && !d_out) return AC_E_INVALID;
    if (!d->parts.empty())
        return scan_partitioned(d, d_text, n, fmt, d_out, capacity, d_count, tune,
                                (hipStream_t)stream);
    if (!d->d_delta) return AC_E_NO_DEVICE;
    int rc = validate_text(d, d_text, n, fmt);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (unsigned long long *)d_count, 1u,
                           0ull);
        HIP_OK(hipGetLastError());
        return AC_OK;
    }
    Geom g;
    rc = resolve_geom(&d, &n, 1, fmt, tune, &g);
    if (rc) return rc;
    uint32_t cus, lds;
    device_limits(&cus, &lds);
    Inst I;
    fill_inst(d, d_text, n, fmt, d_out, capacity, d_count, tune ? tune->placement : 0,
              count_lds_limit(lds), &I);
    I.n_chunks = (uint32_t)g.n_chunks;
    I.n_tiles = (uint32_t)g.n_tiles;
    I.chunk = g.chunk;
    I.warm = g.warm;
    const uint64_t need = ws_layout(g, false, nullptr, nullptr);
    char *ws = (char *)d_workspace;
    bool own = false;
    if (ws) {
        if (workspace_bytes < need) return AC_E_OVERFLOW;
    } else {
        if (test_alloc_fails() || hipMallocAsync((void **)&ws, need, st) != hipSuccess) {
            (void)hipGetLastError();
            return AC_E_NOMEM;
        }
        own = true;
    }
    Workspace w;
    ws_layout(g, false, ws, &w);
    rc = fmt == AC_TEXT_2BIT ? launch_single<AC_TEXT_2BIT>(g, I, w, st)
                             : launch_single<AC_TEXT_U8>(g, I, w, st);
    if (own) (void)hipFreeAsync(ws, st);
    return rc;
}

int ac_scan_noalloc(const ac_dict *d, const void *d_text, uint64_t n, uint32_t fmt,
                    ac_match *d_out, uint64_t capacity, uint64_t *d_count, const ac_tune *tune,
                    void *stream) {
    if (!d || !d_count) return AC_E_INVALID;
    if (capacity && !d_out) return AC_E_INVALID;
    if (!d->parts.empty()) return AC_E_INVALID;  // the partitioned scan allocates
    if (!d->d_delta) return AC_E_NO_DEVICE;
    int rc = validate_text(d, d_text, n, fmt);
    if (rc) return rc;
    uint64_t need = 0;
    if (n) {
        rc = ac_scan_workspace_size(d, n, fmt, tune, &need);
        if (rc) return rc;
    }
    if (need > kScratchBytes) return AC_E_TOO_LARGE;
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    // with a workspace given, ac_scan enqueues kernels only
    return ac_scan(d, d_text, n, fmt, d_out, capacity, d_count, tune, ws, kScratchBytes, stream);
}

int ac_encode(const uint8_t *d_ascii, uint64_t n, uint32_t alphabet, uint32_t fmt, void *d_out,
              uint64_t *d_invalid, void *stream) {
    if (alphabet > AC_ALPHA_PROTEIN || fmt > AC_TEXT_2BIT) return AC_E_INVALID;
    if (alphabet == AC_ALPHA_PROTEIN && fmt == AC_TEXT_2BIT) return AC_E_INVALID;
    if (n && (!d_ascii || !d_out)) return AC_E_INVALID;
    if (n >= kMaxText) return AC_E_TOO_LARGE;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *inv = (unsigned long long *)d_invalid;
    if (inv) hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, inv, 1u, 0ull);
    if (n) {
        KTimer tm(AC_K_ENCODE, st);
        const uint64_t threads = (n + 15) / 16;
        const uint32_t blocks = (uint32_t)((threads + 255) / 256);
        const uint8_t *in = d_ascii;
        uint8_t *out = (uint8_t *)d_out;
        if (alphabet == AC_ALPHA_DNA && fmt == AC_TEXT_2BIT)
            hipLaunchKernelGGL(k_encode_dna2, dim3((uint32_t)((n + 64 * 256 - 1) / (64 * 256))),
                               dim3(256), 0, st, in, n, out, inv);
        else if (alphabet == AC_ALPHA_DNA)
            hipLaunchKernelGGL((k_encode<AC_ALPHA_DNA, AC_TEXT_U8>), dim3(blocks), dim3(256), 0, st,
                               in, n, out, inv);
        else
            hipLaunchKernelGGL((k_encode<AC_ALPHA_PROTEIN, AC_TEXT_U8>), dim3(blocks), dim3(256), 0,
                               st, in, n, out, inv);
    }
    HIP_OK(hipGetLastError());
    return AC_OK;
}

}  // extern "C"

#include "batch.inc"
#include "extra.inc"
