// GPU stage of Aho-Corasick for gfx950 (MI355X): the single-pass scan of the
// paper's section III.A, run as many independent passes over text chunks.
//
// Decomposition (the paper's section IV.A, first design, made exact): lane j
// owns the end positions [j*C, (j+1)*C) of the text.  It starts at the root
// max_len-1 (rounded up to a whole 32-bit text word) symbols before j*C, so
// that by the time it reaches j*C its state is the same one a single pass
// from the start of the text would hold: the state after reading a text
// prefix is its longest suffix that is a trie prefix, and no trie prefix is
// longer than max_len.  Every match is then reported by exactly one lane.
//
// One scan is four launches on the caller's stream:
//   k_count     every lane walks its chunk once with one table lookup per
//               symbol and counts the matches ending in it (sum of output-
//               set sizes of the states it passes through);
//   k_tile_scan one block turns per-tile sums into exclusive offsets;
//   k_scatter   per-chunk output offsets, and the list of chunks that have
//               at least one match;
//   k_emit      only the listed chunks are walked again; matches are written
//               at their final offsets, so the output comes out in
//               (end position, pattern id) order with no sort, and a
//               too-small output buffer still receives the first matches.
// The dense transition table lives in LDS when it fits, in HBM behind the
// L1/L2 caches otherwise, or split (hot first rows in LDS).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

namespace acx {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

enum { PL_LDS = 1, PL_GLOBAL = 2, PL_HYBRID = 3 };

constexpr uint32_t kLdsPad = 1024;     // zero rows past an LDS table (u8 codes >= sigma)
constexpr uint32_t kEmitThreads = 256;
constexpr uint32_t kMaxCountThreads = 1024;

// Per-instance parameters of a scan, shared by host and device.
struct Inst {
    const uint32_t *delta;  // row byte offsets: delta[s*sigma+a] = next*sigma*4
    const uint32_t *out_off;
    const uint32_t *out_ids;
    const uint8_t *text;
    ac_match *out;
    unsigned long long *count;
    uint64_t capacity;
    uint32_t n;            // text symbols
    uint32_t text_bytes4;  // text bytes rounded up to a multiple of 4
    uint32_t table_bytes;
    uint32_t fo_bytes;     // row offset of the first state with output
    uint32_t fo_state;     // its state number
    uint32_t hot_bytes;    // table bytes kept in LDS (0, part, or all)
    uint32_t lds_all;      // 1: whole table in LDS (with zero pad)
    uint32_t n_chunks;
    uint32_t chunk_base;   // first chunk of this instance in the chunk arrays
    uint32_t first_tile;   // first tile of this instance
    uint32_t n_tiles;
    uint32_t div_tz, div_inv;
    uint32_t sigma;
};

struct TileDesc {
    uint32_t inst;
    uint32_t first;  // first chunk (instance-local)
    uint32_t count;  // chunks in this tile
    uint32_t pad;
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ uint32_t lds_load(uint32_t byte_addr) {
    extern __shared__ uint32_t dyn_smem[];
    return *(lds_u32 *)((lds_u8 *)(lds_u32 *)dyn_smem + byte_addr);
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
    } else {
        uint64_t x = __builtin_bit_cast(uint64_t, v);
        uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
        uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of (a, b); returns totals through ta, tb.
// Every thread of the block must call it.  Uses 2*16 words of scratch.
__device__ __forceinline__ void block_excl_scan2(unsigned long long a, uint32_t b,
                                                 unsigned long long *ea, uint32_t *eb,
                                                 unsigned long long *ta, uint32_t *tb) {
    __shared__ unsigned long long s_a[16];
    __shared__ uint32_t s_b[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    unsigned long long ia = wave_incl_scan(a);
    uint32_t ib = wave_incl_scan(b);
    if (lane == 63) {
        s_a[wid] = ia;
        s_b[wid] = ib;
    }
    __syncthreads();
    unsigned long long pa = 0, sa = 0;
    uint32_t pb = 0, sb = 0;
    for (int w = 0; w < nw; ++w) {
        if (w == wid) {
            pa = sa;
            pb = sb;
        }
        sa += s_a[w];
        sb += s_b[w];
    }
    *ea = pa + ia - a;
    *eb = pb + ib - b;
    *ta = sa;
    *tb = sb;
    __syncthreads();
}

// Row byte offset -> state number (exact division by sigma*4).
__device__ __forceinline__ uint32_t row_state(uint32_t e, uint32_t tz, uint32_t inv) {
    return (e >> tz) * inv;
}

// One symbol: bits of the text word at compile-time (k) or run-time slot.
template <int FMT>
__device__ __forceinline__ uint32_t sym_bytes(uint32_t x, uint32_t k) {
    // symbol code * 4 (= its byte offset within a table row)
    if constexpr (FMT == AC_TEXT_2BIT)
        return __builtin_amdgcn_ubfe(x, 2 * k, 2) << 2;
    else
        return __builtin_amdgcn_ubfe(x, 8 * k, 8) << 2;
}

// Table lookups of a uniform (wave-invariant) table.
template <int PLACE>
struct UTable {
    rsrc_t g;
    uint32_t hot;
    __device__ __forceinline__ uint32_t operator()(uint32_t a) const {
        if constexpr (PLACE == PL_LDS) {
            return lds_load(a);
        } else if constexpr (PLACE == PL_GLOBAL) {
            return __builtin_amdgcn_raw_buffer_load_b32(g, a, 0, 0);
        } else {
            uint32_t v;
            if (a < hot)
                v = lds_load(a);
            else
                v = __builtin_amdgcn_raw_buffer_load_b32(g, a, 0, 0);
            return v;
        }
    }
};

// Text reads of a uniform text (bounds from the buffer resource: reads past
// the end return 0).
struct UText {
    rsrc_t r;
    uint32_t bytes4;
    __device__ __forceinline__ uint32_t word(int w) const {
        return w < 0 ? 0u : __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)w * 4u, 0, 0);
    }
    __device__ __forceinline__ u32x4 vec(uint32_t w) const {
        const uint32_t o = w * 4u;
        if (o + 16u <= bytes4) return __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
        u32x4 v;
        v.x = __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0);
        v.y = __builtin_amdgcn_raw_buffer_load_b32(r, o + 4, 0, 0);
        v.z = __builtin_amdgcn_raw_buffer_load_b32(r, o + 8, 0, 0);
        v.w = __builtin_amdgcn_raw_buffer_load_b32(r, o + 12, 0, 0);
        return v;
    }
};

// Per-lane table and text (batched emission: lanes of a wave may work on
// different instances).
struct LTable {
    const uint32_t *t;
    uint32_t bytes;
    __device__ __forceinline__ uint32_t operator()(uint32_t a) const {
        return a < bytes ? t[a >> 2] : 0u;
    }
};
struct LText {
    const uint32_t *t;
    uint32_t bytes4;
    __device__ __forceinline__ uint32_t word(int w) const {
        return (w < 0 || (uint32_t)w * 4u >= bytes4) ? 0u : t[w];
    }
};

template <int FMT>
struct Fmt {
    static constexpr uint32_t SPW = FMT == AC_TEXT_2BIT ? 16 : 4;  // symbols per 32-bit word
};

// Warm-up: walk warm words ending just before word w0 (words before the text
// start are skipped, which leaves the state at the root as it must be).
template <int FMT, class Tab, class Txt>
__device__ __forceinline__ uint32_t warm_up(const Tab &tab, const Txt &txt, int w0, uint32_t warm) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    uint32_t s = 0;
    for (uint32_t i = 0; i < warm; ++i) {
        const int w = w0 - (int)warm + (int)i;
        const uint32_t x = txt.word(w);
        const bool live = w >= 0;
#pragma unroll
        for (uint32_t k = 0; k < SPW; ++k) {
            const uint32_t ns = tab(s + sym_bytes<FMT>(x, k));
            s = live ? ns : s;
        }
    }
    return s;
}

// ------------------------------------------------------------------ count

// Walk chunk j and count the matches that end in it.
template <int FMT, int PLACE>
__device__ __forceinline__ uint32_t walk_count(const UTable<PLACE> &tab, const UText &txt,
                                               const uint32_t *__restrict__ out_off,
                                               uint32_t fo, uint32_t fo_state, uint32_t tz,
                                               uint32_t inv, uint32_t j, uint32_t chunk,
                                               uint32_t warm, uint32_t lim) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    const uint32_t wpc = chunk / SPW;
    const uint32_t w0 = j * wpc;
    uint32_t s = warm_up<FMT>(tab, txt, (int)w0, warm);
    uint32_t cnt = 0;
    u32x4 nx = txt.vec(w0);
    for (uint32_t v = 0; v < wpc; v += 4) {
        const u32x4 x4 = nx;
        if (v + 4 < wpc) nx = txt.vec(w0 + v + 4);
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t x = x4[q];
            const uint32_t s_in = s;
            uint32_t acc = 0;
#pragma unroll
            for (uint32_t k = 0; k < SPW; ++k) {
                s = tab(s + sym_bytes<FMT>(x, k));
                acc = acc > s ? acc : s;
            }
            if (acc >= fo) {
                // rare: walk the word again and add the output-set sizes
                const uint32_t p0 = (v + q) * SPW;
                uint32_t r = s_in;
                for (uint32_t k = 0; k < SPW; ++k) {
                    r = tab(r + sym_bytes<FMT>(x, k));
                    if (r >= fo && p0 + k < lim) {
                        const uint32_t o = row_state(r, tz, inv) - fo_state;
                        cnt += out_off[o + 1] - out_off[o];
                    }
                }
            }
        }
    }
    return cnt;
}

// Copy the LDS part of a table (zero-filled past the table's end).
__device__ __forceinline__ void load_lds_table(rsrc_t g, uint32_t bytes) {
    extern __shared__ uint32_t dyn_smem[];
    for (uint32_t o = threadIdx.x * 4u; o < bytes; o += blockDim.x * 4u)
        ((lds_u32 *)dyn_smem)[o >> 2] = __builtin_amdgcn_raw_buffer_load_b32(g, o, 0, 0);
}

// Persistent count kernel.  Block b takes a contiguous range of tiles; a
// tile is blockDim.x chunks of one instance, one chunk per lane.
template <int FMT, bool BATCH>
__global__ __launch_bounds__(kMaxCountThreads) void k_count(
    Inst single, const Inst *__restrict__ insts, const TileDesc *__restrict__ tiles,
    uint32_t n_tiles, uint32_t chunk, uint32_t warm, uint32_t *__restrict__ cnt,
    unsigned long long *__restrict__ tile_sum, uint32_t *__restrict__ tile_nz) {
    __shared__ unsigned long long red_a[16];
    __shared__ uint32_t red_b[16];
    const uint32_t t0 = (uint32_t)(((uint64_t)n_tiles * blockIdx.x) / gridDim.x);
    const uint32_t t1 = (uint32_t)(((uint64_t)n_tiles * (blockIdx.x + 1)) / gridDim.x);
    int cur = -1;
    for (uint32_t t = t0; t < t1; ++t) {
        uint32_t inst = 0, first, count;
        if constexpr (BATCH) {
            const TileDesc td = tiles[t];
            inst = uniform(td.inst);
            first = uniform(td.first);
            count = uniform(td.count);
        } else {
            first = t * blockDim.x;
            count = min(blockDim.x, single.n_chunks - first);
        }
        const Inst &I = BATCH ? insts[inst] : single;
        const uint32_t *delta = uniform(I.delta);
        const uint32_t table_bytes = uniform(I.table_bytes);
        const uint32_t hot = uniform(I.hot_bytes);
        const uint32_t lds_all = uniform(I.lds_all);
        const rsrc_t gtab = make_rsrc(delta, table_bytes);
        if ((int)inst != cur) {
            if (hot) {
                __syncthreads();
                load_lds_table(gtab, lds_all ? hot + kLdsPad : hot);
                __syncthreads();
            }
            cur = (int)inst;
        }
        const uint32_t n = uniform(I.n);
        const UText txt{make_rsrc(uniform(I.text), uniform(I.text_bytes4)), uniform(I.text_bytes4)};
        const uint32_t *out_off = uniform(I.out_off);
        const uint32_t fo = uniform(I.fo_bytes), fos = uniform(I.fo_state);
        const uint32_t tz = uniform(I.div_tz), inv = uniform(I.div_inv);
        const uint32_t lane_chunk = first + threadIdx.x;
        const bool valid = threadIdx.x < count;
        const uint32_t j = valid ? lane_chunk : first;
        const uint64_t begin = (uint64_t)j * chunk;
        const uint32_t lim = valid ? (uint32_t)min<uint64_t>(chunk, n - begin) : 0u;
        uint32_t c;
        if (lds_all) {
            c = walk_count<FMT, PL_LDS>(UTable<PL_LDS>{gtab, hot}, txt, out_off, fo, fos, tz, inv, j,
                                        chunk, warm, lim);
        } else if (hot == 0) {
            c = walk_count<FMT, PL_GLOBAL>(UTable<PL_GLOBAL>{gtab, 0}, txt, out_off, fo, fos, tz,
                                           inv, j, chunk, warm, lim);
        } else {
            c = walk_count<FMT, PL_HYBRID>(UTable<PL_HYBRID>{gtab, hot}, txt, out_off, fo, fos, tz,
                                           inv, j, chunk, warm, lim);
        }
        if (valid) cnt[uniform(I.chunk_base) + lane_chunk] = c;
        // tile totals
        const unsigned long long ws = wave_sum_u64(c);
        const uint32_t wz = wave_sum_u32(c != 0);
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) {
            red_a[wid] = ws;
            red_b[wid] = wz;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long a = 0;
            uint32_t b = 0;
            for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
                a += red_a[w];
                b += red_b[w];
            }
            tile_sum[t] = a;
            tile_nz[t] = b;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ offsets

// One block: exclusive offsets of the tile sums.  totals[0] = matches,
// totals[1] = chunks with matches; tile_off[n] / tile_nzoff[n] = totals.
__global__ __launch_bounds__(1024) void k_tile_scan(const unsigned long long *__restrict__ tile_sum,
                                                    const uint32_t *__restrict__ tile_nz,
                                                    uint32_t n, unsigned long long *tile_off,
                                                    uint32_t *tile_nzoff,
                                                    unsigned long long *totals,
                                                    unsigned long long *single_count) {
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t b = min(n, threadIdx.x * per), e = min(n, b + per);
    unsigned long long sa = 0;
    uint32_t sb = 0;
    for (uint32_t i = b; i < e; ++i) {
        sa += tile_sum[i];
        sb += tile_nz[i];
    }
    unsigned long long ea, ta;
    uint32_t eb, tb;
    block_excl_scan2(sa, sb, &ea, &eb, &ta, &tb);
    for (uint32_t i = b; i < e; ++i) {
        tile_off[i] = ea;
        tile_nzoff[i] = eb;
        ea += tile_sum[i];
        eb += tile_nz[i];
    }
    if (threadIdx.x == 0) {
        tile_off[n] = ta;
        tile_nzoff[n] = tb;
        totals[0] = ta;
        totals[1] = tb;
        if (single_count) *single_count = ta;
    }
}

// One block per tile: output offset of every chunk with matches, appended
// to the work list of k_emit in text order.
template <bool BATCH>
__global__ __launch_bounds__(kMaxCountThreads) void k_scatter(
    Inst single, const Inst *__restrict__ insts, const TileDesc *__restrict__ tiles,
    const uint32_t *__restrict__ cnt, const unsigned long long *__restrict__ tile_off,
    const uint32_t *__restrict__ tile_nzoff, uint32_t *__restrict__ list_chunk,
    uint32_t *__restrict__ list_inst, unsigned long long *__restrict__ list_off) {
    const uint32_t t = blockIdx.x;
    uint32_t inst = 0, first, count, chunk_base = 0;
    unsigned long long base_off = 0;
    if constexpr (BATCH) {
        const TileDesc td = tiles[t];
        inst = td.inst;
        first = td.first;
        count = td.count;
        chunk_base = insts[inst].chunk_base;
        base_off = tile_off[insts[inst].first_tile];
    } else {
        first = t * blockDim.x;
        count = min(blockDim.x, single.n_chunks - first);
    }
    const bool valid = threadIdx.x < count;
    const uint32_t j = first + threadIdx.x;
    const uint32_t c = valid ? cnt[chunk_base + j] : 0u;
    unsigned long long ea, ta;
    uint32_t eb, tb;
    block_excl_scan2(c, c != 0, &ea, &eb, &ta, &tb);
    if (c != 0) {
        const uint32_t k = tile_nzoff[t] + eb;
        list_chunk[k] = j;
        if constexpr (BATCH) list_inst[k] = inst;
        list_off[k] = tile_off[t] + ea - base_off;
    }
}

__global__ void k_inst_totals(const Inst *__restrict__ insts, uint32_t n_inst,
                              const unsigned long long *__restrict__ tile_off) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const Inst &I = insts[i];
    *I.count = tile_off[I.first_tile + I.n_tiles] - tile_off[I.first_tile];
}

__global__ void k_fill_u64(unsigned long long *p, uint32_t n, unsigned long long v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ emit

// Per-wave record table for cooperative writing of output sets.
struct WaveRecs {
    uint32_t incl[64];   // inclusive prefix of output-set sizes
    uint32_t ids[64];    // first index of the set in out_ids
    uint32_t end[64];    // end position
    uint32_t inst[64];   // instance (batched form)
    unsigned long long off[64];  // output offset of the set's first match
};

// All lanes of the wave call this with `has` set where the lane's state
// (row offset e) is an output state at text position pos.  The wave then
// writes all the matches of all these states together: item k of the
// concatenated sets goes to lane k % 64, so consecutive lanes write
// consecutive 8-byte slots of the output.
template <bool BATCH>
__device__ __forceinline__ void emit_sets(WaveRecs &R, bool has, uint32_t e, uint32_t pos,
                                          unsigned long long &off, uint32_t inst,
                                          const Inst &I0, const Inst *__restrict__ insts,
                                          const uint32_t *out_off, uint32_t fo_state, uint32_t tz,
                                          uint32_t inv) {
    const uint32_t lane = threadIdx.x & 63;
    uint32_t len = 0, first = 0;
    if (has) {
        const uint32_t o = row_state(e, tz, inv) - fo_state;
        first = out_off[o];
        len = out_off[o + 1] - first;
    }
    const uint32_t incl = wave_incl_scan(len);
    const uint32_t total = __shfl(incl, 63, 64);
    R.incl[lane] = incl;
    R.ids[lane] = first;
    R.end[lane] = pos;
    R.off[lane] = off;
    if constexpr (BATCH) R.inst[lane] = inst;
    off += len;
    wave_sync();
    for (uint32_t k = lane; k < total; k += 64) {
        uint32_t r = 0;
#pragma unroll
        for (uint32_t step = 32; step > 0; step >>= 1)
            if (R.incl[r + step - 1] <= k) r += step;
        const uint32_t excl = r ? R.incl[r - 1] : 0u;
        const uint32_t idx = k - excl;
        const unsigned long long dst = R.off[r] + idx;
        const Inst &I = BATCH ? insts[R.inst[r]] : I0;
        if (dst < I.capacity) {
            ac_match m;
            m.pattern_id = I.out_ids[R.ids[r] + idx];
            m.end_pos = R.end[r];
            I.out[dst] = m;
        }
    }
    wave_sync();
}

// Persistent emit kernel over the list of chunks with matches.
template <int FMT, bool BATCH>
__global__ __launch_bounds__(kEmitThreads) void k_emit(
    Inst single, const Inst *__restrict__ insts, uint32_t chunk, uint32_t warm,
    const uint32_t *__restrict__ list_chunk, const uint32_t *__restrict__ list_inst,
    const unsigned long long *__restrict__ list_off, const unsigned long long *__restrict__ totals) {
    constexpr uint32_t SPW = Fmt<FMT>::SPW;
    __shared__ WaveRecs recs[kEmitThreads / 64];
    WaveRecs &R = recs[threadIdx.x >> 6];
    const uint32_t nz = (uint32_t)totals[1];
    const uint32_t wpc = chunk / SPW;
    for (uint32_t base = blockIdx.x * blockDim.x; base < nz; base += gridDim.x * blockDim.x) {
        const uint32_t idx = base + threadIdx.x;
        const bool valid = idx < nz;
        const uint32_t j = valid ? list_chunk[idx] : 0u;
        uint32_t inst = 0;
        if constexpr (BATCH) inst = valid ? list_inst[idx] : 0u;
        unsigned long long off = valid ? list_off[idx] : 0ull;
        const Inst &I = BATCH ? insts[inst] : single;
        const uint32_t n = I.n;
        const uint64_t begin = (uint64_t)j * chunk;
        const uint32_t lim = valid ? (uint32_t)min<uint64_t>(chunk, n - begin) : 0u;
        const uint32_t fo = I.fo_bytes, fos = I.fo_state, tz = I.div_tz, inv = I.div_inv;
        const uint32_t *out_off = I.out_off;
        const uint32_t w0 = j * wpc;
        auto body = [&](const auto &tab, const auto &txt) {
            uint32_t s = warm_up<FMT>(tab, txt, (int)w0, warm);
            for (uint32_t w = 0; w < wpc; ++w) {
                const uint32_t x = txt.word((int)(w0 + w));
                const uint32_t s_in = s;
                uint32_t acc = 0;
#pragma unroll
                for (uint32_t k = 0; k < SPW; ++k) {
                    s = tab(s + sym_bytes<FMT>(x, k));
                    acc = acc > s ? acc : s;
                }
                if (__any(acc >= fo && lim > 0)) {
                    const uint32_t p0 = w * SPW;
                    uint32_t r = s_in;
                    for (uint32_t k = 0; k < SPW; ++k) {
                        r = tab(r + sym_bytes<FMT>(x, k));
                        const bool has = r >= fo && p0 + k < lim;
                        if (__any(has))
                            emit_sets<BATCH>(R, has, r, (uint32_t)(begin + p0 + k), off, inst,
                                             single, insts, out_off, fos, tz, inv);
                    }
                }
            }
        };
        if constexpr (BATCH) {
            LTable tab{I.delta, I.table_bytes};
            LText txt{(const uint32_t *)I.text, I.text_bytes4};
            body(tab, txt);
        } else {
            UTable<PL_GLOBAL> tab{make_rsrc(single.delta, single.table_bytes), 0};
            UText txt{make_rsrc(single.text, single.text_bytes4), single.text_bytes4};
            body(tab, txt);
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

int upload_dict(ac_dict *d) {
    const HostTables &T = d->host;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::vector<uint32_t> rows(T.delta.size());
    const uint32_t row = T.sigma * 4u;
    for (size_t i = 0; i < rows.size(); ++i) rows[i] = T.delta[i] * row;
    const size_t off_bytes = T.out_off.size() * 4;
    const size_t ids_bytes = std::max<size_t>(4, T.out_ids.size() * 4);
    if (hipMalloc((void **)&d->d_delta, rows.size() * 4) != hipSuccess ||
        hipMalloc((void **)&d->d_out_off, off_bytes) != hipSuccess ||
        hipMalloc((void **)&d->d_out_ids, ids_bytes) != hipSuccess) {
        (void)hipGetLastError();
        release_dict(d);
        return AC_E_NOMEM;
    }
    if (hipMemcpy(d->d_delta, rows.data(), rows.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_out_off, T.out_off.data(), off_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        (!T.out_ids.empty() &&
         hipMemcpy(d->d_out_ids, T.out_ids.data(), T.out_ids.size() * 4, hipMemcpyHostToDevice) !=
             hipSuccess)) {
        (void)hipGetLastError();
        release_dict(d);
        return AC_E_HIP;
    }
    d->device = dev;
    return AC_OK;
}

void release_dict(ac_dict *d) {
    if (d->d_delta) (void)hipFree(d->d_delta);
    if (d->d_out_off) (void)hipFree(d->d_out_off);
    if (d->d_out_ids) (void)hipFree(d->d_out_ids);
    d->d_delta = d->d_out_off = d->d_out_ids = nullptr;
    (void)hipGetLastError();
}

// ---------------------------------------------------------- launch geometry

static uint32_t spw_of(uint32_t fmt) { return fmt == AC_TEXT_2BIT ? 16u : 4u; }

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct Geom {
    uint32_t chunk = 0, threads = 0, warm = 0, grid_count = 0, grid_emit = 0;
    uint32_t lds_bytes = 0;  // dynamic LDS of k_count
    uint64_t n_chunks = 0, n_tiles = 0;
};

struct Workspace {
    uint32_t *cnt;
    unsigned long long *tile_sum;
    uint32_t *tile_nz;
    unsigned long long *tile_off;
    uint32_t *tile_nzoff;
    unsigned long long *totals;
    uint32_t *list_chunk;
    uint32_t *list_inst;
    unsigned long long *list_off;
};

static uint64_t ws_layout(uint64_t n_chunks, uint64_t n_tiles, bool batch, char *base,
                          Workspace *w) {
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        char *p = base ? base + o : nullptr;
        o += align256(std::max<uint64_t>(bytes, 8));
        return p;
    };
    Workspace t;
    t.cnt = (uint32_t *)take(4 * n_chunks);
    t.tile_sum = (unsigned long long *)take(8 * n_tiles);
    t.tile_nz = (uint32_t *)take(4 * n_tiles);
    t.tile_off = (unsigned long long *)take(8 * (n_tiles + 1));
    t.tile_nzoff = (uint32_t *)take(4 * (n_tiles + 1));
    t.totals = (unsigned long long *)take(16);
    t.list_chunk = (uint32_t *)take(4 * n_chunks);
    t.list_inst = batch ? (uint32_t *)take(4 * n_chunks) : nullptr;
    t.list_off = (unsigned long long *)take(8 * n_chunks);
    if (w) *w = t;
    return o;
}

// Placement of one dictionary's table: returns hot bytes and lds_all.
static void choose_placement(const ac_dict *d, uint32_t requested, uint32_t lds_limit,
                             uint32_t *hot, uint32_t *lds_all) {
    const uint32_t tb = (uint32_t)d->table_bytes;
    const uint32_t row = d->host.sigma * 4u;
    uint32_t p = requested ? requested : d->placement;
    const bool fits = tb + kLdsPad <= lds_limit;
    if (p == AC_PLACE_AUTO) p = fits ? AC_PLACE_LDS : AC_PLACE_GLOBAL;
    if (p == AC_PLACE_LDS && !fits) p = AC_PLACE_HYBRID;
    if (p == AC_PLACE_LDS) {
        *hot = tb;
        *lds_all = 1;
    } else if (p == AC_PLACE_GLOBAL) {
        *hot = 0;
        *lds_all = 0;
    } else {
        uint32_t rows = d->hot_states ? d->hot_states : lds_limit / row;
        uint64_t h = std::min<uint64_t>((uint64_t)rows * row, lds_limit / row * row);
        if (h >= tb) h = tb;  // the whole table fits: still a split, all hot
        *hot = (uint32_t)h;
        *lds_all = 0;
    }
}

static int resolve_geom(const ac_dict *const *dicts, const uint64_t *ns, uint32_t n_inst,
                        uint32_t fmt, const ac_tune *tune, Geom *g) {
    uint32_t cus = 0, lds = 0;
    int rc = device_limits(&cus, &lds);
    if (rc != AC_OK) return rc;
    const uint32_t lds_limit = lds - 512;  // static LDS of the count kernel
    uint32_t max_len = 1;
    uint64_t total = 0, biggest = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        max_len = std::max(max_len, dicts[i]->host.max_len);
        total += ns[i];
        biggest = std::max(biggest, ns[i]);
    }
    const uint32_t spw = spw_of(fmt);
    g->warm = (max_len - 1 + spw - 1) / spw;
    g->threads = (tune && tune->block_threads) ? tune->block_threads : 1024u;
    if (g->threads < 64 || g->threads > kMaxCountThreads || g->threads % 64) return AC_E_INVALID;
    uint32_t chunk = tune ? tune->chunk : 0;
    if (chunk && (chunk % 64 || chunk > (1u << 20))) return AC_E_INVALID;
    // LDS need of the count kernel
    uint32_t lds_bytes = 0;
    const uint32_t req = tune ? tune->placement : 0;
    if (req > AC_PLACE_HYBRID) return AC_E_INVALID;
    for (uint32_t i = 0; i < n_inst; ++i) {
        uint32_t hot, all;
        choose_placement(dicts[i], req, lds_limit, &hot, &all);
        lds_bytes = std::max(lds_bytes, all ? hot + kLdsPad : hot);
    }
    g->lds_bytes = lds_bytes;
    uint32_t bpc = (tune && tune->blocks_per_cu) ? tune->blocks_per_cu
                                                  : std::max(1u, 2048u / g->threads);
    if (lds_bytes) bpc = std::max(1u, std::min(bpc, (lds + 0u) / (lds_bytes + 512u)));
    const uint64_t slots = (uint64_t)cus * bpc;
    if (!chunk) {
        chunk = 1024;
        while (chunk > 64 && (total / chunk) / g->threads < slots) chunk /= 2;
    }
    g->chunk = chunk;
    g->n_chunks = 0;
    g->n_tiles = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const uint64_t c = (ns[i] + chunk - 1) / chunk;
        g->n_chunks += c;
        g->n_tiles += (c + g->threads - 1) / g->threads;
    }
    if (g->n_chunks >= (1ull << 31) || g->n_tiles >= (1ull << 31)) return AC_E_TOO_LARGE;
    g->grid_count = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g->n_tiles, slots));
    g->grid_emit = cus * 8;
    return AC_OK;
}

static void fill_inst(const ac_dict *d, const void *text, uint64_t n, uint32_t fmt, ac_match *out,
                      uint64_t cap, uint64_t *count, uint32_t req_place, uint32_t lds_limit,
                      Inst *I) {
    memset(I, 0, sizeof(*I));
    I->delta = d->d_delta;
    I->out_off = d->d_out_off;
    I->out_ids = d->d_out_ids;
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
    choose_placement(d, req_place, lds_limit, &I->hot_bytes, &I->lds_all);
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

static const uint64_t kMaxText = (1ull << 32) - 256;

static int validate_text(const ac_dict *d, const void *text, uint64_t n, uint32_t fmt) {
    if (fmt != AC_TEXT_U8 && fmt != AC_TEXT_2BIT) return AC_E_INVALID;
    if (fmt == AC_TEXT_2BIT && d->host.sigma != 4) return AC_E_INVALID;
    if (n >= kMaxText) return AC_E_TOO_LARGE;
    if (n && !text) return AC_E_INVALID;
    return AC_OK;
}

template <int FMT>
static int launch_single(const Geom &g, const Inst &I, const Workspace &w, hipStream_t st) {
    const uint32_t T = (uint32_t)g.n_tiles;
    auto kc = k_count<FMT, false>;
    int rc = allow_lds(kc, g.lds_bytes);
    if (rc) return rc;
    hipLaunchKernelGGL(kc, dim3(g.grid_count), dim3(g.threads), g.lds_bytes, st, I, nullptr,
                       nullptr, T, g.chunk, g.warm, w.cnt, w.tile_sum, w.tile_nz);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, w.tile_sum, w.tile_nz, T,
                       w.tile_off, w.tile_nzoff, w.totals, I.count);
    hipLaunchKernelGGL(k_scatter<false>, dim3(T), dim3(g.threads), 0, st, I, nullptr, nullptr,
                       w.cnt, w.tile_off, w.tile_nzoff, w.list_chunk, nullptr, w.list_off);
    hipLaunchKernelGGL((k_emit<FMT, false>), dim3(g.grid_emit), dim3(kEmitThreads), 0, st, I,
                       nullptr, g.chunk, g.warm, w.list_chunk, nullptr, w.list_off, w.totals);
    HIP_OK(hipGetLastError());
    return AC_OK;
}

}  // namespace acx

using namespace acx;

extern "C" {

int ac_device_info(uint32_t *compute_units, uint32_t *lds_bytes_per_block) {
    return device_limits(compute_units, lds_bytes_per_block);
}

int ac_scan_workspace_size(const ac_dict *d, uint64_t n, uint32_t fmt, const ac_tune *tune,
                           uint64_t *bytes) {
    if (!d || !bytes) return AC_E_INVALID;
    int rc = validate_text(d, (const void *)1, n, fmt);
    if (rc) return rc;
    Geom g;
    rc = resolve_geom(&d, &n, 1, fmt, tune, &g);
    if (rc) return rc;
    *bytes = ws_layout(g.n_chunks, g.n_tiles, false, nullptr, nullptr);
    return AC_OK;
}

int ac_scan(const ac_dict *d, const void *d_text, uint64_t n, uint32_t fmt, ac_match *d_out,
            uint64_t capacity, uint64_t *d_count, const ac_tune *tune, void *d_workspace,
            uint64_t workspace_bytes, void *stream) {
    if (!d || !d_count) return AC_E_INVALID;
    if (!d->d_delta) return AC_E_NO_DEVICE;
    if (capacity && !d_out) return AC_E_INVALID;
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
    fill_inst(d, d_text, n, fmt, d_out, capacity, d_count, tune ? tune->placement : 0, lds - 512,
              &I);
    I.n_chunks = (uint32_t)g.n_chunks;
    I.n_tiles = (uint32_t)g.n_tiles;
    const uint64_t need = ws_layout(g.n_chunks, g.n_tiles, false, nullptr, nullptr);
    char *ws = (char *)d_workspace;
    bool own = false;
    if (ws) {
        if (workspace_bytes < need) return AC_E_OVERFLOW;
    } else {
        if (hipMallocAsync((void **)&ws, need, st) != hipSuccess) {
            (void)hipGetLastError();
            return AC_E_NOMEM;
        }
        own = true;
    }
    Workspace w;
    ws_layout(g.n_chunks, g.n_tiles, false, ws, &w);
    rc = fmt == AC_TEXT_2BIT ? launch_single<AC_TEXT_2BIT>(g, I, w, st)
                             : launch_single<AC_TEXT_U8>(g, I, w, st);
    if (own) (void)hipFreeAsync(ws, st);
    return rc;
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
        const uint64_t threads = (n + 15) / 16;
        const uint32_t blocks = (uint32_t)((threads + 255) / 256);
        const uint8_t *in = d_ascii;
        uint8_t *out = (uint8_t *)d_out;
        if (alphabet == AC_ALPHA_DNA && fmt == AC_TEXT_2BIT)
            hipLaunchKernelGGL((k_encode<AC_ALPHA_DNA, AC_TEXT_2BIT>), dim3(blocks), dim3(256), 0, st,
                               in, n, out, inv);
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
