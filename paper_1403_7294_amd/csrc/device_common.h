// Device-side helpers of the gfx950 scan kernels: buffer-resource loads,
// LDS access, wave-level reductions and scans, and the table / text access
// policies the walking loops are templated on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ac.h"

namespace acx {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

enum { PL_LDS = 1, PL_GLOBAL = 2, PL_HYBRID = 3, PL_LDS16 = 4 };

// A raw buffer resource over [p, p + bytes): loads at offsets >= bytes
// return 0 instead of touching memory (gfx9 buffer range checking).
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ uint32_t buf_load(rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// Byte-addressed read of the dynamic LDS region.
__device__ __forceinline__ uint32_t lds_load(uint32_t byte_addr) {
    extern __shared__ uint32_t dyn_smem[];
    return *(lds_u32 *)((lds_u8 *)(lds_u32 *)dyn_smem + byte_addr);
}

// Force a value the compiler cannot prove uniform into a scalar register.
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

// Make a wave's LDS writes visible to the other lanes of the same wave.
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

// Block-wide exclusive scan of three values (one 64-bit, two 32-bit), with
// block totals.  Every thread of the block must call it.
struct Scan3 {
    unsigned long long a;
    uint32_t b, c;
};
__device__ __forceinline__ void block_excl_scan3(Scan3 v, Scan3 *excl, Scan3 *total) {
    __shared__ unsigned long long s_a[16];
    __shared__ uint32_t s_b[16], s_c[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    const unsigned long long ia = wave_incl_scan(v.a);
    const uint32_t ib = wave_incl_scan(v.b), ic = wave_incl_scan(v.c);
    if (lane == 63) {
        s_a[wid] = ia;
        s_b[wid] = ib;
        s_c[wid] = ic;
    }
    __syncthreads();
    Scan3 pre = {0, 0, 0}, tot = {0, 0, 0};
    for (int w = 0; w < nw; ++w) {
        if (w == wid) pre = tot;
        tot.a += s_a[w];
        tot.b += s_b[w];
        tot.c += s_c[w];
    }
    excl->a = pre.a + ia - v.a;
    excl->b = pre.b + ib - v.b;
    excl->c = pre.c + ic - v.c;
    *total = tot;
    __syncthreads();
}

// Row byte offset (state * sigma * 4) -> state number: exact division by
// sigma * 4 = 2^tz * odd, as a shift and a multiply by the odd part's
// inverse modulo 2^32.
__device__ __forceinline__ uint32_t row_state(uint32_t e, uint32_t tz, uint32_t inv) {
    return (e >> tz) * inv;
}
// The same where the text format fixes sigma: 2-bit text means sigma 4,
// rows of 16 bytes, so the state is a shift (no multiply).
template <int FMT>
__device__ __forceinline__ uint32_t row_state_f(uint32_t e, uint32_t tz, uint32_t inv) {
    if constexpr (FMT == AC_TEXT_2BIT)
        return e >> 4;
    else
        return row_state(e, tz, inv);
}

template <int FMT>
struct Fmt {
    static constexpr uint32_t SPW = FMT == AC_TEXT_2BIT ? 16 : 4;  // symbols per 32-bit word
};

// Symbol k of text word x, times 4 (its byte offset within a table row).
template <int FMT>
__device__ __forceinline__ uint32_t sym_bytes(uint32_t x, uint32_t k) {
    if constexpr (FMT == AC_TEXT_2BIT)
        return __builtin_amdgcn_ubfe(x, 2 * k, 2) << 2;
    else
        return __builtin_amdgcn_ubfe(x, 8 * k, 8) << 2;
}

// Byte-addressed 16-bit read of the dynamic LDS region.
__device__ __forceinline__ uint32_t lds_load_u16(uint32_t byte_addr) {
    extern __shared__ uint32_t dyn_smem[];
    typedef __attribute__((address_space(3))) uint16_t lds_u16;
    return *(lds_u16 *)((lds_u8 *)(lds_u32 *)dyn_smem + byte_addr);
}

// Table of one wave-uniform dictionary.  Lookups take the byte address
// a = row offset + 4 * symbol in the 32-bit table and return the next
// state's row offset.
//   PL_LDS     the whole 32-bit table is in LDS;
//   PL_LDS16   the whole table is in LDS as 16-bit state ids, at half the
//              byte address;
//   PL_GLOBAL  the table is read through the L1/L2 caches;
//   PL_HYBRID  rows below `hot` (a byte bound in the 32-bit table) are in
//              LDS as 16-bit state ids, at half the byte address; an id of
//              0xFFFF (a state too far down the numbering for 16 bits) and
//              every other row are read from the 32-bit table.
template <int PLACE, bool ROW16 = false>
struct UTable {
    rsrc_t g;
    uint32_t hot;  // hybrid: first row offset not held in LDS
    uint32_t row;  // hybrid: sigma * 4, bytes of a 32-bit row (16 when ROW16)
    __device__ __forceinline__ uint32_t operator()(uint32_t a) const {
        if constexpr (PLACE == PL_LDS) {
            return lds_load(a);
        } else if constexpr (PLACE == PL_LDS16) {
            const uint32_t h = lds_load_u16(a >> 1);
            return ROW16 ? h << 4 : h * row;
        } else if constexpr (PLACE == PL_GLOBAL) {
            return buf_load(g, a);
        } else {
            // rows past the LDS part go to the cache hierarchy first, so
            // their latency overlaps the LDS read of the other lanes; a hot
            // row entry 0xFFFF (target id beyond 16 bits) is read again from
            // the 32-bit table.  Lanes that need no global read give the
            // load an offset past the buffer's end: the load returns 0
            // without a memory access, and the step stays straight-line
            // code, so the loads of independent chains can be in flight
            // together instead of each waiting behind an exec-mask branch.
            constexpr uint32_t kNoRead = 0xFFFFFFF0u;
            const bool in = a < hot;
            const uint32_t v1 = buf_load(g, in ? kNoRead : a);
            const uint32_t h = lds_load_u16((in ? a : 0u) >> 1);
            const bool esc = in && h == 0xFFFFu;
            uint32_t v2 = 0;
            if (esc) v2 = buf_load(g, a);
            return in ? (esc ? v2 : (ROW16 ? h << 4 : h * row)) : v1;
        }
    }
};

// Text of one wave-uniform instance; reads past the end return 0.
struct UText {
    rsrc_t r;
    uint32_t bytes4;  // readable bytes, rounded up to 4
    __device__ __forceinline__ uint32_t word(int w) const {
        return w < 0 ? 0u : buf_load(r, (uint32_t)w * 4u);
    }
    __device__ __forceinline__ u32x4 vec(uint32_t w) const {
        const uint32_t o = w * 4u;
        if (o + 16u <= bytes4) return __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
        u32x4 v;
        v.x = buf_load(r, o);
        v.y = buf_load(r, o + 4);
        v.z = buf_load(r, o + 8);
        v.w = buf_load(r, o + 12);
        return v;
    }
    // Same, marked non-temporal: text read once should not push the
    // transition table out of the L2 cache.
    __device__ __forceinline__ u32x4 vec_once(uint32_t w) const {
        constexpr int kNonTemporal = 2;  // cache-policy bit "nt" of gfx94x/gfx950
        const uint32_t o = w * 4u;
        if (o + 16u <= bytes4)
            return __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, kNonTemporal);
        u32x4 v;
        v.x = __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, kNonTemporal);
        v.y = __builtin_amdgcn_raw_buffer_load_b32(r, o + 4, 0, kNonTemporal);
        v.z = __builtin_amdgcn_raw_buffer_load_b32(r, o + 8, 0, kNonTemporal);
        v.w = __builtin_amdgcn_raw_buffer_load_b32(r, o + 12, 0, kNonTemporal);
        return v;
    }
};

// Per-lane table and text (batched kernels whose lanes may belong to
// different instances).  Bounds are checked explicitly.
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
    __device__ __forceinline__ u32x4 vec(uint32_t w) const {
        u32x4 v;
        v.x = word((int)w);
        v.y = word((int)w + 1);
        v.z = word((int)w + 2);
        v.w = word((int)w + 3);
        return v;
    }
};

// Walk `warm` text words ending just before word w0 from the root.  Words
// before the text start are skipped, leaving the state at the root.
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

}  // namespace acx
