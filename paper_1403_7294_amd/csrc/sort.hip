// Canonical (end position, pattern id) order for match records that were
// produced in another order: the partitioned scan (one machine per pattern
// slice, the paper's second design of section IV.A) and the failure-less
// kernel.  A record {pattern_id, end_pos} read as a little-endian 64-bit
// word is end_pos * 2^32 + pattern_id, so a radix sort of those words over
// the significant bits gives the order; records whose ties on end_pos are
// already in id order need only the end bits (radix sort is stable).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <hipcub/device/device_radix_sort.hpp>
#include <hipcub/device/device_scan.hpp>

#include "internal.h"

namespace acx {

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static size_t radix_temp_bytes(uint64_t n) {
    size_t bytes = 0;
    hipcub::DoubleBuffer<unsigned long long> db(nullptr, nullptr);
    if (hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, db, (int)n, 0, 64) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return bytes;
}

uint64_t sort_workspace_bytes(uint64_t n) { return align256(n * 8) + align256(radix_temp_bytes(n)); }

int sort_matches(ac_match *d, uint64_t n, uint32_t flags, uint32_t end_bits, void *ws,
                 uint64_t ws_bytes, hipStream_t st) {
    if (n < 2) return AC_OK;
    if (n >= (1ull << 31)) return AC_E_TOO_LARGE;
    if (end_bits == 0 || end_bits > 32) end_bits = 32;
    const uint64_t need = sort_workspace_bytes(n);
    if (ws_bytes < need) return AC_E_OVERFLOW;
    unsigned long long *keys = (unsigned long long *)d;
    unsigned long long *alt = (unsigned long long *)ws;
    void *temp = (char *)ws + align256(n * 8);
    size_t temp_bytes = need - align256(n * 8);
    hipcub::DoubleBuffer<unsigned long long> db(keys, alt);
    const int begin = (flags & AC_SORT_BY_END) ? 32 : 0;
    if (hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, db, (int)n, begin, 32 + (int)end_bits,
                                          st) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_HIP;
    }
    if (db.Current() != keys &&
        hipMemcpyAsync(keys, db.Current(), n * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_HIP;
    }
    return AC_OK;
}

// out[i] = in[0] + ... + in[i-1] over n 64-bit counts (stream-ordered; the
// temporary storage is taken from and returned to the stream's pool).
int exclusive_sum_u64(const unsigned long long *in, unsigned long long *out, uint64_t n,
                      hipStream_t st) {
    if (n == 0) return AC_OK;
    if (n >= (1ull << 31)) return AC_E_TOO_LARGE;
    size_t bytes = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, st) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_HIP;
    }
    void *temp = nullptr;
    if (hipMallocAsync(&temp, std::max<size_t>(bytes, 8), st) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_NOMEM;
    }
    const hipError_t e = hipcub::DeviceScan::ExclusiveSum(temp, bytes, in, out, (int)n, st);
    (void)hipFreeAsync(temp, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_HIP;
    }
    return AC_OK;
}

}  // namespace acx

extern "C" {

int ac_sort_workspace_size(uint64_t n, uint64_t *bytes) {
    if (!bytes) return AC_E_INVALID;
    if (n >= (1ull << 31)) return AC_E_TOO_LARGE;
    *bytes = acx::sort_workspace_bytes(n);
    return AC_OK;
}

int ac_sort_matches(ac_match *d_matches, uint64_t n, uint32_t flags, uint32_t end_bits,
                    void *d_workspace, uint64_t workspace_bytes, void *stream) {
    if (n && !d_matches) return AC_E_INVALID;
    if (flags & ~AC_SORT_BY_END) return AC_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    if (n < 2) return AC_OK;
    if (n >= (1ull << 31)) return AC_E_TOO_LARGE;
    if (d_workspace) return acx::sort_matches(d_matches, n, flags, end_bits, d_workspace,
                                              workspace_bytes, st);
    const uint64_t need = acx::sort_workspace_bytes(n);
    void *ws = nullptr;
    if (hipMallocAsync(&ws, need, st) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_NOMEM;
    }
    const int rc = acx::sort_matches(d_matches, n, flags, end_bits, ws, need, st);
    (void)hipFreeAsync(ws, st);
    return rc;
}

}  // extern "C"
