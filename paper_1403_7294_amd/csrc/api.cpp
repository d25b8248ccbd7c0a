// C-ABI entry points that run on the host only: building, inspecting and
// releasing dictionaries.  The scan entry points live in scan.hip.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <new>

#include "internal.h"

namespace acx {

bool test_alloc_fails() {
    static const long long nth = [] {
        const char *e = getenv("AC_TEST_FAIL_ALLOC");
        return e ? atoll(e) : 0LL;
    }();
    if (nth <= 0) return false;
    static std::atomic<long long> seen{0};
    return ++seen == nth;
}

}  // namespace acx

extern "C" {

int ac_build(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
             const ac_build_opts *opts, ac_dict **out) {
    if (!out) return AC_E_INVALID;
    *out = nullptr;
    ac_build_opts o = {4, AC_PLACE_AUTO, 0, 0};
    if (opts) o = *opts;
    if (o.placement > AC_PLACE_LDS16 || (o.flags & ~(AC_BUILD_HOST_ONLY | AC_BUILD_SERIAL)))
        return AC_E_INVALID;
    ac_dict *d = acx::test_alloc_fails() ? nullptr : new (std::nothrow) ac_dict();
    if (!d) return AC_E_NOMEM;
    const auto t0 = std::chrono::steady_clock::now();
    int rc;
    try {
        rc = acx::compile_automaton(symbols, offsets, n_patterns, o.sigma, &d->host,
                                    (o.flags & AC_BUILD_SERIAL) ? 1u : 0u);
    } catch (const std::bad_alloc &) {
        rc = AC_E_NOMEM;
    }
    const auto t1 = std::chrono::steady_clock::now();
    if (rc != AC_OK) {
        delete d;
        return rc;
    }
    d->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    d->placement = o.placement;
    d->hot_states = o.hot_states;
    d->table_bytes = (uint64_t)d->host.states * d->host.sigma * 4u;
    if (!(o.flags & AC_BUILD_HOST_ONLY)) {
        rc = acx::upload_dict(d);
        if (rc != AC_OK) {
            delete d;
            return rc;
        }
    }
    *out = d;
    return AC_OK;
}

void ac_destroy(ac_dict *d) {
    if (!d) return;
    for (ac_dict *p : d->parts) ac_destroy(p);
    acx::release_dict(d);
    delete d;
}

int ac_build_partitioned(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
                         const ac_build_opts *opts, uint32_t parts, ac_dict **out) {
    if (!out) return AC_E_INVALID;
    *out = nullptr;
    if (!offsets || n_patterns == 0 || offsets[0] != 0) return AC_E_INVALID;
    ac_build_opts o = {4, AC_PLACE_AUTO, 0, 0};
    if (opts) o = *opts;
    if (o.sigma < 2 || o.sigma > 256 || o.placement > AC_PLACE_LDS16 ||
        (o.flags & ~(AC_BUILD_HOST_ONLY | AC_BUILD_SERIAL)))
        return AC_E_INVALID;
    if (parts > n_patterns) parts = n_patterns;
    const uint64_t total = offsets[n_patterns];
    // a slice of c characters has at most c + 1 states; LDS holds this many
    // 16-bit rows
    uint32_t cus = 0, lds = 160 * 1024;
    if (!(o.flags & AC_BUILD_HOST_ONLY) && acx::device_limits(&cus, &lds) != AC_OK)
        lds = 160 * 1024;
    const uint64_t rows = (lds - 2048u) / (o.sigma * 2u);
    uint32_t k = parts ? parts : (uint32_t)std::max<uint64_t>(1, (total + rows - 1) / rows);
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        k = std::min(k, n_patterns);
        std::vector<ac_dict *> built;
        std::vector<uint32_t> base;
        bool fits = true;
        int rc = AC_OK;
        uint32_t first = 0;
        for (uint32_t i = 0; i < k && rc == AC_OK; ++i) {
            // slice i ends at the first pattern boundary reaching (i+1)/k of
            // the characters (at least one pattern per slice)
            uint32_t last = first + 1;
            const uint64_t goal = total * (i + 1) / k;
            while (last < n_patterns && offsets[last] < goal && n_patterns - last > k - 1 - i)
                ++last;
            if (i == k - 1) last = n_patterns;
            std::vector<uint64_t> off(last - first + 1);
            for (uint32_t j = first; j <= last; ++j) off[j - first] = offsets[j] - offsets[first];
            const ac_build_opts po = o;
            ac_dict *p = nullptr;
            rc = ac_build(symbols + offsets[first], off.data(), last - first, &po, &p);
            if (rc != AC_OK) break;
            fits = fits && p->host.states <= rows;
            built.push_back(p);
            base.push_back(first);
            first = last;
        }
        if (rc != AC_OK || (!fits && !parts && k < n_patterns)) {
            for (ac_dict *p : built) ac_destroy(p);
            if (rc != AC_OK) return rc;
            ++k;
            continue;
        }
        ac_dict *d = acx::test_alloc_fails() ? nullptr : new (std::nothrow) ac_dict();
        if (!d) {
            for (ac_dict *p : built) ac_destroy(p);
            return AC_E_NOMEM;
        }
        d->parts = std::move(built);
        d->part_base = std::move(base);
        d->placement = o.placement;
        acx::HostTables &T = d->host;
        T.sigma = o.sigma;
        T.patterns = n_patterns;
        T.min_len = UINT32_MAX;
        for (ac_dict *p : d->parts) {
            T.states += p->host.states;
            T.min_len = std::min(T.min_len, p->host.min_len);
            T.max_len = std::max(T.max_len, p->host.max_len);
            T.max_output = std::max(T.max_output, p->host.max_output);
            d->table_bytes += p->table_bytes;
        }
        d->build_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = d;
        return AC_OK;
    }
}

int ac_dict_parts(const ac_dict *d, uint32_t *parts, uint32_t *first_ids) {
    if (!d || !parts) return AC_E_INVALID;
    *parts = (uint32_t)d->parts.size();
    if (first_ids)
        for (size_t i = 0; i < d->parts.size(); ++i) first_ids[i] = d->part_base[i];
    return AC_OK;
}

int ac_dict_get_info(const ac_dict *d, ac_dict_info *info) {
    if (!d || !info) return AC_E_INVALID;
    memset(info, 0, sizeof(*info));
    const acx::HostTables &T = d->host;
    info->states = T.states;
    info->patterns = T.patterns;
    info->sigma = T.sigma;
    info->min_len = T.min_len;
    info->max_len = T.max_len;
    info->first_output_state = T.first_output;
    info->max_output = T.max_output;
    info->placement = d->placement;
    info->hot_states = d->hot_states ? std::min(d->hot_states, d->hot16_rows) : d->hot16_rows;
    info->has_device = d->d_delta != nullptr;
    info->output_entries = T.out_ids.size();
    if (!d->parts.empty()) info->has_device = 1;
    for (const ac_dict *p : d->parts) {
        info->has_device = info->has_device && p->d_delta != nullptr;
        info->output_entries += p->host.out_ids.size();
    }
    info->table_bytes = d->table_bytes;
    info->build_ms = d->build_ms;
    return AC_OK;
}

int ac_debug_export(const ac_dict *d, uint32_t *delta, uint32_t *out_off, uint32_t *out_ids,
                    uint32_t *depth) {
    if (!d || !d->parts.empty()) return AC_E_INVALID;
    const acx::HostTables &T = d->host;
    if (delta) memcpy(delta, T.delta.data(), T.delta.size() * 4);
    if (out_off) memcpy(out_off, T.out_off.data(), T.out_off.size() * 4);
    if (out_ids && !T.out_ids.empty()) memcpy(out_ids, T.out_ids.data(), T.out_ids.size() * 4);
    if (depth) memcpy(depth, T.depth.data(), T.depth.size() * 4);
    return AC_OK;
}

const char *ac_status_str(int s) {
    switch (s) {
        case AC_OK: return "ok";
        case AC_E_INVALID: return "invalid argument";
        case AC_E_EMPTY_PATTERN: return "empty pattern";
        case AC_E_SYMBOL: return "pattern symbol outside the alphabet";
        case AC_E_TOO_LARGE: return "input too large";
        case AC_E_NOMEM: return "out of memory";
        case AC_E_OVERFLOW: return "workspace too small";
        case AC_E_HIP: return "HIP runtime error";
        case AC_E_NO_DEVICE: return "dictionary has no device tables";
        case AC_E_TIMEOUT: return "wait timed out";
        default: return "unknown status";
    }
}

}  // extern "C"
