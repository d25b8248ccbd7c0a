// C-ABI entry points that run on the host only: building, inspecting and
// releasing dictionaries.  The scan entry points live in scan.hip.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>

#include "internal.h"

extern "C" {

int ac_build(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
             const ac_build_opts *opts, ac_dict **out) {
    if (!out) return AC_E_INVALID;
    *out = nullptr;
    ac_build_opts o = {4, AC_PLACE_AUTO, 0, 0};
    if (opts) o = *opts;
    if (o.placement > AC_PLACE_LDS2 || (o.flags & ~(AC_BUILD_HOST_ONLY | AC_BUILD_SERIAL)))
        return AC_E_INVALID;
    ac_dict *d = new (std::nothrow) ac_dict();
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
    acx::release_dict(d);
    delete d;
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
    info->table_bytes = d->table_bytes;
    info->build_ms = d->build_ms;
    return AC_OK;
}

int ac_debug_export(const ac_dict *d, uint32_t *delta, uint32_t *out_off, uint32_t *out_ids,
                    uint32_t *depth) {
    if (!d) return AC_E_INVALID;
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
        default: return "unknown status";
    }
}

}  // extern "C"
