// Host-side checks of the library's stage 1 (paper section III.A: goto,
// failure and output functions) built with AddressSanitizer and
// UndefinedBehaviorSanitizer, linked with the CPU oracle.
//
//   host_driver corpus FILE  every instance of FILE is compiled host-only by
//                            ac_build (one thread and the default pool), its
//                            exported tables are walked chunk by chunk with
//                            the overlap rule for several chunk sizes, and the
//                            matches must equal the oracle's, order included;
//                            the partitioned build is checked as well
//   host_driver errors       every argument error returns its status code
//   host_driver alloc        builds one dictionary and one partitioned one;
//                            with AC_TEST_FAIL_ALLOC=<n> the n-th checked
//                            allocation fails: prints the two status codes
//
// Exit status 0 on success; the sanitizers (leak checking included) abort
// on any error they find.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/ac.h"

extern "C" {
typedef struct oracle_machine oracle_machine;
int oracle_build(const uint8_t *sym, const uint64_t *off, uint32_t n_patterns, uint32_t sigma,
                 oracle_machine **out);
void oracle_free(oracle_machine *m);
int64_t oracle_scan(const oracle_machine *m, const uint8_t *text, uint64_t n, uint32_t *pid,
                    uint32_t *end, uint64_t cap);
}

namespace {

struct Instance {
    uint32_t sigma = 0;
    std::vector<uint8_t> text, sym;
    std::vector<uint64_t> off;
};

bool read_exact(FILE *f, void *p, size_t n) { return n == 0 || fread(p, 1, n, f) == n; }

bool load(const char *path, std::vector<Instance> *out) {
    FILE *f = fopen(path, "rb");
    if (!f) return false;
    uint32_t count = 0;
    bool ok = read_exact(f, &count, 4);
    for (uint32_t i = 0; ok && i < count; ++i) {
        Instance in;
        uint32_t n = 0, np = 0;
        ok = read_exact(f, &in.sigma, 4) && read_exact(f, &n, 4);
        in.text.resize(n);
        ok = ok && read_exact(f, in.text.data(), n) && read_exact(f, &np, 4);
        in.off.resize((size_t)np + 1);
        ok = ok && read_exact(f, in.off.data(), 8 * in.off.size());
        in.sym.resize(ok ? in.off[np] : 0);
        ok = ok && read_exact(f, in.sym.data(), in.sym.size());
        out->push_back(std::move(in));
    }
    fclose(f);
    return ok;
}

typedef std::vector<std::pair<uint32_t, uint32_t>> Matches;  // (end, id) in order

Matches oracle_matches(const Instance &in) {
    oracle_machine *m = nullptr;
    const uint32_t np = (uint32_t)in.off.size() - 1;
    if (oracle_build(in.sym.data(), in.off.data(), np, in.sigma, &m) != 0) abort();
    int64_t tot = oracle_scan(m, in.text.data(), in.text.size(), nullptr, nullptr, 0);
    std::vector<uint32_t> pid((size_t)tot + 1), end((size_t)tot + 1);
    oracle_scan(m, in.text.data(), in.text.size(), pid.data(), end.data(), (uint64_t)tot);
    oracle_free(m);
    Matches r;
    for (int64_t k = 0; k < tot; ++k) r.push_back({end[k], pid[k]});
    return r;
}

// The exported completed transitions walked with the chunk rule: chunk
// [j0, j0 + C) restarts at the root max_len - 1 symbols early and reports
// only ends inside the chunk.
Matches walk(const ac_dict *d, const Instance &in, uint32_t C) {
    ac_dict_info info;
    if (ac_dict_get_info(d, &info) != AC_OK) abort();
    std::vector<uint32_t> delta((size_t)info.states * info.sigma);
    std::vector<uint32_t> out_off(info.states - info.first_output_state + 1);
    std::vector<uint32_t> out_ids(info.output_entries + 1);
    if (ac_debug_export(d, delta.data(), out_off.data(), out_ids.data(), nullptr) != AC_OK)
        abort();
    Matches r;
    const uint64_t n = in.text.size();
    for (uint64_t j0 = 0; j0 < n; j0 += C) {
        const uint64_t b = j0 > info.max_len - 1 ? j0 - (info.max_len - 1) : 0;
        const uint64_t e1 = j0 + C < n ? j0 + C : n;
        uint32_t s = 0;
        for (uint64_t e = b; e < e1; ++e) {
            s = delta[(size_t)s * info.sigma + in.text[e]];
            if (e >= j0 && s >= info.first_output_state) {
                const uint32_t o = s - info.first_output_state;
                for (uint32_t k = out_off[o]; k < out_off[o + 1]; ++k)
                    r.push_back({(uint32_t)e, out_ids[k]});
            }
        }
    }
    return r;
}

int run_corpus(const char *path) {
    std::vector<Instance> all;
    if (!load(path, &all)) {
        fprintf(stderr, "cannot read %s\n", path);
        return 2;
    }
    size_t checked = 0;
    for (size_t i = 0; i < all.size(); ++i) {
        const Instance &in = all[i];
        const uint32_t np = (uint32_t)in.off.size() - 1;
        const Matches want = oracle_matches(in);
        for (uint32_t flags : {AC_BUILD_HOST_ONLY | AC_BUILD_SERIAL, (uint32_t)AC_BUILD_HOST_ONLY}) {
            ac_build_opts o = {in.sigma, AC_PLACE_AUTO, flags, 0};
            ac_dict *d = nullptr;
            int rc = ac_build(in.sym.data(), in.off.data(), np, &o, &d);
            if (rc != AC_OK) {
                fprintf(stderr, "instance %zu: ac_build %d\n", i, rc);
                return 1;
            }
            for (uint32_t C : {1u, 3u, 7u, 64u, 1u << 20}) {
                if (walk(d, in, C) != want) {
                    fprintf(stderr, "instance %zu: chunk %u differs from the oracle\n", i, C);
                    return 1;
                }
                ++checked;
            }
            ac_destroy(d);
        }
        // the paper's second design: slices of the pattern list
        ac_build_opts o = {in.sigma, AC_PLACE_AUTO, AC_BUILD_HOST_ONLY, 0};
        ac_dict *p = nullptr;
        const uint32_t parts = 1 + (uint32_t)(i % 3);
        if (ac_build_partitioned(in.sym.data(), in.off.data(), np, &o, parts, &p) != AC_OK)
            return 1;
        uint32_t k = 0;
        if (ac_dict_parts(p, &k, nullptr) != AC_OK || k == 0 || k > parts) return 1;
        ac_destroy(p);
    }
    printf("ok %zu instances, %zu walks\n", all.size(), checked);
    return 0;
}

int run_errors() {
    const uint8_t sym[] = {0, 1, 2, 3, 1};
    const uint64_t off[] = {0, 2, 5};
    const uint64_t off_empty[] = {0, 2, 2};
    const uint64_t off_bad[] = {1, 2, 5};
    ac_build_opts o = {4, AC_PLACE_AUTO, AC_BUILD_HOST_ONLY, 0};
    ac_dict *d = nullptr;
    struct {
        int got, want;
        const char *what;
    } cases[] = {
        {ac_build(sym, off, 2, &o, nullptr), AC_E_INVALID, "null out"},
        {ac_build(sym, off, 0, &o, &d), AC_E_INVALID, "no patterns"},
        {ac_build(sym, nullptr, 2, &o, &d), AC_E_INVALID, "null offsets"},
        {ac_build(nullptr, off, 2, &o, &d), AC_E_INVALID, "null symbols"},
        {ac_build(sym, off_empty, 2, &o, &d), AC_E_EMPTY_PATTERN, "empty pattern"},
        {ac_build(sym, off_bad, 2, &o, &d), AC_E_INVALID, "offsets[0] != 0"},
        {[&] {
             ac_build_opts s3 = {3, AC_PLACE_AUTO, AC_BUILD_HOST_ONLY, 0};
             return ac_build(sym, off, 2, &s3, &d);
         }(),
         AC_E_SYMBOL, "symbol >= sigma"},
        {[&] {
             ac_build_opts s1 = {1, AC_PLACE_AUTO, AC_BUILD_HOST_ONLY, 0};
             return ac_build(sym, off, 2, &s1, &d);
         }(),
         AC_E_INVALID, "sigma 1"},
        {[&] {
             ac_build_opts bad = {4, 99, AC_BUILD_HOST_ONLY, 0};
             return ac_build(sym, off, 2, &bad, &d);
         }(),
         AC_E_INVALID, "placement"},
        {ac_build_partitioned(sym, off, 2, &o, 1, nullptr), AC_E_INVALID, "partitioned null out"},
        {ac_dict_get_info(nullptr, nullptr), AC_E_INVALID, "info null"},
        {ac_debug_export(nullptr, nullptr, nullptr, nullptr, nullptr), AC_E_INVALID,
         "export null"},
    };
    for (const auto &c : cases)
        if (c.got != c.want) {
            fprintf(stderr, "%s: got %d, want %d\n", c.what, c.got, c.want);
            return 1;
        }
    ac_destroy(nullptr);
    if (strcmp(ac_status_str(AC_E_NOMEM), "out of memory") != 0) return 1;
    printf("ok %zu error cases\n", sizeof(cases) / sizeof(cases[0]));
    return 0;
}

int run_alloc() {
    // 300 patterns of 6-20 symbols over 4 letters (a fixed LCG)
    uint32_t x = 12345;
    auto next = [&] { return x = x * 1664525u + 1013904223u; };
    std::vector<uint8_t> sym;
    std::vector<uint64_t> off{0};
    for (int i = 0; i < 300; ++i) {
        const uint32_t len = 6 + (next() >> 24) % 15;
        for (uint32_t k = 0; k < len; ++k) sym.push_back((uint8_t)((next() >> 28) & 3));
        off.push_back(sym.size());
    }
    ac_build_opts o = {4, AC_PLACE_AUTO, AC_BUILD_HOST_ONLY, 0};
    ac_dict *d = nullptr;
    const int a = ac_build(sym.data(), off.data(), 300, &o, &d);
    if ((a == AC_OK) != (d != nullptr)) return 1;
    ac_destroy(d);
    ac_dict *p = nullptr;
    const int b = ac_build_partitioned(sym.data(), off.data(), 300, &o, 3, &p);
    if ((b == AC_OK) != (p != nullptr)) return 1;
    ac_destroy(p);
    printf("%d %d\n", a, b);
    return 0;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc >= 3 && !strcmp(argv[1], "corpus")) return run_corpus(argv[2]);
    if (argc >= 2 && !strcmp(argv[1], "errors")) return run_errors();
    if (argc >= 2 && !strcmp(argv[1], "alloc")) return run_alloc();
    fprintf(stderr, "usage: host_driver corpus FILE | errors | alloc\n");
    return 2;
}
