// Host automaton compiler: stage 1 of Aho-Corasick (paper, section III.A,
// Figure 1), producing the tables the GPU scan reads.
//
//  1. goto function: a keyword trie; each inserted keyword walks existing
//     edges and creates a state per new prefix.  Keyword i ends in state
//     end_state[i].
//  2. failure function, breadth first: depth-1 states fail to the root; the
//     failure state of child s = g(r, a) is reached by following failure
//     links from f(r) until a state with an a-edge appears.
//  3. completed transitions: delta(s, a) = g(s, a) when the edge exists,
//     otherwise delta(f(s), a) (delta(0, a) = 0 without an edge).  Reading a
//     symbol is then one table lookup, which is what the paper's failure
//     loop ("read the same input character again") amounts to.  Rows are
//     filled in breadth-first order, so delta(f(s), .) is complete before s.
//  4. output sets: out(s) = keywords ending at s plus out(f(s)), ids sorted.
//  5. renumbering: root 0, then output-free states from most to least
//     likely to be visited, then output states in breadth-first order.  The
//     visit likelihood of a state is estimated as the probability of its
//     string under independent symbols with the frequencies of the pattern
//     symbols (the shallow, common prefixes first); the scan keeps the first
//     rows of the table in LDS.
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"

namespace acx {

RowDiv make_row_div(uint32_t sigma) {
    RowDiv r;
    uint32_t d = sigma * 4u;
    while ((d & 1u) == 0) {
        d >>= 1;
        ++r.tz;
    }
    // Newton iteration for the inverse of an odd number modulo 2^32
    uint32_t x = d;  // correct to 3 bits
    for (int i = 0; i < 5; ++i) x *= 2u - d * x;
    r.inv = x;
    return r;
}

int compile_automaton(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
                      uint32_t sigma, HostTables *out) {
    if (!offsets || !out || sigma < 2 || sigma > 256 || n_patterns == 0) return AC_E_INVALID;
    if (offsets[0] != 0) return AC_E_INVALID;
    uint64_t total = 0;
    uint32_t min_len = UINT32_MAX, max_len = 0;
    for (uint32_t i = 0; i < n_patterns; ++i) {
        if (offsets[i + 1] < offsets[i]) return AC_E_INVALID;
        uint64_t len = offsets[i + 1] - offsets[i];
        if (len == 0) return AC_E_EMPTY_PATTERN;
        if (len > (1u << 24)) return AC_E_TOO_LARGE;
        min_len = std::min<uint32_t>(min_len, (uint32_t)len);
        max_len = std::max<uint32_t>(max_len, (uint32_t)len);
        total += len;
    }
    if (!symbols) return AC_E_INVALID;
    for (uint64_t k = 0; k < total; ++k)
        if (symbols[k] >= sigma) return AC_E_SYMBOL;
    // one state per character at most, plus the root
    if (total + 1 > (1ull << 27) || (total + 1) * sigma * 4ull >= (1ull << 32))
        return AC_E_TOO_LARGE;

    // ---- 1. trie (goto function); -1 = no edge
    std::vector<int32_t> child;
    child.reserve(std::min<uint64_t>(total + 1, 1u << 20) * sigma);
    child.assign(sigma, -1);
    std::vector<uint32_t> depth(1, 0);
    std::vector<uint32_t> end_state(n_patterns);
    for (uint32_t i = 0; i < n_patterns; ++i) {
        uint32_t s = 0;
        for (uint64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            const uint32_t a = symbols[k];
            int32_t t = child[(size_t)s * sigma + a];
            if (t < 0) {
                t = (int32_t)depth.size();
                child[(size_t)s * sigma + a] = t;
                child.insert(child.end(), sigma, -1);
                depth.push_back(depth[s] + 1);
            }
            s = (uint32_t)t;
        }
        end_state[i] = s;
    }
    const uint32_t S = (uint32_t)depth.size();

    // ---- 2./3. breadth-first order, failure links and completed rows
    std::vector<uint32_t> bfs;
    bfs.reserve(S);
    bfs.push_back(0);
    std::vector<uint32_t> fail(S, 0);
    std::vector<uint32_t> delta((size_t)S * sigma);
    for (uint32_t a = 0; a < sigma; ++a) {
        const int32_t t = child[a];
        delta[a] = t < 0 ? 0u : (uint32_t)t;
    }
    for (size_t head = 0; head < bfs.size(); ++head) {
        const uint32_t r = bfs[head];
        for (uint32_t a = 0; a < sigma; ++a) {
            const int32_t t = child[(size_t)r * sigma + a];
            if (t < 0) continue;
            const uint32_t s = (uint32_t)t;
            // r's row is complete, so delta(f(r), a) is the failure target
            // reached by the failure-link walk for a child of a non-root r
            fail[s] = (r == 0) ? 0u : delta[(size_t)fail[r] * sigma + a];
            bfs.push_back(s);
        }
        if (r != 0) {
            const uint32_t f = fail[r];
            for (uint32_t a = 0; a < sigma; ++a) {
                const int32_t t = child[(size_t)r * sigma + a];
                delta[(size_t)r * sigma + a] =
                    t >= 0 ? (uint32_t)t : delta[(size_t)f * sigma + a];
            }
        }
    }

    // ---- 4. output sets, in breadth-first order (f(s) before s)
    std::vector<uint32_t> own_cnt(S + 1, 0);
    for (uint32_t i = 0; i < n_patterns; ++i) own_cnt[end_state[i] + 1]++;
    for (uint32_t s = 0; s < S; ++s) own_cnt[s + 1] += own_cnt[s];
    std::vector<uint32_t> own_ids(n_patterns);
    {
        std::vector<uint32_t> fill(own_cnt.begin(), own_cnt.end() - 1);
        for (uint32_t i = 0; i < n_patterns; ++i) own_ids[fill[end_state[i]]++] = i;  // ascending
    }
    std::vector<uint64_t> set_begin(S, 0);
    std::vector<uint32_t> set_len(S, 0);
    std::vector<uint32_t> sets;
    for (uint32_t s : bfs) {
        const uint32_t *a = own_ids.data() + own_cnt[s];
        const uint32_t na = own_cnt[s + 1] - own_cnt[s];
        const uint32_t inh_len = (s == 0) ? 0 : set_len[fail[s]];
        if (na + inh_len == 0) continue;
        if ((uint64_t)na + inh_len > UINT32_MAX) return AC_E_TOO_LARGE;
        const uint64_t b = sets.size();
        const uint64_t inh_begin = (s == 0) ? 0 : set_begin[fail[s]];
        sets.resize(b + na + inh_len);
        // merge own ids with the inherited set (both ascending, disjoint)
        uint32_t x = 0, y = 0;
        uint64_t o = b;
        while (x < na || y < inh_len) {
            if (y == inh_len || (x < na && a[x] < sets[inh_begin + y]))
                sets[o++] = a[x++];
            else
                sets[o++] = sets[inh_begin + y++];
        }
        set_begin[s] = b;
        set_len[s] = na + inh_len;
    }

    // ---- 5. renumbering
    std::vector<double> logp_sym(sigma, 0.0);
    {
        std::vector<uint64_t> freq(sigma, 1);  // add-one smoothing
        for (uint64_t k = 0; k < total; ++k) freq[symbols[k]]++;
        const double all = (double)(total + sigma);
        for (uint32_t a = 0; a < sigma; ++a) logp_sym[a] = std::log((double)freq[a] / all);
    }
    std::vector<double> logp(S, 0.0);
    for (uint32_t s : bfs)
        for (uint32_t a = 0; a < sigma; ++a) {
            const int32_t t = child[(size_t)s * sigma + a];
            if (t >= 0) logp[t] = logp[s] + logp_sym[a];
        }
    child.clear();
    child.shrink_to_fit();
    std::vector<uint32_t> order;
    order.reserve(S);
    for (uint32_t s : bfs)
        if (set_len[s] == 0) order.push_back(s);
    // root first (log-probability 0), then by decreasing probability; the
    // stable sort keeps breadth-first order among equals
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return logp[x] > logp[y]; });
    const uint32_t first_output = (uint32_t)order.size();
    for (uint32_t s : bfs)
        if (set_len[s] != 0) order.push_back(s);
    std::vector<uint32_t> new_id(S);
    for (uint32_t k = 0; k < S; ++k) new_id[order[k]] = k;

    HostTables &T = *out;
    T.sigma = sigma;
    T.states = S;
    T.patterns = n_patterns;
    T.min_len = min_len;
    T.max_len = max_len;
    T.first_output = first_output;
    T.delta.assign((size_t)S * sigma, 0);
    T.depth.assign(S, 0);
    for (uint32_t k = 0; k < S; ++k) {
        const uint32_t s = order[k];
        T.depth[k] = depth[s];
        for (uint32_t a = 0; a < sigma; ++a)
            T.delta[(size_t)k * sigma + a] = new_id[delta[(size_t)s * sigma + a]];
    }
    T.out_off.assign(S - first_output + 1, 0);
    T.out_ids.clear();
    T.max_output = 0;
    for (uint32_t k = first_output; k < S; ++k) {
        const uint32_t s = order[k];
        T.out_ids.insert(T.out_ids.end(), sets.begin() + set_begin[s],
                         sets.begin() + set_begin[s] + set_len[s]);
        T.max_output = std::max(T.max_output, set_len[s]);
        if (T.out_ids.size() > UINT32_MAX) return AC_E_TOO_LARGE;
        T.out_off[k - first_output + 1] = (uint32_t)T.out_ids.size();
    }
    return AC_OK;
}

}  // namespace acx
