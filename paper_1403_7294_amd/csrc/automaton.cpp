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
//     symbol is then one table lookup, which is what the failure loop of
//     section III.A (take failure transitions, then retry the symbol)
//     amounts to.
//  4. output sets: out(s) = keywords ending at s plus out(f(s)), ids sorted.
//  5. renumbering: root 0, then output-free states from most to least
//     likely to be visited, then output states in breadth-first order.  The
//     visit probability of a state is the chance that the walk sits in it
//     when the text has independent symbols with the frequencies of the
//     pattern symbols (its string's probability less that of the strings
//     whose failure link points straight to it); the scan keeps the first
//     rows of the table in LDS (and, in
//     16-bit form, rows whose targets are among the first 65,535 states).
//     Only the first 65,536 output-free states are ranked this way; any
//     further ones follow in breadth-first order.
//
// Steps 2-5 depend only on shallower states (f(s) is shallower than s), so
// each breadth-first level is processed by up to 16 host threads at once --
// the paper's own remedy for slow machine construction (section IV.A,
// second design: build in parallel) applied inside one machine.  The
// result does not depend on the thread count.
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
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

namespace {

// Worker threads that live for one compilation; parallel_for() hands every
// thread (the caller included) its part of one job and returns when all are
// done.
class Pool {
  public:
    explicit Pool(uint32_t threads) : n_(std::max(1u, threads)) {
        for (uint32_t i = 1; i < n_; ++i) workers_.emplace_back([this, i] { loop(i); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }
    uint32_t size() const { return n_; }
    // fn(begin, end) over [0, n) in contiguous ranges; small n runs inline
    void parallel_for(size_t n, const std::function<void(size_t, size_t)> &fn) {
        constexpr size_t kMinPerThread = 4096;
        const size_t t = std::min<size_t>(n_, std::max<size_t>(1, n / kMinPerThread));
        if (t <= 1) {
            fn(0, n);
            return;
        }
        {
            std::lock_guard<std::mutex> g(m_);
            job_ = [&fn, n, t](size_t i) {
                if (i < t) fn(n * i / t, n * (i + 1) / t);
            };
            pending_ = n_ - 1;
            ++gen_;
        }
        cv_.notify_all();
        job_(0);
        std::unique_lock<std::mutex> g(m_);
        done_.wait(g, [this] { return pending_ == 0; });
    }

  private:
    void loop(uint32_t i) {
        uint64_t seen = 0;
        for (;;) {
            std::function<void(size_t)> job;
            {
                std::unique_lock<std::mutex> g(m_);
                cv_.wait(g, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                job = job_;
            }
            job(i);
            std::lock_guard<std::mutex> g(m_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    uint32_t n_;
    std::vector<std::thread> workers_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    std::function<void(size_t)> job_;
    uint64_t gen_ = 0;
    uint32_t pending_ = 0;
    bool stop_ = false;
};

}  // namespace

int compile_automaton(const uint8_t *symbols, const uint64_t *offsets, uint32_t n_patterns,
                      uint32_t sigma, HostTables *out, uint32_t threads) {
    if (!offsets || !out || sigma < 2 || sigma > 256 || n_patterns == 0) return AC_E_INVALID;
    if (offsets[0] != 0) return AC_E_INVALID;
    if (threads == 0) threads = std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
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

    // small dictionaries compile faster than threads start
    Pool pool(total < (1u << 16) ? 1u : threads);
    auto parallel_for = [&pool](uint32_t, size_t n, const std::function<void(size_t, size_t)> &fn) {
        pool.parallel_for(n, fn);
    };

    // ---- 1. trie (goto function); -1 = no edge
    // (each phase's allocations may be failed by the test hook: the caller
    // turns std::bad_alloc into AC_E_NOMEM, and every vector is released)
    if (test_alloc_fails()) throw std::bad_alloc();
    std::vector<int32_t> child;
    child.reserve((size_t)(total + 1) * sigma);
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

    // ---- 2./3. breadth-first levels, failure links and completed rows
    if (test_alloc_fails()) throw std::bad_alloc();
    std::vector<uint32_t> bfs(S);
    std::vector<uint32_t> level_begin{0, 1};  // level d = bfs[level_begin[d] .. level_begin[d+1])
    bfs[0] = 0;
    std::vector<uint32_t> fail(S, 0);
    std::vector<uint32_t> delta((size_t)S * sigma);
    for (uint32_t a = 0; a < sigma; ++a) {
        const int32_t t = child[a];
        delta[a] = t < 0 ? 0u : (uint32_t)t;
    }
    std::vector<uint32_t> nkids;
    for (size_t d = 0; level_begin[d] < level_begin[d + 1]; ++d) {
        const uint32_t b = level_begin[d], e = level_begin[d + 1];
        // children per state of the level, then their places in the next level
        nkids.assign(e - b + 1, 0);
        parallel_for(threads, e - b, [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const uint32_t r = bfs[b + i];
                uint32_t c = 0;
                for (uint32_t a = 0; a < sigma; ++a) c += child[(size_t)r * sigma + a] >= 0;
                nkids[i + 1] = c;
            }
        });
        for (size_t i = 0; i < e - b; ++i) nkids[i + 1] += nkids[i];
        parallel_for(threads, e - b, [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const uint32_t r = bfs[b + i];
                uint32_t o = e + nkids[i];
                const uint32_t f = fail[r];
                for (uint32_t a = 0; a < sigma; ++a) {
                    const int32_t t = child[(size_t)r * sigma + a];
                    if (t < 0) {
                        // rows of shallower states are complete
                        if (r != 0) delta[(size_t)r * sigma + a] = delta[(size_t)f * sigma + a];
                        continue;
                    }
                    const uint32_t s = (uint32_t)t;
                    if (r != 0) delta[(size_t)r * sigma + a] = s;
                    // the failure-link walk from f(r) ends at delta(f(r), a)
                    fail[s] = (r == 0) ? 0u : delta[(size_t)f * sigma + a];
                    bfs[o++] = s;
                }
            }
        });
        level_begin.push_back(e + nkids[e - b]);
    }
    const size_t levels = level_begin.size() - 2;

    // ---- 4. output sets, level by level (f(s) is shallower than s)
    if (test_alloc_fails()) throw std::bad_alloc();
    std::vector<uint32_t> own_cnt(S + 1, 0);
    for (uint32_t i = 0; i < n_patterns; ++i) own_cnt[end_state[i] + 1]++;
    for (uint32_t s = 0; s < S; ++s) own_cnt[s + 1] += own_cnt[s];
    std::vector<uint32_t> own_ids(n_patterns);
    {
        std::vector<uint32_t> fill(own_cnt.begin(), own_cnt.end() - 1);
        for (uint32_t i = 0; i < n_patterns; ++i) own_ids[fill[end_state[i]]++] = i;  // ascending
    }
    std::vector<uint64_t> set_len(S, 0);
    for (size_t d = 0; d < levels; ++d) {
        const uint32_t b = level_begin[d], e = level_begin[d + 1];
        parallel_for(threads, e - b, [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const uint32_t s = bfs[b + i];
                set_len[s] = (uint64_t)(own_cnt[s + 1] - own_cnt[s]) + (s ? set_len[fail[s]] : 0);
            }
        });
    }
    std::vector<uint64_t> set_begin(S, 0);
    uint64_t n_sets = 0;
    for (uint32_t k = 0; k < S; ++k) {
        const uint32_t s = bfs[k];
        if (set_len[s] > UINT32_MAX) return AC_E_TOO_LARGE;
        set_begin[s] = n_sets;
        n_sets += set_len[s];
    }
    std::vector<uint32_t> sets(n_sets);
    for (size_t d = 0; d < levels; ++d) {
        const uint32_t b = level_begin[d], e = level_begin[d + 1];
        parallel_for(threads, e - b, [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const uint32_t s = bfs[b + i];
                if (!set_len[s]) continue;
                // merge own ids with the inherited set (both ascending, disjoint)
                const uint32_t *a = own_ids.data() + own_cnt[s];
                const uint64_t na = own_cnt[s + 1] - own_cnt[s];
                const uint32_t *h = s ? sets.data() + set_begin[fail[s]] : nullptr;
                const uint64_t nh = s ? set_len[fail[s]] : 0;
                uint32_t *o = sets.data() + set_begin[s];
                uint64_t x = 0, y = 0;
                while (x < na || y < nh) {
                    if (y == nh || (x < na && a[x] < h[y]))
                        *o++ = a[x++];
                    else
                        *o++ = h[y++];
                }
            }
        });
    }

    // ---- 5. renumbering
    if (test_alloc_fails()) throw std::bad_alloc();
    // Visit probability of each state under text drawn i.i.d. from the
    // patterns' symbol frequencies: the walk is in s exactly when the text
    // read so far ends with s's string but with no longer trie string, and
    // the longer trie strings that end with s's string and fail straight to
    // s are disjoint events, so P(s) = p(s) - sum of p(t) over the states t
    // with f(t) = s, where p(x) is the probability of x's string.  Shallow
    // states with every one-symbol extension in the trie are never entered
    // after the first few symbols and rank low; the states the walk really
    // sits in rank high.
    std::vector<double> p_sym(sigma, 0.0);
    {
        std::vector<uint64_t> freq(sigma, 1);  // add-one smoothing
        for (uint64_t k = 0; k < total; ++k) freq[symbols[k]]++;
        const double all = (double)(total + sigma);
        for (uint32_t a = 0; a < sigma; ++a) p_sym[a] = (double)freq[a] / all;
    }
    std::vector<double> pstr(S, 0.0);
    pstr[0] = 1.0;
    for (size_t d = 0; d < levels; ++d) {
        const uint32_t b = level_begin[d], e = level_begin[d + 1];
        parallel_for(threads, e - b, [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const uint32_t s = bfs[b + i];
                for (uint32_t a = 0; a < sigma; ++a) {
                    const int32_t t = child[(size_t)s * sigma + a];
                    if (t >= 0) pstr[t] = pstr[s] * p_sym[a];
                }
            }
        });
    }
    std::vector<double> visit(pstr);
    for (uint32_t s = 1; s < S; ++s) visit[fail[s]] -= pstr[s];
    visit[0] = 2.0;  // the root is state 0: every chain starts there
    struct Rank {
        double lp;
        uint32_t pos;
    };
    std::vector<Rank> free_states;
    free_states.reserve(S);
    for (uint32_t k = 0; k < S; ++k)
        if (set_len[bfs[k]] == 0) free_states.push_back(Rank{visit[bfs[k]], k});
    const auto before = [](const Rank &x, const Rank &y) {
        return x.lp > y.lp || (x.lp == y.lp && x.pos < y.pos);
    };
    constexpr size_t kRanked = 65536;
    if (free_states.size() > kRanked) {
        std::nth_element(free_states.begin(), free_states.begin() + kRanked, free_states.end(),
                         before);
        std::sort(free_states.begin(), free_states.begin() + kRanked, before);
        // the rest in breadth-first order: positions not ranked, ascending
        std::vector<uint8_t> ranked(S, 0);
        for (size_t i = 0; i < kRanked; ++i) ranked[free_states[i].pos] = 1;
        size_t o = kRanked;
        for (uint32_t k = 0; k < S; ++k)
            if (!ranked[k] && set_len[bfs[k]] == 0) free_states[o++].pos = k;
    } else {
        std::sort(free_states.begin(), free_states.end(), before);
    }
    std::vector<uint32_t> order;
    order.reserve(S);
    for (const Rank &r : free_states) order.push_back(bfs[r.pos]);
    const uint32_t first_output = (uint32_t)order.size();
    for (uint32_t k = 0; k < S; ++k)
        if (set_len[bfs[k]] != 0) order.push_back(bfs[k]);
    std::vector<uint32_t> new_id(S);
    parallel_for(threads, S, [&](size_t k0, size_t k1) {
        for (size_t k = k0; k < k1; ++k) new_id[order[k]] = (uint32_t)k;
    });

    HostTables &T = *out;
    T.sigma = sigma;
    T.states = S;
    T.patterns = n_patterns;
    T.min_len = min_len;
    T.max_len = max_len;
    T.first_output = first_output;
    if (test_alloc_fails()) throw std::bad_alloc();
    T.delta.assign((size_t)S * sigma, 0);
    T.depth.assign(S, 0);
    parallel_for(threads, S, [&](size_t k0, size_t k1) {
        for (size_t k = k0; k < k1; ++k) {
            const uint32_t s = order[k];
            T.depth[k] = depth[s];
            for (uint32_t a = 0; a < sigma; ++a)
                T.delta[k * sigma + a] = new_id[delta[(size_t)s * sigma + a]];
        }
    });
    // the trie alone and each state's own patterns, renumbered
    T.go.assign((size_t)S * sigma, 0);
    T.own_off.assign(S + 1, 0);
    for (uint32_t k = 0; k < S; ++k)
        T.own_off[k + 1] = T.own_off[k] + (own_cnt[order[k] + 1] - own_cnt[order[k]]);
    T.own_ids.assign(n_patterns, 0);
    parallel_for(threads, S, [&](size_t k0, size_t k1) {
        for (size_t k = k0; k < k1; ++k) {
            const uint32_t s = order[k];
            for (uint32_t a = 0; a < sigma; ++a) {
                const int32_t t = child[(size_t)s * sigma + a];
                T.go[k * sigma + a] = t < 0 ? 0u : new_id[t];
            }
            std::copy(own_ids.begin() + own_cnt[s], own_ids.begin() + own_cnt[s + 1],
                      T.own_ids.begin() + T.own_off[k]);
        }
    });
    child.clear();
    child.shrink_to_fit();
    const uint32_t n_out = S - first_output;
    T.out_off.assign(n_out + 1, 0);
    T.max_output = 0;
    uint64_t ids = 0;
    for (uint32_t k = 0; k < n_out; ++k) {
        const uint64_t len = set_len[order[first_output + k]];
        T.max_output = std::max<uint32_t>(T.max_output, (uint32_t)len);
        ids += len;
        if (ids > UINT32_MAX) return AC_E_TOO_LARGE;
        T.out_off[k + 1] = (uint32_t)ids;
    }
    T.out_ids.assign(ids, 0);
    parallel_for(threads, n_out, [&](size_t k0, size_t k1) {
        for (size_t k = k0; k < k1; ++k) {
            const uint32_t s = order[first_output + k];
            std::copy(sets.begin() + set_begin[s], sets.begin() + set_begin[s] + set_len[s],
                      T.out_ids.begin() + T.out_off[k]);
        }
    });
    return AC_OK;
}

}  // namespace acx
