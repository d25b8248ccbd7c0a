// Continuous-batching serving core: requests (DNA letters and the index of
// one of the server's dictionaries) arrive at any time; the server groups
// waiting requests into batches and runs each batch as one set of
// independent scans (the paper's section IV.A: the work is split into
// independent matching jobs run in parallel) on one of several streams, so
// that batches admitted while others run overlap them on the GPU.
//
// Threads:
//   caller    ac_server_submit reserves room for the letters in a pinned
//             staging ring (waiting while it is full) and queues the request;
//             ac_server_wait blocks until a request's matches are on the host
//   copiers   copy queued letters into their ring regions
//   worker    admits staged requests while device memory (a budget, capped by
//             the free device memory) and a free in-flight slot allow; per
//             batch: one letters copy to the device, one ac_encode, one
//             ac_scan_batch, copies of the counts and the matches back; on
//             completion, results move to per-request host buffers and ring
//             space and memory are released.  A request whose matches
//             overflow its reservation is scanned again, alone, exactly sized.
//
// Output space is reserved per request from a running estimate of each
// dictionary's matches per base, started at the expected rate on uniform
// random DNA: the sum over patterns of 4^-length.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace acx {
namespace {

typedef std::chrono::steady_clock Clock;

double seconds(Clock::time_point t) {
    return std::chrono::duration<double>(t.time_since_epoch()).count();
}

uint64_t pad16(uint64_t n) { return (n + 15) & ~uint64_t(15); }
uint64_t al256(uint64_t n) { return (n + 255) & ~uint64_t(255); }

// Upper bound of one request's share of a batch workspace: 68 bytes of
// per-segment records per 64 bases (1.0625 bytes per base), up to one chunk
// of padding (at most 2,048 bases), its descriptor and chunk counters, and a
// few KiB of per-batch arrays: 1.5 bytes per base plus 64 KiB.
uint64_t ws_bound(uint64_t n) { return n + n / 2 + (64u << 10); }

bool dna_letters(const uint8_t *p, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i) {
        const uint8_t c = p[i] | 0x20;
        if (c != 'a' && c != 'c' && c != 'g' && c != 't') return false;
    }
    return true;
}

// A ring region; the ring keeps them in order until the oldest are done.
struct Region {
    uint64_t start = 0, padded = 0;
    bool done = false;
};

struct Req {
    uint64_t ticket = 0;
    uint32_t dict = 0;
    const uint8_t *src = nullptr;  // caller's letters (valid until copied)
    uint64_t n = 0, padded = 0;
    uint64_t start = 0;            // ring offset of the letters
    uint8_t *oneoff = nullptr;     // pinned buffer when larger than the ring
    Region *region = nullptr;      // its ring region (null: a one-off buffer)
    bool ready = false;            // letters staged
    bool in_copy = false;          // queued for a copier or being copied
    uint64_t cap = 0;              // reserved matches
    uint64_t charge = 0;           // device bytes counted against the budget
    int status = 1;                // 1 pending, AC_OK, or an AC_E_* code
    std::vector<ac_match> out;
    double t_arrive = 0, t_done = 0;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    int64_t *counts = nullptr;     // pinned: max_batch counts + the invalid-letter count
    ac_match *out = nullptr;       // pinned, grown as needed
    uint64_t out_cap = 0;
    std::vector<Req *> batch;
    std::vector<uint64_t> moff, offs;
    char *mem = nullptr;           // device memory of the batch in flight
    uint64_t a_pack = 0;
    uint64_t charged = 0;
};

}  // namespace
}  // namespace acx

struct ac_server {
    std::vector<ac_dict *> dicts;
    std::vector<double> rate;      // matches per base, per dictionary
    ac_server_opts o{};
    uint64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_copy;
    std::deque<acx::Req *> queue;  // submitted, in ring order
    std::deque<acx::Req *> to_copy;
    std::unordered_map<uint64_t, std::unique_ptr<acx::Req>> reqs;
    uint64_t next_ticket = 1;
    // staging ring
    uint8_t *ring = nullptr;
    uint64_t ring_size = 0;
    std::deque<acx::Region> ring_live;  // regions in use, oldest first
    std::vector<acx::Slot> slots;
    uint64_t used = 0, peak = 0;
    bool stopping = false;
    int failed = AC_OK;
    // statistics
    std::vector<double> lat;
    uint64_t bases = 0, matches = 0, batches = 0, reruns = 0, overlapped = 0;
    double t_first = -1, t_last = 0;
    uint32_t launches = 0;
    std::thread worker;
    std::vector<std::thread> copiers;
};

namespace acx {
namespace {

// Ring regions are taken in submission order and given back as requests
// finish; a region never wraps (the rest of the ring is skipped).
bool ring_reserve(ac_server *s, Req *r) {
    if (r->padded > s->ring_size) return false;
    uint64_t start = 0;
    if (!s->ring_live.empty()) {
        const uint64_t tail = s->ring_live.front().start;
        const uint64_t head = s->ring_live.back().start + s->ring_live.back().padded;
        const bool wrapped = s->ring_live.front().start > s->ring_live.back().start;
        if (!wrapped && head + r->padded <= s->ring_size)
            start = head;
        else if (!wrapped && r->padded <= tail)
            start = 0;
        else if (wrapped && head + r->padded <= tail)
            start = head;
        else
            return false;
    }
    r->start = start;
    s->ring_live.push_back(Region{start, r->padded, false});
    r->region = &s->ring_live.back();  // deque elements stay put on push_back/pop_front
    return true;
}

void ring_release(ac_server *s) {
    while (!s->ring_live.empty() && s->ring_live.front().done) s->ring_live.pop_front();
}

uint64_t reserve_matches(const ac_server *s, uint32_t dict, uint64_t n) {
    const double mean = s->rate[dict] * (double)n;
    return (uint64_t)(s->o.margin * (mean + 2.0 * sqrt(mean))) + 64;
}

uint64_t charge_of(uint64_t n, uint64_t cap) {
    const uint64_t p = pad16(n);
    return p + p / 4 + 8 * cap + 8 + ws_bound(n) + 1024;
}

void copier_main(ac_server *s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_copy.wait(lk, [&] { return s->stopping || !s->to_copy.empty(); });
        if (s->to_copy.empty()) return;
        Req *r = s->to_copy.front();
        s->to_copy.pop_front();
        uint8_t *dst = r->oneoff ? r->oneoff : s->ring + r->start;
        lk.unlock();
        if (r->n) memcpy(dst, r->src, r->n);
        memset(dst + r->n, 'A', r->padded - r->n);  // padding: valid letters
        lk.lock();
        r->ready = true;
        r->in_copy = false;
        r->src = nullptr;
        s->cv_work.notify_one();
        s->cv_done.notify_all();  // a release may wait for the copy to end
    }
}

// Consecutive staged requests whose letters are contiguous in the ring,
// while memory and the batch size allow (lock held).
std::vector<Req *> take(ac_server *s) {
    std::vector<Req *> b;
    uint64_t need = 0;
    for (Req *r : s->queue) {
        if (b.size() >= s->o.max_batch || !r->ready) break;
        if (!b.empty() && (r->oneoff || b[0]->oneoff || r->start != b.back()->start + b.back()->padded))
            break;
        if (s->used + need + r->charge > s->budget) break;
        need += r->charge;
        b.push_back(r);
    }
    return b;
}

void finish_request(ac_server *s, Req *r, int status) {
    // (lock held)
    if (r->status != 1) return;
    r->status = status;
    r->t_done = seconds(Clock::now());
    if (r->region) {
        r->region->done = true;
        r->region = nullptr;
    }
    if (r->oneoff) {
        (void)hipHostFree(r->oneoff);
        r->oneoff = nullptr;
    }
    if (status == AC_OK) {
        s->lat.push_back(r->t_done - r->t_arrive);
        s->bases += r->n;
        s->matches += r->out.size();
    }
    s->t_last = r->t_done;
}

int launch(ac_server *s, Slot &sl, std::vector<Req *> &batch) {
    const uint32_t L = (uint32_t)batch.size();
    sl.offs.assign(L + 1, 0);
    sl.moff.assign(L + 1, 0);
    uint64_t ws = 0;
    for (uint32_t i = 0; i < L; ++i) {
        sl.offs[i + 1] = sl.offs[i] + batch[i]->padded;
        sl.moff[i + 1] = sl.moff[i] + batch[i]->cap;
        ws += ws_bound(batch[i]->n);
        sl.charged += batch[i]->charge;
    }
    const uint64_t total = sl.offs[L], m_total = sl.moff[L];
    sl.a_pack = al256(total);
    const uint64_t a_cnt = sl.a_pack + al256(total / 4);
    const uint64_t a_out = a_cnt + al256(8 * (L + 1));
    const uint64_t a_ws = a_out + al256(8 * m_total);
    const uint64_t bytes = a_ws + ws;
    if (sl.out_cap < m_total) {
        if (sl.out) (void)hipHostFree(sl.out);
        sl.out = nullptr;
        uint64_t c = 1u << 16;
        while (c < m_total) c *= 2;
        if (hipHostMalloc((void **)&sl.out, c * sizeof(ac_match), hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            sl.out_cap = 0;
            return AC_E_NOMEM;
        }
        sl.out_cap = c;
    }
    s->launches++;
    if ((s->o.fail_batch && s->launches == s->o.fail_batch) || test_alloc_fails() ||
        hipMallocAsync((void **)&sl.mem, bytes, sl.st) != hipSuccess) {
        (void)hipGetLastError();
        sl.mem = nullptr;
        return AC_E_NOMEM;
    }
    const uint8_t *host = batch[0]->oneoff ? batch[0]->oneoff : s->ring + batch[0]->start;
    int64_t *d_cnt = (int64_t *)(sl.mem + a_cnt);
    if (total && hipMemcpyAsync(sl.mem, host, total, hipMemcpyHostToDevice, sl.st) != hipSuccess)
        return AC_E_HIP;
    // (with no letters this only clears the invalid-letter count)
    int rc = ac_encode((const uint8_t *)sl.mem, total, AC_ALPHA_DNA, AC_TEXT_2BIT,
                       sl.mem + sl.a_pack, (uint64_t *)(d_cnt + L), sl.st);
    if (rc) return rc;
    std::vector<ac_batch_item> items(L);
    for (uint32_t i = 0; i < L; ++i) {
        ac_batch_item &it = items[i];
        it.dict = s->dicts[batch[i]->dict];
        it.d_text = sl.mem + sl.a_pack + sl.offs[i] / 4;
        it.n = batch[i]->n;
        it.fmt = AC_TEXT_2BIT;
        it.reserved = 0;
        it.d_out = (ac_match *)(sl.mem + a_out) + sl.moff[i];
        it.capacity = batch[i]->cap;
        it.d_count = (uint64_t *)(d_cnt + i);
    }
    const ac_tune *tune = s->o.tune.chunk || s->o.tune.block_threads || s->o.tune.placement ||
                                  s->o.tune.blocks_per_cu || s->o.tune.chains
                              ? &s->o.tune
                              : nullptr;
    rc = ac_scan_batch(items.data(), L, tune, sl.mem + a_ws, ws, sl.st);
    if (rc) return rc;
    if (hipMemcpyAsync(sl.counts, d_cnt, 8 * (L + 1), hipMemcpyDeviceToHost, sl.st) !=
            hipSuccess ||
        (m_total && hipMemcpyAsync(sl.out, sl.mem + a_out, 8 * m_total, hipMemcpyDeviceToHost,
                                   sl.st) != hipSuccess) ||
        hipEventRecord(sl.ev, sl.st) != hipSuccess)
        return AC_E_HIP;
    return AC_OK;
}

// Results of a completed batch (lock not held on entry).
void finish(ac_server *s, Slot &sl) {
    (void)hipEventSynchronize(sl.ev);
    const uint32_t L = (uint32_t)sl.batch.size();
    const bool invalid = sl.counts[L] != 0;
    std::vector<int> st(L, AC_OK);
    std::vector<double> got(s->dicts.size(), 0.0), seen(s->dicts.size(), 0.0);
    for (uint32_t i = 0; i < L; ++i) {
        Req *r = sl.batch[i];
        const uint64_t c = (uint64_t)sl.counts[i];
        const uint8_t *letters = r->oneoff ? r->oneoff : s->ring + r->start;
        if (invalid && !dna_letters(letters, r->n)) {
            st[i] = AC_E_SYMBOL;
            continue;
        }
        if (c <= r->cap) {
            r->out.assign(sl.out + sl.moff[i], sl.out + sl.moff[i] + c);
        } else {
            // overflow: again, alone, exactly sized (memory counted)
            uint64_t wsb = 0;
            int rc = ac_scan_workspace_size(s->dicts[r->dict], r->n, AC_TEXT_2BIT, nullptr, &wsb);
            const uint64_t need = 8 * c + 8 + wsb;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->used += need;
                s->peak = std::max(s->peak, s->used);
                s->reruns++;
            }
            char *m = nullptr;
            if (rc == AC_OK && hipMallocAsync((void **)&m, need, sl.st) != hipSuccess) {
                (void)hipGetLastError();
                rc = AC_E_NOMEM;
            }
            if (rc == AC_OK) {
                rc = ac_scan(s->dicts[r->dict], sl.mem + sl.a_pack + sl.offs[i] / 4, r->n,
                             AC_TEXT_2BIT, (ac_match *)(m + wsb), c, (uint64_t *)(m + wsb + 8 * c),
                             nullptr, m, wsb, sl.st);
                r->out.resize(c);
                if (rc == AC_OK &&
                    (hipMemcpyAsync(r->out.data(), m + wsb, 8 * c, hipMemcpyDeviceToHost,
                                    sl.st) != hipSuccess ||
                     hipStreamSynchronize(sl.st) != hipSuccess))
                    rc = AC_E_HIP;
            }
            if (m) (void)hipFreeAsync(m, sl.st);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->used -= need;
            }
            st[i] = rc;
        }
        got[r->dict] += (double)c;
        seen[r->dict] += (double)r->n;
    }
    if (sl.mem) (void)hipFreeAsync(sl.mem, sl.st);
    sl.mem = nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t d = 0; d < got.size(); ++d)
        if (seen[d] > 0) s->rate[d] = 0.8 * s->rate[d] + 0.2 * got[d] / seen[d];
    for (uint32_t i = 0; i < L; ++i) finish_request(s, sl.batch[i], st[i]);
    s->used -= sl.charged;
    sl.charged = 0;
    sl.batch.clear();
    s->batches++;
    ring_release(s);
    s->cv_done.notify_all();
}

void fail_all(ac_server *s, int rc) {
    // (lock held; no batch in flight) every request not finished gets rc
    for (Req *r : s->to_copy) r->in_copy = false;
    s->to_copy.clear();
    for (auto &kv : s->reqs)
        if (kv.second->status == 1) finish_request(s, kv.second.get(), rc);
    s->queue.clear();
    ring_release(s);
    s->cv_done.notify_all();
}

void worker_main(ac_server *s) {
    std::deque<Slot *> inflight;
    std::vector<Slot *> free;
    for (Slot &sl : s->slots) free.push_back(&sl);
    const auto max_wait = std::chrono::microseconds(s->o.max_wait_us);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions, in launch order
        while (!inflight.empty() && hipEventQuery(inflight.front()->ev) == hipSuccess) {
            Slot *sl = inflight.front();
            inflight.pop_front();
            lk.unlock();
            finish(s, *sl);
            lk.lock();
            free.push_back(sl);
        }
        if (s->failed) {
            // finish what is in flight, then fail everything else
            while (!inflight.empty()) {
                Slot *sl = inflight.front();
                inflight.pop_front();
                lk.unlock();
                finish(s, *sl);
                lk.lock();
                free.push_back(sl);
            }
            fail_all(s, s->failed);
            if (s->stopping) return;
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        std::vector<Req *> batch;
        if (!free.empty() && !s->failed) batch = take(s);
        // with batches in flight, let a short batch fill while its requests
        // are still being staged (for at most max_wait)
        if (!batch.empty() && !inflight.empty() && batch.size() < s->o.max_batch &&
            batch.size() < s->queue.size() && !s->queue[batch.size()]->ready &&
            seconds(Clock::now()) - batch[0]->t_arrive < 1e-6 * s->o.max_wait_us) {
            s->cv_work.wait_for(lk, max_wait / 4);
            continue;
        }
        if (batch.empty()) {
            if (inflight.empty()) {
                if (s->stopping && s->queue.empty() && s->to_copy.empty()) return;
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
            const bool blocked = !s->queue.empty() && s->queue.front()->ready;
            if (!blocked) {
                s->cv_work.wait_for(lk, std::chrono::microseconds(50));
                continue;
            }
            // slots or memory exhausted: wait for the oldest batch
            Slot *sl = inflight.front();
            inflight.pop_front();
            lk.unlock();
            finish(s, *sl);
            lk.lock();
            free.push_back(sl);
            continue;
        }
        for (size_t i = 0; i < batch.size(); ++i) s->queue.pop_front();
        Slot *sl = free.back();
        free.pop_back();
        uint64_t need = 0;
        for (Req *r : batch) need += r->charge;
        s->used += need;
        s->peak = std::max(s->peak, s->used);
        if (!inflight.empty()) s->overlapped++;
        sl->batch = batch;
        lk.unlock();
        int rc = launch(s, *sl, sl->batch);
        lk.lock();
        if (rc == AC_OK) {
            inflight.push_back(sl);
            continue;
        }
        // the batch did not start: its requests fail with rc; a HIP error
        // stops the server
        if (sl->mem) (void)hipFreeAsync(sl->mem, sl->st);
        sl->mem = nullptr;
        for (Req *r : sl->batch) finish_request(s, r, rc);
        s->used -= sl->charged;
        sl->charged = 0;
        sl->batch.clear();
        free.push_back(sl);
        ring_release(s);
        s->cv_done.notify_all();
        if (rc == AC_E_HIP) s->failed = rc;
    }
}

}  // namespace
}  // namespace acx

using namespace acx;

extern "C" {

int ac_server_create(ac_dict *const *dicts, uint32_t n_dicts, const ac_server_opts *opts,
                     ac_server **out) {
    if (!out || !dicts || !n_dicts) return AC_E_INVALID;
    *out = nullptr;
    for (uint32_t i = 0; i < n_dicts; ++i)
        if (!dicts[i] || dicts[i]->host.sigma != 4 || !dicts[i]->parts.empty())
            return AC_E_INVALID;
        else if (!dicts[i]->d_delta)
            return AC_E_NO_DEVICE;
    std::unique_ptr<ac_server> s(test_alloc_fails() ? nullptr : new (std::nothrow) ac_server());
    if (!s) return AC_E_NOMEM;
    ac_server_opts o{};
    if (opts) o = *opts;
    if (!o.max_batch) o.max_batch = 256;
    if (!o.streams) o.streams = 4;
    if (!o.staging_bytes) o.staging_bytes = 256ull << 20;
    if (o.margin < 0) o.margin = 2.0;
    if (!o.copy_threads) o.copy_threads = 8;
    if (o.max_batch > 4096 || o.streams > 16 || o.copy_threads > 64) return AC_E_INVALID;
    s->o = o;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_HIP;
    }
    const uint64_t cap = (uint64_t)(0.9 * (double)free_b);
    s->budget = o.budget_bytes ? std::min<uint64_t>(o.budget_bytes, cap) : cap;
    s->dicts.assign(dicts, dicts + n_dicts);
    for (uint32_t i = 0; i < n_dicts; ++i) {
        // expected matches per position of uniform random DNA: sum of 4^-len
        const HostTables &T = dicts[i]->host;
        double r = 0;
        // a pattern's length is the depth of the state where it ends
        for (uint32_t st = 0; st < T.states; ++st)
            for (uint32_t k = T.own_off.empty() ? 0 : T.own_off[st];
                 !T.own_off.empty() && k < T.own_off[st + 1]; ++k)
                r += pow(4.0, -(double)T.depth[st]);
        s->rate.push_back(r > 0 ? r : 1e-3);
    }
    s->ring_size = pad16(o.staging_bytes);
    if (test_alloc_fails() ||
        hipHostMalloc((void **)&s->ring, s->ring_size, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return AC_E_NOMEM;
    }
    s->slots.resize(o.streams);
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.counts, 8 * (o.max_batch + 1), hipHostMallocDefault) !=
                hipSuccess) {
            (void)hipGetLastError();
            ac_server *raw = s.release();
            raw->stopping = true;
            ac_server_destroy(raw);
            return AC_E_HIP;
        }
    }
    ac_server *raw = s.release();
    for (uint32_t i = 0; i < o.copy_threads; ++i) raw->copiers.emplace_back(copier_main, raw);
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return AC_OK;
}

int ac_server_submit(ac_server *s, const uint8_t *letters, uint64_t n, uint32_t dict_id,
                     uint64_t *ticket) {
    if (!s || !ticket || (n && !letters) || dict_id >= s->dicts.size()) return AC_E_INVALID;
    if (n >= (1ull << 32) - 256) return AC_E_TOO_LARGE;
    std::unique_ptr<Req> q(new (std::nothrow) Req());
    if (!q) return AC_E_NOMEM;
    Req *r = q.get();
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->failed) return s->failed;
    if (s->stopping) return AC_E_INVALID;
    r->ticket = s->next_ticket++;
    r->dict = dict_id;
    r->src = letters;
    r->n = n;
    r->padded = pad16(n);
    r->t_arrive = seconds(Clock::now());
    if (s->t_first < 0) s->t_first = r->t_arrive;
    r->cap = reserve_matches(s, dict_id, n);
    r->charge = charge_of(n, r->cap);
    *ticket = r->ticket;
    if (r->charge > s->budget) {
        r->status = AC_E_NOMEM;  // can never fit: refused, not queued
        s->reqs.emplace(r->ticket, std::move(q));
        return AC_OK;
    }
    if (r->padded > s->ring_size) {
        if (hipHostMalloc((void **)&r->oneoff, r->padded, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return AC_E_NOMEM;
        }
    } else {
        while (!ring_reserve(s, r)) {
            if (s->failed) return s->failed;
            s->cv_done.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
    r->in_copy = true;
    s->queue.push_back(r);
    s->to_copy.push_back(r);
    s->reqs.emplace(r->ticket, std::move(q));
    s->cv_copy.notify_one();
    return AC_OK;
}

int ac_server_wait(ac_server *s, uint64_t ticket, int64_t timeout_us, const ac_match **matches,
                   uint64_t *count, double *latency_s) {
    if (!s || !matches || !count) return AC_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return AC_E_INVALID;
    Req *r = it->second.get();
    auto done = [&] { return r->status != 1 && !r->in_copy; };
    if (timeout_us < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done))
        return AC_E_TIMEOUT;
    if (latency_s) *latency_s = r->t_done - r->t_arrive;
    if (r->status != AC_OK) return r->status;
    *matches = r->out.data();
    *count = r->out.size();
    return AC_OK;
}

int ac_server_request_charge(ac_server *s, uint64_t n, uint32_t dict_id, uint64_t *bytes) {
    if (!s || !bytes || dict_id >= s->dicts.size()) return AC_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    *bytes = charge_of(n, reserve_matches(s, dict_id, n));
    return AC_OK;
}

int ac_server_release(ac_server *s, uint64_t ticket) {
    if (!s) return AC_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->status == 1) return AC_E_INVALID;
    Req *r = it->second.get();
    s->cv_done.wait(lk, [&] { return !r->in_copy; });
    s->reqs.erase(it);
    return AC_OK;
}

int ac_server_stats(ac_server *s, ac_server_counters *st, double *latencies,
                    uint64_t max_latencies) {
    if (!s || !st) return AC_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    st->requests = s->lat.size();
    st->bases = s->bases;
    st->matches = s->matches;
    st->batches = s->batches;
    st->reruns = s->reruns;
    st->overlapped = s->overlapped;
    st->peak_bytes = s->peak;
    st->budget_bytes = s->budget;
    st->wall_s = s->t_first >= 0 ? s->t_last - s->t_first : 0.0;
    st->failed = s->failed;
    if (latencies)
        for (uint64_t i = 0; i < std::min<uint64_t>(max_latencies, s->lat.size()); ++i)
            latencies[i] = s->lat[i];
    return AC_OK;
}

int ac_server_destroy(ac_server *s) {
    if (!s) return AC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    s->cv_copy.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &t : s->copiers) t.join();
    const int failed = s->failed;
    for (Slot &sl : s->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.counts) (void)hipHostFree(sl.counts);
        if (sl.out) (void)hipHostFree(sl.out);
    }
    for (auto &kv : s->reqs)
        if (kv.second->oneoff) (void)hipHostFree(kv.second->oneoff);
    if (s->ring) (void)hipHostFree(s->ring);
    (void)hipGetLastError();
    delete s;
    return failed;
}

}  // extern "C"
