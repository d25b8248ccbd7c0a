"""GPU tests of the continuous-batching server: every request's matches in
the mix equal its matches from a scan alone and from the oracle, including
requests admitted while other batches run, requests whose output overflows
the server's reservation, and a memory budget that admits a few requests
at a time."""
import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _workload(seed, requests, dicts=4):
    """Serving-shaped requests (log-uniform lengths, uniform dictionary) with
    dictionaries that do match: random patterns of 10-30 bases, as in the
    served workload, plus substrings cut from the requests and short
    patterns of 6-8 bases that occur every few kilobases."""
    rng = W.rng_for(seed)
    lens = np.maximum(16, np.round(np.exp(rng.uniform(np.log(1000), np.log(200_000),
                                                      requests))).astype(np.int64))
    lens[:3] = [16, 17, 1000]            # tiny and ragged requests
    texts = [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in lens]
    dict_of = rng.integers(0, dicts, size=requests)
    pats = []
    for k in range(dicts):
        mine = [t for t, d in zip(texts, dict_of) if d == k] or texts[:1]
        p = [rng.integers(0, 4, size=int(L), dtype=np.uint8)
             for L in rng.integers(10, 31, size=200 * (k + 1))]
        for t in mine:
            p += W._cut(rng, t, rng.integers(10, 31, size=3))
        p += [rng.integers(0, 4, size=int(L), dtype=np.uint8)
              for L in rng.integers(6, 9, size=4 * (k + 1))]
        pats.append(W.PatternSet.from_list(p))
    return pats, texts, dict_of, rng.exponential(1.0, size=requests)


def _expected(pats, texts, dict_of):
    machines = [oracle.Machine(p, 4) for p in pats]
    return [machines[d].scan_keys(t) for t, d in zip(texts, dict_of)]


def _letters(t):
    return W.to_ascii(t, W.DNA)


def test_serve_mix_equals_alone():
    torch = torch_cuda()
    pats, texts, dict_of, gaps = _workload(11, 120)
    want = _expected(pats, texts, dict_of)
    # alone: each request scanned by itself through ac_scan
    dicts = [ac.ac_build(p, sigma=4) for p in pats]
    for t, d, w in zip(texts, dict_of, want):
        dev = torch.from_numpy(t.copy()).cuda()
        out, total = ac.scan(dicts[d], dev, ac.AC_TEXT_U8)
        assert total == len(w)
        assert np.array_equal(ac.match_keys(out), w)
    # in the mix: all queued at once, small batches, two streams
    from paper_1403_7294_amd.serve import Server
    srv = Server(pats, max_batch=8, streams=2)
    futs = [srv.submit(_letters(t), int(d)) for t, d in zip(texts, dict_of)]
    got = [f.result(timeout=60) for f in futs]
    st = srv.close()
    for k, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), k
    assert st.batches >= len(texts) // 8
    assert st.overlapped > 0          # batches admitted while others ran
    assert len(st.latencies_s) == len(texts)


def test_serve_poisson_arrivals_and_overflow():
    torch_cuda()
    from paper_1403_7294_amd.serve import Server, run_poisson
    pats, texts, dict_of, gaps = _workload(12, 150)
    want = _expected(pats, texts, dict_of)
    # margin 0: every reservation is the 64-match floor, so requests with
    # more matches overflow and are scanned again exactly sized
    srv = Server(pats, max_batch=16, streams=3, margin=0.0)
    futs = run_poisson(srv, [_letters(t) for t in texts], dict_of, gaps, rate=3000.0)
    got = [f.result(timeout=60) for f in futs]
    st = srv.close()
    for k, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), k
    assert st.reruns == sum(len(w) > 64 for w in want) > 0
    s = st.summary()
    assert s["requests"] == len(texts) and s["p99_ms"] >= s["p50_ms"] > 0


def test_serve_memory_budget():
    torch_cuda()
    from paper_1403_7294_amd.serve import Server
    pats, texts, dict_of, _ = _workload(13, 40)
    want = _expected(pats, texts, dict_of)
    big = max(len(t) for t in texts)
    probe = Server(pats)
    budget = 3 * max(probe.request_charge(big, d) for d in range(len(pats)))
    probe.close()
    srv = Server(pats, budget_bytes=budget, max_batch=64, streams=2)
    futs = [srv.submit(_letters(t), int(d)) for t, d in zip(texts, dict_of)]
    got = [f.result(timeout=60) for f in futs]
    st = srv.close()
    for k, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), k
    assert 0 < st.peak_bytes <= budget
    assert st.batches > 2
    # a request that can never fit is refused, not queued forever
    srv = Server(pats, budget_bytes=1024)
    f = srv.submit(_letters(np.zeros(4096, np.uint8)), 0)
    with pytest.raises(MemoryError):
        f.result(timeout=10)
    srv.close()


def test_serve_invalid_letters_and_empty():
    torch_cuda()
    from paper_1403_7294_amd.serve import Server
    pats, texts, dict_of, _ = _workload(14, 12)
    want = _expected(pats, texts, dict_of)
    srv = Server(pats, max_batch=64)
    good = [srv.submit(_letters(t), int(d)) for t, d in zip(texts, dict_of)]
    bad_text = _letters(texts[5]).copy()
    bad_text[len(bad_text) // 2] = ord("N")
    bad = srv.submit(bad_text, int(dict_of[5]))
    empty = srv.submit(np.zeros(0, np.uint8), 0)
    with pytest.raises(ValueError):
        bad.result(timeout=60)
    assert len(empty.result(timeout=60)) == 0
    for k, (f, w) in enumerate(zip(good, want)):
        assert np.array_equal(f.result(timeout=60), w), k
    srv.close()


def test_serve_failed_batch_allocation():
    # the third batch's device allocation is reported failed (fault
    # injection from the host; no GPU fault): exactly that batch's requests
    # get MemoryError, every other request is served correctly, and the
    # server keeps going
    torch_cuda()
    from paper_1403_7294_amd.serve import Server
    pats, texts, dict_of, _ = _workload(15, 40)
    want = _expected(pats, texts, dict_of)
    srv = Server(pats, max_batch=4, streams=2, fail_batch=3)
    futs = [srv.submit(_letters(t), int(d)) for t, d in zip(texts, dict_of)]
    failed = 0
    for k, (f, w) in enumerate(zip(futs, want)):
        try:
            got = f.result(timeout=60)
        except MemoryError:
            failed += 1
            continue
        assert np.array_equal(got, w), k
    assert 1 <= failed <= 4
    late = srv.submit(_letters(texts[0]), int(dict_of[0]))
    assert np.array_equal(late.result(timeout=60), want[0])
    st = srv.close()
    assert len(st.latencies_s) == len(texts) - failed + 1


def test_serve_accounts_batch_workspace():
    # the budget counts each request's share of the batch workspace: a
    # budget just above one request's letters, text and reservation, but
    # below that plus its workspace bound, refuses it
    torch_cuda()
    from paper_1403_7294_amd.serve import Server
    pats, texts, dict_of, _ = _workload(16, 8)
    n = 100_000
    srv = Server(pats, budget_bytes=n + n // 4 + 8 * 300 + 4096)
    assert srv.request_charge(n, 0) > 1.5 * n + n + n // 4
    f = srv.submit(_letters(np.zeros(n, np.uint8)), 0)
    with pytest.raises(MemoryError):
        f.result(timeout=10)
    srv.close()
