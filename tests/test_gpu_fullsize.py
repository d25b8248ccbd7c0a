"""GPU parity at the full sizes of the batched and the served workloads.

Every instance is compared element by element, order included, with the
oracle's single pass over the same text (section III.A: every occurrence in
one pass, Fig. 2):

* the batch workload at its full size: 512 independent DNA instances (text
  log-uniform 4 Ki-4 Mi bases, 10-2,000 patterns of 8-24 each; about 356 M
  bases in all), through one plan (``ac_batch_create`` / ``ac_batch_run``),
  its replay, and a hipGraph capture of the plan replayed with eager work
  between replays;
* the eight serving dictionaries at their full size (1,000-50,000 random
  10-30-mers, 15,592-649,494 states, hybrid or global placement), each
  against a request of just over 1 M bases, scanned alone through ``ac_scan``
  and through the continuous-batching server mixed with other requests.
"""
import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, torch_cuda

pytestmark = pytest.mark.gpu


def _check(wants, outs, counts, tag):
    c = counts.cpu().numpy()
    for k, w in enumerate(wants):
        assert c[k] == len(w), (tag, k, int(c[k]), len(w))
        assert np.array_equal(ac.match_keys(outs[k][:len(w)]), w), (tag, k)


def test_batch_full_size_plan_replay_and_graph():
    torch = torch_cuda()
    insts = W.batch()
    assert len(insts) == 512
    wants = [oracle.Machine(i.patterns, 4).scan_keys(i.text) for i in insts]
    dicts = [ac.ac_build(i.patterns, sigma=4) for i in insts]
    texts = [device_text(i, ac.AC_TEXT_2BIT) for i in insts]
    outs = [torch.full((len(w) + 4, 2), -1, dtype=torch.int32, device="cuda") for w in wants]
    counts = torch.full((len(insts),), -1, dtype=torch.int64, device="cuda")
    items = [(d, t, len(i.text), ac.AC_TEXT_2BIT, o, len(w) + 4, counts[k:k + 1])
             for k, (d, t, i, o, w) in enumerate(zip(dicts, texts, insts, outs, wants))]
    print(f"batch: {sum(len(i.text) for i in insts)} bases, "
          f"{sum(len(w) for w in wants)} matches", flush=True)

    def reset():
        counts.fill_(-1)
        for o in outs:
            o.fill_(-1)
        torch.cuda.synchronize()

    plan = ac.ac_batch_create(items)
    for rep in range(2):
        reset()
        ac.ac_batch_run(plan)
        torch.cuda.synchronize()
        _check(wants, outs, counts, f"plan run {rep}")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        ac.ac_batch_run(plan, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            ac.ac_batch_run(plan, stream=s)
    for rep in range(3):
        reset()
        g.replay()
        torch.cuda.synchronize()
        _check(wants, outs, counts, f"graph replay {rep}")
    plan.close()
    # the one-call form with the library's default shape
    reset()
    ac.ac_scan_batch(items)
    torch.cuda.synchronize()
    _check(wants, outs, counts, "ac_scan_batch")


def _serve_requests():
    """The serving dictionaries at full size, one request of just over 1 M
    bases per dictionary (ragged lengths), and 48 further requests of the
    serving length mix (shrunk 4x so that the oracle stays quick)."""
    wl = W.serve(requests=48, scale=0.25)
    rng = W.rng_for(55)
    big = [rng.integers(0, 4, size=1_048_576 + 13 * k + 3, dtype=np.uint8) for k in range(8)]
    return wl, big


def test_serve_dictionaries_full_size_alone():
    torch = torch_cuda()
    wl, big = _serve_requests()
    for k, (pats, t) in enumerate(zip(wl.dictionaries, big)):
        want = oracle.Machine(pats, 4).scan_keys(t)
        d = ac.ac_build(pats, sigma=4)
        print(f"dictionary {k}: {pats.count} patterns, {d.info.states} states, "
              f"placement {d.info.placement}, {len(want)} matches", flush=True)
        for fmt in (ac.AC_TEXT_2BIT, ac.AC_TEXT_U8):
            inst = W.Instance(t, pats, 4, W.DNA)
            dev = device_text(inst, fmt)
            out, total = ac.scan(d, dev, fmt, n=len(t))
            assert total == len(want), (k, fmt, total, len(want))
            assert np.array_equal(ac.match_keys(out), want), (k, fmt)
        torch.cuda.synchronize()


def test_serve_dictionaries_full_size_in_the_mix():
    torch_cuda()
    from paper_1403_7294_amd.serve import Server
    wl, big = _serve_requests()
    machines = [oracle.Machine(p, 4) for p in wl.dictionaries]
    texts = list(wl.texts)
    dict_of = [int(x) for x in wl.dict_of]
    # the big requests interleaved with the others
    for k, t in enumerate(big):
        pos = 6 * k + 3
        texts.insert(pos, t)
        dict_of.insert(pos, k)
    want = [machines[d].scan_keys(t) for t, d in zip(texts, dict_of)]
    srv = Server(wl.dictionaries, max_batch=8, streams=2)
    futs = [srv.submit(W.to_ascii(t, W.DNA), d) for t, d in zip(texts, dict_of)]
    got = [f.result(timeout=300) for f in futs]
    st = srv.close()
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), (i, dict_of[i], len(texts[i]), len(g), len(w))
    assert st.overlapped > 0
