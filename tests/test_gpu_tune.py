"""GPU tests of the autotuner: the shape it picks gives the oracle's exact
result, the choice is cached by shape key and reused without timing, and
the batch tuner's shape gives every instance's exact result."""
import json

import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture
def cache(tmp_path, monkeypatch):
    p = tmp_path / "tune.json"
    monkeypatch.setenv("AC_TUNE_CACHE", str(p))
    from paper_1403_7294_amd import tune
    tune._mem.clear()
    return p


@pytest.mark.parametrize("which", ["dna_small", "protein", "dna_dense"])
def test_autotune_exact_and_cached(cache, which):
    torch_cuda()
    from paper_1403_7294_amd import tune
    if which == "dna_small":
        inst, fmt = W.dna_small(), ac.AC_TEXT_2BIT
    elif which == "protein":
        inst, fmt = W.protein(scale=1 / 16), ac.AC_TEXT_U8
    else:
        inst, fmt = W.dna_dense(scale=1 / 128), ac.AC_TEXT_2BIT
    d = ac.ac_build(inst.patterns, sigma=inst.sigma)
    text = device_text(inst, fmt)
    n = len(inst.text)
    timed = tune.stats["timed"]
    t = tune.autotune(d, text, n, fmt, reps=2)
    assert tune.stats["timed"] == timed + 1
    entry = json.loads(cache.read_text())[tune.key_for(d, n, fmt)]
    assert entry["tune"] == t and entry["candidates"] > 1
    want = oracle.Machine(inst.patterns, inst.sigma).scan_keys(inst.text)
    out, total = ac.scan(d, text, fmt, n=n, tune=t)
    assert total == len(want) and np.array_equal(ac.match_keys(out), want)
    # the same shape key is served from the cache, in memory and on disk
    hits = tune.stats["hits"]
    out, total = ac.scan(d, text, fmt, n=n, tune="auto")
    assert tune.stats["timed"] == timed + 1 and tune.stats["hits"] == hits + 1
    assert np.array_equal(ac.match_keys(out), want)
    tune._mem.clear()
    assert tune.autotune(d, text, n, fmt) == t and tune.stats["hits"] == hits + 2


def test_autotune_batch_exact():
    torch = torch_cuda()
    from paper_1403_7294_amd import tune
    insts = W.batch(scale=1 / 64, count=24)
    fmt = ac.AC_TEXT_2BIT
    dicts = [ac.ac_build(i.patterns, sigma=4) for i in insts]
    wants = [oracle.Machine(i.patterns, 4).scan_keys(i.text) for i in insts]
    texts = [device_text(i, fmt) for i in insts]
    outs = [torch.full((len(w) + 1, 2), -1, dtype=torch.int32, device="cuda") for w in wants]
    counts = torch.full((len(insts),), -1, dtype=torch.int64, device="cuda")
    items = [(d, t, len(i.text), fmt, o, len(w) + 1, counts[k:k + 1])
             for k, (d, t, i, o, w) in enumerate(zip(dicts, texts, insts, outs, wants))]
    best = tune.autotune_batch(items, reps=2)
    counts.fill_(-1)
    ac.ac_scan_batch(items, tune=best)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    for k, w in enumerate(wants):
        assert c[k] == len(w)
        assert np.array_equal(ac.match_keys(outs[k][:len(w)]), w), k


def test_timing_of_chosen_kinds_only():
    # with a kind mask, only those kernels are timed (the others record no
    # events); the scan's result does not depend on timing
    torch = torch_cuda()
    inst = W.dna_small()
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    ac.ac_timing_enable(True, kinds=[ac.AC_K_COUNT, ac.AC_K_EMIT_DENSE])
    ac.ac_timing_read(reset=True)
    out, total = ac.scan(d, t, ac.AC_TEXT_2BIT, n=len(inst.text))
    torch.cuda.synchronize()
    tm = ac.ac_timing_read(reset=True)
    ac.ac_timing_enable(False)
    assert total == len(want) and np.array_equal(ac.match_keys(out), want)
    assert tm["count"][1] >= 1 and tm["emit_dense"][1] >= 1
    assert tm["scatter"][1] == 0 and tm["emit"][1] == 0 and tm["offsets"][1] == 0
