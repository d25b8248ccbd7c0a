"""GPU parity of the batched form: every instance of a batch against the
oracle run on that instance alone, one-shot and as a replayed plan, and a
replayed hipGraph capture of the plan."""
import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(insts, fmt):
    torch = torch_cuda()
    dicts = [ac.ac_build(i.patterns, sigma=i.sigma) for i in insts]
    wants = [oracle.Machine(i.patterns, i.sigma).scan_keys(i.text) for i in insts]
    texts = [device_text(i, fmt) for i in insts]
    outs = [torch.full((len(w) + 4, 2), -1, dtype=torch.int32, device="cuda") for w in wants]
    counts = torch.full((len(insts),), -1, dtype=torch.int64, device="cuda")
    items = [(d, t, len(i.text), fmt, o, len(w) + 4, counts[k:k + 1])
             for k, (d, t, i, o, w) in enumerate(zip(dicts, texts, insts, outs, wants))]
    return dicts, wants, outs, counts, items


def _check(wants, outs, counts):
    c = counts.cpu().numpy()
    for k, w in enumerate(wants):
        assert c[k] == len(w), k
        assert np.array_equal(ac.match_keys(outs[k][:len(w)]), w), k


@pytest.mark.parametrize("fmt", [ac.AC_TEXT_2BIT, ac.AC_TEXT_U8])
def test_batch_one_shot(fmt):
    torch = torch_cuda()
    insts = W.batch(scale=1 / 64, count=48)
    dicts, wants, outs, counts, items = _setup(insts, fmt)
    ac.ac_scan_batch(items)
    torch.cuda.synchronize()
    _check(wants, outs, counts)


def test_batch_mixed_placements_and_empty():
    torch = torch_cuda()
    insts = W.batch(scale=1 / 32, count=12)
    insts.append(W.Instance(np.zeros(0, dtype=np.uint8), insts[0].patterns, 4, W.DNA))
    insts.append(W.dna_dense(scale=1 / 1024))   # big table: not in LDS
    insts.append(W.Instance(np.zeros(0, dtype=np.uint8), insts[1].patterns, 4, W.DNA))
    dicts, wants, outs, counts, items = _setup(insts, ac.AC_TEXT_2BIT)
    for tune in (None, {"chunk": 64, "block_threads": 256}, {"placement": ac.AC_PLACE_GLOBAL},
                 {"placement": ac.AC_PLACE_HYBRID, "chunk": 128},
                 {"placement": ac.AC_PLACE_LDS2}, {"placement": ac.AC_PLACE_LDS2, "chains": 4}):
        counts.fill_(-1)
        ac.ac_scan_batch(items, tune=tune)
        torch.cuda.synchronize()
        _check(wants, outs, counts)


def test_batch_protein_u8():
    torch = torch_cuda()
    insts = [W.protein(seed=30 + k, scale=1 / 2048) for k in range(6)]
    dicts, wants, outs, counts, items = _setup(insts, ac.AC_TEXT_U8)
    ac.ac_scan_batch(items)
    torch.cuda.synchronize()
    _check(wants, outs, counts)


def test_batch_plan_replay_and_graph():
    torch = torch_cuda()
    insts = W.batch(scale=1 / 64, count=32)
    dicts, wants, outs, counts, items = _setup(insts, ac.AC_TEXT_2BIT)
    plan = ac.ac_batch_create(items)
    for _ in range(3):
        counts.fill_(-1)
        for o in outs:
            o.fill_(-1)
        ac.ac_batch_run(plan)
        torch.cuda.synchronize()
        _check(wants, outs, counts)
    # capture the launches in a graph and replay it, with eager work between
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        ac.ac_batch_run(plan, stream=s)      # warm-up on the capture stream
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            ac.ac_batch_run(plan, stream=s)
    for _ in range(3):
        counts.fill_(-1)
        for o in outs:
            o.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check(wants, outs, counts)
    plan.close()


def test_batch_with_lds16_instances():
    # instances whose 32-bit table exceeds LDS while the 16-bit one fits are
    # counted with the whole-table LDS instances
    torch = torch_cuda()
    rng = W.rng_for(77)
    insts = W.batch(scale=1 / 64, count=10)
    for k in range(4):
        n = int(rng.integers(20_000, 200_000))
        text = rng.integers(0, 4, size=n, dtype=np.uint8)
        text[n // 3:n // 3 + 300] = 0
        pats = [np.zeros(10, np.uint8)]
        pats += W._cut(rng, text, rng.integers(8, 21, size=500))
        pats += [rng.integers(0, 4, size=int(L), dtype=np.uint8)
                 for L in rng.integers(8, 21, size=600 + 50 * k)]
        insts.insert(3 * k, W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA, "lds16"))
    dicts, wants, outs, counts, items = _setup(insts, ac.AC_TEXT_2BIT)
    _, lds = ac.ac_device_info()
    assert sum(1 for d in dicts if d.info.states * 16 + 1024 > lds - 512
               and d.info.states * 8 + 512 <= lds - 512) >= 3
    for tune in (None, {"chunk": 64, "block_threads": 512}, {"chains": 2}):
        counts.fill_(-1)
        ac.ac_scan_batch(items, tune=tune)
        torch.cuda.synchronize()
        _check(wants, outs, counts)
