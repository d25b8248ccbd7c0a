"""GPU parity of the alternative forms of stage 2: the radix sort into
(end, id) order, the failure-less scan (one thread per start position) and
the partitioned dictionary (one machine per pattern slice), each against the
oracle or numpy, bit-exact and in order."""
import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, torch_cuda

pytestmark = pytest.mark.gpu


def _want(inst):
    return oracle.Machine(inst.patterns, inst.sigma).scan_keys(inst.text)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 1000, 65537, 1 << 20])
def test_sort_matches(n):
    torch = torch_cuda()
    rng = W.rng_for(900 + n)
    ends = rng.integers(0, 1 << 22, size=n, dtype=np.uint64)
    ids = rng.integers(0, 1 << 20, size=n, dtype=np.uint64)
    keys = (ends << np.uint64(32)) | ids
    dev = torch.from_numpy(keys.view(np.int32).reshape(n, 2).copy()).cuda()
    ac.ac_sort_matches(dev, n, end_bits=22)
    torch.cuda.synchronize()
    assert np.array_equal(ac.match_keys(dev), np.sort(keys))
    # stable sort on end alone keeps equal-end records in their order
    order = np.lexsort((ids, ends))
    pre = keys[order]
    rot = np.roll(pre, n // 3)  # tie order inside equal ends preserved, ends shuffled
    dev = torch.from_numpy(rot.view(np.int32).reshape(n, 2).copy()).cuda()
    ws = torch.empty(max(1, ac.ac_sort_workspace_size(n)), dtype=torch.uint8, device="cuda")
    ac.ac_sort_matches(dev, n, flags=ac.AC_SORT_BY_END, end_bits=22, workspace_dev=ws)
    torch.cuda.synchronize()
    want = rot[np.argsort(rot >> np.uint64(32), kind="stable")]
    assert np.array_equal(ac.match_keys(dev), want)


def _pfac(d, t, n, fmt, cap=None):
    torch = torch_cuda()
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    cap = cap if cap is not None else max(1024, n // 2)
    out = torch.full((max(1, cap), 2), -1, dtype=torch.int32, device="cuda")
    ac.ac_scan_pfac(d, t, n, fmt, out, cap, cnt)
    torch.cuda.synchronize()
    total = int(cnt.item())
    if total > cap:
        return _pfac(d, t, n, fmt, total) if cap else (None, total)
    return ac.match_keys(out[:total]), total


@pytest.mark.parametrize("sigma", [4, 20])
def test_pfac_tiny_corpus(sigma):
    for seed in range(60):
        inst = W.tiny(7000 + seed * 5 + sigma, sigma, max_text=300, max_pats=20, max_len=9)
        inst.alphabet = W.DNA if sigma == 4 else ""
        d = ac.ac_build(inst.patterns, sigma=sigma)
        want = _want(inst)
        for fmt in ([ac.AC_TEXT_U8, ac.AC_TEXT_2BIT] if sigma == 4 else [ac.AC_TEXT_U8]):
            t = device_text(inst, fmt)
            got, total = _pfac(d, t, len(inst.text), fmt)
            assert total == len(want), (seed, fmt)
            assert np.array_equal(got, want), (seed, fmt)


@pytest.mark.parametrize("which", ["dna_small", "protein", "dna_dense"])
def test_pfac_workloads(which):
    if which == "dna_small":
        inst, fmt = W.dna_small(), ac.AC_TEXT_2BIT
    elif which == "protein":
        inst, fmt = W.protein(scale=1 / 16), ac.AC_TEXT_U8
    else:
        inst, fmt = W.dna_dense(scale=1 / 64), ac.AC_TEXT_2BIT
    d = ac.ac_build(inst.patterns, sigma=inst.sigma)
    got, total = _pfac(d, device_text(inst, fmt), len(inst.text), fmt)
    want = _want(inst)
    assert total == len(want) and np.array_equal(got, want)


def test_pfac_overflow_prefix_and_empty():
    torch = torch_cuda()
    inst = W.dna_dense(scale=1 / 256)
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = _want(inst)
    cap = len(want) // 3
    out = torch.full((cap + 8, 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan_pfac(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, cap, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(ac.match_keys(out[:cap]), want[:cap])
    assert (out[cap:].cpu().numpy() == -1).all()
    ac.ac_scan_pfac(d, t, 0, ac.AC_TEXT_2BIT, out, cap, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


@pytest.mark.parametrize("parts", [0, 1, 3, 7])
def test_partitioned_dna(parts):
    inst = W.dna_dense(scale=1 / 64)
    d = ac.ac_build_partitioned(inst.patterns, sigma=4, parts=parts)
    bases = ac.ac_dict_parts(d)
    assert bases[0] == 0 and bases == sorted(bases)
    if parts:
        assert len(bases) == parts
    else:
        _, lds = ac.ac_device_info()
        assert len(bases) >= d.info.states * 8 // lds
    t = device_text(inst, ac.AC_TEXT_2BIT)
    out, total = ac.scan(d, t, ac.AC_TEXT_2BIT, n=len(inst.text))
    want = _want(inst)
    assert total == len(want) and np.array_equal(ac.match_keys(out), want)


def test_partitioned_protein_and_overflow():
    torch = torch_cuda()
    inst = W.protein(scale=1 / 16)
    d = ac.ac_build_partitioned(inst.patterns, sigma=20)
    assert len(ac.ac_dict_parts(d)) > 1
    t = device_text(inst, ac.AC_TEXT_U8)
    want = _want(inst)
    out, total = ac.scan(d, t, ac.AC_TEXT_U8, n=len(inst.text))
    assert total == len(want) and np.array_equal(ac.match_keys(out), want)
    cap = len(want) // 2
    o = torch.full((cap + 4, 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan(d, t, len(inst.text), ac.AC_TEXT_U8, o, cap, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(ac.match_keys(o[:cap]), want[:cap])


def test_partitioned_rejected_where_unsupported():
    torch = torch_cuda()
    inst = W.dna_small(scale=1 / 16)
    d = ac.ac_build_partitioned(inst.patterns, sigma=4, parts=2)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(ac.ACError):
        ac.ac_scan_batch([(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, 16, cnt)])
    with pytest.raises(ac.ACError):
        ac.ac_scan_workspace_size(d, len(inst.text), ac.AC_TEXT_2BIT)
    with pytest.raises(ac.ACError):
        ac.ac_scan_pfac(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, 16, cnt)
