"""ac_scan_noalloc: the scan that allocates nothing, against ac_scan.

Two calls in a row share the library's device scratch array; the second
has a smaller input, so stale records of the first call would show up in
it.  Each call's output must equal ac_scan's (and the oracle's) element by
element, order included.  A text whose workspace exceeds the array is
rejected before anything is enqueued."""
import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, torch_cuda

pytestmark = pytest.mark.gpu


def _both(d, text_dev, n, fmt, want, tune=None):
    """(no-alloc keys, ac_scan keys) for one text, each in its own buffer."""
    torch = torch_cuda()
    cap = len(want) + 16
    got = []
    for fn in (ac.ac_scan_noalloc, None):
        out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        if fn is None:
            ac.ac_scan(d, text_dev, n, fmt, out, cap, cnt, tune=tune)
        else:
            fn(d, text_dev, n, fmt, out, cap, cnt, tune=tune)
        torch.cuda.synchronize()
        c = int(cnt.item())
        assert c == len(want), (fn, c, len(want))
        assert bool((out[c:] == -1).all()), "slots past the total were written"
        got.append(ac.match_keys(out[:c]))
    return got


@pytest.mark.parametrize("which", ["dna_dense", "dna_small", "protein"])
def test_noalloc_two_calls_second_smaller(which):
    torch_cuda()
    if which == "dna_dense":
        inst = W.dna_dense(scale=1 / 64)          # hybrid table, dense poly-A output
        fmt = ac.AC_TEXT_2BIT
    elif which == "dna_small":
        inst = W.dna_small()                      # whole table in LDS
        fmt = ac.AC_TEXT_2BIT
    else:
        inst = W.protein(scale=1 / 32)            # bytes, hybrid table
        fmt = ac.AC_TEXT_U8
    d = ac.ac_build(inst.patterns, sigma=inst.sigma)
    m = oracle.Machine(inst.patterns, inst.sigma)
    n1 = len(inst.text)
    n2 = n1 // 3 + 37                             # smaller, ragged
    print(f"{which}: n1={n1} n2={n2} states={d.info.states}", flush=True)
    text_dev = device_text(inst, fmt)
    for n in (n1, n2):
        want = m.scan_keys(inst.text[:n])
        noalloc, plain = _both(d, text_dev, n, fmt, want)
        assert np.array_equal(noalloc, plain), n
        assert np.array_equal(noalloc, want), n


def test_noalloc_overflow_and_empty():
    torch = torch_cuda()
    inst = W.dna_small(scale=1 / 4)
    d = ac.ac_build(inst.patterns, sigma=4)
    text_dev = device_text(inst, ac.AC_TEXT_2BIT)
    n = len(inst.text)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    # capacity below the total: the total is reported, the canonical prefix written
    cap = max(1, len(want) // 2)
    out = torch.full((len(want), 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan_noalloc(d, text_dev, n, ac.AC_TEXT_2BIT, out, cap, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(ac.match_keys(out[:cap]), want[:cap])
    assert bool((out[cap:] == -1).all())
    # empty text: total 0
    cnt.fill_(7)
    ac.ac_scan_noalloc(d, text_dev, 0, ac.AC_TEXT_2BIT, out, cap, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


def test_noalloc_rejects_text_beyond_scratch():
    torch = torch_cuda()
    inst = W.dna_small(scale=1 / 16)
    d = ac.ac_build(inst.patterns, sigma=4)
    limit = 64 << 20
    n = 1 << 27                                    # 128 Mi bases
    assert ac.ac_scan_workspace_size(d, n, ac.AC_TEXT_2BIT) > limit
    # a real buffer of that size, so that even a wrong launch stays in bounds
    text_dev = torch.zeros(n // 4, dtype=torch.uint8, device="cuda")
    out = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(ac.ACError) as e:
        ac.ac_scan_noalloc(d, text_dev, n, ac.AC_TEXT_2BIT, out, 16, cnt)
    assert e.value.status == ac.AC_E_TOO_LARGE
    torch.cuda.synchronize()
    assert int(cnt.item()) == -5                   # nothing was enqueued
