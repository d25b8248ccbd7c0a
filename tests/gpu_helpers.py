"""Helpers for the GPU tests: put synthetic instances on the device through
the library's own encoder and run scans through the C ABI."""
import numpy as np

import paper_1403_7294_amd as ac
import workloads as W


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def alphabet_id(inst):
    return ac.AC_ALPHA_PROTEIN if inst.alphabet == W.PROTEIN else ac.AC_ALPHA_DNA


def device_text(inst, fmt):
    """The instance's text on the GPU in format fmt, produced from letters by
    ac_encode when the instance has an alphabet, else uploaded as codes."""
    torch = torch_cuda()
    n = len(inst.text)
    if not inst.alphabet:
        assert fmt == ac.AC_TEXT_U8
        return torch.from_numpy(inst.text.copy()).cuda() if n else torch.empty(1, dtype=torch.uint8,
                                                                               device="cuda")
    letters = torch.from_numpy(W.to_ascii(inst.text, inst.alphabet)).cuda()
    nbytes = (n + 3) // 4 if fmt == ac.AC_TEXT_2BIT else n
    out = torch.empty(max(1, nbytes), dtype=torch.uint8, device="cuda")
    bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    if n:
        ac.ac_encode(letters, alphabet_id(inst), fmt, out, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    return out


def gpu_keys(d, text_dev, n, fmt, tune=None, capacity=None):
    out, total = ac.scan(d, text_dev, fmt, n=n, tune=tune, capacity=capacity)
    keys = ac.match_keys(out)
    return keys, total
