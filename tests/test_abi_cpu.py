"""Host-side checks of the C-ABI library (no GPU needed): every declared
symbol is exported, arguments are validated, and the compiled tables are
the automaton the paper describes (checked by walking them on the CPU with
the chunk/overlap rule and comparing with the oracle)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from conftest import ROOT
from emulate import emulate_scan


def _declared():
    src = open(os.path.join(ROOT, "include", "ac.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(ac_\w+)\(", src, re.M)))


def test_header_declares_binding_symbols():
    assert _declared() == sorted(ac.ABI_SYMBOLS)


def test_library_exports_every_symbol():
    L = ac.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_no_oracle_in_product():
    # the product library and binding never touch the oracle
    pkg = os.path.join(ROOT, "paper_1403_7294_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h", ".inc")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "ac_oracle" not in txt and "liboracle" not in txt, f


def test_status_strings():
    assert ac.ac_status_str(ac.AC_OK) == "ok"
    assert "empty" in ac.ac_status_str(ac.AC_E_EMPTY_PATTERN)


@pytest.mark.parametrize("pats,sigma,code", [
    ([[0, 1], []], 4, ac.AC_E_EMPTY_PATTERN),
    ([[0, 4]], 4, ac.AC_E_SYMBOL),
    ([[0]], 1, ac.AC_E_INVALID),
    ([[0]], 300, ac.AC_E_INVALID),
    ([], 4, ac.AC_E_INVALID),
])
def test_build_rejects(pats, sigma, code):
    with pytest.raises(ac.ACError) as e:
        ac.ac_build(pats, sigma=sigma, host_only=True)
    assert e.value.status == code


def test_timing_mask_validation():
    # a mask naming kinds past AC_K_KINDS, or a negative value, is rejected
    assert ac.lib().ac_timing_enable(ac.AC_TIMING_KIND(ac.AC_K_KINDS)) == ac.AC_E_INVALID
    assert ac.lib().ac_timing_enable(-2) == ac.AC_E_INVALID
    assert ac.lib().ac_timing_enable(ac.AC_TIMING_KIND(ac.AC_K_COUNT)) == ac.AC_OK
    assert ac.lib().ac_timing_enable(0) == ac.AC_OK


def test_scan_needs_device_tables():
    d = ac.ac_build([[0, 1]], sigma=4, host_only=True)
    assert d.info.has_device == 0
    cnt = ctypes.c_uint64()
    rc = ac.lib().ac_scan(d.handle, None, 0, 0, None, 0, ctypes.addressof(cnt), None, None, 0,
                          None)
    assert rc == ac.AC_E_NO_DEVICE


def test_fig2_tables():
    # HIS, HERS, SHE over E H I R S: ten states, SHE and HERS end in output
    # states, and the completed transition of SHE's state on R is HER's
    alpha = "EHIRS"
    names = ["HIS", "HERS", "SHE"]
    d = ac.ac_build([[alpha.index(c) for c in p] for p in names], sigma=5, host_only=True)
    delta, off, ids, depth = ac.ac_debug_export(d)
    info = d.info
    assert info.states == 10 and info.max_len == 4 and info.min_len == 3
    def walk(word):
        s = 0
        for ch in word:
            s = int(delta[s, alpha.index(ch)])
        return s
    she, hers = walk("SHE"), walk("HERS")
    assert she >= info.first_output_state and hers >= info.first_output_state
    fo = info.first_output_state
    assert list(ids[off[she - fo]:off[she - fo + 1]]) == [2]
    assert list(ids[off[hers - fo]:off[hers - fo + 1]]) == [1]
    assert delta[she, alpha.index("R")] == walk("HER")
    assert depth[she] == 3 and depth[0] == 0


def _check_instance(inst, chunks=(64, 128, 1024)):
    d = ac.ac_build(inst.patterns, sigma=inst.sigma, host_only=True)
    delta, off, ids, _ = ac.ac_debug_export(d)
    fo = d.info.first_output_state
    # output-set invariants of the renumbering
    sizes = np.diff(off.astype(np.int64))
    assert (sizes > 0).all()
    want = oracle.Machine(inst.patterns, inst.sigma).scan_keys(inst.text)
    warm = int(inst.patterns.lengths.max()) - 1
    for c in chunks:
        got = emulate_scan(delta, off, ids, fo, inst.text, c, warm)
        assert np.array_equal(got, want), c
    return d


def test_compiled_tables_tiny():
    for seed in range(300):
        inst = W.tiny(seed, 2 + seed % 3, max_text=40)
        if len(inst.text) == 0:
            continue
        _check_instance(inst, chunks=(1, 3, 64))


def test_compiled_tables_dna_small():
    _check_instance(W.dna_small(scale=1 / 64))


def test_compiled_tables_dna_dense():
    _check_instance(W.dna_dense(scale=1 / 2048), chunks=(64, 512))


def test_compiled_tables_protein():
    _check_instance(W.protein(scale=1 / 512), chunks=(64, 256))


def test_build_info_full_configs():
    for inst in (W.dna_small(), W.protein(scale=1 / 64)):
        d = ac.ac_build(inst.patterns, sigma=inst.sigma, host_only=True)
        i = d.info
        assert i.patterns == inst.patterns.count
        assert i.max_len == int(inst.patterns.lengths.max())
        assert i.table_bytes == i.states * i.sigma * 4
        assert i.output_entries >= i.patterns


def test_info_struct_layout():
    # the ctypes mirrors must match the C layout (sizes checked against the
    # header's field lists)
    assert ctypes.sizeof(ac.ac_match) == 8
    assert ctypes.sizeof(ac.ac_build_opts) == 16
    assert ctypes.sizeof(ac.ac_tune) == 20
    assert ctypes.sizeof(ac.ac_batch_item) == 56


@pytest.mark.parametrize("which", ["tiny", "dna_dense", "protein", "serve_large"])
def test_parallel_build_equals_serial(which):
    """The level-parallel host build gives exactly the serial build's tables
    (the serve dictionary has more than 65,536 output-free states, so the
    partial ranking path is taken too)."""
    if which == "tiny":
        pats, sigma = W.tiny(77, 4, max_pats=12).patterns, 4
    elif which == "dna_dense":
        pats, sigma = W.dna_dense(scale=1 / 4096).patterns, 4
    elif which == "protein":
        pats, sigma = W.protein(scale=1 / 64).patterns, 20
    else:
        pats, sigma = W.serve(requests=1).dictionaries[5], 4
    a = ac.ac_build(pats, sigma=sigma, host_only=True, serial=True)
    b = ac.ac_build(pats, sigma=sigma, host_only=True)
    for x, y in zip(ac.ac_debug_export(a), ac.ac_debug_export(b)):
        assert np.array_equal(x, y)
    assert a.info.states == b.info.states and a.info.first_output_state == b.info.first_output_state
    if which == "serve_large":
        assert a.info.first_output_state > 65536
        # the scan behaviour is the oracle's on a sample text
        rng = W.rng_for(9)
        text = rng.integers(0, 4, size=20000, dtype=np.uint8)
        sub = W.PatternSet.from_list(W._cut(rng, text, rng.integers(10, 31, size=50)) +
                                     pats.as_list()[:2000])
        c = ac.ac_build(sub, sigma=4, host_only=True)
        delta, out_off, out_ids, depth = ac.ac_debug_export(c)
        want = oracle.Machine(sub, 4).scan_keys(text)
        got = emulate_scan(delta, out_off, out_ids, c.info.first_output_state, text, 1024,
                           c.info.max_len - 1)
        assert np.array_equal(got, want)


def test_partitioned_build_host():
    """Slices are contiguous, start at pattern 0, and each slice's table fits
    LDS as 16-bit rows when the count is chosen automatically."""
    pats = W.dna_dense(scale=1 / 4096).patterns
    d = ac.ac_build_partitioned(pats, sigma=4, host_only=True)
    bases = ac.ac_dict_parts(d)
    assert bases[0] == 0 and all(a < b for a, b in zip(bases, bases[1:]))
    assert len(bases) >= 2
    assert d.info.patterns == pats.count
    with pytest.raises(ac.ACError):
        ac.ac_debug_export(d)
    d3 = ac.ac_build_partitioned(pats, sigma=4, parts=3, host_only=True)
    assert len(ac.ac_dict_parts(d3)) == 3
    assert ac.ac_dict_parts(ac.ac_build(pats, sigma=4, host_only=True)) == []


def test_microbench_library_exports_every_declared_symbol():
    from paper_1403_7294_amd import microbench
    src = open(os.path.join(ROOT, "include", "ac_microbench.h")).read()
    declared = sorted(set(re.findall(r"^\s*int\s+(acb_\w+)\(", src, re.M)))
    assert declared == sorted(microbench.SYMBOLS)
    L = microbench.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_microbench_cycle_is_one_permutation_cycle():
    from paper_1403_7294_amd.microbench import _cyclic_permutation
    nxt = _cyclic_permutation(4096, 3)
    assert np.array_equal(np.sort(nxt), np.arange(4096, dtype=np.uint32))
    s, seen = 0, 0
    while True:
        s = int(nxt[s])
        seen += 1
        if s == 0:
            break
    assert seen == 4096


def test_batch_item_record_layout_matches_the_c_struct():
    import ctypes as C
    dt = ac.BATCH_ITEM_DTYPE
    assert dt.itemsize == C.sizeof(ac.ac_batch_item)
    for name, ctype in ac.ac_batch_item._fields_:
        rec = {"d_text": "text", "d_out": "out", "d_count": "count"}.get(name, name)
        assert dt.fields[rec][1] == getattr(ac.ac_batch_item, name).offset, name
