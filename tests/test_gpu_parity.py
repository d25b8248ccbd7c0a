"""GPU parity: the HIP scan against the CPU oracle, element by element, on
the same seeded inputs (bit-exact: matches are integers)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, gpu_keys, torch_cuda

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _parity(inst, fmt, tune=None, d=None):
    torch = torch_cuda()
    if d is None:
        d = ac.ac_build(inst.patterns, sigma=inst.sigma)
    t = device_text(inst, fmt)
    got, total = gpu_keys(d, t, len(inst.text), fmt, tune=tune)
    want = oracle.Machine(inst.patterns, inst.sigma).scan_keys(inst.text)
    assert total == len(want)
    assert np.array_equal(got, want)
    return d, total


def test_device_info():
    cu, lds = ac.ac_device_info()
    _say("compute units", cu, "lds per block", lds)
    assert cu >= 1 and lds >= 64 * 1024


# ------------------------------------------------------------ encoding

@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 15, 16, 17, 63, 64, 65, 1000, 1 << 20, (1 << 20) + 7])
def test_encode_dna(n):
    torch = torch_cuda()
    rng = W.rng_for(100 + n)
    codes = rng.integers(0, 4, size=n, dtype=np.uint8)
    letters = W.to_ascii(codes, W.DNA)
    low = rng.random(n) < 0.3
    letters = np.where(low, letters | 0x20, letters).astype(np.uint8)
    a = torch.from_numpy(letters).cuda() if n else torch.empty(0, dtype=torch.uint8, device="cuda")
    out8 = torch.full((max(1, n),), 77, dtype=torch.uint8, device="cuda")
    out2 = torch.full((max(1, (n + 3) // 4),), 77, dtype=torch.uint8, device="cuda")
    bad = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    ac.ac_encode(a, ac.AC_ALPHA_DNA, ac.AC_TEXT_U8, out8, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    ac.ac_encode(a, ac.AC_ALPHA_DNA, ac.AC_TEXT_2BIT, out2, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    want = oracle.encode(letters, W.DNA)
    assert np.array_equal(out8.cpu().numpy()[:n], want)
    assert np.array_equal(out2.cpu().numpy()[:(n + 3) // 4], oracle.pack2(want))


@pytest.mark.parametrize("n,offset", [(1, 0), (63, 1), (64, 0), (65, 3), (4096, 0), (4097, 5),
                                      ((1 << 20) + 13, 0), ((1 << 20) + 13, 7)])
def test_encode_dna_invalid_and_unaligned(n, offset):
    """Invalid letters become code 0 and are counted; the input may start at
    any byte (a view into a larger tensor); ragged tails."""
    torch = torch_cuda()
    rng = W.rng_for(300 + n + offset)
    letters = W.to_ascii(rng.integers(0, 4, size=n, dtype=np.uint8), W.DNA).copy()
    letters[rng.random(n) < 0.3] |= 0x20
    bad_at = rng.random(n) < 0.02
    letters[bad_at] = rng.choice(np.frombuffer(b"NXnx*bB\x00\xff", np.uint8), int(bad_at.sum()))
    clean = letters.copy()
    clean[bad_at] = ord("A")
    want = oracle.pack2(oracle.encode(clean, W.DNA))
    big = torch.zeros(n + offset + 64, dtype=torch.uint8, device="cuda")
    big[offset:offset + n] = torch.from_numpy(letters).cuda()
    out = torch.full(((n + 3) // 4,), 77, dtype=torch.uint8, device="cuda")
    bad = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    ac.ac_encode(big[offset:offset + n], ac.AC_ALPHA_DNA, ac.AC_TEXT_2BIT, out, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == int(bad_at.sum())
    assert np.array_equal(out.cpu().numpy(), want)


def test_encode_protein_and_invalid():
    torch = torch_cuda()
    rng = W.rng_for(7)
    n = 100_003
    codes = rng.integers(0, 20, size=n, dtype=np.uint8)
    letters = W.to_ascii(codes, W.PROTEIN)
    letters[::7] |= 0x20
    a = torch.from_numpy(letters).cuda()
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_encode(a, ac.AC_ALPHA_PROTEIN, ac.AC_TEXT_U8, out, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    assert np.array_equal(out.cpu().numpy(), oracle.encode(letters, W.PROTEIN))
    # letters outside the alphabet are counted
    bad_letters = letters.copy()
    bad_letters[[5, 77, 1000, n - 1]] = [ord("B"), ord("X"), ord("*"), ord("j")]
    a2 = torch.from_numpy(bad_letters).cuda()
    ac.ac_encode(a2, ac.AC_ALPHA_PROTEIN, ac.AC_TEXT_U8, out, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 4
    dna_bad = np.frombuffer(b"ACGTNACGTRYacgtn", dtype=np.uint8).copy()
    a3 = torch.from_numpy(dna_bad).cuda()
    out3 = torch.empty(4, dtype=torch.uint8, device="cuda")
    ac.ac_encode(a3, ac.AC_ALPHA_DNA, ac.AC_TEXT_2BIT, out3, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 4


# ------------------------------------------------------------ scan parity

@pytest.mark.parametrize("sigma", [2, 3, 4])
def test_tiny_corpus(sigma):
    torch = torch_cuda()
    for seed in range(150):
        inst = W.tiny(5000 + seed * 3 + sigma, sigma, max_text=300, max_pats=20, max_len=9)
        inst.alphabet = W.DNA if sigma == 4 else ""
        d = ac.ac_build(inst.patterns, sigma=sigma)
        n = len(inst.text)
        want = oracle.Machine(inst.patterns, sigma).scan_keys(inst.text)
        for fmt in ([ac.AC_TEXT_U8, ac.AC_TEXT_2BIT] if sigma == 4 else [ac.AC_TEXT_U8]):
            t = device_text(inst, fmt)
            tunes = [{"chunk": 64}]
            if fmt == ac.AC_TEXT_2BIT:
                tunes.append({"chunk": 64, "placement": ac.AC_PLACE_LDS2})
            for tune in tunes:
                got, total = gpu_keys(d, t, n, fmt, tune=tune)
                assert total == len(want), (seed, fmt, tune)
                assert np.array_equal(got, want), (seed, fmt, tune)


@pytest.mark.parametrize("fmt", [0, 1])
def test_dna_small_full(fmt):
    _say("dna_small fmt", fmt)
    d, total = _parity(W.dna_small(), fmt)
    assert total > 0


def test_protein_scaled():
    _say("protein 1/8")
    _parity(W.protein(scale=1 / 8), ac.AC_TEXT_U8)


def test_dna_dense_scaled():
    _say("dna_dense 1/64")
    _parity(W.dna_dense(scale=1 / 64), ac.AC_TEXT_2BIT)


@pytest.mark.parametrize("place", [ac.AC_PLACE_LDS, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_HYBRID])
@pytest.mark.parametrize("chunk,threads", [(64, 64), (128, 1024), (512, 256), (2048, 512)])
def test_launch_shapes_and_placements(place, chunk, threads):
    # the result must not depend on chunk size, block size or table placement
    inst = W.dna_dense(scale=1 / 512)
    d = ac.ac_build(inst.patterns, sigma=4, hot_states=1500)
    _say("placement", place, "chunk", chunk, "threads", threads, "states", d.info.states)
    _parity(inst, ac.AC_TEXT_2BIT, tune={"chunk": chunk, "block_threads": threads,
                                         "placement": place}, d=d)


def _two_symbol_dict_fits(d):
    _, lds = ac.ac_device_info()
    return d.info.states * 64 <= lds - 512


@pytest.mark.parametrize("chunk,threads,chains", [(64, 64, 1), (256, 1024, 2), (512, 256, 4),
                                                  (2048, 1024, 1)])
def test_two_symbol_stride_dna_small(chunk, threads, chains):
    inst = W.dna_small()
    d = ac.ac_build(inst.patterns, sigma=4)
    assert _two_symbol_dict_fits(d)
    _parity(inst, ac.AC_TEXT_2BIT, tune={"chunk": chunk, "block_threads": threads,
                                         "chains": chains, "placement": ac.AC_PLACE_LDS2}, d=d)


def test_two_symbol_stride_dense_and_odd_lengths():
    # poly-A text with A^k for odd and even k: outputs after the first symbol
    # of a pair (flagged entries) and after the second, in dense segments
    rng = W.rng_for(41)
    text = rng.integers(0, 4, size=300_000, dtype=np.uint8)
    for start in range(1000, 290_000, 9000):
        text[start:start + int(rng.integers(50, 700))] = 0
    pats = [np.zeros(k, np.uint8) for k in range(3, 17)]
    pats += W._cut(rng, text, rng.integers(5, 14, size=120))
    pats += [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in rng.integers(5, 14, size=60)]
    inst = W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA, "poly_a_odd")
    d = ac.ac_build(inst.patterns, sigma=4)
    assert _two_symbol_dict_fits(d)
    for tune in ({"placement": ac.AC_PLACE_LDS2}, {"placement": ac.AC_PLACE_LDS2, "chunk": 64},
                 {"placement": ac.AC_PLACE_LDS2, "chains": 4, "chunk": 1024}):
        _parity(inst, ac.AC_TEXT_2BIT, tune=tune, d=d)


def test_two_symbol_stride_falls_back():
    # tables that do not fit (or byte text) take the single-symbol path
    inst = W.dna_dense(scale=1 / 512)
    _parity(inst, ac.AC_TEXT_2BIT, tune={"placement": ac.AC_PLACE_LDS2})
    small = W.dna_small(scale=1 / 8)
    _parity(small, ac.AC_TEXT_U8, tune={"placement": ac.AC_PLACE_LDS2})


@pytest.mark.parametrize("place", [ac.AC_PLACE_LDS, ac.AC_PLACE_GLOBAL, ac.AC_PLACE_HYBRID])
def test_protein_placements(place):
    inst = W.protein(scale=1 / 256)
    d = ac.ac_build(inst.patterns, sigma=20, hot_states=300)
    _parity(inst, ac.AC_TEXT_U8, tune={"chunk": 128, "placement": place}, d=d)


def test_overflow_writes_canonical_prefix():
    torch = torch_cuda()
    inst = W.dna_dense(scale=1 / 256)
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    cap = len(want) // 3
    out = torch.full((cap + 16, 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, cap, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(ac.match_keys(out[:cap]), want[:cap])
    assert (out[cap:] == -1).all()          # nothing written past capacity
    # capacity 0: count only
    ac.ac_scan(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, 0, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)


def test_edge_cases():
    torch = torch_cuda()
    d = ac.ac_build([[0, 1, 2, 3, 0]], sigma=4)
    cnt = torch.full((1,), 9, dtype=torch.int64, device="cuda")
    out = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    t = torch.zeros(8, dtype=torch.uint8, device="cuda")
    ac.ac_scan(d, t, 0, ac.AC_TEXT_U8, out, 4, cnt)          # empty text
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    for n in (1, 3, 4):                                       # pattern longer than text
        ac.ac_scan(d, t, n, ac.AC_TEXT_U8, out, 4, cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == 0
    # a match ending on the very last symbol, 2-bit text of ragged length
    for n in (5, 6, 7, 9, 63, 64, 65, 127, 1029):
        codes = np.zeros(n, dtype=np.uint8)
        codes[-5:] = [0, 1, 2, 3, 0]
        inst = W.Instance(codes, W.PatternSet.from_list([[0, 1, 2, 3, 0], [0]]), 4, W.DNA)
        _parity(inst, ac.AC_TEXT_2BIT)
        _parity(inst, ac.AC_TEXT_U8)


def test_chunk_smaller_than_pattern():
    # chunks of 64 symbols against patterns of up to 200: the warm-up spans
    # several earlier chunks
    rng = W.rng_for(21)
    text = rng.integers(0, 4, size=20_000, dtype=np.uint8)
    pats = [text[o:o + L].copy() for o, L in zip(rng.integers(0, 19_000, 40),
                                                 rng.integers(60, 201, 40))]
    inst = W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA)
    for fmt in (0, 1):
        _parity(inst, fmt, tune={"chunk": 64})


def test_determinism():
    torch = torch_cuda()
    inst = W.dna_dense(scale=1 / 128)
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    ref, _ = gpu_keys(d, t, len(inst.text), ac.AC_TEXT_2BIT)
    for _ in range(5):
        got, _ = gpu_keys(d, t, len(inst.text), ac.AC_TEXT_2BIT)
        assert np.array_equal(got, ref)


def test_caller_workspace():
    torch = torch_cuda()
    inst = W.dna_small(scale=1 / 4)
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_U8)
    n = len(inst.text)
    need = ac.ac_scan_workspace_size(d, n, ac.AC_TEXT_U8)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    out = torch.empty((len(want) + 8, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan(d, t, n, ac.AC_TEXT_U8, out, len(want) + 8, cnt, workspace_dev=ws)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(ac.match_keys(out[:len(want)]), want)
    with pytest.raises(ac.ACError) as e:
        ac.ac_scan(d, t, n, ac.AC_TEXT_U8, out, 8, cnt, workspace_dev=ws[:need // 2])
    assert e.value.status == ac.AC_E_OVERFLOW


# ------------------------------------------------------------ full sizes

def test_protein_full():
    _say("protein full")
    _parity(W.protein(), ac.AC_TEXT_U8)


def test_dna_dense_full():
    # the benchmark's workload, in the launch configuration it times
    _say("dna_dense full")
    torch = torch_cuda()
    inst = W.dna_dense()
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    _say("oracle matches", len(want))
    got, total = gpu_keys(d, t, len(inst.text), ac.AC_TEXT_2BIT, capacity=len(want) + 1024)
    assert total == len(want)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("pats,n", [
    ([[0]], 1000),                       # 64 events per segment, 64 matches: sparse, > 16 events
    ([[0], [0, 0]], 1000),               # 127 matches per segment: sparse
    ([[0], [0], [0], [0]], 1000),        # exactly 256 matches per full segment: dense
    ([[0], [0], [0], [0], [0, 0]], 777),  # dense, ragged tail
    ([[0, 0, 0]] * 3 + [[1]], 5000),     # mixed
])
def test_event_overflow_and_dense_threshold(pats, n):
    rng = W.rng_for(n)
    text = np.zeros(n, dtype=np.uint8)
    text[rng.integers(0, n, n // 10)] = 1          # a few breaks in the runs
    inst = W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA)
    for fmt in (0, 1):
        _parity(inst, fmt, tune={"chunk": 128})


@pytest.mark.parametrize("chains", [1, 2, 4])
def test_chains_per_lane(chains):
    for inst, fmt in ((W.dna_dense(scale=1 / 512), ac.AC_TEXT_2BIT),
                      (W.protein(scale=1 / 256), ac.AC_TEXT_U8),
                      (W.dna_small(scale=1 / 8), ac.AC_TEXT_U8)):
        for place in (ac.AC_PLACE_AUTO, ac.AC_PLACE_GLOBAL):
            _parity(inst, fmt, tune={"chains": chains, "placement": place, "chunk": 128,
                                     "block_threads": 256})


def test_output_buffer_not_16_byte_aligned():
    # the dense writer pairs slots into 16-byte stores by address; start the
    # output one slot (8 bytes) into a buffer
    torch = torch_cuda()
    inst = W.dna_dense(scale=1 / 256)
    d = ac.ac_build(inst.patterns, sigma=4)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    buf = torch.full((len(want) + 3, 2), -1, dtype=torch.int32, device="cuda")
    out = buf[1:]
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ac.ac_scan(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, len(want), cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(want)
    assert np.array_equal(ac.match_keys(out[:len(want)]), want)
    assert (buf[0] == -1).all() and (buf[len(want) + 1:] == -1).all()


# ------------------------------------------------------------ 16-bit whole table in LDS

def _lds16_instance(seed=61, n=600_000):
    # about 13 K states: the 32-bit table (16 B a row) exceeds LDS, the
    # 16-bit one (8 B a row) fits; poly-A runs and A^k patterns give dense
    # segments, cut patterns give sparse ones
    rng = W.rng_for(seed)
    text = rng.integers(0, 4, size=n, dtype=np.uint8)
    for start in range(5000, n - 1000, 40_000):
        text[start:start + int(rng.integers(50, 500))] = 0
    pats = [np.zeros(k, np.uint8) for k in range(8, 17)]
    pats += W._cut(rng, text, rng.integers(8, 21, size=560))
    pats += [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in rng.integers(8, 21, size=560)]
    return W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA, "lds16")


def _lds16_fits(d):
    _, lds = ac.ac_device_info()
    limit = lds - 512
    return d.info.states * 16 + 1024 > limit and d.info.states * 8 + 512 <= limit


@pytest.mark.parametrize("fmt", [ac.AC_TEXT_2BIT, ac.AC_TEXT_U8])
@pytest.mark.parametrize("chunk,threads,chains", [(None, None, None), (64, 256, 1),
                                                  (256, 1024, 2), (1024, 512, 4)])
def test_lds16_whole_table(fmt, chunk, threads, chains):
    inst = _lds16_instance()
    d = ac.ac_build(inst.patterns, sigma=4)
    assert _lds16_fits(d), d.info.states
    _say("lds16 states", d.info.states, "fmt", fmt, "chunk", chunk, "threads", threads,
         "chains", chains)
    tune = None if chunk is None else {"chunk": chunk, "block_threads": threads, "chains": chains}
    _parity(inst, fmt, tune=tune, d=d)
    _parity(inst, fmt, tune=dict(tune or {}, placement=ac.AC_PLACE_LDS16), d=d)


def test_lds16_requested_on_small_and_large_tables():
    # a small table may be asked for 16-bit rows; a table too large for them
    # falls back to the hybrid placement
    small = W.dna_small(scale=1 / 4)
    _parity(small, ac.AC_TEXT_2BIT, tune={"placement": ac.AC_PLACE_LDS16})
    _parity(small, ac.AC_TEXT_U8, tune={"placement": ac.AC_PLACE_LDS16, "chunk": 128})
    big = W.dna_dense(scale=1 / 1024)
    _parity(big, ac.AC_TEXT_2BIT, tune={"placement": ac.AC_PLACE_LDS16})
