"""GPU parity of the other Table 1 rules (Wolf, Feng, Rais, Khurshid/NICK,
Phansalkar) and of the global statistics they use, against the oracle.

Wolf, Rais and NICK use only +, -, *, /, sqrt and max, which round the same
way on both sides: their masks must be bit-exact.  Feng (pow) and Phansalkar
(exp) call the device's and the C library's transcendental functions, which
may differ in the last bit: their masks may disagree only where the oracle's
|I - t| < 1e-4, and the count of such pixels is printed."""
import numpy as np
import pytest
import torch

import oracle
from docgen import gen_document

pytestmark = pytest.mark.gpu

REL = 1e-6
NEAR = 1e-4

CASES = {
    "wolf": (oracle.WOLF, (0.5, 128.0), True),
    "feng": (oracle.FENG, (0.9, 0.2, 0.3, 0.5, 128.0), False),
    "rais": (oracle.RAIS, (), True),
    "nick": (oracle.NICK, (-0.1,), True),
    "phansalkar": (oracle.PHANSALKAR, (2.0, 0.04, 0.25, 128.0), False),
}


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(bz, I, h, w, name, view=None, params=None):
    code, p, exact = CASES[name]
    p = p if params is None else params
    print("table1", name, I.shape, h, w, p, flush=True)
    mask, m, s = bz.table1_threshold(dev(I) if view is None else view, h, w, name, p)
    torch.cuda.synchronize()
    ref = oracle.table1(I, h, w, code, p)
    got = mask.cpu().numpy()
    bad = got != ref["mask"]
    near = np.abs(I.astype(np.float64) - ref["t"]) < NEAR
    print("  mask disagreements", int(bad.sum()), "oracle near-ties", int(near.sum()), flush=True)
    if exact:
        assert not bad.any()
    else:
        assert not (bad & ~near).any()
    m = m.cpu().numpy().astype(np.float64)
    s = s.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(m - ref["m"]) <= REL * np.abs(ref["m"]))
    assert np.all(np.abs(s - ref["s"]) <= REL * np.abs(ref["s"]))


@pytest.mark.parametrize("H,W", [(384, 512), (1, 1), (203, 301), (70, 4100), (1000, 512), (3072, 4096)])
def test_global_stats_match_oracle(bz, H, W):
    I = gen_document(H, W, 80 + H, noise=10.0, stain=True)
    g = bz.read_global_stats(bz.global_stats(dev(I)))
    r = oracle.global_stats(I)
    assert (g["n"], g["sum"], g["sumsq"]) == (r["N"], r["T1"], r["T2"])
    assert (g["min"], g["max"]) == (r["L"], r["max"])
    assert g["mean"] == r["M"] and g["std"] == r["S"]


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_page(bz, name):
    check(bz, gen_document(384, 512, 1, noise=10.0, stain=True), 31, 31, name)


@pytest.mark.parametrize("name", sorted(CASES))
def test_ragged_strided_page(bz, name):
    # odd sizes, a window wider than tall, rows at an odd stride and offset
    I = gen_document(203, 301, 5, noise=10.0, stain=True)
    big = torch.zeros((203, 311), dtype=torch.uint8, device="cuda")
    big[:, 3:304] = dev(I)
    check(bz, I, 9, 40, name, view=big[:, 3:304])


@pytest.mark.parametrize("name", sorted(CASES))
def test_headline_page_w75(bz, name):
    check(bz, gen_document(3072, 4096, 2, noise=10.0, stain=True), 75, 75, name)


def test_feng_integer_exponent_and_constant_image(bz):
    # gamma = 2: powers of s/R; a constant image: s = 0 and S = 0 everywhere
    check(bz, gen_document(120, 160, 7, noise=10.0, stain=True), 15, 15, "feng",
          params=(0.85, 0.15, 0.05, 2.0, 128.0))
    C = np.full((40, 50), 133, np.uint8)
    for name in sorted(CASES):
        check(bz, C, 7, 9, name)


@pytest.mark.parametrize("gamma", [0.0, -0.5, 0.25, 2.5])
def test_feng_powers_on_flat_and_textured_windows(bz, monkeypatch, gamma):
    # x^g on the float32 path comes from the native log2 and exp2; flat
    # windows (x = 0) take pow's value at 0, which for g < 0 is infinite.
    # A noiseless page (flat background) with a noisy block: masks equal the
    # oracle's (up to its near-ties) and the binary64 sequence's everywhere
    I = gen_document(300, 400, 13, noise=0.0, stain=False)
    I[100:220, 120:320] = gen_document(120, 200, 14, noise=12.0, stain=True)
    p = (0.85, 0.15, 0.05, gamma, 96.0)
    check(bz, I, 11, 13, "feng", params=p)
    d = dev(I)
    rec = bz.global_stats(d)
    fast = bz.table1_threshold(d, 11, 13, "feng", p, stats=rec)
    monkeypatch.setenv("BZ_FORCE_REFERENCE", "1")
    ref = bz.table1_threshold(d, 11, 13, "feng", p, stats=rec)
    torch.cuda.synchronize()
    assert torch.equal(fast[0], ref[0])


def test_global_record_is_reused(bz):
    # a record computed once serves several calls; outputs equal the
    # call that computes its own record
    I = dev(gen_document(200, 260, 9, noise=10.0, stain=True))
    rec = bz.global_stats(I)
    a = bz.table1_threshold(I, 21, 21, "wolf", (0.4, 100.0), stats=rec)
    b = bz.table1_threshold(I, 21, 21, "wolf", (0.4, 100.0))
    assert all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("name", sorted(CASES))
def test_guarded_float32_path_equals_binary64_everywhere(bz, monkeypatch, name):
    # BZ_FORCE_REFERENCE=1 decides every pixel with the binary64 sequence;
    # the default path decides in float32 outside the guard: same masks
    I = dev(gen_document(600, 800, 12, noise=10.0, stain=True))
    code, p, _ = CASES[name]
    rec = bz.global_stats(I)
    fast = bz.table1_threshold(I, 45, 45, name, p, stats=rec)
    monkeypatch.setenv("BZ_FORCE_REFERENCE", "1")
    ref = bz.table1_threshold(I, 45, 45, name, p, stats=rec)
    torch.cuda.synchronize()
    assert torch.equal(fast[0], ref[0])


def test_global_stats_graph_replays(bz):
    # during the call the record's count tallies the finished workgroups and
    # the last one forms mean and std; every replay of a captured call leaves
    # the complete record again, with other work in between
    H, W = 700, 900
    host = gen_document(H, W, 21, noise=10.0, stain=True)
    I = dev(host)
    r = oracle.global_stats(host)
    rec = torch.empty(bz.GLOBAL_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

    def call():
        st = torch.cuda.current_stream().cuda_stream
        assert bz.lib.bz_global_stats(I.data_ptr(), H, W, W, rec.data_ptr(), st) == 0

    call()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for _ in range(3):
        rec.fill_(0xAB)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = bz.read_global_stats(rec)
        assert (got["n"], got["sum"], got["sumsq"], got["min"], got["max"]) == (r["N"], r["T1"], r["T2"], r["L"],
                                                                                r["max"])
        assert got["mean"] == r["M"] and got["std"] == r["S"]


@pytest.mark.parametrize("blocks", ["1", "3", "128", "1000"])
def test_global_stats_any_grid(bz, monkeypatch, blocks):
    # the last of the accumulating workgroups forms mean and std, whatever
    # their number (BZ_GSTATS_BLOCKS, capped at the row count)
    monkeypatch.setenv("BZ_GSTATS_BLOCKS", blocks)
    for H, W in ((257, 300), (5, 4100)):
        I = gen_document(H, W, 90 + H, noise=10.0, stain=True)
        g = bz.read_global_stats(bz.global_stats(dev(I)))
        r = oracle.global_stats(I)
        assert (g["n"], g["sum"], g["sumsq"], g["min"], g["max"]) == (r["N"], r["T1"], r["T2"], r["L"], r["max"])
        assert g["mean"] == r["M"] and g["std"] == r["S"]
