"""The C-ABI library on the host: it loads, exports every declared symbol, and
rejects invalid arguments before touching the device (no compute calls)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "binarize.h")


@pytest.fixture(scope="module")
def bz():
    import paper_1905_13038_amd as pkg
    return pkg


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bz_[a-z_0-9]+)\s*\(", text)))


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "binarize.h"\nint main(void){return bz_version()<0;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-c", "-I", os.path.dirname(HEADER),
                    str(src), "-o", str(tmp_path / "t.o")], check=True)


def test_every_declared_symbol_is_exported(bz):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(bz.lib, n), n


def test_static_queries(bz):
    assert bz.lib.bz_version() >= 100
    assert bz.lib.bz_max_window() == 257
    assert bz.lib.bz_status_string(0) == b"BZ_OK"
    assert bz.lib.bz_status_string(3) == b"BZ_ERR_ALIAS"


# Fake device addresses: validation inspects only the numeric values.
IMG = 0x100000
OUT = 0x900000
OUT2 = 0xA00000
OUT3 = 0xB00000


def test_validation_sauvola(bz):
    L = bz.lib
    ok = dict(I=IMG, H=64, W=64, ld=64, h=15, w=15, k=0.5, R=128.0, mask=OUT, ldm=64,
              mean=OUT2, std=OUT3, ldms=64)

    def call(**kw):
        a = dict(ok, **kw)
        return L.bz_sauvola(a["I"], a["H"], a["W"], a["ld"], a["h"], a["w"], a["k"], a["R"],
                            a["mask"], a["ldm"], a["mean"], a["std"], a["ldms"], None)

    assert call(I=None) == 1
    assert call(H=0) == 1
    assert call(W=-3) == 1
    assert call(ld=63) == 1
    assert call(h=0) == 1
    assert call(h=258) == 2
    assert call(w=300) == 2
    assert call(k=-0.1) == 1            # Sauvola needs k >= 0
    assert call(k=float("nan")) == 1
    assert call(R=0.0) == 1
    assert call(R=float("inf")) == 1
    assert call(mask=None) == 1
    assert call(ldm=10) == 1
    assert call(mean=OUT2 + 2) == 1     # float outputs must be 4-byte aligned
    assert call(std=None) == 1          # mean and std come together
    assert call(mask=IMG + 100) == 3    # output overlaps input
    assert call(mean=IMG + 64 * 63) == 3
    assert call(mean=OUT, mask=OUT + 4) == 3   # outputs overlap each other


def test_validation_other_entry_points(bz):
    L = bz.lib
    assert L.bz_niblack(IMG, 64, 64, 64, 15, 15, float("inf"), OUT, 64, None, None, 0, None) == 1
    assert L.bz_window_sums(IMG, 64, 64, 64, 15, 15, OUT, OUT + 64 * 64, 64, None) == 3
    assert L.bz_window_sums(IMG, 64, 64, 64, 15, 15, OUT, None, 64, None) == 1
    assert L.bz_window_mean_std(IMG, 64, 64, 64, 15, 15, OUT, OUT2, 60, None) == 1
    assert L.bz_window_quantile(IMG, 64, 64, 64, 15, 15, 1.5, OUT, 64, None, 64, None) == 1
    assert L.bz_window_quantile(IMG, 64, 64, 64, 15, 15, float("nan"), OUT, 64, None, 64, None) == 1
    assert L.bz_window_quantile(IMG, 64, 64, 64, 15, 15, 0.5, IMG + 1, 64, None, 64, None) == 3
    assert L.bz_window_quantile(IMG, 64, 64, 64, 300, 15, 0.5, OUT, 64, None, 64, None) == 2
    # the binary64 sums of the soft calls: 8-byte aligned outputs, no overlap
    big = 0x40000000
    assert L.bz_soft_window_sums(IMG, 2, 64, 64, 64, 15, 15, big + 4, big + 2 * 64 * 64 * 8, 64, None) == 1
    assert L.bz_soft_window_sums(IMG, 2, 64, 64, 64, 15, 15, big, big + 64 * 8, 64, None) == 3
    assert L.bz_soft_window_sums(IMG, 2, 64, 64, 64, 15, 15, big, None, 64, None) == 1
    assert L.bz_soft_window_sums(IMG, 2, 64, 64, 64, 15, 258, big, big + 2 * 64 * 64 * 8, 64, None) == 2
    assert L.bz_soft_window_sums(IMG, 2, 64, 64, 64, 15, 15, big, big + 2 * 64 * 64 * 8, 63, None) == 1
    assert L.bz_soft_window_sums(IMG, 1, 40000, 8, 8, 15, 15, big, big + 2 ** 33, 8000, None) == 2


def test_fault_injection_maps_to_hip_error():
    # BZ_FAULT_INJECT=launch makes a valid call report BZ_ERR_HIP without
    # launching; run in a child so the environment of this process is untouched.
    code = (
        "import paper_1905_13038_amd as b;"
        "print(b.lib.bz_sauvola(0x100000, 8, 8, 8, 3, 3, 0.5, 128.0, 0x900000, 8, None, None, 0, None))"
    )
    env = dict(os.environ, BZ_FAULT_INJECT="launch")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, check=True)
    assert out.stdout.strip() == "5"


def test_python_binding_refuses_host_tensors(bz):
    import torch
    with pytest.raises(ValueError):
        bz.sauvola(torch.zeros((8, 8), dtype=torch.uint8), 3, 3)


def test_batch_rejects_cross_item_aliasing():
    # the items of a batch run concurrently: an output overlapping another
    # item's output or input is rejected before any device work; items may
    # share an input.  Run in a child with BZ_FAULT_INJECT=launch, so a batch
    # that passes validation reports BZ_ERR_HIP instead of touching a device.
    code = r'''
import ctypes
import paper_1905_13038_amd as b
L = b.lib
def item(I, mask, mean, std):
    return b.bz_item(I, mask, mean, std, 32, 40, 7, 9, 40, 40, 40 if mean else 0, 0.3, 128.0,
                     b.METHOD_SAUVOLA)
WS = 0x4000000
nb = L.bz_batched_workspace_size(2)
def plan(a, c):
    arr = (b.bz_item * 2)(a, c)
    return L.bz_batched_plan(arr, 2, None, WS, nb, None)
A = item(0x100000, 0x200000, 0x300000, 0x400000)
print(plan(A, item(0x110000, 0x300000 + 64, None, None)))        # mask inside A's mean
print(plan(A, item(0x110000, 0x210000, 0x400000 + 4 * 40, 0x500000)))  # mean inside A's std
print(plan(A, item(0x110000, 0x100000 + 8, None, None)))         # mask inside A's input
print(plan(A, item(0x100000, 0x210000, 0x310000, 0x410000)))     # shares A's input: valid
print(plan(A, item(0x110000, 0x210000, None, None)))             # disjoint: valid
'''
    env = dict(os.environ, BZ_FAULT_INJECT="launch")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, check=True)
    assert out.stdout.split() == ["3", "3", "3", "5", "5"]


def test_validation_table1_and_global_stats(bz):
    L = bz.lib
    P5 = ctypes.c_double * 5
    good = P5(0.5, 128.0, 0, 0, 0)
    STATS = 0xC00000  # 8-byte aligned fake device record

    def thr(method=3, params=good, stats=STATS, mask=OUT, mean=OUT2, std=OUT3, h=15):
        return L.bz_threshold(IMG, 64, 64, 64, h, 15, method, params, stats, mask, 64, mean, std, 64, None)

    assert thr(method=1) == 1                      # Sauvola/Niblack have their own calls
    assert thr(method=8) == 1
    assert thr(params=None) == 1                   # Wolf takes {k, R}
    assert thr(params=P5(0.5, 0.0, 0, 0, 0)) == 1  # R > 0
    assert thr(params=P5(float("nan"), 128.0, 0, 0, 0)) == 1
    assert thr(stats=None) == 1                    # Wolf reads L
    assert thr(stats=STATS + 4) == 1               # record alignment
    assert thr(method=5, params=None, stats=OUT + 8) == 3   # Rais: record inside the mask
    assert thr(method=4, params=P5(1, 0.2, 0.3, 2.0, -1.0)) == 1  # Feng's R
    assert thr(method=7, params=P5(2.0, 0.04, 0.25, 0.0, 0)) == 1  # Phansalkar's R
    assert thr(h=258) == 2
    assert thr(mask=IMG + 10) == 3
    assert L.bz_global_stats(None, 8, 8, 8, STATS, None) == 1
    assert L.bz_global_stats(IMG, 8, 8, 8, STATS + 2, None) == 1
    assert L.bz_global_stats(IMG, 8, 8, 8, IMG + 16, None) == 3


def test_table1_valid_calls_reach_the_launch():
    # NICK and Phansalkar need no record; Rais takes no parameters.  Valid
    # calls pass validation (BZ_FAULT_INJECT=launch reports BZ_ERR_HIP there).
    code = r'''
import ctypes
import paper_1905_13038_amd as b
L = b.lib
P5 = ctypes.c_double * 5
print(L.bz_threshold(0x100000, 64, 64, 64, 15, 15, 6, P5(-0.1, 0, 0, 0, 0), None, 0x900000, 64, None, None, 0, None))
print(L.bz_threshold(0x100000, 64, 64, 64, 15, 15, 7, P5(2.0, 0.04, 0.25, 128.0, 0), None, 0x900000, 64, None, None, 0, None))
print(L.bz_threshold(0x100000, 64, 64, 64, 15, 15, 5, None, 0xC00000, 0x900000, 64, None, None, 0, None))
print(L.bz_global_stats(0x100000, 64, 64, 64, 0xC00000, None))
'''
    env = dict(os.environ, BZ_FAULT_INJECT="launch")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, check=True)
    assert out.stdout.split() == ["5", "5", "5", "5"]


def test_validation_minmax_and_bernsen(bz):
    L = bz.lib
    MN, MX, WS = 0xD00000, 0xE00000, 0xF00000
    nb = L.bz_extremes_workspace_size(64, 64)
    assert nb == 2 * 64 * 64
    mm = lambda mn=MN, mx=MX, ws=WS, n=nb, w=9: L.bz_window_minmax(IMG, 64, 64, 64, 9, w, mn, mx, 64, ws, n, None)
    assert mm(mx=MN + 64) == 3            # mn, mx overlap
    assert mm(mn=IMG + 5) == 3            # output inside the input
    assert mm(w=300) == 2
    assert mm(mn=None) == 1
    assert mm(ws=None) == 1
    assert mm(ws=WS + 2) == 1             # workspace alignment
    assert mm(n=nb - 1) == 4              # workspace too small
    assert mm(ws=MN + 100) == 3           # workspace over an output
    bs = lambda c=15, mask=OUT: L.bz_bernsen(IMG, 64, 64, 64, 9, 9, c, mask, 64, MN, MX, 64, WS, nb, None)
    assert bs(mask=None) == 1
    assert bs(c=-1) == 1
    assert bs(c=257) == 1
    assert bs(mask=MN + 3) == 3


def test_validation_streamed(bz):
    # host image and mask, device workspace: statuses before any HIP call
    L = bz.lib
    H_, W_, BAND = 64, 48, 16
    nb = L.bz_stream_workspace_size(H_, W_, 9, 9, BAND, 0)
    # rows: slots of BAND + h - 1 rows at a 64-byte pitch, 256-byte rounded
    assert nb == 4 * (((BAND + 8) * 64 + 255) // 256 * 256)
    # auto takes rows also for a wide image; columns on request: H rows at a
    # pitch of BAND + w - 1 rounded up to 64
    assert L.bz_stream_workspace_size(20, 300, 5, 9, 16, 0) == 4 * (20 * 320)
    assert L.bz_stream_workspace_size(20, 300, 5, 9, 16, 2) == 4 * ((20 * 64 + 255) // 256 * 256)
    assert L.bz_stream_workspace_size(0, 8, 3, 3, 4, 0) == 0
    assert L.bz_stream_workspace_size(8, 8, 3, 3, 0, 0) == 0
    assert L.bz_stream_workspace_size(8, 8, 3, 3, 4, 3) == 0
    # rows of 2^28 bytes: h + 1 = 10 of them span more than 2^31 bytes, so
    # auto sweeps columns
    wide = 1 << 28
    assert L.bz_stream_workspace_size(8, wide, 9, 9, 16, 0) == L.bz_stream_workspace_size(8, wide, 9, 9, 16, 2)
    WS, HOUT = 0xF00000, 0x900000

    def call(I=IMG, ld=W_, mask=HOUT, ldm=W_, h=9, w=9, method=1, k=0.5, R=128.0, band=BAND, axis=0, ws=WS,
             n=nb):
        return L.bz_binarize_streamed(I, H_, W_, ld, h, w, method, k, R, mask, ldm, band, axis, ws, n, None,
                                      None, None)

    assert call(I=None) == 1
    assert call(mask=None) == 1
    assert call(ld=W_ - 1) == 1
    assert call(band=0) == 1
    assert call(axis=-1) == 1
    assert call(axis=3) == 1
    assert call(method=3) == 1           # only Sauvola and Niblack stream
    assert call(k=-0.1) == 1             # Sauvola needs k >= 0
    assert call(R=0.0) == 1
    assert call(h=258) == 2
    assert call(mask=IMG + 7) == 3       # partial overlap
    assert call(mask=IMG, ldm=W_ + 1) == 3   # the same buffer at another stride
    assert call(ws=None) == 1
    assert call(ws=WS + 64) == 1         # workspace alignment
    assert call(n=nb - 1) == 4
    # a band slot above 2^46 bytes while the host image is within them: rows
    # of 65537 bytes take a 65600-byte pitch on the device (in place, one band)
    Hb, Wb = 1073700000, 65537
    assert Hb * Wb <= 1 << 46 < Hb * 65600
    assert L.bz_binarize_streamed(IMG, Hb, Wb, Wb, 9, 9, 1, 0.5, 128.0, IMG, Wb, Hb, 1, WS, nb,
                                  None, None, None) == 2
    # in place and Niblack with any k pass validation (launch fault injected)
    code = (
        "import paper_1905_13038_amd as b; L = b.lib;"
        "n = L.bz_stream_workspace_size(64, 48, 9, 9, 16, 2);"
        "print(L.bz_binarize_streamed(0x100000, 64, 48, 48, 9, 9, 1, 0.5, 128.0, 0x100000, 48, 16, 2,"
        " 0xF00000, n, None, None, None));"
        "print(L.bz_binarize_streamed(0x100000, 64, 48, 48, 9, 9, 2, -0.3, 0.0, 0x900000, 48, 16, 1,"
        " 0xF00000, n, None, None, None))"
    )
    env = dict(os.environ, BZ_FAULT_INJECT="launch")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, check=True)
    assert out.stdout.split() == ["5", "5"]


def test_streamed_binding_refuses_device_arguments(bz):
    import torch
    with pytest.raises(ValueError):
        bz.binarize_streamed(torch.zeros((8, 8), dtype=torch.int16), 3, 3)
    with pytest.raises(ValueError):
        bz.binarize_streamed(torch.zeros((8, 8), dtype=torch.uint8), 3, 3, method="wolf")
    with pytest.raises(ValueError):
        bz.binarize_streamed(torch.zeros((8, 8), dtype=torch.uint8)[:, ::2], 3, 3)
    with pytest.raises(ValueError):
        bz.binarize_streamed(torch.zeros((8, 8), dtype=torch.uint8), 3, 3, axis="diagonal")


def test_validation_haar(bz):
    L = bz.lib
    F, WS = 0xD00000, 0xF00000
    nb = L.bz_haar_workspace_size(64, 48, 5, 1)
    assert nb == (64 - 5 + 1) * 64 * 2                  # 16-bit column sums only
    # rows too wide for the row kernel (kv * W > 12288) add 32-bit prefixes
    assert L.bz_haar_workspace_size(64, 13000, 5, 1) == ((60 * 13056 * 2 + 255) // 256 * 256) + 60 * 13056 * 4
    assert L.bz_haar_workspace_size(64, 4096, 5, 4) == 60 * 4096 * 2   # three rows of 4096 fit
    assert L.bz_haar_workspace_size(4, 48, 5, 1) == 0
    assert L.bz_haar_workspace_size(64, 48, 5, 9) == 0

    def call(I=IMG, H=64, W=48, ld=48, a=5, b=6, kind=1, out=F, ldF=48, ws=WS, n=nb):
        return L.bz_haar_features(I, H, W, ld, a, b, kind, out, ldF, ws, n, None)

    assert call(I=None) == 1
    assert call(out=None) == 1
    assert call(kind=0) == 1
    assert call(kind=6) == 1
    assert call(ld=47) == 1
    assert call(a=0) == 1
    assert call(a=258) == 2
    assert call(b=25) == 1            # two cells of 25 columns exceed W = 48
    assert call(kind=4, a=22) == 1    # three cells of 22 rows exceed H = 64
    assert call(ldF=36) == 1          # ld_F below the W - 2 b + 1 = 37 outputs per row
    assert call(out=F + 2) == 1       # int32 output alignment
    assert call(out=IMG + 64) == 3    # output over the input
    assert call(ws=None) == 1
    assert call(ws=WS + 4) == 1       # workspace alignment
    assert call(n=nb - 1) == 4
    assert call(ws=F + 256) == 3      # workspace over the output
    code = (
        "import paper_1905_13038_amd as b; L = b.lib;"
        "print(L.bz_haar_features(0x100000, 64, 48, 48, 5, 6, 5, 0xD00000, 48, 0xF00000,"
        " L.bz_haar_workspace_size(64, 48, 5, 5), None))"
    )
    env = dict(os.environ, BZ_FAULT_INJECT="launch")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                         text=True, check=True)
    assert out.stdout.strip() == "5"
