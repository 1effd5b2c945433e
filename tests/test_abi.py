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
