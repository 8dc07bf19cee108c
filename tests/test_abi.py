"""The C ABI boundary on the CPU: the HIP library loads without a GPU, exports
every function that include/fenc.h declares, the Python binding covers each
of them, and the host-only entry points (prime search, planner, slot map,
sampler, encoder) agree with the oracle.  No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2606_16359_amd import build as B
from paper_2606_16359_amd import fenc as F
from paper_2606_16359_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fenc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s+(fenc_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def hiplib():
    if not os.path.exists(B.LIB):
        B.build_hip()
    return F.load()


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("fenc_keygen", "fenc_encode_fragment", "fenc_encrypt", "fenc_conv2d", "fenc_fc",
              "fenc_poly_act", "fenc_compress", "fenc_decrypt", "fenc_avgpool2", "fenc_plan_layout"):
        assert n in names
    assert len(names) >= 35


def test_library_exports_every_declared_symbol(hiplib):
    missing = [n for n in declared_functions() if not hasattr(hiplib, n)]
    assert not missing, missing
    # the raw ELF symbol table agrees (no lazily resolved stubs)
    raw = C.CDLL(B.LIB)
    for n in declared_functions():
        assert C.cast(getattr(raw, n), C.c_void_p).value


def test_binding_covers_every_declared_function():
    src = open(os.path.join(ROOT, "paper_2606_16359_amd", "fenc.py")).read()
    missing = [n for n in declared_functions() if f'"{n}"' not in src]
    assert not missing, missing


def test_host_entry_points_match_the_oracle(hiplib):
    from oracle import pyoracle as P
    for name in ("conv1_small", "lenet"):
        prm = W.PARAMS[name]
        fe = F.Fenc(*prm)
        o = P.Oracle(*prm)
        assert fe.primes() == list(o.primes())
    # planner and slot map at the benchmark shapes (LeNet input, 64 images)
    prm = W.PARAMS["lenet"]
    fe, o = F.Fenc(*prm), P.Oracle(*prm)
    lay = fe.plan_layout(64, 1, 28, 28, 5, 6)
    ol = o.plan_layout(64, 1, 28, 28, 5, 6)
    assert (lay.S, lay.m, lay.bs_g, lay.chan_per_ct, lay.n_ct()) == (ol["S"], ol["m"], ol["bsg"], ol["cpc"],
                                                                    ol["nbg"] * ol["ncg"] * ol["S"] ** 2)
    rng = np.random.default_rng(7)
    for _ in range(50):
        b, y, x = int(rng.integers(64)), int(rng.integers(28)), int(rng.integers(28))
        ct, slot = fe.layout_slot(lay, b, 0, y, x)
        assert (ct, slot) in [tuple(p) for p in o.element_slots(ol, b, 0, y, x)]


def test_sampler_and_integer_encoder_match_the_oracle(hiplib):
    from oracle import pyoracle as P
    o = P.Oracle(*W.PARAMS["conv1_small"])
    for seed, tag, i in [(3, 1 << 56, 0), (3, (2 << 56) | (5 << 24) | (1 << 16) | 2, 77), (9, 5 << 56, 12345)]:
        assert F.sample_word(seed, tag, i) == P.lib().orc_rng(seed, tag, i)
        assert F.sample_gauss(seed, tag, i) == P.lib().orc_gauss(seed, tag, i)
    z = np.random.default_rng(1).uniform(-1, 1, 1 << 12)
    m_lib = F.encode_int(13, z, 2.0 ** 30)
    m_orc = np.array(o.encode_int(z, None, 2.0 ** 30), np.int64)
    # the library's double-double FFT and the oracle's binary128 transform
    # round to the same integers
    assert np.array_equal(m_lib, m_orc)


def test_errors_before_any_launch(hiplib):
    fe = F.Fenc(*W.PARAMS["conv1_small"])
    with pytest.raises(F.FencError):
        fe.plan_layout(1, 1, 28, 28, 5, 6, s_override=3)   # S must divide M
    bad = F.Params(13, 1, 40, 1, 40, 1, 30, 3)               # one prime: no level to rescale
    h = C.c_void_p()
    assert hiplib.fenc_ctx_create(C.byref(bad), C.byref(h)) != 0
    assert hiplib.fenc_last_error()
