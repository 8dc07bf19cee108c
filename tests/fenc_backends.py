"""Shared helpers for tests that run the library's kernels.

Backend "emu" runs the kernel bodies through the CPU emulator (CPU suite);
backend "hip" runs the gfx950 library on the GPU (marked gpu).
"""
import os

import numpy as np
import pytest

from paper_2606_16359_amd import build as B
from paper_2606_16359_amd import fenc as F

BACKENDS = ["emu", pytest.param("hip", marks=pytest.mark.gpu)]

_built_emu = False


def lib_path(backend):
    global _built_emu
    if backend == "emu":
        if os.environ.get("FENC_EMU_LIB"):   # a prebuilt emulator (the sanitizer build)
            return os.environ["FENC_EMU_LIB"]
        if not _built_emu and not os.environ.get("FENC_SKIP_EMU_BUILD"):
            B.build_emu()
            _built_emu = True
        return B.EMU_LIB
    if not os.path.exists(B.LIB):
        raise RuntimeError("HIP library missing: build before running GPU tests")
    return None


def make(backend, *params, server=False):
    return F.Fenc(*params, lib_path=lib_path(backend), server=server)


def rng(seed):
    return np.random.default_rng(seed)
