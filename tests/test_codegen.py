"""The gfx950 code of every kernel keeps its working arrays in registers: no
kernel uses private (scratch) memory and none spills registers.  The kernel
bodies pass small arrays between always-inlined helpers; if the compiler stops
inlining one of them (a second call site, a larger instantiation), the arrays
move to scratch memory and the kernel slows down several times while its
results stay correct, so only this check catches it.  Compiles the device code
to assembly on the CPU (about 40 s)."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2606_16359_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_kernels_use_no_scratch_and_do_not_spill():
    src = os.path.join(ROOT, "paper_2606_16359_amd", "csrc", "backend_hip.hip")
    out = tempfile.mkdtemp()
    try:
        asm = os.path.join(out, "backend.s")
        cmd = [HIPCC] + B.COMMON + ["-x", "hip", "--offload-arch=" + B.ARCH, "-munsafe-fp-atomics",
                                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                    "--cuda-device-only", "-S", "-o", asm, src]
        subprocess.run(cmd, check=True, capture_output=True)
        text = open(asm).read()
    finally:
        shutil.rmtree(out)
    # kernel metadata blocks: name, private segment size, spill counts
    kernels = re.findall(r"\.name:\s+(_Z\w+)\n(.*?)(?=\n  - \.|\Z)", text, flags=re.S)
    names = [n for n, _ in kernels]
    assert any("k_kip" in n for n in names) and any("k_gmac_pt_fast" in n for n in names)
    bad = []
    for name, meta in kernels:
        priv = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", meta).group(1))
        vsp = int(re.search(r"\.vgpr_spill_count:\s+(\d+)", meta).group(1))
        if priv or vsp:
            bad.append((name, priv, vsp))
    assert not bad, bad
