"""The kernel emulator and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

Both are rebuilt with -fsanitize=address,undefined (host code; the emulator
runs the same kernel bodies as the GPU build, one CPU thread per block, and
allocates every device buffer at its exact size, so a read of a padded table
slot, a spare MAC slot or a tail word past the end of its buffer is reported).
A subset of the parity and oracle tests that reaches every kernel variant then
runs in a child interpreter with the sanitizer runtime preloaded; any report
ends it with a non-zero status.
"""
import os
import subprocess
import sys
import threading

import pytest

from oracle import build as OB
from paper_2606_16359_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# conv variants (masks, outer rotations, both hoisting schedules, every MAC
# kernel form), fused and standalone compression, batch-group tiles, the LeNet
# chain (pool, square, compress, FC with bias), the cubic stack, the server
# context, NTT round trips; oracle: conv decryption, border rotations, the
# pool/square/compress/FC chain and the bias
SUBSET = " or ".join([
    "test_conv_variants_bit_exact", "test_conv_large_weight_codes_bit_exact", "test_mini_lenet_layers_bit_exact",
    "test_fused_compression_bottleneck_bit_exact", "test_batch_group_tiles_give_identical_residues",
    "test_cifar_shaped_stack_small_bit_exact", "test_server_context", "test_ntt_roundtrip_and_product",
    "test_conv2d_decrypts_to_float64_conv", "test_conv2d_border_rotations_match_brute_force",
    "test_avgpool_square_compress_fc_decrypt_to_float64", "test_bias_is_added_at_the_output_scale",
])


def _runtime(name):
    return subprocess.check_output(["g++", "-print-file-name=" + name], text=True).strip()


def test_parity_subset_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan, cxx = _runtime("libasan.so"), _runtime("libstdc++.so")
    if not all(os.path.isabs(p) and os.path.exists(p) for p in (asan, cxx)):
        pytest.skip("no AddressSanitizer runtime for g++")
    built, errs = {}, []

    def job(key, fn):
        try:
            built[key] = fn()
        except Exception as e:   # reported below
            errs.append(f"{key}: {e}")

    # built outside the tree: nothing else loads them
    ts = [threading.Thread(target=job, args=("emu", lambda: B.build_emu(sanitize=True,
                                                                         out=str(tmp_path / "libfenc_emu_san.so")))),
          threading.Thread(target=job, args=("orc", lambda: OB.build(sanitize=True,
                                                                     out=str(tmp_path / "liborc_san.so"))))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs, errs
    env = dict(os.environ)
    # the runtime first; then libstdc++, which the interpreter does not link, so
    # that the runtime finds the C++ exception entry points it intercepts
    env["LD_PRELOAD"] = asan + ":" + cxx + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    logs = str(tmp_path / "san")
    env["ASAN_OPTIONS"] = f"detect_leaks=0:halt_on_error=1:exitcode=97:log_path={logs}"
    env["UBSAN_OPTIONS"] = f"halt_on_error=1:print_stacktrace=1:exitcode=98:log_path={logs}"
    env["FENC_EMU_LIB"] = built["emu"]
    env["ORC_LIB"] = built["orc"]
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_parity.py", "tests/test_oracle_method.py",
                        "-m", "not gpu", "-x", "-q", "-p", "no:cacheprovider", "-k", SUBSET],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    print(r.stdout[-2000:])
    reports = "".join(open(tmp_path / f).read()[:6000] for f in sorted(os.listdir(tmp_path))
                      if f.startswith("san."))
    assert r.returncode == 0 and not reports, (r.stdout[-3000:] + "\n" + r.stderr[-4000:] + "\n" + reports)
    assert " passed" in r.stdout and " failed" not in r.stdout
