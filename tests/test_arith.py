"""The library's binary64 modular arithmetic and NTT register rounds against
128-bit integer arithmetic (CPU only).

tests/arith/arith_check.cpp includes the product headers fenc_arith.h and
fenc_kernels.h unchanged and checks, for NTT primes of 30, 40 and 50 bits:
mulmod exact for |a*b/q| < 2^51; mulmod_c exact for a*w/q > -2^51 with the
stated remainder bounds, and inexact somewhere below -2^51 (the precondition
is tight); red, full_norm, norm, centre, u2d and d2u; and the forward and
inverse radix-8/16 register rounds on adversarial inputs (all 0 / q-1, all
+-(q/2+1), twiddles 1, q-1, (q+-1)/2) and random ones, against exact integer
butterfly networks.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2606_16359_amd", "csrc")


def test_modular_arithmetic_and_ntt_rounds_are_exact(tmp_path):
    exe = str(tmp_path / "arith_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-w", "-I", CSRC, "-o", exe,
                           os.path.join(HERE, "arith", "arith_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "ok (0 failures)" in r.stdout
