"""Build the CPU oracle (test infrastructure) into oracle/_build/liborc.so.

Plain g++; no HIP, no code shared with the product library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_core.cpp", "orc_encode.cpp", "orc_method.cpp", "orc_capi.cpp"]
OUT = os.path.join(HERE, "_build", "liborc.so")


def build(verbose=False):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["g++", "-O2", "-std=gnu++17", "-fPIC", "-shared", "-pthread", "-Wall", "-Wno-sign-compare",
           "-o", OUT] + [os.path.join(HERE, s) for s in SOURCES] + ["-lquadmath"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
