"""Build the CPU oracle (test infrastructure) into oracle/_build/liborc.so.

Plain g++; no HIP, no code shared with the product library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_core.cpp", "orc_encode.cpp", "orc_method.cpp", "orc_capi.cpp"]
OUT = os.path.join(HERE, "_build", "liborc.so")
SAN_OUT = os.path.join(HERE, "_build", "liborc_san.so")


def build(verbose=False, sanitize=False, out=None):
    """liborc.so; with sanitize, liborc_san.so under AddressSanitizer and
    UndefinedBehaviorSanitizer."""
    out = out or (SAN_OUT if sanitize else OUT)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    base = ["g++"] + opt + ["-std=gnu++17", "-fPIC", "-pthread", "-Wall", "-Wno-sign-compare"]
    objs, procs = [], []
    for src in SOURCES:   # one compiler per source, then the link
        obj = out + "." + src + ".o"
        objs.append(obj)
        cmd = base + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append(subprocess.Popen(cmd))
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("oracle build failed")
    subprocess.check_call(base + ["-shared", "-o", out] + objs + ["-lquadmath"])
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--san" in sys.argv))
