"""Build the HIP library for gfx950 (and, for the CPU test suite, the emulator).

    python -m paper_2606_16359_amd.build            # libfenc.so + libfenc_peaks.so (HIP, gfx950)
    python -m paper_2606_16359_amd.build --emu      # tests/emu/_build/libfenc_emu.so
    python -m paper_2606_16359_amd.build --emu-san  # the same under ASan + UBSan
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "_build", "libfenc.so")
PEAKS_LIB = os.path.join(PKG, "_build", "libfenc_peaks.so")
EMU_LIB = os.path.join(ROOT, "tests", "emu", "_build", "libfenc_emu.so")
HOST_SOURCES = ["runtime.cpp", "ops.cpp", "host_math.cpp"]
ARCH = os.environ.get("FENC_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_hip(verbose=False, jobs=8):
    """Compile every source with hipcc for gfx950 and link libfenc.so."""
    out_dir = os.path.dirname(LIB)
    os.makedirs(out_dir, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, procs = [], []
    for src in ["backend_hip.hip"] + HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        objs.append(obj)
        if src.endswith(".hip"):
            flags = ["-x", "hip", "--offload-arch=" + ARCH, "-munsafe-fp-atomics",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        else:
            flags = ["-x", "c++"]
        cmd = [hipcc] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("hipcc failed")
    _run([hipcc, "-shared", "--offload-arch=" + ARCH, "-o", LIB] + objs + ["-lpthread"], verbose)
    # peak-rate microbenchmarks: a separate library, not part of libfenc
    _run([hipcc] + COMMON + ["-x", "hip", "--offload-arch=" + ARCH, "-Wno-unused-result",
                             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-shared",
                             os.path.join(CSRC, "peaks.hip"), "-o", PEAKS_LIB], verbose)
    return LIB


EMU_SAN_LIB = os.path.join(ROOT, "tests", "emu", "_build", "libfenc_emu_san.so")
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build_emu(verbose=False, sanitize=False, out=None):
    """CPU emulator of the kernels (test infrastructure); with sanitize, an
    AddressSanitizer + UndefinedBehaviorSanitizer build (host code only)."""
    out = out or (EMU_SAN_LIB if sanitize else EMU_LIB)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    srcs = [os.path.join(ROOT, "tests", "emu", "backend_cpu.cpp")] + [os.path.join(CSRC, s) for s in HOST_SOURCES]
    flags = ["g++"] + ([f for f in COMMON if f != "-O3"] + SANITIZE if sanitize else COMMON) + \
        ["-Wno-unknown-pragmas", "-fopenmp", "-I", CSRC]
    objs, procs = [], []
    for src in srcs:   # one compiler per source, then the link
        obj = out + "." + os.path.basename(src) + ".o"
        objs.append(obj)
        cmd = flags + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("emulator build failed")
    _run(flags + ["-shared", "-o", out] + objs + ["-lpthread"], verbose)
    return out


if __name__ == "__main__":
    v = "-v" in sys.argv
    if "--emu-san" in sys.argv:
        print(build_emu(v, sanitize=True))
    else:
        print(build_emu(v) if "--emu" in sys.argv else build_hip(v))
