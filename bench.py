"""Benchmark: encrypted CNN inference on one MI355X.

Headline (`value`): the largest configuration that fits one GPU, the three
MobileNet-V1-shaped early blocks at ImageNet shape (224x224x3 input; conv 3->32
stride 2; depthwise 3x3 32 + pointwise 32->64; depthwise 3x3 stride 2 64 +
pointwise 64->128; a quadratic after each conv), each block from a fresh
encryption, with the largest batch that fits HBM (64 images); RNS-CKKS
N=2^16, 24 x 50-bit primes + 6 special, dnum 4, scale 2^40.  Inputs are
encrypted and resident in HBM before timing; a step is the whole server-side
circuit of the batch, captured once as a hipGraph and replayed.

Beside it: the same step in the per-op form (every homomorphic operation of
every ciphertext launched separately) and the batch/per-op ratio; every
kernel's time and algorithmic bytes from HIP events on its launch stream, the
roofline of the dominant one; the smaller configurations (the single 28x28
conv layer at N=2^13, the LeNet-5-shaped network of 64 images at N=2^15, the
CIFAR-shaped stack of 256 images at N=2^16), each graph-replayed beside its
per-op form; and the CPU oracle, per-operation times on the host cores scaled
by the step's operation counts (extrapolated).
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# measured on this device by `bench.py --peaks` (profiles/gfx950_peaks.md): a
# 4 GiB device-to-device copy and the library's binary64 modular multiply
COPY_CEILING_GBS = 5202.0
MODMUL_PEAK = 6.223e12
COPY_BYTES = 256 << 20
PEAKS_BYTES = 4 << 30          # buffer size of the --peaks HBM ceilings
MOBILENET_BATCH = 64
WORKSPACE_LIMIT = 24 << 30
METRIC = "encrypted images/sec (batched hipGraph, bit-exact)"
DTYPE = "u64 RNS residues (50-bit primes), binary64 FMA modular arithmetic"
# HBM bytes per launch of each workload's dominant kernel, from FETCH_SIZE +
# WRITE_SIZE counters scaled by a copy of known size (profiles/*_hbm_traffic.md);
# an entry is kept only while its kernel is unchanged since the counters were taken
TRAFFIC = {
    ("mobilenet", "ntt_fwd_cols"): 1.7878e9,
    ("cifar", "gmac_pt_fast"): 9.4836e9,
    ("lenet", "kip"): 0.8760e9,
    ("ffn", "gmac_diag"): 6.9616e9,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fingerprint(outs):
    """Checksum of a step's output ciphertexts: the wrapped int64 sum of every
    word and every 7919th word, computed on the device."""
    import torch
    fp = []
    for ct in outs:
        t = ct.buf
        fp.append((int(t.sum().item()), int(t[::7919].sum().item()), int(t.numel())))
    return fp


def measure(fe, step, imgs, steps, warmup, per_op_steps, tag, graph=True):
    """Warm-up, counters, eager and per-op timings, the per-kernel table, then
    the hipGraph capture and its timed replays."""
    import torch
    from paper_2606_16359_amd import fenc as F
    out = None
    for i in range(max(1, warmup)):
        t0 = time.time()
        out = None           # the previous step's outputs go before the next step allocates its own
        out = step()
        torch.cuda.synchronize()
        log(f"[{tag}] warmup {i} {time.time() - t0:.2f}s")
    ref_fp = fingerprint(out)
    out = None
    fe.stats_reset()
    step()
    torch.cuda.synchronize()
    st = fe.stats()
    n_eager = max(1, min(3, steps // 4))
    t0 = time.perf_counter()
    for _ in range(n_eager):
        step()
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / n_eager
    fe.set_mode(F.FENC_MODE_PER_OP)
    out = step()
    torch.cuda.synchronize()
    per_op_identical = fingerprint(out) == ref_fp
    del out
    t0 = time.perf_counter()
    for _ in range(per_op_steps):
        step()
    torch.cuda.synchronize()
    t_perop = (time.perf_counter() - t0) / per_op_steps
    fe.set_mode(F.FENC_MODE_BATCHED)
    kernels = kernel_table(fe, step)
    gc.collect()
    torch.cuda.empty_cache()
    res = {"images": imgs, "step_counters": st, "keyswitches_per_step": st["keyswitch"],
           "launches_per_step": st["launches"],
           "batched_eager": {"images_per_s": round(imgs / t_eager, 3), "ms_per_step": round(t_eager * 1e3, 3)},
           "per_op": {"images_per_s": round(imgs / t_perop, 3), "ms_per_step": round(t_perop * 1e3, 3),
                      "keyswitches_per_s": round(st["keyswitch"] / t_perop, 1)},
           "kernels": kernels}
    t_best, graph_identical = t_eager, None
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out_graph = step()
        for _ in range(2):     # replays interleaved with eager device work
            g.replay()
            torch.cuda.synchronize()
        graph_identical = fingerprint(out_graph) == ref_fp
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        t_best = (time.perf_counter() - t0) / steps
        res["graph"] = {"images_per_s": round(imgs / t_best, 3), "ms_per_step": round(t_best * 1e3, 3)}
        del g, out_graph
        gc.collect()
        torch.cuda.empty_cache()
    res["images_per_s"] = round(imgs / t_best, 3)
    res["ms_per_step"] = round(t_best * 1e3, 3)
    res["keyswitches_per_s"] = round(st["keyswitch"] / t_best, 1)
    res["batched_vs_per_op"] = round(t_perop / t_best, 3)
    res["bit_identical"] = {"per_op_vs_batched": per_op_identical, "graph_vs_eager": graph_identical}
    log(f"[{tag}] {json.dumps({k: v for k, v in res.items() if k != 'kernels'})}")
    return res


def kernel_table(fe, step):
    """Per-kernel time and algorithmic bytes of one batched step: HIP events
    around every launch, on the launch stream."""
    import torch
    fe.profile_kernel("*")
    step()
    torch.cuda.synchronize()
    summ = fe.profile_summary()
    fe.profile_kernel(None)
    kernels = {}
    for name, (kms, klaunch, kbytes, kops) in sorted(summ.items(), key=lambda kv: -kv[1][0]):
        avg_s = kms / 1e3 / klaunch
        gbs = kbytes / klaunch / avg_s / 1e9
        kernels[name] = {"launches": klaunch, "ms_per_step": round(kms, 4), "avg_launch_us": round(avg_s * 1e6, 2),
                         "bytes_per_launch": round(kbytes / klaunch), "achieved_GBs": round(gbs, 1),
                         "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                         "frac_copy_ceiling": round(gbs / COPY_CEILING_GBS, 4)}
        if kops > 0:
            rate = kops / klaunch / avg_s
            kernels[name].update({"modmul_per_launch": round(kops / klaunch), "modmul_per_s": round(rate, -6),
                                  "frac_modmul_peak": round(rate / MODMUL_PEAK, 4)})
    return kernels


def roofline(kernels, workload):
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    r = {"kernel": dom, "bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": TRAFFIC.get((workload, dom)),
         "avg_launch_us": kd["avg_launch_us"], "launches": kd["launches"],
         "bytes_per_launch": kd["bytes_per_launch"],
         "measured_copy_ceiling_GBs": COPY_CEILING_GBS, "frac_of_measured_ceiling": kd["frac_copy_ceiling"]}
    if "modmul_per_s" in kd:
        r["alu"] = {"achieved": kd["modmul_per_s"], "peak": MODMUL_PEAK, "unit": "modmul/s",
                    "frac": kd["frac_modmul_peak"], "peak_source": "measured binary64 mulmod rate"}
    return r


# ---------------------------------------------------------------- workloads
def run_conv1(args):
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["conv1_small"])
    W.bench_config(fe)
    x, w = W.conv1_inputs()
    lay = fe.plan_layout(1, 1, 28, 28, 5, 6)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    r = measure(fe, lambda: [fe.conv2d(ct, w)], 1, max(10, args.steps), 2, 5, "conv1")
    r["workload"] = "single conv 1->6 5x5 on one 28x28 image, N=2^13, 4 x 40-bit + 1 special, scale 2^30"
    return r


def run_lenet(args):
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["lenet"])
    W.bench_config(fe)
    x, w = W.lenet_inputs(64)
    lay = W.lenet_layout(fe, 64)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    r = measure(fe, lambda: [W.lenet_forward(fe, ct, w)], 64, max(10, args.steps), 2, 2, "lenet")
    r["workload"] = ("LeNet-5-shaped network, 64 images 28x28, N=2^15, 20 x 50-bit + 7 special, dnum 3, "
                     "scale 2^40, fragment S=%d" % lay.S)
    r["roofline"] = roofline(r["kernels"], "lenet")
    return r


def run_cifar(args):
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["cifar"])
    W.bench_config(fe)
    x, w = W.cifar_inputs(256)
    lay = fe.plan_layout(256, 16, 32, 32, 3, 16)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    r = measure(fe, lambda: [W.cifar_forward(fe, ct, w)], 256, max(3, args.steps // 4), 2, 1, "cifar")
    r["workload"] = ("CIFAR-shaped stack, 256 images 16x32x32 (3 x conv 16->16, conv 16->32 s2, conv 32->32, "
                     "a cubic after each), N=2^16, 24 x 50-bit + 6 special, dnum 4, scale 2^40")
    r["roofline"] = roofline(r["kernels"], "cifar")
    return r


def run_ffn(args):
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["ffn"])
    W.bench_config(fe)
    x, w = W.ffn_inputs()
    lay = fe.plan_tokens(W.FFN_TOKENS, W.FFN_E, W.FFN_S)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    r = measure(fe, lambda: [W.ffn_forward(fe, ct, w)], W.FFN_TOKENS, max(10, args.steps), 2, 1, "ffn")
    r["tokens_per_s"] = r.pop("images_per_s")
    r["unit"] = "tokens/s (the images fields count tokens)"
    r["workload"] = ("BERT-base-shaped feed-forward block on token fragments: 128 tokens, FC 768->3072 with bias, "
                     "x^2, FC 3072->768 with bias; S=4 (%d input ciphertexts), N=2^16, 4 x 50-bit + 2 special, "
                     "dnum 2, scale 2^40" % lay.n_ct())
    r["roofline"] = roofline(r["kernels"], "ffn")
    return r


def ffn_sweep(args):
    """The FFN block at every admissible block size S: key switches, plaintext
    products and time per step (graph replay), each S on a fresh context."""
    import torch
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    x, w = W.ffn_inputs()
    rows = []
    print("| S | tokens per group | d | input cts | key switches | plaintext products | context GB | "
          "ms per step (graph) | tokens/s |")
    print("|---|---|---|---|---|---|---|---|---|")
    for S in (1, 2, 4, 8):
        fe = F.Fenc(*W.PARAMS["ffn"])
        W.bench_config(fe)
        lay = fe.plan_tokens(W.FFN_TOKENS, W.FFN_E, S)
        ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
        t0 = time.time()
        W.ffn_forward(fe, ct, w)
        torch.cuda.synchronize()
        log(f"[ffn S={S}] plans and keys {time.time() - t0:.1f}s")
        W.ffn_forward(fe, ct, w)
        fe.stats_reset()
        W.ffn_forward(fe, ct, w)
        torch.cuda.synchronize()
        st = fe.stats()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out = W.ffn_forward(fe, ct, w)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        err = float(np.max(np.abs(fe.decrypt(out).reshape(W.FFN_TOKENS, W.FFN_E) - W.ffn_reference(x, w))))
        r = {"S": S, "bs_g": lay.bs_g, "d": lay.d, "input_cts": lay.n_ct(), "keyswitch": st["keyswitch"],
             "pmult": st["pmult"], "device_bytes": fe.device_bytes(), "ms_per_step": round(t * 1e3, 3),
             "tokens_per_s": round(W.FFN_TOKENS / t, 1), "max_abs_err": err}
        rows.append(r)
        print(f"| {S} | {lay.bs_g} | {lay.d} | {lay.n_ct()} | {st['keyswitch']} | {st['pmult']} | "
              f"{fe.device_bytes() / 1e9:.1f} | {r['ms_per_step']} | {r['tokens_per_s']} |", flush=True)
        del g, out, ct, fe
        gc.collect()
        torch.cuda.empty_cache()
    print(json.dumps({"ffn_sweep": rows}), flush=True)


def mobilenet_context(batch):
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["cifar"])
    fe.set_workspace_limit(WORKSPACE_LIMIT)
    W.bench_config(fe)
    t0 = time.time()
    cts = W.mobilenet_encrypt(fe, batch)
    log(f"[mobilenet] encode+encrypt of {batch} images: {time.time() - t0:.1f}s")
    return fe, cts, W.mobilenet_weights()


def cpu_baseline(counters, imgs, level):
    """The oracle (plain C++ with 128-bit integers) on the host cores: its
    per-operation times at the headline's parameters (ModUp with a hoisted
    rotation, further hoisted rotations, plaintext and scalar products,
    rescale, square with relinearisation), single-threaded and with one thread
    per core over independent ciphertexts, scaled by the operation counts of
    one step (extrapolated; the ops are timed at the top level)."""
    from oracle import pyoracle as P
    from paper_2606_16359_amd import workloads as W
    t0 = time.time()
    o = P.Oracle(*W.PARAMS["cifar"])
    cores = max(1, min(16, os.cpu_count() or 1))
    t1 = P.time_ops(o, level, 1, 1)
    tn = P.time_ops(o, level, cores, 1)
    rot = counters["rot_inner"] + counters["rot_outer"] + counters["rot_other"]

    def step_s(t):
        return (counters["modup"] * t["modup_rot"] + max(0, rot - counters["modup"]) * t["rot"]
                + counters["pmult"] * t["pmult"] + counters["smult"] * t["smult"]
                + counters["rescale"] * t["rescale"] + counters["relin"] * t["square_relin"])
    s1, sn = step_s(t1), step_s(tn)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    log(f"oracle per-op seconds (1 thread) {t1}; ({cores} threads) {tn}; {time.time() - t0:.1f}s in all")
    return {"value": round(imgs / sn, 6), "unit": "images/s", "cores": cores, "kind": "oracle",
            "single_thread_images_per_s": round(imgs / s1, 6), "cpu": model,
            "sample": (f"oracle per-operation times at N=2^16, 24 limbs (one op per thread, {cores} threads and 1), "
                       f"times the step's counts (modup {counters['modup']}, rotations {rot}, "
                       f"pmult {counters['pmult']}, smult {counters['smult']}, rescale {counters['rescale']}, "
                       f"relin {counters['relin']}); extrapolated")}


def workload_step(workload, batch):
    """(context, step) of a benchmark workload in its benchmark configuration."""
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    if workload == "mobilenet":
        fe, cts, ws = mobilenet_context(batch)
        return fe, lambda: W.mobilenet_forward(fe, cts, ws)
    if workload == "cifar":
        fe = F.Fenc(*W.PARAMS["cifar"])
        W.bench_config(fe)
        x, w = W.cifar_inputs(256)
        lay = fe.plan_layout(256, 16, 32, 32, 3, 16)
        ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
        return fe, lambda: W.cifar_forward(fe, ct, w)
    if workload == "ffn":
        fe = F.Fenc(*W.PARAMS["ffn"])
        W.bench_config(fe)
        x, w = W.ffn_inputs()
        lay = fe.plan_tokens(W.FFN_TOKENS, W.FFN_E, W.FFN_S)
        ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
        return fe, lambda: [W.ffn_forward(fe, ct, w)]
    fe = F.Fenc(*W.PARAMS["lenet"])
    W.bench_config(fe)
    x, w = W.lenet_inputs(64)
    lay = W.lenet_layout(fe, 64)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    return fe, lambda: W.lenet_forward(fe, ct, w)


def counters_run(args):
    """Short run for hardware-counter passes: one warm-up step, a 256 MiB
    device copy (calibrates the byte counters), one batched step; no timing."""
    import torch
    fe, step = workload_step(args.workload, args.batch)
    out = step()
    torch.cuda.synchronize()
    out = None
    src = torch.empty(COPY_BYTES // 8, dtype=torch.int64, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    step()
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": True, "workload": args.workload, "copy_bytes": COPY_BYTES}), flush=True)


def pmc_summary(fetch_csv, write_csv):
    """HBM bytes per dispatch of every kernel of the measured step of a
    --counters run, from a FETCH_SIZE and a WRITE_SIZE pass (rocprofv3
    counter_collection CSVs, KiB per dispatch).  Each counter is calibrated by
    the run's COPY_BYTES device copy (the largest runtime copy dispatch), and
    only the dispatches after that copy (the step that follows it) count.
    Radix variants of an NTT pass are merged under the pass's name."""
    import csv
    import re

    def load(path):
        rows = list(csv.DictReader(open(path)))
        keys = rows[0].keys()
        kcol = next(k for k in keys if k.lower().replace("-", "_") in ("kernel_name", "kernelname"))
        vcol = next(k for k in keys if k.lower() in ("counter_value", "value"))
        icol = next(k for k in keys if "dispatch" in k.lower() and "id" in k.lower())
        out = {}
        for r in rows:   # one row per dispatch (and counter instance): sum the instances
            d = int(r[icol])
            name = r[kcol].split("(")[0].split("<")[0].strip()
            out.setdefault(d, [name, 0.0])[1] += float(r[vcol])
        copy = max((d for d, (n, v) in out.items() if "copyBuffer" in n), key=lambda d: out[d][1])
        factor = COPY_BYTES / 1024.0 / out[copy][1]
        return {d: (n, v) for d, (n, v) in out.items() if d > copy}, factor, out[copy][1]

    def norm(name):
        name = re.sub(r"^k_", "", name)
        return name.replace("16", "") if name.startswith("ntt_") else name

    fetch, ff, fc = load(fetch_csv)
    write, fw, wc = load(write_csv)
    agg = {}
    for d, (n, v) in fetch.items():
        a = agg.setdefault(norm(n), [0, 0.0, 0.0])
        a[0] += 1
        a[1] += v
        a[2] += write.get(d, (n, 0.0))[1]
    print(f"calibration copy of {COPY_BYTES >> 10} KiB: FETCH_SIZE {fc:.0f} KiB (factor {ff:.3f}), "
          f"WRITE_SIZE {wc:.0f} KiB (factor {fw:.3f})")
    print("| Kernel | Dispatches | FETCH KiB (mean) | WRITE KiB (mean) | HBM GB per dispatch (calibrated) |")
    print("|---|---|---|---|---|")
    res = {}
    for name, (n, fs, ws) in sorted(agg.items(), key=lambda kv: -(kv[1][1] * ff + kv[1][2] * fw)):
        gb = (fs * ff + ws * fw) / n * 1024 / 1e9
        res[name] = round(gb, 4)
        print(f"| {name} | {n} | {fs / n:.4g} | {ws / n:.4g} | {gb:.4f} |")
    print(json.dumps({"hbm_GB_per_dispatch": res}))


def peaks_run(args):
    """Measured gfx950 peaks: instruction issue rates, modular-multiply rates
    of the binary64 and the 64-bit integer designs, and HBM ceilings."""
    import ctypes
    from paper_2606_16359_amd import build as B
    if not os.path.exists(B.PEAKS_LIB):
        raise RuntimeError(f"{B.PEAKS_LIB} is not built")
    L = ctypes.CDLL(B.PEAKS_LIB)
    L.fenc_peaks_name.restype = ctypes.c_char_p
    L.fenc_peaks_run.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    rows = []
    for i in range(L.fenc_peaks_count()):
        name, unit = L.fenc_peaks_name(i).decode().split("|")
        arg = float(PEAKS_BYTES) if unit == "byte" else 0.02
        sec, work, exact = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        if L.fenc_peaks_run(i, arg, ctypes.byref(sec), ctypes.byref(work), ctypes.byref(exact)) != 0:
            raise RuntimeError(f"peaks test {name} failed")
        rate = work.value / sec.value
        rows.append({"test": name, "unit": unit + "/s", "rate": rate, "seconds": sec.value,
                     "work": work.value, "exact": {1: True, 0: False}.get(exact.value)})
        log(f"{name:55s} {rate / 1e12:9.3f} T{unit}/s  ({sec.value * 1e3:.3f} ms, exact={rows[-1]['exact']})")
    print(json.dumps({"peaks": rows, "buffer_bytes": PEAKS_BYTES, "device": torch_device_name()}), flush=True)


def torch_device_name():
    import torch
    return torch.cuda.get_device_properties(0).name


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3,
                    help="untimed steps (the first builds plans and keys; the workspace settles by the third)")
    ap.add_argument("--per-op-steps", type=int, default=1)
    ap.add_argument("--batch", type=int, default=MOBILENET_BATCH, help="MobileNet images per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--workload", choices=["mobilenet", "cifar", "lenet", "ffn"], default="mobilenet",
                    help="workload of the --counters and --trace runs")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="reduce the two counter passes of a --counters run to HBM bytes per dispatch and exit")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter passes (one warm-up step, a 256 MiB copy, one step)")
    ap.add_argument("--ffn-sweep", action="store_true",
                    help="the Transformer FFN block at block sizes 1, 2, 4, 8 (key switches, time)")
    ap.add_argument("--peaks", action="store_true",
                    help="measure instruction, modular-multiply and HBM peaks of the device and exit")
    ap.add_argument("--trace", action="store_true",
                    help="run for a kernel trace: three warm-up steps, then --steps batched eager steps of the "
                         "workload (--workload) and nothing else")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: this build runs every configuration on a single MI355X; the "
                                   "path would shard by independent batch groups, which is not implemented"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.counters:
        counters_run(args)
        return
    if args.peaks:
        peaks_run(args)
        return
    if args.ffn_sweep:
        ffn_sweep(args)
        return
    if args.trace:
        fe, step = workload_step(args.workload, args.batch)
        out = None
        for i in range(3 + args.steps):
            out = None
            out = step()
            torch.cuda.synchronize()
        print(json.dumps({"trace_run": True, "workload": args.workload, "batched_steps": args.steps,
                          "warmup_steps": 3}), flush=True)
        return

    extras = {}
    if not args.no_extras:
        for name, fn in [("single_conv_n2p13", run_conv1), ("lenet64_n2p15", run_lenet),
                         ("cifar256_n2p16", run_cifar), ("bert_ffn128_n2p16", run_ffn)]:
            t0 = time.time()
            extras[name] = fn(args)
            gc.collect()
            torch.cuda.empty_cache()
            log(f"[{name}] done in {time.time() - t0:.1f}s")

    from paper_2606_16359_amd import workloads as W
    fe, cts, ws = mobilenet_context(args.batch)
    r = measure(fe, lambda: W.mobilenet_forward(fe, cts, ws), args.batch, args.steps, args.warmup,
                args.per_op_steps, "mobilenet")
    res = {
        "metric": METRIC,
        "value": r["images_per_s"],
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic (uniform [0,1) images of the ImageNet/CIFAR/MNIST shapes, N(0,0.1) weights, seeded)",
        "config": {"workload": ("MobileNet-V1-shaped early blocks at ImageNet shape 224x224x3 (conv 3->32 s2; "
                                "dw 3x3 32 + pw 32->64; dw 3x3 s2 64 + pw 64->128; a quadratic after each conv), "
                                f"{args.batch} images (the largest batch that fits HBM), each block from a fresh "
                                "encryption, RNS-CKKS N=2^16, 24x50-bit limbs + 6 special, dnum 4, scale 2^40"),
                   "batch_images": args.batch, "log_n": 16, "limbs": 24, "dnum": 4,
                   "workspace_limit_bytes": WORKSPACE_LIMIT},
        "keyswitches_per_s": r["keyswitches_per_s"],
        "keyswitches_per_step": r["keyswitches_per_step"],
        "per_op": r["per_op"],
        "batched_eager": r["batched_eager"],
        "graph_vs_per_op": r["batched_vs_per_op"],
        "bit_identical": r["bit_identical"],
        "launches_per_step": r["launches_per_step"],
        "step_counters": r["step_counters"],
        "ntt_config": fe.ntt_config(),
        "device_bytes_context": fe.device_bytes(),
        "roofline": roofline(r["kernels"], "mobilenet"),
        "kernels": r["kernels"],
        "other_configs": {k: {kk: vv for kk, vv in v.items() if kk != "kernels"} for k, v in extras.items()},
    }
    level = cts[0].lay.level
    del cts, fe
    gc.collect()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(r["step_counters"], args.batch, level)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
