"""Serving loop: encrypted inference requests of several tenants and networks,
admitted by HBM footprint and continuously batched into the library's stage
launches.

Each tenant owns a context (its own keys, resident in HBM), a network and a
serving layout whose batch group holds `capacity` images.  A request is one
client's batch of images, encrypted by the client into up to `max_groups`
whole batch groups.  A tenant's executor takes every request queued when it becomes idle
(up to its batch-size limit and the memory budget), concatenates their batch
groups into one ciphertext batch and runs the network once for all of them:
every stage launch covers the requests together.  Batch groups never mix
inside a ciphertext, so each request's output ciphertexts are bit-identical to
a run of that request alone.  Tenants run on their own HIP streams, so their
batches overlap on the device.

This module holds scheduling and bookkeeping only; all arithmetic runs in the
library.  Arrival traces are seeded and synthetic.
"""
import sys
import threading
import time
from collections import deque

import numpy as np

from . import fenc as F
from . import workloads as W


class Request:
    __slots__ = ("rid", "tenant", "n_images", "ct", "t_arrival", "t_start", "t_done", "out", "footprint")

    def __init__(self, rid, tenant, n_images, ct, t_arrival=0.0):
        self.rid, self.tenant, self.n_images, self.ct = rid, tenant, n_images, ct
        self.t_arrival, self.t_start, self.t_done, self.out = t_arrival, None, None, None
        self.footprint = 0


class Tenant:
    """A network served for one key owner.

    net: "lenet" (LeNet-5-shaped, N = 2^15), "cifar" (CIFAR-shaped stack,
    N = 2^16) or "mobilenet" (the first MobileNet-V1-shaped block at
    224x224: conv 3->32 stride 2 and the quadratic activation, N = 2^16).
    capacity: images per batch group; max_groups: batch groups per request;
    max_batch: requests merged into one run."""

    NETS = {
        "lenet": dict(params="lenet", in_shape=(1, 28, 28), block_size=0),
        "cifar": dict(params="cifar", in_shape=(16, 32, 32), block_size=0),
        # S = 2: two images per batch group, the request granularity
        "mobilenet": dict(params="cifar", in_shape=W.MOBILENET_INPUTS[0], block_size=2),
    }

    def __init__(self, name, net, seed, capacity, max_batch=4, lib_path=None, params=None, shapes=None,
                 strides=None, in_shape=None, block_size=None, max_groups=1):
        spec = self.NETS[net]
        self.name, self.net, self.capacity, self.max_batch = name, net, capacity, max_batch
        self.max_groups = max_groups
        prm = list(params or W.PARAMS[spec["params"]])
        prm[-1] = seed
        self.fe = F.Fenc(*prm, lib_path=lib_path)
        c, h, w = in_shape or spec["in_shape"]
        self.in_shape = (c, h, w)
        if net == "mobilenet":
            self.w = W.mobilenet_weights(seed=seed + 100)[0]
        else:
            self.w = W.weights(shapes or (W.LENET_SHAPES if net == "lenet" else W.CIFAR_SHAPES), seed=seed + 100)
        self.strides = strides or W.CIFAR_STRIDES
        self.k0 = self.w[0].shape[2]
        self.block_size = spec["block_size"] if block_size is None else block_size
        self.layouts = {}
        self.lay = self.layout(1)
        self.stream = None
        if not self.fe.emulated:
            import torch
            self.stream = torch.cuda.Stream()
        self.queue = deque()
        self.lock = threading.Lock()

    def layout(self, groups):
        """Serving layout of `groups` whole batch groups of `capacity` images."""
        if groups not in self.layouts:
            c, h, w = self.in_shape
            lay = self.fe.plan_layout(groups * self.capacity, c, h, w, self.k0, self.w[0].shape[0], self.block_size)
            if lay.n_bg != groups or lay.bs != groups * self.capacity:
                raise ValueError("capacity must be the layout's images per batch group")
            self.layouts[groups] = lay
        return self.layouts[groups]

    def groups_of(self, n_images):
        g = -(-n_images // self.capacity)
        if n_images < 1 or g > self.max_groups:
            raise ValueError("request size out of range")
        return g

    # ---- client side
    def encrypt_request(self, x, seed):
        """Encode and encrypt images x[n][c][h][w] into whole batch groups."""
        g = self.groups_of(x.shape[0])
        full = np.zeros((g * self.capacity,) + self.in_shape)
        full[:x.shape[0]] = x
        lay = self.layout(g)
        return self.fe.encrypt(self.fe.encode_fragment(full, lay), lay, seed)

    def leading_groups(self, ct, g):
        """The first g batch groups of an encrypted request (ciphertexts are
        batch-group major, so this is a prefix of the buffer, shared)."""
        if g == ct.lay.n_bg:
            return ct
        lay = ct.lay.copy()
        lay.n_bg, lay.bs = g, g * self.capacity
        return F.Ciphertexts(self.fe, lay, ct.buf[:g * (ct.n_ct // ct.lay.n_bg) * 2 * (lay.level + 1) * self.fe.N])

    def decrypt_request(self, req):
        y = self.fe.decrypt(req.out)
        return y.reshape(y.shape[0], -1)[:req.n_images]

    # ---- server side
    def forward(self, ct):
        if self.net == "lenet":
            return W.lenet_forward(self.fe, ct, self.w)
        if self.net == "mobilenet":
            return W.mobilenet_block(self.fe, ct, W.MOBILENET_BLOCKS[0], self.w)
        return W.cifar_forward(self.fe, ct, self.w, self.strides)

    # HBM held while a request runs, in units of its input ciphertext bytes
    # (rotated copies, extended digits and outputs).  The MobileNet-shaped
    # block writes 32 output ciphertexts per 12 input ones and relinearises
    # them all at once: extended digits of ~2.5 ciphertexts each.
    WORKING_SET = {"lenet": 5, "cifar": 5, "mobilenet": 16}

    def footprint(self, ct):
        """HBM bytes a request holds while in flight."""
        return self.WORKING_SET[self.net] * ct.n_ct * 2 * (ct.lay.level + 1) * self.fe.N * 8

    def run_batch(self, reqs):
        """Concatenate the requests' batch groups, run the network once, split."""
        groups = [r.ct.lay.n_bg for r in reqs]
        G = sum(groups)
        if len(reqs) == 1:
            ct = reqs[0].ct
        else:
            lay = reqs[0].ct.lay.copy()
            lay.n_bg = G
            lay.bs = G * self.capacity
            bufs = [r.ct.buf for r in reqs]
            if self.fe.emulated:
                buf = np.concatenate(bufs)
            else:
                import torch
                buf = torch.cat(bufs)
            ct = F.Ciphertexts(self.fe, lay, buf)
        out = self.forward(ct)
        per = out.n_ct // G * 2 * (out.lay.level + 1) * self.fe.N   # elements per batch group
        g0 = 0
        for r, g in zip(reqs, groups):
            lay = out.lay.copy()
            lay.n_bg = g
            lay.bs = out.lay.bs // G * g
            r.out = F.Ciphertexts(self.fe, lay, out.buf[g0 * per:(g0 + g) * per])
            g0 += g
        return out


class Server:
    """Continuous batching over tenants with HBM-footprint admission."""

    def __init__(self, tenants, hbm_budget=200 << 30, keep_outputs=True):
        """keep_outputs=False drops each request's output ciphertexts once it
        is done (a benchmark without clients to hand them to)."""
        self.tenants = {t.name: t for t in tenants}
        self.budget = hbm_budget
        self.keep_outputs = keep_outputs
        self.in_flight = 0
        self.mem = threading.Lock()
        self.done = []
        self.done_lock = threading.Lock()
        self.batches = []

    def warmup(self, seed=1, group_counts=None, progress=None):
        """Build a tenant's plans for the batch-group counts it may run (all
        counts up to max_batch * max_groups unless given; not timed).
        progress(tenant name, group count) is called after each run."""
        for t in self.tenants.values():
            x = np.zeros((t.capacity,) + t.in_shape)
            ct = t.encrypt_request(x, seed)
            for G in (group_counts or {}).get(t.name, range(1, t.max_batch * t.max_groups + 1)):
                reqs = [Request(-1, t.name, t.capacity, ct) for _ in range(G)]
                self._run(t, reqs)
                if progress:
                    progress(t.name, G)

    @staticmethod
    def _run(t, reqs):
        """One batch on the tenant's stream, ordered after the work that wrote
        the requests' ciphertexts, synchronised at the end."""
        if t.stream is None:
            t.run_batch(reqs)
            return
        import torch
        t.stream.wait_stream(torch.cuda.default_stream())
        with torch.cuda.stream(t.stream):
            t.run_batch(reqs)
        t.stream.synchronize()

    def submit(self, req):
        t = self.tenants[req.tenant]
        req.footprint = t.footprint(req.ct)
        with t.lock:
            t.queue.append(req)

    def _take(self, t):
        """Requests for the next batch of tenant t: FIFO while the batch limit
        and the memory budget allow (at least one, if it fits at all)."""
        with t.lock, self.mem:
            reqs = []
            while t.queue and len(reqs) < t.max_batch:
                r = t.queue[0]
                if self.in_flight + r.footprint > self.budget and (reqs or self.in_flight):
                    break
                t.queue.popleft()
                self.in_flight += r.footprint
                reqs.append(r)
            return reqs

    def step(self, t, clock):
        """Run one batch of tenant t if it has queued requests; returns the batch size."""
        reqs = self._take(t)
        if not reqs:
            return 0
        t0 = clock()
        for r in reqs:
            r.t_start = t0
        self._run(t, reqs)
        t1 = clock()
        with self.mem:
            self.in_flight -= sum(r.footprint for r in reqs)
        with self.done_lock:
            for r in reqs:
                r.t_done = t1
                if not self.keep_outputs:
                    r.out = None
                self.done.append(r)
            self.batches.append((t.name, len(reqs), sum(r.n_images for r in reqs), t0, t1))
        return len(reqs)

    def serve(self, arrivals, clock=time.perf_counter):
        """arrivals: list of (t_offset_seconds, Request) sorted by time.  One
        executor thread per tenant; the calling thread releases requests at
        their arrival times.  Returns when every request is done."""
        total = len(arrivals)
        stop = threading.Event()
        t_begin = clock()

        errors = []

        def worker(ts):
            try:
                while not stop.is_set():
                    if not sum(self.step(t, clock) for t in ts):
                        time.sleep(0.0005)
            except Exception as e:   # reported by serve(); the other executors stop
                errors.append(e)
                stop.set()

        # one executor per tenant on the GPU (their streams overlap); the CPU
        # emulator runs every tenant from one executor
        ts = list(self.tenants.values())
        groups = [[t] for t in ts] if all(t.stream is not None for t in ts) else [ts]
        threads = [threading.Thread(target=worker, args=(g,), daemon=True) for g in groups]
        for th in threads:
            th.start()
        for off, req in arrivals:
            now = clock() - t_begin
            if off > now:
                time.sleep(off - now)
            req.t_arrival = clock()
            self.submit(req)
        while not stop.is_set():
            with self.done_lock:
                if len(self.done) >= total:
                    break
            time.sleep(0.001)
        stop.set()
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        return clock() - t_begin


def poisson_trace(rate, duration, mix, sizes, seed=7):
    """Seeded Poisson arrivals: (time, tenant name, n_images) with tenant drawn
    from `mix` ({name: probability}) and n_images from `sizes` ({name: (lo, hi)})."""
    r = np.random.default_rng(seed)
    names = list(mix)
    p = np.array([mix[n] for n in names], float)
    p /= p.sum()
    t, out = 0.0, []
    while True:
        t += r.exponential(1.0 / rate)
        if t > duration:
            return out
        name = names[r.choice(len(names), p=p)]
        lo, hi = sizes[name]
        out.append((t, name, int(r.integers(lo, hi + 1))))


def latency_summary(done):
    lat = np.array([r.t_done - r.t_arrival for r in done])
    imgs = sum(r.n_images for r in done)
    return {"requests": len(done), "images": imgs,
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(lat.mean()) * 1e3, 3)}


def main():
    """Serving benchmark: Poisson arrivals over LeNet-shaped, CIFAR-shaped and
    MobileNet-block tenants; prints one JSON line with latency percentiles and
    throughput."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=5.0)
    ap.add_argument("--lenet-tenants", type=int, default=2)
    ap.add_argument("--cifar-tenants", type=int, default=1)
    ap.add_argument("--mobilenet-tenants", type=int, default=1)
    ap.add_argument("--mobilenet-max-images", type=int, default=16,
                    help="largest MobileNet request (two 224x224 images per batch group)")
    ap.add_argument("--max-batch", type=int, default=4)
    ap.add_argument("--cifar-capacity", type=int, default=64)
    ap.add_argument("--pool", type=int, default=4, help="distinct pre-encrypted requests per tenant")
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    import torch
    tenants = [Tenant(f"lenet{i}", "lenet", 11 + i, 64, args.max_batch) for i in range(args.lenet_tenants)]
    tenants += [Tenant(f"cifar{i}", "cifar", 31 + i, args.cifar_capacity, 2) for i in range(args.cifar_tenants)]
    tenants += [Tenant(f"mobilenet{i}", "mobilenet", 41 + i, 2, 1, max_groups=-(-args.mobilenet_max_images // 2))
                for i in range(args.mobilenet_tenants)]
    srv = Server(tenants, keep_outputs=False)
    share = {"lenet": 0.6, "cifar": 0.3, "mobilenet": 0.1}
    count = {net: sum(t.net == net for t in tenants) for net in share}
    mix = {t.name: share[t.net] / count[t.net] for t in tenants}
    sizes = {t.name: (1, min(64, t.capacity * t.max_groups)) for t in tenants}
    trace = poisson_trace(args.rate, args.duration, mix, sizes, args.seed)
    # plans for every batch-group count a run can reach
    t0 = time.perf_counter()
    srv.warmup(progress=lambda n, G: print(
        f"warm-up {n}: {G} batch groups, {time.perf_counter() - t0:.1f}s, library GiB "
        f"{srv.tenants[n].fe.device_bytes() / 2**30:.1f}, torch GiB {torch.cuda.memory_reserved() / 2**30:.1f}",
        file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    held = {t.name: round(t.fe.device_bytes() / 2**30, 2) for t in tenants}
    print(f"warm-up {t_warm:.1f}s; device GiB held per tenant {held}", file=sys.stderr, flush=True)
    # clients encrypt before sending (outside the served latency); each tenant
    # has a pool of distinct encrypted requests of its largest size, and an
    # arrival of n images takes the leading batch groups it needs (read-only:
    # the network never writes its input)
    pool = {t.name: [t.encrypt_request(W.images((t.capacity * t.max_groups,) + t.in_shape, seed=1000 + j),
                                       5000 + j) for j in range(args.pool)] for t in tenants}
    arrivals = []
    for i, (off, name, n) in enumerate(trace):
        t = srv.tenants[name]
        ct = t.leading_groups(pool[name][i % args.pool], t.groups_of(n))
        arrivals.append((off, Request(i, name, n, ct)))
    # the tenants' workspaces were sized in the warm-up; admission budgets what
    # is left for the ciphertexts that runs allocate between layers
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    srv.budget = int(0.8 * torch.cuda.mem_get_info()[0])
    torch.cuda.synchronize()
    wall = srv.serve(arrivals)
    res = latency_summary(srv.done)
    res.update({"metric": "served encrypted images/s (continuous batching, per-tenant keys resident)",
                "images_per_s": round(res["images"] / wall, 2), "wall_s": round(wall, 3),
                "rate_req_per_s": args.rate, "batches": len(srv.batches),
                "mean_batch": round(float(np.mean([b[1] for b in srv.batches])), 2),
                "tenants": {t.name: t.net for t in tenants}, "warmup_s": round(t_warm, 1),
                "device_GiB_after_warmup": held, "admission_budget_GiB": round(srv.budget / 2**30, 1),
                "per_net": {}})
    for net in ("lenet", "cifar", "mobilenet"):
        d = [r for r in srv.done if srv.tenants[r.tenant].net == net]
        if d:
            res["per_net"][net] = latency_summary(d)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
