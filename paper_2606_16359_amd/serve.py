"""Serving loop: encrypted inference requests of several tenants and networks,
admitted by HBM footprint and continuously batched into the library's stage
launches.

Each tenant owns a context (its own keys, resident in HBM), a network and a
serving layout whose batch group holds `capacity` images.  A request is one
client's batch of images, encrypted by the client into up to `max_groups`
whole batch groups.  Requests queued together (up to a batch-size limit and
the memory budget) are concatenated into one ciphertext batch and the network
runs once for all of them: every stage launch covers the requests together.
Batch groups never mix inside a ciphertext, so each request's output
ciphertexts are bit-identical to a run of that request alone.

On the GPU a tenant has several lanes: contexts of their own with the
tenant's parameters and key seed (so the same keys and the same residues),
each with its own HIP stream and workspace, and the network's stages
(layers) captured as hipGraphs for every batch-group count.  The tenant's
executor replays each running batch stage by stage and, at every stage
boundary, admits the requests that arrived meanwhile into a free lane: a new
batch starts while earlier ones are at later layers, and the batches of all
lanes and all tenants overlap on the device.

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
                 strides=None, in_shape=None, block_size=None, max_groups=1, ws_limit=None):
        """ws_limit: the workspace limit of each of the tenant's contexts (bytes;
        None: the library's default); operations tile by batch groups within it."""
        spec = self.NETS[net]
        self.name, self.net, self.capacity, self.max_batch = name, net, capacity, max_batch
        self.max_groups = max_groups
        prm = list(params or W.PARAMS[spec["params"]])
        prm[-1] = seed
        self.prm, self.lib_path, self.ws_limit = prm, lib_path, ws_limit
        self.fe = self._context()
        self.lanes = []
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
    def stages(self, fe):
        """The network as a list of stages (one layer each) on context fe; the
        same calls as workloads' lenet_forward / cifar_forward / mobilenet_block."""
        w = self.w
        if self.net == "lenet":
            return [lambda c: fe.conv2d(c, w[0]), fe.poly_act, fe.avgpool2,
                    lambda c: fe.conv2d(c, w[1]), fe.poly_act, fe.avgpool2, fe.compress,
                    lambda c: fe.fc(c, w[2]), lambda c: fe.fc(c, w[3]), lambda c: fe.fc(c, w[4])]
        if self.net == "mobilenet":
            ly = W.MOBILENET_BLOCKS[0][0]
            return [lambda c: fe.conv2d(c, w[0], stride=ly["stride"], pad=ly["pad"], groups=ly["groups"]),
                    lambda c: fe.poly_act(c, W.QUADRATIC, inplace=True)]
        out = []
        for wi, st in zip(w, self.strides):
            out += [lambda c, wi=wi, st=st: fe.conv2d(c, wi, stride=st, pad=wi.shape[2] // 2),
                    lambda c: fe.poly_act(c, W.CUBIC, inplace=True)]
        return out

    def forward(self, ct):
        y = ct
        for st in self.stages(self.fe):
            y = st(y)
        return y

    def _context(self):
        fe = F.Fenc(*self.prm, lib_path=self.lib_path)
        if self.ws_limit is not None:
            fe.set_workspace_limit(self.ws_limit)
        return fe

    def make_lanes(self, n):
        """n lanes (GPU): the first on the tenant's own context, the others on
        new contexts with the same parameters and key seed."""
        self.lanes = [Lane(self, self.fe if i == 0 else self._context()) for i in range(n)]
        return self.lanes

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


class Lane:
    """One pipeline slot of a tenant on the GPU: a context, a HIP stream (default
    priority) and, per batch-group count G, the network's stages captured as
    hipGraphs on that stream, reading a fixed input buffer of G groups."""

    def __init__(self, tenant, fe):
        import torch
        self.t, self.fe = tenant, fe
        self.stream = torch.cuda.Stream()
        self.graphs = {}         # G -> (input Ciphertexts, [CUDAGraph per stage], output Ciphertexts)
        self.reqs = None         # the running batch
        self.G = 0
        self.next = 0            # next stage to launch
        self.events = deque()    # one per launched, unfinished stage
        self.t_admit = 0.0

    def capture(self, G):
        """An eager run of G groups (plans, keys, workspace), then one graph per
        stage.  The stages' buffers come from one private pool and stay
        referenced, so replays find them where the capture left them."""
        import torch
        lay = self.t.layout(1).copy()   # G groups side by side, as a merged batch is laid out
        lay.n_bg, lay.bs = G, G * self.t.capacity
        x = self.fe.alloc_cts(lay)
        x.buf.zero_()
        stages = self.t.stages(self.fe)
        self.stream.wait_stream(torch.cuda.current_stream())
        # eager passes until the workspace stops changing: an operation may
        # replace the unpinned chunks an earlier one used, and a capture
        # cannot grow the workspace
        size = -1
        for _ in range(4):
            with torch.cuda.stream(self.stream):
                y = x
                for st in stages:
                    y = st(y)
            self.stream.synchronize()
            del y
            if self.fe.device_bytes() == size:
                break
            size = self.fe.device_bytes()
        graphs, cur, pool = [], x, None
        for st in stages:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, pool=pool, stream=self.stream):
                cur = st(cur)
            pool = g.pool()
            graphs.append(g)
        self.graphs[G] = (x, graphs, cur)

    def launch(self):
        """Replay the next stage on the lane's stream; an event marks its end."""
        import torch
        g = self.graphs[self.G][1][self.next]
        with torch.cuda.stream(self.stream):
            g.replay()
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.events.append(ev)
        self.next += 1


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
        self.admissions = []   # lanes: (tenant, time, stages the tenant's other running batches are at)

    def warmup(self, seed=1, group_counts=None, progress=None, lanes=0):
        """Build a tenant's plans for the batch-group counts it may run (all
        counts up to max_batch * max_groups unless given; not timed).  With
        lanes > 0 (GPU), each tenant gets that many lanes and every lane
        captures its stage graphs for those counts.  progress(tenant name,
        group count) is called after each count."""
        for t in self.tenants.values():
            counts = list((group_counts or {}).get(t.name, range(1, t.max_batch * t.max_groups + 1)))
            if lanes and t.stream is not None:
                t.make_lanes(lanes)
                # graphs for powers of two (and the largest count): a batch runs
                # in the smallest captured count that holds it
                counts = sorted({1 << i for i in range(max(counts).bit_length()) if (1 << i) <= max(counts)}
                                | {max(counts)})
                for G in counts:
                    for ln in t.lanes:
                        ln.capture(G)
                    if progress:
                        progress(t.name, G)
                continue
            x = np.zeros((t.capacity,) + t.in_shape)
            ct = t.encrypt_request(x, seed)
            for G in counts:
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

    # ---- lanes (GPU): stage-by-stage replay, admission at stage boundaries
    def _admit(self, t, ln, reqs, clock):
        """Copy the batch's input groups into the lane's buffer (after the work
        that wrote them) and launch its first stages."""
        import torch
        need = sum(r.ct.lay.n_bg for r in reqs)
        G = min(g for g in ln.graphs if g >= need)   # groups past `need` hold stale data; their outputs are dropped
        x = ln.graphs[G][0]
        ln.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(ln.stream):
            off = 0
            for r in reqs:
                n = r.ct.buf.numel()
                x.buf[off:off + n].copy_(r.ct.buf)
                off += n
        ln.reqs, ln.G, ln.next, ln.t_admit = reqs, G, 0, clock()
        for r in reqs:
            r.t_start = ln.t_admit
        # the stage each other running batch of this tenant is executing
        others = [o.next - len(o.events) for o in t.lanes if o is not ln and o.reqs is not None]
        self.admissions.append((t.name, ln.t_admit, others))
        self._advance(t, ln, clock)

    def _advance(self, t, ln, clock, ahead=2):
        """Retire finished stages, keep up to `ahead` stages queued; when the
        last stage is done, hand out the outputs and free the lane."""
        while ln.events and ln.events[0].query():
            ln.events.popleft()
        n_st = len(ln.graphs[ln.G][1])
        while len(ln.events) < ahead and ln.next < n_st:
            ln.launch()
        if ln.next < n_st or ln.events:
            return
        import torch
        reqs, out, G = ln.reqs, ln.graphs[ln.G][2], ln.G
        if self.keep_outputs:   # the next replay overwrites the output buffer
            per = out.n_ct // G * 2 * (out.lay.level + 1) * t.fe.N
            g0 = 0
            with torch.cuda.stream(ln.stream):
                for r in reqs:
                    g = r.ct.lay.n_bg
                    lay = out.lay.copy()
                    lay.n_bg, lay.bs = g, out.lay.bs // G * g
                    r.out = F.Ciphertexts(t.fe, lay, out.buf[g0 * per:(g0 + g) * per].clone())
                    g0 += g
            ln.stream.synchronize()
        t1 = clock()
        ln.reqs = None
        with self.mem:
            self.in_flight -= sum(r.footprint for r in reqs)
        with self.done_lock:
            for r in reqs:
                r.t_done = t1
                self.done.append(r)
            self.batches.append((t.name, len(reqs), sum(r.n_images for r in reqs), ln.t_admit, t1))

    def lane_step(self, t, clock):
        """One pass of tenant t's lane executor: advance every running batch,
        then admit queued requests into a free lane.  Returns True if any lane
        is busy."""
        busy = False
        for ln in t.lanes:
            if ln.reqs is not None:
                self._advance(t, ln, clock)
                busy = busy or ln.reqs is not None
        for ln in t.lanes:
            if ln.reqs is None:
                reqs = self._take(t)
                if not reqs:
                    break
                self._admit(t, ln, reqs, clock)
                busy = True
        return busy

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
                    if all(t.lanes for t in ts):
                        if not any([self.lane_step(t, clock) for t in ts]):
                            time.sleep(0.0002)
                    elif not sum(self.step(t, clock) for t in ts):
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
    MobileNet-block tenants at one or more offered rates (the same warmed
    server); prints one JSON line with latency percentiles and throughput per
    rate."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", type=float, nargs="+", default=[200.0],
                    help="offered request rates (requests/s), each a run of --duration seconds")
    ap.add_argument("--duration", type=float, default=5.0)
    ap.add_argument("--lenet-tenants", type=int, default=2)
    ap.add_argument("--cifar-tenants", type=int, default=1)
    ap.add_argument("--mobilenet-tenants", type=int, default=1)
    ap.add_argument("--mobilenet-max-images", type=int, default=16,
                    help="largest MobileNet request (two 224x224 images per batch group)")
    ap.add_argument("--max-batch", type=int, default=4)
    ap.add_argument("--cifar-capacity", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=2, help="pipeline lanes per tenant (0: eager runs, one per tenant)")
    ap.add_argument("--pool", type=int, default=4, help="distinct pre-encrypted requests per tenant")
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    import torch
    # every lane is a context with its own workspace: bound them so that all
    # tenants' lanes, keys, plans and stage graphs fit in HBM together
    ws = {"lenet": 6 << 30, "cifar": 12 << 30, "mobilenet": 8 << 30}
    tenants = [Tenant(f"lenet{i}", "lenet", 11 + i, 64, args.max_batch, ws_limit=ws["lenet"])
               for i in range(args.lenet_tenants)]
    tenants += [Tenant(f"cifar{i}", "cifar", 31 + i, args.cifar_capacity, 2, ws_limit=ws["cifar"])
                for i in range(args.cifar_tenants)]
    tenants += [Tenant(f"mobilenet{i}", "mobilenet", 41 + i, 2, 1, max_groups=-(-args.mobilenet_max_images // 2),
                       ws_limit=ws["mobilenet"]) for i in range(args.mobilenet_tenants)]
    srv = Server(tenants, keep_outputs=False)
    share = {"lenet": 0.6, "cifar": 0.3, "mobilenet": 0.1}
    count = {net: sum(t.net == net for t in tenants) for net in share}
    mix = {t.name: share[t.net] / count[t.net] for t in tenants}
    sizes = {t.name: (1, min(64, t.capacity * t.max_groups)) for t in tenants}
    # plans (and, with lanes, the stage graphs) for every batch-group count a run can reach
    t0 = time.perf_counter()
    srv.warmup(lanes=args.lanes, progress=lambda n, G: print(
        f"warm-up {n}: {G} batch groups, {time.perf_counter() - t0:.1f}s, library GiB "
        f"{srv.tenants[n].fe.device_bytes() / 2**30:.1f}, torch GiB {torch.cuda.memory_reserved() / 2**30:.1f}",
        file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    held = {t.name: round(sum(ln.fe.device_bytes() for ln in t.lanes) / 2**30 if t.lanes
                          else t.fe.device_bytes() / 2**30, 2) for t in tenants}
    print(f"warm-up {t_warm:.1f}s; device GiB held per tenant {held}", file=sys.stderr, flush=True)
    # clients encrypt before sending (outside the served latency); each tenant
    # has a pool of distinct encrypted requests of its largest size, and an
    # arrival of n images takes the leading batch groups it needs (read-only:
    # the network never writes its input)
    pool = {t.name: [t.encrypt_request(W.images((t.capacity * t.max_groups,) + t.in_shape, seed=1000 + j),
                                       5000 + j) for j in range(args.pool)] for t in tenants}
    # the workspaces and graphs were sized in the warm-up; admission budgets what
    # is left for the ciphertexts that runs allocate between layers
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    srv.budget = int(0.8 * torch.cuda.mem_get_info()[0])
    runs = []
    for k, rate in enumerate(args.rates):
        trace = poisson_trace(rate, args.duration, mix, sizes, args.seed + k)
        arrivals = []
        for i, (off, name, n) in enumerate(trace):
            t = srv.tenants[name]
            ct = t.leading_groups(pool[name][i % args.pool], t.groups_of(n))
            arrivals.append((off, Request(i, name, n, ct)))
        srv.done, srv.batches = [], []
        torch.cuda.synchronize()
        wall = srv.serve(arrivals)
        res = latency_summary(srv.done)
        offered = sum(n for _, _, n in trace) / args.duration
        res.update({"rate_req_per_s": rate, "offered_images_per_s": round(offered, 1),
                    "images_per_s": round(res["images"] / wall, 2), "wall_s": round(wall, 3),
                    "batches": len(srv.batches), "mean_batch": round(float(np.mean([b[1] for b in srv.batches])), 2),
                    "per_net": {}})
        for net in ("lenet", "cifar", "mobilenet"):
            d = [r for r in srv.done if srv.tenants[r.tenant].net == net]
            if d:
                res["per_net"][net] = latency_summary(d)
        runs.append(res)
        print(f"rate {rate}: {json.dumps(res)}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "served encrypted images/s (continuous batching, per-tenant keys resident)",
                      "lanes_per_tenant": args.lanes, "tenants": {t.name: t.net for t in tenants},
                      "warmup_s": round(t_warm, 1), "device_GiB_after_warmup": held,
                      "admission_budget_GiB": round(srv.budget / 2**30, 1), "duration_s": args.duration,
                      "runs": runs}), flush=True)


if __name__ == "__main__":
    main()
