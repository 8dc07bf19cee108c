"""Serving loop: requests of several tenants, continuously batched, give the
same ciphertexts as each request run alone (batch groups never share a
ciphertext), and decrypt to the float64 network."""
import time

import numpy as np
import pytest

from oracle import cnn_ref
from paper_2606_16359_amd import serve as S
from paper_2606_16359_amd import workloads as W

from fenc_backends import BACKENDS, lib_path

SMALL_NET = dict(params=(11, 12, 50, 4, 50, 3, 0, 0), shapes=[(4, 4, 3, 3), (8, 4, 3, 3), (8, 8, 3, 3)],
                 strides=[1, 2, 1], in_shape=(4, 8, 8))


def small_tenant(name, seed, backend, max_batch=2):
    prm = list(SMALL_NET["params"])
    prm[6] = 40
    return S.Tenant(name, "cifar", seed, 2, max_batch, lib_path=lib_path(backend), params=prm,
                    shapes=SMALL_NET["shapes"], strides=SMALL_NET["strides"], in_shape=SMALL_NET["in_shape"],
                    block_size=2)


def reference(t, x):
    y = x
    for wi, s in zip(t.w, t.strides):
        y = np.polynomial.polynomial.polyval(cnn_ref.conv2d(y, wi, s, 1), W.CUBIC)
    return y.reshape(x.shape[0], -1)


@pytest.mark.parametrize("backend", BACKENDS)
def test_requests_batched_across_arrivals_match_each_alone(backend):
    tenants = [small_tenant("a", 21, backend), small_tenant("b", 22, backend)]
    srv = S.Server(tenants)
    trace = [(0.0, "a", 1), (0.0, "b", 2), (0.0, "a", 2), (0.0, "a", 1), (0.0, "b", 1)]
    reqs, xs = [], []
    for i, (off, name, n) in enumerate(trace):
        t = srv.tenants[name]
        x = W.images((n,) + t.in_shape, seed=300 + i)
        xs.append(x)
        reqs.append((off, S.Request(i, name, n, t.encrypt_request(x, 900 + i))))
    srv.serve(reqs)
    assert len(srv.done) == len(trace)
    assert max(b[1] for b in srv.batches) == 2            # at least one batch merged two requests
    for (off, r), x in zip(reqs, xs):
        t = srv.tenants[r.tenant]
        mixed = t.fe.export(r.out)
        alone = S.Request(r.rid, r.tenant, r.n_images, r.ct)
        srv._run(t, [alone])
        assert np.array_equal(t.fe.export(alone.out), mixed)
        got = t.decrypt_request(r)
        assert np.max(np.abs(got - reference(t, x))) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_served_request_equals_the_oracle(backend):
    """A request served in a merged batch (on the GPU: replayed from a lane's
    stage graphs) equals, word for word, the oracle's run of the same
    encryption through the same network."""
    from oracle import pyoracle as P
    t = small_tenant("a", 25, backend)
    srv = S.Server([t])
    if backend == "hip":
        srv.warmup(lanes=2)
    xs = [W.images((n,) + t.in_shape, seed=330 + i) for i, n in enumerate((2, 1))]
    reqs = [(0.0, S.Request(i, "a", len(x), t.encrypt_request(x, 930 + i))) for i, x in enumerate(xs)]
    srv.serve(reqs)
    assert len(srv.done) == 2
    o = P.Oracle(*t.prm)
    for (_, r), x, seed in zip(reqs, xs, (930, 931)):
        full = np.zeros((t.capacity,) + t.in_shape)
        full[:len(x)] = x
        ob = o.encrypt_tensor(o.fragment_layout(t.capacity, *t.in_shape, t.block_size), full, seed)
        for wi, st in zip(t.w, t.strides):
            ob, _ = o.conv2d(ob, wi, st, wi.shape[2] // 2, 1, hoist=t.fe.hoist)
            ob, _ = o.poly_act(ob, list(W.CUBIC))
        assert np.array_equal(t.fe.export(r.out), ob.data())


@pytest.mark.parametrize("backend", BACKENDS)
def test_admission_respects_the_memory_budget(backend):
    t = small_tenant("a", 23, backend, max_batch=4)
    x = W.images((1,) + t.in_shape, seed=5)
    reqs = [S.Request(i, "a", 1, t.encrypt_request(x, 40 + i)) for i in range(4)]
    fp = t.footprint(reqs[0].ct)
    srv = S.Server([t], hbm_budget=2 * fp)                 # two requests fit at once
    for r in reqs:
        srv.submit(r)
    first = srv._take(t)
    assert len(first) == 2 and srv.in_flight == 2 * fp
    assert srv._take(t) == []                               # nothing more fits until they finish
    srv.in_flight = 0
    assert len(srv._take(t)) == 2


@pytest.mark.parametrize("backend", BACKENDS)
def test_requests_of_several_batch_groups(backend):
    """A tenant whose batch group holds 16 images takes requests of up to two
    groups; merged runs cover up to four groups and each request's output is
    bit-identical to its run alone."""
    prm = list(SMALL_NET["params"])
    prm[6] = 40
    t = S.Tenant("m", "cifar", 24, 16, 2, lib_path=lib_path(backend), params=prm, shapes=SMALL_NET["shapes"],
                 strides=[1, 1, 1], in_shape=SMALL_NET["in_shape"], block_size=1, max_groups=2)
    assert t.layout(2).n_bg == 2 and t.groups_of(17) == 2 and t.groups_of(16) == 1
    with pytest.raises(ValueError):
        t.groups_of(33)
    srv = S.Server([t])
    reqs, xs = [], []
    for i, n in enumerate((20, 5, 32, 16)):
        x = W.images((n,) + t.in_shape, seed=310 + i)
        xs.append(x)
        reqs.append((0.0, S.Request(i, "m", n, t.encrypt_request(x, 910 + i))))
        srv.submit(reqs[-1][1])
    # two requests per run: groups 2 + 1, then 2 + 1
    assert srv.step(t, time.perf_counter) == 2 and srv.step(t, time.perf_counter) == 2
    assert [b[2] for b in srv.batches] == [25, 48]
    for (off, r), x in zip(reqs, xs):
        mixed = t.fe.export(r.out)
        alone = S.Request(r.rid, r.tenant, r.n_images, r.ct)
        srv._run(t, [alone])
        assert np.array_equal(t.fe.export(alone.out), mixed)
        assert np.max(np.abs(t.decrypt_request(r) - reference(t, x))) < 1e-4
    # the leading groups of a request are a view of its buffer
    c = reqs[2][1].ct
    one = t.leading_groups(c, 1)
    assert one.lay.n_bg == 1 and one.n_ct == c.n_ct // 2


def test_poisson_trace_is_seeded_and_mixed():
    a = S.poisson_trace(200, 1.0, {"x": 0.6, "y": 0.4}, {"x": (1, 64), "y": (1, 8)}, seed=3)
    b = S.poisson_trace(200, 1.0, {"x": 0.6, "y": 0.4}, {"x": (1, 64), "y": (1, 8)}, seed=3)
    assert a == b and 150 < len(a) < 250
    assert all(0 < t <= 1.0 for t, _, _ in a) and all(a[i][0] < a[i + 1][0] for i in range(len(a) - 1))
    assert {n for _, n, _ in a} == {"x", "y"} and all(1 <= k <= 8 for _, n, k in a if n == "y")


@pytest.mark.gpu
def test_lenet_tenants_served_in_batches_match_alone_at_full_size():
    """Two LeNet-shaped tenants (N = 2^15, 64-image batch groups): ten requests
    arriving together are served in merged batches; sampled requests are
    bit-identical to their runs alone and decrypt to the float64 network."""
    import torch
    ts = [S.Tenant("l0", "lenet", 11, 64, 4), S.Tenant("l1", "lenet", 12, 64, 4)]
    srv = S.Server(ts)
    reqs, xs = [], []
    for i in range(10):
        t = ts[i % 2]
        n = 1 + (7 * i) % 64
        x = W.images((n, 1, 28, 28), seed=500 + i)
        xs.append(x)
        reqs.append((0.0, S.Request(i, t.name, n, t.encrypt_request(x, 700 + i))))
    torch.cuda.synchronize()
    srv.serve(reqs)
    assert len(srv.done) == 10 and max(b[1] for b in srv.batches) > 1
    for k in (0, 3, 8):
        r, x = reqs[k][1], xs[k]
        t = srv.tenants[r.tenant]
        mixed = t.fe.export(r.out)
        alone = S.Request(r.rid, r.tenant, r.n_images, r.ct)
        srv._run(t, [alone])
        assert np.array_equal(t.fe.export(alone.out), mixed)
        want = cnn_ref.lenet(x, *t.w).reshape(r.n_images, -1)
        assert np.max(np.abs(t.decrypt_request(r)[:, :want.shape[1]] - want)) < 1e-4
    s = S.latency_summary(srv.done)
    assert s["requests"] == 10 and s["p99_ms"] >= s["p50_ms"] > 0


@pytest.mark.gpu
def test_mobilenet_tenant_requests_of_several_groups_at_full_size():
    """The first MobileNet-V1-shaped block at 224x224 (N = 2^16, two images per
    batch group): a three-image and a two-image request are merged into one
    three-group run; each matches its run alone and the float64 block."""
    import torch
    t = S.Tenant("mb", "mobilenet", 41, 2, 2, max_groups=2)
    srv = S.Server([t])
    reqs, xs = [], []
    for i, n in enumerate((3, 2)):
        x = W.images((n,) + t.in_shape, seed=520 + i)
        xs.append(x)
        reqs.append((0.0, S.Request(i, t.name, n, t.encrypt_request(x, 720 + i))))
        srv.submit(reqs[-1][1])
    torch.cuda.synchronize()
    assert srv.step(t, time.perf_counter) == 2 and len(srv.done) == 2
    for (off, r), x in zip(reqs, xs):
        mixed = t.fe.export(r.out)
        alone = S.Request(r.rid, r.tenant, r.n_images, r.ct)
        srv._run(t, [alone])
        assert np.array_equal(t.fe.export(alone.out), mixed)
        layer = W.MOBILENET_BLOCKS[0][0]
        want = np.polynomial.polynomial.polyval(
            cnn_ref.conv2d(x, t.w[0], layer["stride"], layer["pad"], layer["groups"]), W.QUADRATIC)
        assert np.max(np.abs(t.decrypt_request(r) - want.reshape(x.shape[0], -1))) < 1e-4


@pytest.mark.gpu
def test_lanes_admit_a_batch_while_another_is_at_a_later_layer():
    """A LeNet-shaped tenant with two lanes (stage graphs, N = 2^15): a request
    arriving while another batch of the same tenant is mid-network is admitted
    at the next stage boundary into the free lane and runs concurrently; both
    outputs equal their runs alone and the float64 network."""
    import torch
    t = S.Tenant("l", "lenet", 13, 64, 1)
    srv = S.Server([t])
    srv.warmup(lanes=2, group_counts={"l": [1]})
    xs = [W.images((n, 1, 28, 28), seed=540 + i) for i, n in enumerate((64, 40))]
    cts = [t.encrypt_request(x, 740 + i) for i, x in enumerate(xs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a = S.Request(0, "l", 64, cts[0])
    srv.submit(a)
    srv.lane_step(t, time.perf_counter)                    # a: lane 0, first stages queued
    ln0 = t.lanes[0]
    while ln0.reqs is not None and ln0.next - len(ln0.events) < 3:
        srv.lane_step(t, time.perf_counter)                # until a is executing its fourth stage or later
    assert ln0.reqs is not None, "the first batch finished before the second could arrive"
    b = S.Request(1, "l", 40, cts[1])
    srv.submit(b)
    srv.lane_step(t, time.perf_counter)
    assert t.lanes[1].reqs == [b]                          # admitted into the free lane
    assert srv.admissions[-1][2] and srv.admissions[-1][2][0] >= 3   # while a was at a later layer
    while any(ln.reqs is not None for ln in t.lanes):
        srv.lane_step(t, time.perf_counter)
    assert len(srv.done) == 2 and time.perf_counter() > t0
    for r, x in zip((a, b), xs):
        alone = S.Request(r.rid, r.tenant, r.n_images, r.ct)
        srv._run(t, [alone])
        assert np.array_equal(t.fe.export(alone.out), t.fe.export(r.out))
        want = cnn_ref.lenet(x, *t.w).reshape(r.n_images, -1)
        assert np.max(np.abs(t.decrypt_request(r)[:, :want.shape[1]] - want)) < 1e-4
