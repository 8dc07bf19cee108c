"""Element-by-element parity of the library's kernels with the oracle.

Every test runs twice: through the CPU emulator of the kernel bodies (CPU
suite) and on the MI355X (marked gpu).  Ciphertext limbs must be bit-exact in
coefficient form; decrypted values are compared with float64 references.
"""
import numpy as np
import pytest

from oracle import cnn_ref
from oracle import pyoracle as P

from fenc_backends import BACKENDS, make, rng
from paper_2606_16359_amd import fenc as F

# toy parameters: N = 2^10, 8 x 50-bit primes, 3 special primes, dnum 3 (3 limbs per digit)
SMALL = (10, 8, 50, 3, 50, 3, 40, 17)


@pytest.fixture(scope="module")
def orc():
    return P.Oracle(*SMALL)


def cmp(lib_ct, orc_batch, fenc):
    a = fenc.export(lib_ct)
    b = orc_batch if isinstance(orc_batch, np.ndarray) else orc_batch.data()
    assert a.shape == b.shape
    bad = np.argwhere(a != b)
    assert bad.size == 0, f"{len(bad)} limbs words differ, first at {bad[0]}"


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("logn", [10, 13, 16])
def test_ntt_roundtrip_and_product(backend, logn):
    o = P.Oracle(logn, 4, 50, 2, 50, 2, 40, 3)
    f = make(backend, logn, 4, 50, 2, 50, 2, 40, 3)
    r = rng(logn)
    primes = o.primes()
    rows = np.array([r.integers(0, primes[i % 6], o.N, dtype=np.uint64) for i in range(7)])   # 7 rows: ragged
    pidx = [i % 6 for i in range(7)]
    A = f.ntt_rows(rows, pidx)
    assert np.array_equal(f.ntt_rows(A, pidx, inverse=True), rows)
    for i in range(0, 6, 2):
        q = primes[pidx[i]]
        prod = (A[i].astype(object) * A[i + 1].astype(object) % q).astype(np.uint64)
        got = f.ntt_rows(prod[None], [pidx[i]], inverse=True)[0]
        assert np.array_equal(got, o.polymul(pidx[i], rows[i], rows[i + 1])) if pidx[i] == pidx[i + 1] else True
    # evaluation order: slot k holds a(psi^(2 brev(k) + 1))
    psi, q = o.psi()[0], primes[0]
    a = rows[0]
    for k in [0, 1, 5, o.N - 1]:
        e = 2 * int(format(k, f"0{logn}b")[::-1], 2) + 1
        assert int(A[0][k]) == sum(int(a[i]) * pow(psi, e * i, q) for i in range(o.N)) % q


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("logn", [11, 15, 16])
def test_ntt_pass_shapes_give_identical_residues(backend, logn):
    """Radix-8 and radix-16 rounds and every tile size compute the same NTT
    (log N = 16: the column pass with eight stage bits of the N = 2^16 sets)."""
    f = make(backend, logn, 3, 50, 1, 50, 3, 40, 3)
    o = P.Oracle(logn, 3, 50, 1, 50, 3, 40, 3)
    r = rng(logn + 1)
    primes = o.primes()
    pidx = [0, 1, 2, 3, 1]                       # 5 rows: ragged against any batch shape
    rows = np.array([r.integers(0, primes[p], o.N, dtype=np.uint64) for p in pidx])
    n2 = (logn + 1) // 2
    n1 = logn - n2
    shapes = [[(3, -1)] * 4, [(4, -1)] * 4, [(4, 0), (4, 0), (3, 0), (3, 0)],
              [(3, min(5, n2)), (4, min(3, n1)), (4, min(2, n1)), (3, 2)]]
    shapes = [[(rb, t if t < 0 or 8 << ((n1 if k in (0, 3) else n2) + t) <= 65536 else 0)
               for k, (rb, t) in enumerate(sh)] for sh in shapes]
    want_f = want_i = None
    for sh in shapes:
        f.set_ntt_config(sh)
        assert f.ntt_config() == [tuple(x) for x in sh]
        A = f.ntt_rows(rows, pidx)
        B = f.ntt_rows(A, pidx, inverse=True)
        assert np.array_equal(B, rows)
        if want_f is None:
            want_f = A
            # a spot check against the oracle's NTT (natural order there, bit-reversed here)
            nat = o.ntt(pidx[0], rows[0])
            br = [int(format(k, f"0{logn}b")[::-1], 2) for k in range(o.N)]
            assert np.array_equal(A[0], nat[br])
        assert np.array_equal(A, want_f)
    with pytest.raises(F.FencError):
        f.set_ntt_config([(5, -1)] * 4)


@pytest.mark.parametrize("backend", BACKENDS)
def test_encrypt_keys_and_keyswitch_building_blocks(backend, orc):
    o, f = orc, make(backend, *SMALL)
    assert f.primes() == o.primes()
    z = rng(1).uniform(-1, 1, o.ns)
    pt = o.encode(z, None, 2.0 ** 40)
    assert np.array_equal(f.encode_slots(z, o.L, 2.0 ** 40), pt)
    lay = f.plan_layout(1, 1, 16, 16, 3, 1)
    ct = f.encrypt(pt[None], lay, 7)
    oc = o.encrypt(pt, o.L, 2.0 ** 40, 7, 0)
    cmp(ct, oc[None], f)
    for shift in (1, 37):
        assert np.array_equal(f.key_export(shift), o.switch_key(o.galois(shift)))
    assert np.array_equal(f.key_export(F.RELIN), o.switch_key(0))
    shifts = [1, 37, o.ns - 5]
    cmp(f.rotate(ct, shifts), o.rotate(oc, shifts), f)
    r = f.rotate(ct, [3, 9])
    orr = o.rotate(oc, [3, 9])
    cmp(f.rotate_sum(ct, r, [1, 2]), o.rotate_sum(oc, orr, [1, 2])[None], f)
    cmp(f.rotate_sum(None, r, [1, 2]), o.rotate_sum(None, orr, [1, 2])[None], f)
    cmp(f.rescale(ct), o.rescale(oc)[None], f)
    assert np.array_equal(f.decrypt_raw(ct)[0], o.decrypt(oc))


@pytest.mark.parametrize("backend", BACKENDS)
def test_device_bytes_return_after_encrypt_and_decrypt(backend, orc):
    """Temporaries of encryption, decryption and transfers are returned and
    taken off the context's device byte count."""
    f = make(backend, *SMALL)
    lay = f.plan_layout(1, 1, 16, 16, 3, 1)
    x = rng(3).uniform(0, 1, (1, 1, 16, 16))
    ct = f.encrypt(f.encode_fragment(x, lay), lay, 7)
    f.decrypt(ct)
    before = f.device_bytes()
    for _ in range(3):
        ct = f.encrypt(f.encode_fragment(x, lay), lay, 7)
        f.decrypt(ct)
        f.decrypt_raw(ct)
        f.export(ct)
    assert f.device_bytes() == before


@pytest.mark.parametrize("backend", BACKENDS)
def test_batch_group_tiles_give_identical_residues(backend, orc):
    """A workspace limit that forces one batch group per tile: convolution
    (hoisted rotations, masks, outer rotations), S = 1 pooling and the
    quadratic run tile by tile and give the untiled residues, which equal the
    oracle's."""
    o, f = orc, make(backend, *SMALL)
    x = rng(11).uniform(0, 1, (16, 2, 8, 8))     # 512 slots, 64-slot fragments: 8 images per ct
    w = rng(12).normal(0, 0.1, (3, 2, 3, 3))
    lay = f.plan_layout(16, 2, 8, 8, 3, 3, 1)
    assert lay.n_bg == 2
    ct = f.encrypt(f.encode_fragment(x, lay), lay, 5)

    def net():
        y = f.conv2d(ct, w, pad=1)
        return f.avgpool2(f.poly_act(y, (0.1, 0.5, 0.25)))
    ref = f.export(net())
    f.set_workspace_limit(1)
    assert np.array_equal(f.export(net()), ref)

    def net_inplace():    # the activation overwrites the convolution's output
        y = f.conv2d(ct, w, pad=1)
        return f.avgpool2(f.poly_act(y, (0.1, 0.5, 0.25), inplace=True))
    assert np.array_equal(f.export(net_inplace()), ref)
    f.set_workspace_limit(0)
    assert np.array_equal(f.export(net_inplace()), ref)
    cub = f.poly_act(f.conv2d(ct, w, pad=1), (0.1, 0.5, 0.25, -0.02))
    assert np.array_equal(f.export(f.poly_act(f.conv2d(ct, w, pad=1), (0.1, 0.5, 0.25, -0.02), inplace=True)),
                          f.export(cub))
    Lo = o.fragment_layout(16, 2, 8, 8, 1)
    ob = o.encrypt_tensor(Lo, x, 5)
    yo, _ = o.conv2d(ob, w, pad=1, hoist=f.hoist)
    yo, _ = o.poly_act(yo, (0.1, 0.5, 0.25))
    yo, _ = o.avgpool2(yo, hoist=f.hoist)
    assert np.array_equal(ref, yo.data())


def _layout_dict(o, lay):
    d = o.fragment_layout(lay.bs, lay.c, lay.h, lay.w, lay.S)
    assert (d["bsg"], d["cpc"], d["rep"], d["M"]) == (lay.bs_g, lay.chan_per_ct, lay.replicate, lay.M)
    return d


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("budget,hoist", [(1 << 30, 1), (0, 1), (1 << 30, 0), (0, 0)])
def test_fused_compression_bottleneck_bit_exact(backend, budget, hoist, orc):
    """8 -> 2 -> 8 bottleneck: the reduction writes its output straight into
    the dense repeated-channel layout (the repack fused with the convolution,
    same level), then the expansion runs with a bias; both bit-exact against
    the oracle, with the oracle's rotation counts."""
    o, f = orc, make(backend, *SMALL)
    f.set_plaintext_budget(budget)
    f.set_hoisting(hoist)
    r = rng(21)
    x, w1, w2 = r.uniform(0, 1, (4, 8, 4, 4)), r.normal(0, 0.1, (2, 8, 1, 1)), r.normal(0, 0.1, (8, 2, 1, 1))
    bias = np.linspace(-0.5, 0.5, 8)
    lay = f.plan_layout(4, 8, 4, 4, 1, 2, 1)
    Lo = o.fragment_layout(4, 8, 4, 4, 1)
    fb, ob = f.encrypt(f.encode_fragment(x, lay), lay, 3), o.encrypt_tensor(Lo, x, 3)
    f.stats_reset()
    y = f.conv2d(fb, w1, s_out=1)
    assert (y.lay.replicate, y.n_ct, y.lay.level) == (1, 1, lay.level - 1)
    yo, cnt = o.conv2d(ob, w1, pt_budget=budget, hoist=hoist, target=o.fragment_layout(4, 2, 4, 4, 1))
    cmp(y, yo, f)
    st = f.stats()
    assert (st["rot_inner"], st["rot_outer"]) == (cnt["inner_rot"], cnt["outer_rot"])
    z = f.conv2d(y, w2, bias=bias)
    zo, _ = o.conv2d(yo, w2, pt_budget=budget, hoist=hoist, bias=bias)
    cmp(z, zo, f)
    ref = cnn_ref.conv2d(cnn_ref.conv2d(x, w1), w2) + bias[None, :, None, None]
    assert np.max(np.abs(f.decrypt(z) - ref)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_compression_targets_and_fused_block_size_change_bit_exact(backend, orc):
    """Standalone compression into fragment targets of three block sizes and
    into the library's vector; a convolution fused with a block-size change
    (S = 2 -> 1); an FC layer with a bias."""
    o, f = orc, make(backend, *SMALL)
    r = rng(31)
    x = r.uniform(0, 1, (4, 2, 4, 4))
    lay = f.plan_layout(4, 2, 4, 4, 3, 2, 2)
    Lo = o.fragment_layout(4, 2, 4, 4, 2)
    fb, ob = f.encrypt(f.encode_fragment(x, lay), lay, 5), o.encrypt_tensor(Lo, x, 5)
    for S_t in (1, 2, 4):
        T = f.plan_layout(4, 2, 4, 4, 3, 2, S_t)
        c = f.compress(fb, T)
        co, _ = o.compress(ob, target=_layout_dict(o, T), hoist=f.hoist)
        assert (c.lay.S, c.lay.level) == (S_t, lay.level - 1)
        cmp(c, co, f)
        assert np.max(np.abs(f.decrypt(c) - x)) < 1e-6
    v = f.compress(fb)
    vo, _ = o.compress(ob, hoist=f.hoist)
    cmp(v, vo, f)
    fw, fbias = r.normal(0, 0.1, (5, 32)), np.linspace(-1, 1, 5)
    cmp(f.fc(v, fw, bias=fbias), o.fc(vo, fw, bias=fbias)[0], f)
    # fused S = 2 -> 1 (8 images, 2 channels of 8 x 8)
    x8 = r.uniform(0, 1, (8, 2, 8, 8))
    w = r.normal(0, 0.1, (2, 2, 3, 3))
    lay8 = f.plan_layout(8, 2, 8, 8, 3, 2, 2)
    L8 = o.fragment_layout(8, 2, 8, 8, 2)
    y = f.conv2d(f.encrypt(f.encode_fragment(x8, lay8), lay8, 6), w, pad=1, s_out=1)
    yo, _ = o.conv2d(o.encrypt_tensor(L8, x8, 6), w, 1, 1, 1, hoist=f.hoist, target=o.fragment_layout(8, 2, 8, 8, 1))
    assert y.lay.S == 1
    cmp(y, yo, f)
    assert np.max(np.abs(f.decrypt(y) - cnn_ref.conv2d(x8, w, 1, 1))) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_server_context_evaluates_with_imported_keys_and_holds_no_secret(backend):
    """Client/server protocol (Design Overview): the client encrypts and
    generates the evaluation keys; a server context without a secret key
    imports them and the ciphertexts, evaluates a convolution, an activation,
    pooling, compression and an FC layer, and returns ciphertexts identical
    to the client's own evaluation; it cannot encrypt, decrypt or make keys."""
    client, server = make(backend, *SMALL), make(backend, *SMALL, server=True)
    r = rng(41)
    x, w, fw = r.uniform(0, 1, (4, 2, 8, 8)), r.normal(0, 0.1, (2, 2, 3, 3)), r.normal(0, 0.1, (3, 32))
    lay = client.plan_layout(4, 2, 8, 8, 3, 2, 2)
    ct = client.encrypt(client.encode_fragment(x, lay), lay, 9)

    def net(f, c):
        y = f.avgpool2(f.poly_act(f.conv2d(c, w, pad=1)))
        return f.fc(f.compress(y), fw)
    ref = client.export(net(client, ct))
    keys = client.key_list()
    assert 0 in keys and len(keys) > 2
    for g in keys:
        server.key_import(g, client.key_export_galois(g))
    assert sorted(server.key_list()) == sorted(keys)
    sct = server.import_cts(client.export(ct), ct.lay.copy())
    out = net(server, sct)
    assert np.array_equal(server.export(out), ref)
    back = client.import_cts(server.export(out), out.lay.copy())
    want = cnn_ref.fc(cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(x, w, 1, 1))), fw)
    assert np.max(np.abs(client.decrypt(back).reshape(4, 3) - want.reshape(4, 3))) < 1e-4
    for call in (lambda: server.decrypt(out), lambda: server.decrypt_raw(out),
                 lambda: server.encrypt(client.encode_fragment(x, lay), lay, 9),
                 lambda: server.rotate(sct, [5])):            # no key for this shift, and none can be made
        with pytest.raises(F.FencError) as e:
            call()
        assert e.value.code == -3
    with pytest.raises(F.FencError) as e:
        server.key_import(keys[0], client.key_export_galois(keys[0]))   # already held
    assert e.value.code == -1


WIDE = (10, 10, 40, 10, 40, 1, 30, 19)   # one digit of 10 limbs, 10 special primes


@pytest.mark.parametrize("backend", BACKENDS)
def test_keyswitch_with_digits_and_special_primes_above_eight(backend):
    """A digit of 10 limbs and 10 special primes: the base conversions run in
    their wide form (more than 8 limbs)."""
    from oracle import pyoracle as P
    o, f = P.Oracle(*WIDE), make(backend, *WIDE)
    assert f.primes() == o.primes()
    z = rng(2).uniform(-1, 1, o.ns)
    pt = o.encode(z, None, 2.0 ** 30)
    lay = f.plan_layout(1, 1, 16, 16, 3, 1)
    ct = f.encrypt(pt[None], lay, 7)
    oc = o.encrypt(pt, o.L, 2.0 ** 30, 7, 0)
    cmp(ct, oc[None], f)
    shifts = [1, 37, o.ns - 5]
    cmp(f.rotate(ct, shifts), o.rotate(oc, shifts), f)
    r = f.rotate(ct, [3, 9])
    cmp(f.rotate_sum(ct, r, [1, 2]), o.rotate_sum(oc, o.rotate(oc, [3, 9]), [1, 2])[None], f)
    cmp(f.rescale(ct), o.rescale(oc)[None], f)


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("mode,budget,hoist,own", [(F.FENC_MODE_BATCHED, 1 << 30, 1, None),
                                                   (F.FENC_MODE_PER_OP, 1 << 30, 1, 0),
                                                   (F.FENC_MODE_BATCHED, 0, 1, 0), (F.FENC_MODE_BATCHED, 1 << 30, 0, None),
                                                   (F.FENC_MODE_PER_OP, 0, 0, None),
                                                   (F.FENC_MODE_BATCHED, 1 << 30, 2, 0)])
def test_mini_lenet_layers_bit_exact(backend, mode, budget, hoist, own, orc):
    """Two conv/x^2/pool blocks, compression and two FC layers at N = 2^10, in
    both hoisting schedules and in the per-layer choice (mode 2: the oracle
    runs each layer in the schedule the library reports it chose); with the
    digits' own limbs copied into the extended digits (the default at this
    size) and read from the input ciphertexts (own-copy limit 0)."""
    o, f = orc, make(backend, *SMALL)
    if own is not None:
        f.set_own_copy_limit(own)
    f.set_mode(mode)
    f.set_plaintext_budget(budget)
    f.set_hoisting(hoist)
    r = rng(2)
    x = r.uniform(0, 1, (4, 1, 14, 14))
    w1, w2 = r.normal(0, 0.1, (3, 1, 3, 3)), r.normal(0, 0.1, (4, 3, 3, 3))
    f1, f2 = r.normal(0, 0.1, (8, 16)), r.normal(0, 0.1, (4, 8))
    Lo = o.fragment_layout(4, 1, 14, 14, 2)
    lay = f.plan_layout(4, 1, 14, 14, 3, 3, 2)
    pt = f.encode_fragment(x, lay)
    assert np.array_equal(pt, o.encode_tensor(Lo, x))
    ob, fb = o.encrypt_tensor(Lo, x, 3), f.encrypt(pt, lay, 3)
    cmp(fb, ob, f)
    # h: the schedule the library's layer ran with
    steps = [("conv", lambda c: f.conv2d(c, w1), lambda b, h: o.conv2d(b, w1, pt_budget=budget, hoist=h)[0]),
             ("square", f.poly_act, lambda b, h: o.square(b)[0]),
             ("pool-fragments", f.avgpool2, lambda b, h: o.avgpool2(b, h)[0]),
             ("conv", lambda c: f.conv2d(c, w2), lambda b, h: o.conv2d(b, w2, pt_budget=budget, hoist=h)[0]),
             ("square", f.poly_act, lambda b, h: o.square(b)[0]),
             ("pool-rotations", f.avgpool2, lambda b, h: o.avgpool2(b, h)[0]),
             ("compress", f.compress, lambda b, h: o.compress(b, hoist=h)[0]),
             ("fc", lambda c: f.fc(c, f1), lambda b, h: o.fc(b, f1)[0]),
             ("fc", lambda c: f.fc(c, f2), lambda b, h: o.fc(b, f2)[0])]
    chosen = []
    for name, fl, ol in steps:
        fb = fl(fb)
        h = f.last_hoisting() if hoist == 2 else hoist
        chosen.append(h)
        ob = ol(ob, h)
        cmp(fb, ob, f)
    if hoist != 2:
        assert f.last_hoisting() == hoist   # the compression has rotated copies
    ref = cnn_ref.fc(cnn_ref.fc(cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(
        cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(x, w1))), w2))), f1), f2)
    assert np.max(np.abs(f.decrypt(fb) - ref)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("budget", [1 << 30, 0])
@pytest.mark.parametrize("case", [
    dict(x=(2, 4, 8, 8), w=(4, 4, 3, 3), stride=2, pad=1, groups=1, S=2),    # stride by discarding, masks
    dict(x=(2, 4, 8, 8), w=(4, 1, 3, 3), stride=1, pad=1, groups=4, S=2),    # depthwise
    dict(x=(2, 3, 8, 8), w=(5, 3, 3, 3), stride=1, pad=1, groups=1, S=1),    # outer rotations, ragged channels
    dict(x=(16, 2, 8, 8), w=(5, 2, 5, 5), stride=1, pad=0, groups=1, S=1),   # C' = 1: scalar MAC only
    dict(x=(1, 1, 12, 12), w=(6, 1, 5, 5), stride=1, pad=0, groups=1, S=1),  # replicated single channel
    dict(x=(2, 4, 8, 8), w=(6, 4, 1, 1), stride=1, pad=0, groups=1, S=1),    # pointwise: outer rotations only
    dict(x=(2, 4, 8, 8), w=(4, 1, 3, 3), stride=2, pad=1, groups=4, S=2),    # depthwise with stride
])
@pytest.mark.parametrize("hoist", [1, 0, 2])
def test_conv_variants_bit_exact(backend, budget, case, hoist, orc):
    o, f = orc, make(backend, *SMALL)
    f.set_own_copy_limit(0 if hoist != 1 else 1 << 40)   # own limbs read from the input / always copied
    f.set_plaintext_budget(budget)
    f.set_hoisting(hoist)
    r = rng(3)
    x, w = r.uniform(0, 1, case["x"]), r.normal(0, 0.1, case["w"])
    Lo = o.fragment_layout(*case["x"], case["S"])
    lay = f.plan_layout(*case["x"], case["w"][2], case["w"][0], case["S"])
    ob, fb = o.encrypt_tensor(Lo, x, 5), f.encrypt(f.encode_fragment(x, lay), lay, 5)
    f.stats_reset()
    yf = f.conv2d(fb, w, case["stride"], case["pad"], case["groups"])
    h = f.last_hoisting()
    assert h in (0, 1) and (hoist == 2 or h == hoist or (h == 0 and f.stats()["rot_inner"] == 0))
    yo, cnt = o.conv2d(ob, w, case["stride"], case["pad"], case["groups"], pt_budget=budget, hoist=h)
    cmp(yf, yo, f)
    st = f.stats()
    assert (st["rot_inner"], st["rot_outer"], st["moddown"]) == (cnt["inner_rot"], cnt["outer_rot"], cnt["moddown"])
    want = cnn_ref.conv2d(x, w, case["stride"], case["pad"], case["groups"])
    assert np.max(np.abs(f.decrypt(yf) - want)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("case", [
    dict(x=(2, 4, 8, 8), w=(4, 4, 3, 3), stride=1, pad=1, groups=1, S=2),    # one mask per group and class
    dict(x=(2, 4, 8, 8), w=(4, 1, 3, 3), stride=2, pad=1, groups=4, S=2),    # masks differing per output
])
@pytest.mark.parametrize("hoist", [1, 0])
def test_conv_large_weight_codes_bit_exact(backend, case, hoist, orc):
    """Weights of magnitude ~10 give codes above 2^23 after the scale split,
    so the MAC takes a modular product per term instead of the small-code
    path; the mask-basis form (plaintext budget 0) is forced."""
    o, f = orc, make(backend, *SMALL)
    f.set_plaintext_budget(0)
    f.set_hoisting(hoist)
    r = rng(4)
    x, w = r.uniform(0, 1, case["x"]), r.normal(0, 10.0, case["w"])
    Lo = o.fragment_layout(*case["x"], case["S"])
    lay = f.plan_layout(*case["x"], case["w"][2], case["w"][0], case["S"])
    ob, fb = o.encrypt_tensor(Lo, x, 5), f.encrypt(f.encode_fragment(x, lay), lay, 5)
    yo, _ = o.conv2d(ob, w, case["stride"], case["pad"], case["groups"], pt_budget=0, hoist=hoist)
    yf = f.conv2d(fb, w, case["stride"], case["pad"], case["groups"])
    cmp(yf, yo, f)
    want = cnn_ref.conv2d(x, w, case["stride"], case["pad"], case["groups"])
    assert np.max(np.abs(f.decrypt(yf) - want)) < 1e-4 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("backend", BACKENDS)
def test_single_conv_layer_benchmark_small_config(backend):
    """1x28x28 image, conv 1->6 5x5 valid, N=2^13, 4 x 40-bit primes + 1 special, scale 2^30."""
    params = (13, 4, 40, 1, 40, 4, 30, 1)
    o, f = P.Oracle(*params), make(backend, *params)
    r = rng(4)
    x, w = r.uniform(0, 1, (1, 1, 28, 28)), r.normal(0, 0.1, (6, 1, 5, 5))
    Lo = o.plan_layout(1, 1, 28, 28, 5, 6)
    lay = f.plan_layout(1, 1, 28, 28, 5, 6)
    assert (lay.S, lay.chan_per_ct, lay.replicate) == (Lo["S"], Lo["cpc"], Lo["rep"]) == (1, 4, 1)
    ob, fb = o.encrypt_tensor(Lo, x, 9), f.encrypt(f.encode_fragment(x, lay), lay, 9)
    cmp(fb, ob, f)
    yo, cnt = o.conv2d(ob, w, hoist=f.hoist)
    yf = f.conv2d(fb, w)
    cmp(yf, yo, f)
    assert cnt["inner_rot"] == 24 and cnt["outer_rot"] == 0 and yf.n_ct == 2
    # The target bound 1e-4 holds at Delta = 2^30: the 24 key switches (one
    # 40-bit special prime) each add slot noise of a few 1e-5, weighted by
    # |w| ~ 0.1 in the sum; measured maxima are near 2e-5.
    assert np.max(np.abs(f.decrypt(yf) - cnn_ref.conv2d(x, w))) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_errors_are_reported_not_launched(backend, orc):
    f = make(backend, *SMALL)
    with pytest.raises(F.FencError) as e:
        F.Fenc(10, 8, 50, 1, 50, 3, 40, 1, lib_path=f.lib._name if backend == "emu" else None)
    assert e.value.code == -1          # fewer special primes than digit limbs
    lay = f.plan_layout(2, 4, 8, 8, 3, 4, 2)
    ct = f.encrypt(f.encode_fragment(np.zeros((2, 4, 8, 8)), lay), lay, 1)
    with pytest.raises(F.FencError) as e:
        f.conv2d(ct, np.zeros((4, 4, 3, 3)), stride=4)       # stride must divide S
    assert e.value.code == -8
    with pytest.raises(F.FencError) as e:
        f.poly_act(ct, (0.5, 0.0, 1.0, 0.0, 1.0))                 # degree 4
    assert e.value.code == -8
    with pytest.raises(F.FencError) as e:
        f.fc(ct, np.zeros((4, 4)))                            # fc needs a vector layout
    assert e.value.code == -6
    lay0 = lay.copy()
    lay0.level = 0
    c0 = f.encrypt(f.encode_fragment(np.zeros((2, 4, 8, 8)), lay0)[:, :1], lay0, 1)
    with pytest.raises(F.FencError) as e:
        f.conv2d(c0, np.zeros((4, 4, 3, 3)), pad=1)
    assert e.value.code == -4
    f.keygen([1], relin=False, strict=True)
    with pytest.raises(F.FencError) as e:
        f.rotate(ct, [2])
    assert e.value.code == -3


@pytest.mark.parametrize("backend", BACKENDS)
def test_scalar_weights_after_activation_scale_drop(backend, orc):
    """x^2 leaves the scale near Delta; after a second conv the activation's scale
    drift is absorbed by the next convolution's T = q_l Delta / s_in split."""
    o, f = orc, make(backend, *SMALL)
    r = rng(5)
    x = r.uniform(0, 1, (16, 2, 8, 8))
    w1, w2 = r.normal(0, 0.1, (2, 2, 3, 3)), r.normal(0, 0.1, (3, 2, 3, 3))
    Lo = o.fragment_layout(16, 2, 8, 8, 1)
    lay = f.plan_layout(16, 2, 8, 8, 3, 2, 1)
    ob, fb = o.encrypt_tensor(Lo, x, 6), f.encrypt(f.encode_fragment(x, lay), lay, 6)
    ob = o.conv2d(o.square(o.conv2d(ob, w1, hoist=f.hoist)[0])[0], w2, hoist=f.hoist)[0]
    fb = f.conv2d(f.poly_act(f.conv2d(fb, w1)), w2)
    cmp(fb, ob, f)
    want = cnn_ref.conv2d(cnn_ref.square(cnn_ref.conv2d(x, w1)), w2)
    assert np.max(np.abs(f.decrypt(fb) - want)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("coeffs", [
    (0.25, -1.5),                          # affine
    (0.1471, 0.5, 0.1196),                 # a x^2 + b x + c, ReLU-shaped
    (-0.3, 0.0, -2.0),                     # negative leading coefficient
    (0.02, 0.5, 0.2, -0.04),               # cubic
    (0.0, 0.0, 0.0, 1.0),                  # x^3 alone
])
def test_poly_act_bit_exact(backend, orc, coeffs):
    """Polynomial activations of degree 1-3 on a 3-ct fragment batch, batched and per-op."""
    o, f = orc, make(backend, *SMALL)
    x = 2.0 * rng(21).uniform(0, 1, (4, 3, 8, 8)) - 1.0
    Lo = o.fragment_layout(4, 3, 8, 8, 2)
    lay = f.plan_layout(4, 3, 8, 8, 3, 3, 2)
    ob, fb = o.encrypt_tensor(Lo, x, 3), f.encrypt(f.encode_fragment(x, lay), lay, 3)
    yo, cnt = o.poly_act(ob, list(coeffs))
    for mode in (F.FENC_MODE_BATCHED, F.FENC_MODE_PER_OP):
        f.set_mode(mode)
        f.set_own_copy_limit(0 if mode == F.FENC_MODE_PER_OP else 1 << 40)
        yf = f.poly_act(fb, coeffs)
        Ly = yo.layout()
        assert (yf.lay.level, yf.lay.scale) == (Ly["level"], Ly["scale"])
        cmp(yf, yo, f)
    f.set_mode(F.FENC_MODE_BATCHED)
    ref = np.polynomial.polynomial.polyval(x, coeffs)
    assert np.max(np.abs(f.decrypt(yf) - ref)) < 1e-5


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("params", [(10, 8, 50, 8, 50, 1, 40, 17), (10, 9, 50, 7, 50, 2, 40, 17),
                                    (10, 4, 40, 1, 40, 4, 30, 17)])
def test_activation_modulus_shapes_bit_exact(backend, params):
    """The square and the cubic (relinearisation and rescale by one ModDown by
    P q_l) where the conversion has K + 1 = 9 sources (past the unrolled
    forms), 8, and 2 (one special prime, one-limb digits)."""
    o, f = P.Oracle(*params), make(backend, *params)
    x = 2.0 * rng(24).uniform(0, 1, (2, 2, 8, 8)) - 1.0
    Lo = o.fragment_layout(2, 2, 8, 8, 2)
    lay = f.plan_layout(2, 2, 8, 8, 3, 2, 2)
    ob, fb = o.encrypt_tensor(Lo, x, 5), f.encrypt(f.encode_fragment(x, lay), lay, 5)
    for coeffs in ((0.0, 0.0, 1.0), (0.1, 0.5, 0.25, -0.02)):
        yo, _ = o.poly_act(ob, list(coeffs))
        yf = f.poly_act(fb, coeffs)
        cmp(yf, yo, f)
        assert np.max(np.abs(f.decrypt(yf) - np.polynomial.polynomial.polyval(x, coeffs))) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_cifar_shaped_stack_small_bit_exact(backend):
    """The CIFAR-shaped stack scaled down: 3x3 convs with padding, a stride-2 conv
    (fragments discarded) and a cubic activation after each conv; N = 2^11."""
    from paper_2606_16359_amd import workloads as W
    params = (11, 12, 50, 4, 50, 3, 40, 17)
    o, f = P.Oracle(*params), make(backend, *params)
    shapes, strides = [(4, 4, 3, 3), (8, 4, 3, 3), (8, 8, 3, 3)], [1, 2, 1]
    x, w = W.cifar_inputs(2, 4, 8, shapes)
    Lo = o.fragment_layout(2, 4, 8, 8, 2)
    lay = f.plan_layout(2, 4, 8, 8, 3, 4, 2)
    ob, fb = o.encrypt_tensor(Lo, x, 7), f.encrypt(f.encode_fragment(x, lay), lay, 7)
    ref = x
    for wi, s in zip(w, strides):
        ob = o.poly_act(o.conv2d(ob, wi, s, 1, hoist=f.hoist)[0], list(W.CUBIC))[0]
        ref = np.polynomial.polynomial.polyval(cnn_ref.conv2d(ref, wi, s, 1), W.CUBIC)
    fb = W.cifar_forward(f, fb, w, strides)
    cmp(fb, ob, f)
    assert fb.lay.level == 11 - 9
    assert np.max(np.abs(f.decrypt(fb) - ref)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("case", [dict(x=(1, 16, 4, 4), w=(16, 16, 1, 1), pad=0),
                                  dict(x=(1, 16, 4, 4), w=(16, 16, 3, 3), pad=1),
                                  dict(x=(2, 8, 8, 8), w=(8, 8, 3, 3), pad=1)])
@pytest.mark.parametrize("n1", [1, 2, 4, 0])
@pytest.mark.parametrize("budget,hoist", [(1 << 30, 1), (0, 0)])
def test_conv_bsgs_outer_rotations_bit_exact(backend, case, n1, budget, hoist, orc):
    """Outer rotations by baby-step giant-step: a fixed baby step or the
    per-layer choice (0) gives the oracle's words for the same baby step, in
    both plaintext forms and both hoisting schedules; the key switches equal
    the oracle's and the no-build count, and the choice is the count's
    minimum over powers of two."""
    o, f = orc, make(backend, *SMALL)
    f.set_baby_step(n1)
    f.set_plaintext_budget(budget)
    f.set_hoisting(hoist)
    r = rng(41)
    x, w = r.uniform(0, 1, case["x"]), r.normal(0, 0.1, case["w"])
    lay = f.plan_layout(*case["x"], case["w"][2], case["w"][0], 1)
    ob, fb = o.encrypt_tensor(o.fragment_layout(*case["x"], 1), x, 5), f.encrypt(f.encode_fragment(x, lay), lay, 5)
    inner, outer, _ = f.conv2d_keyswitches(lay, case["w"][0], case["w"][2], 1, case["pad"])
    f.stats_reset()
    yf = f.conv2d(fb, w, 1, case["pad"])
    nb = f.last_baby_step()
    nd = lay.chan_per_ct if not lay.replicate else case["x"][1]
    assert nb == (min(n1, nd) if n1 else nb)
    yo, cnt = o.conv2d(ob, w, 1, case["pad"], 1, pt_budget=budget, hoist=f.last_hoisting(), baby=nb)
    cmp(yf, yo, f)
    st = f.stats()
    assert (st["rot_inner"], st["rot_outer"]) == (cnt["inner_rot"], cnt["outer_rot"]) == (inner, outer)
    if n1 == 0:
        ks = {}
        for p in (1, 2, 4, 8, 16, 32):
            if p <= nd:
                f.set_baby_step(p)
                a, b, _ = f.conv2d_keyswitches(lay, case["w"][0], case["w"][2], 1, case["pad"])
                ks[p] = a + b
        assert inner + outer == min(ks.values()) and nb == min(p for p in ks if ks[p] == min(ks.values()))
    ref = cnn_ref.conv2d(x, w, 1, case["pad"])
    assert np.max(np.abs(f.decrypt(yf) - ref)) < 1e-4
