"""Full-size runs on the MI355X (LeNet-5-shaped benchmark configuration)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lenet():
    import torch
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["lenet"])
    W.bench_config(fe)   # the benchmark's per-layer schedule choice
    x, w = W.lenet_inputs(64)
    lay = W.lenet_layout(fe, 64)          # the benchmark's block size (chain planner)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    torch.cuda.synchronize()
    return fe, x, w, lay, ct


def test_lenet_decrypts_to_float64_cnn(lenet):
    from oracle import cnn_ref
    from paper_2606_16359_amd import workloads as W
    fe, x, w, lay, ct = lenet
    # chain planner: S = 2 (S = 4 would save key switches but replicate the
    # single input channel four times per ciphertext and quadruple the MAC terms)
    assert lay.S == 2 and lay.n_ct() == 4
    out = W.lenet_forward(fe, ct, w)
    got = fe.decrypt(out).reshape(64, 10)
    want = cnn_ref.lenet(x, *w).reshape(64, 10)
    assert np.max(np.abs(got - want)) < 1e-4


def test_lenet_modes_and_graph_replays_are_bit_identical(lenet):
    import torch
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe, x, w, lay, ct = lenet
    ref = fe.export(W.lenet_forward(fe, ct, w))
    fe.set_mode(F.FENC_MODE_PER_OP)
    assert np.array_equal(fe.export(W.lenet_forward(fe, ct, w)), ref)
    fe.set_mode(F.FENC_MODE_BATCHED)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = W.lenet_forward(fe, ct, w)
    for _ in range(3):       # replays interleaved with eager work
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(fe.export(out), ref)
        assert np.array_equal(fe.export(W.lenet_forward(fe, ct, w)), ref)


def test_graph_replay_survives_workspace_growth():
    """A captured rescale keeps its workspace when a much larger operation in
    the same context later grows the arena: chunks used during a capture are
    never returned, so replays after the growth still give the eager result."""
    import torch
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["lenet"])
    W.bench_config(fe)   # the benchmark's per-layer schedule choice
    x, w = W.lenet_inputs(64)
    lay = fe.plan_layout(64, 1, 28, 28, 5, 6)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    ref = fe.export(fe.rescale(ct))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = fe.rescale(ct)
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(fe.export(out), ref)
    before = fe.device_bytes()
    y = W.lenet_forward(fe, ct, w)          # hundreds of MB of workspace
    torch.cuda.synchronize()
    assert fe.device_bytes() > before
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(fe.export(out), ref)
    assert fe.export(y).shape[0] == y.n_ct


def test_lenet_every_layer_matches_oracle_at_full_size(lenet):
    """The whole LeNet-shaped network at N = 2^15, 20 limbs, 64 images, element
    by element after every layer: encryption, conv1 (32 hoisted key switches),
    x^2, the fragment-sum pool, conv2 (144), x^2, the rotation pool (48),
    compression (15) and the three FC layers.  The oracle runs its own chain
    from its own encryption (a thread per independent ciphertext)."""
    import time
    from oracle import pyoracle as P
    from paper_2606_16359_amd import workloads as W
    fe, x, w, lay, ct = lenet
    o = P.Oracle(*W.PARAMS["lenet"])
    ob = o.encrypt_tensor(o.fragment_layout(64, 1, 28, 28, lay.S), x, W.SEED_ENC)
    assert np.array_equal(fe.export(ct), ob.data())
    # h: the schedule the library's layer ran with
    steps = [("conv1", lambda c: fe.conv2d(c, w[0]), lambda b, h: o.conv2d(b, w[0], hoist=h, baby=fe.last_baby_step())),
             ("x^2", lambda c: fe.poly_act(c), lambda b, h: o.poly_act(b, [0.0, 0.0, 1.0])),
             ("pool1", fe.avgpool2, lambda b, h: o.avgpool2(b, hoist=h)),
             ("conv2", lambda c: fe.conv2d(c, w[1]), lambda b, h: o.conv2d(b, w[1], hoist=h, baby=fe.last_baby_step())),
             ("x^2", lambda c: fe.poly_act(c), lambda b, h: o.poly_act(b, [0.0, 0.0, 1.0])),
             ("pool2", fe.avgpool2, lambda b, h: o.avgpool2(b, hoist=h)),
             ("compress", fe.compress, lambda b, h: o.compress(b, hoist=h)),
             ("fc1", lambda c: fe.fc(c, w[2]), lambda b, h: o.fc(b, w[2])),
             ("fc2", lambda c: fe.fc(c, w[3]), lambda b, h: o.fc(b, w[3])),
             ("fc3", lambda c: fe.fc(c, w[4]), lambda b, h: o.fc(b, w[4]))]
    y, yo = ct, ob
    for name, lib_op, orc_op in steps:
        t0 = time.time()
        y = lib_op(y)
        yo, cnt = orc_op(yo, fe.last_hoisting())
        got, want = fe.export(y), yo.data()
        print(f"{name}: {want.shape[0]} cts, oracle {time.time() - t0:.1f}s, {cnt['ks']} key switches", flush=True)
        assert got.shape == want.shape, name
        assert np.array_equal(got, want), name


def _container(layout, n, level):
    """An oracle layout dict holding n ciphertexts of `layout` at `level` (for
    per-ciphertext operations on sampled outputs)."""
    d = dict(layout)
    d.update(nbg=n, ncg=1, S=1, level=level)
    return d


def test_cifar_first_layer_and_cubic_sampled_cones_match_oracle():
    """CIFAR-shaped stack at its real parameters (256 images, N = 2^16, 24 limbs,
    dnum 4): the first layer (S = 4, C' = 2: masks, hoisted inner rotations,
    one outer rotation per output) and its cubic activation, compared element
    by element on seeded sampled output ciphertexts whose input cones the
    oracle recomputes; sampled input ciphertexts equal the oracle's own
    encryption."""
    import time
    from oracle import pyoracle as P
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["cifar"])
    W.bench_config(fe)
    o = P.Oracle(*W.PARAMS["cifar"])
    x, w = W.cifar_inputs(256)
    lay = fe.plan_layout(256, 16, 32, 32, 3, 16)
    Lo = o.plan_layout(256, 16, 32, 32, 3, 16)
    assert (lay.S, lay.chan_per_ct, lay.n_ct()) == (Lo["S"], Lo["cpc"], 128) == (4, 2, 128)
    pt = fe.encode_fragment(x, lay)
    ct = fe.encrypt(pt, lay, W.SEED_ENC)
    xin = fe.export(ct)
    for t in (0, 77, 127):
        assert np.array_equal(xin[t], o.encrypt(pt[t], Lo["level"], Lo["scale"], W.SEED_ENC, t))
    outs = sorted(np.random.default_rng(2026).choice(128, 2, replace=False).tolist())
    y = fe.conv2d(ct, w[0], pad=1)
    t0 = time.time()
    yo, cnt = o.conv2d(o.batch(Lo, xin), w[0], 1, 1, 1, hoist=fe.last_hoisting(), outputs=outs,
                       baby=fe.last_baby_step())
    print(f"oracle cone of outputs {outs} (schedule {fe.last_hoisting()}): {cnt}, {time.time() - t0:.1f}s",
          flush=True)
    del xin
    assert np.array_equal(fe.export(y)[outs], yo)
    z = fe.export(fe.poly_act(y, W.CUBIC))[outs]
    t0 = time.time()
    zo, _ = o.poly_act(o.batch(_container(Lo, len(outs), y.lay.level), yo), W.CUBIC)
    print(f"oracle cubic on the sampled outputs: {time.time() - t0:.1f}s", flush=True)
    assert np.array_equal(z, zo.data())


def test_mobilenet_block_a_sampled_cones_match_oracle():
    """MobileNet-V1 block A at ImageNet shape as the benchmark runs it
    (224x224x3, conv 3->32 stride 2, 64 images at the planned block size,
    N = 2^16, 24 limbs) and its quadratic, compared element by element on
    seeded sampled output ciphertexts."""
    import time
    from oracle import pyoracle as P
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["cifar"])
    W.bench_config(fe)
    o = P.Oracle(*W.PARAMS["cifar"])
    blk = W.MOBILENET_BLOCKS[0][0]
    wa = W.mobilenet_weights()[0][0]
    x = W.images((64, 3, 224, 224))
    lay = W.mobilenet_layout(fe, 0, 64)
    Lo = o.fragment_layout(64, 3, 224, 224, lay.S)
    assert (lay.bs_g, lay.chan_per_ct, lay.n_ct()) == (Lo["bsg"], Lo["cpc"], Lo["nbg"] * Lo["ncg"] * lay.S ** 2)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    xin = fe.export(ct)
    y = fe.conv2d(ct, wa, stride=blk["stride"], pad=blk["pad"])
    outs = sorted(np.random.default_rng(2027).choice(y.n_ct, 2, replace=False).tolist())
    t0 = time.time()
    yo, cnt = o.conv2d(o.batch(Lo, xin), wa, blk["stride"], blk["pad"], 1, hoist=fe.last_hoisting(), outputs=outs,
                       baby=fe.last_baby_step())
    print(f"oracle cone of outputs {outs} (schedule {fe.last_hoisting()}): {cnt}, {time.time() - t0:.1f}s",
          flush=True)
    del xin
    assert np.array_equal(fe.export(y)[outs], yo)
    z = fe.export(fe.poly_act(y, W.QUADRATIC))[outs]
    zo, _ = o.poly_act(o.batch(_container(Lo, len(outs), y.lay.level), yo), W.QUADRATIC)
    assert np.array_equal(z, zo.data())


def test_cifar_stack_full_size_decrypts_to_float64():
    """CIFAR-shaped stack at its full size: 256 images 16x32x32, N = 2^16, 24 limbs,
    dnum 4; three 3x3 convs 16->16, a stride-2 conv 16->32, a conv 32->32, each
    followed by the cubic activation (two levels each)."""
    import time
    import torch
    from oracle import cnn_ref
    from oracle import pyoracle as P
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["cifar"])
    x, w = W.cifar_inputs(256)
    lay = fe.plan_layout(256, 16, 32, 32, 3, 16)
    ol = P.Oracle(*W.PARAMS["cifar"]).plan_layout(256, 16, 32, 32, 3, 16)
    assert (lay.S, lay.n_ct()) == (ol["S"], ol["nbg"] * ol["ncg"] * ol["S"] ** 2) == (4, 128)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    t0 = time.time()
    out = W.cifar_forward(fe, ct, w)
    torch.cuda.synchronize()
    print(f"cifar stack first pass (plans, keys) {time.time() - t0:.2f}s", flush=True)
    t0 = time.time()
    out = W.cifar_forward(fe, ct, w)
    torch.cuda.synchronize()
    print(f"cifar stack {time.time() - t0:.3f}s for 256 images, {fe.stats()}", flush=True)
    ref = x
    for wi, s in zip(w, W.CIFAR_STRIDES):
        ref = np.polynomial.polynomial.polyval(cnn_ref.conv2d(ref, wi, s, 1), W.CUBIC)
    assert out.lay.level == 23 - 15
    assert np.max(np.abs(fe.decrypt(out) - ref)) < 1e-4


def test_mobilenet_blocks_at_imagenet_shape_decrypt_to_float64():
    """MobileNet-V1-shaped early blocks at 224x224 (N = 2^16, 24 limbs), each from
    a fresh encryption of the float64 output of the previous block, 2 images."""
    import time
    import torch
    from oracle import cnn_ref
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["cifar"])
    ws = W.mobilenet_weights()
    x = W.images((2, 3, 224, 224))
    for b, (blk, w, (c, h, wd)) in enumerate(zip(W.MOBILENET_BLOCKS, ws, W.MOBILENET_INPUTS)):
        assert x.shape[1:] == (c, h, wd)
        lay = W.mobilenet_layout(fe, b, 2)
        ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC + b)
        t0 = time.time()
        y = W.mobilenet_block(fe, ct, blk, w)
        torch.cuda.synchronize()
        print(f"block {b}: {lay.n_ct()} input cts, S={lay.S}, {time.time() - t0:.2f}s (first run)", flush=True)
        ref = x
        for layer, wi in zip(blk, w):
            ref = np.polynomial.polynomial.polyval(
                cnn_ref.conv2d(ref, wi, layer["stride"], layer["pad"], layer["groups"]), W.QUADRATIC)
        got = fe.decrypt(y)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) < 1e-4, (b, np.max(np.abs(got - ref)))
        x = ref


def test_bert_ffn_block_on_token_fragments_decrypts_to_float64():
    """The BERT-base-shaped feed-forward block of the benchmark (128 tokens,
    768 -> 3072 -> 768 with biases, x^2 between, S = 4, N = 2^16): the
    output decrypts to the float64 block; a second pass is bit-identical."""
    import time
    import torch
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["ffn"])
    W.bench_config(fe)
    x, w = W.ffn_inputs()
    lay = fe.plan_tokens(W.FFN_TOKENS, W.FFN_E, W.FFN_S)
    assert (lay.kind, lay.S, lay.bs_g, lay.d, lay.n_ct()) == (2, 4, 128, 256, 4)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    t0 = time.time()
    out = W.ffn_forward(fe, ct, w)
    torch.cuda.synchronize()
    print(f"ffn first pass (plans, keys) {time.time() - t0:.2f}s", flush=True)
    fe.stats_reset()
    t0 = time.time()
    again = W.ffn_forward(fe, ct, w)
    torch.cuda.synchronize()
    print(f"ffn {time.time() - t0:.3f}s for 128 tokens, {fe.stats()}", flush=True)
    assert np.array_equal(fe.export(out), fe.export(again))
    got = fe.decrypt(out).reshape(W.FFN_TOKENS, W.FFN_E)
    ref = W.ffn_reference(x, w)
    assert np.max(np.abs(got - ref)) < 1e-4, np.max(np.abs(got - ref))


def _orc_layout(lay):
    """The oracle's layout dict of a library layout (token and vector kinds)."""
    return {"kind": lay.kind, "bs": lay.bs, "c": lay.c, "h": lay.h, "w": lay.w, "M": lay.M, "S": lay.S, "m": lay.m,
            "bsg": lay.bs_g, "cpc": lay.chan_per_ct, "nbg": lay.n_bg, "ncg": lay.n_cg, "rep": lay.replicate,
            "dil": lay.dil, "level": lay.level, "d": lay.d, "nfeat": lay.n_feat, "scale": lay.scale, "pos": None}


def test_bert_ffn_sampled_outputs_match_oracle_at_full_size():
    """Both linear layers of the BERT-base-shaped feed-forward block at their
    benchmark size (128 tokens, 768 -> 3072 -> 768, S = 4, N = 2^16): the
    last output ciphertext of the first and the first of the second (other
    fragments and chunks) equal, word for word, the oracle computing just
    that output from the library's own input words (every input ciphertext
    with the baby steps the output uses)."""
    import time
    import torch
    from oracle import pyoracle as P
    from paper_2606_16359_amd import fenc as F
    from paper_2606_16359_amd import workloads as W
    fe = F.Fenc(*W.PARAMS["ffn"])
    W.bench_config(fe)
    o = P.Oracle(*W.PARAMS["ffn"])
    x, w = W.ffn_inputs()
    lay = fe.plan_tokens(W.FFN_TOKENS, W.FFN_E, W.FFN_S)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    h = fe.fc(ct, w[0], bias=w[1])
    a = fe.poly_act(h)
    y = fe.fc(a, w[2], bias=w[3])
    torch.cuda.synchronize()
    for src, out, wi, bi, pick in ((ct, h, w[0], w[1], [h.lay.n_ct() - 1]), (a, y, w[2], w[3], [0])):
        t0 = time.time()
        ref, _ = o.fc(o.batch(_orc_layout(src.lay), fe.export(src)), wi, bias=bi, outputs=pick)
        print(f"oracle fc {wi.shape}: output {pick} of {out.lay.n_ct()} in {time.time() - t0:.1f}s", flush=True)
        assert np.array_equal(fe.export(out)[pick], ref)
