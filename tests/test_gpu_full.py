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
    x, w = W.lenet_inputs(64)
    lay = fe.plan_layout(64, 1, 28, 28, 5, 6)
    ct = fe.encrypt(fe.encode_fragment(x, lay), lay, W.SEED_ENC)
    torch.cuda.synchronize()
    return fe, x, w, lay, ct


def test_lenet_decrypts_to_float64_cnn(lenet):
    from oracle import cnn_ref
    from paper_2606_16359_amd import workloads as W
    fe, x, w, lay, ct = lenet
    assert lay.S == 2 and lay.n_ct() == 4          # planner: S = 2 fills the slots (eq. opt)
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


def test_lenet_first_layer_matches_oracle_at_full_size(lenet):
    """Encryption and the whole first convolution (4 -> 24 ciphertexts, 32
    hoisted key switches) at N = 2^15, 20 limbs, element by element."""
    from oracle import pyoracle as P
    from paper_2606_16359_amd import workloads as W
    fe, x, w, lay, ct = lenet
    o = P.Oracle(*W.PARAMS["lenet"])
    Lo = o.plan_layout(64, 1, 28, 28, 5, 6)
    ob = o.encrypt_tensor(Lo, x, W.SEED_ENC)
    assert np.array_equal(fe.export(ct), ob.data())
    yo, cnt = o.conv2d(ob, w[0], hoist=fe.hoist)
    y = fe.conv2d(ct, w[0])
    assert cnt["ks"] == 32
    assert np.array_equal(fe.export(y), yo.data())


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
    for b, (blk, w, ((c, h, wd), S)) in enumerate(zip(W.MOBILENET_BLOCKS, ws, W.MOBILENET_INPUTS)):
        assert x.shape[1:] == (c, h, wd)
        lay = fe.plan_layout(2, c, h, wd, blk[0]["w"][2], blk[0]["w"][0], S)
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
