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
    yo, cnt = o.conv2d(ob, w[0])
    y = fe.conv2d(ct, w[0])
    assert cnt["ks"] == 32
    assert np.array_equal(fe.export(y), yo.data())
