"""The layer-chain block-size planner (the paper adapts the block size between
layers, Evaluation Methodology; eq. total-rot prices one layer).

Its key-switch counts are checked against the library's own runs and the
oracle's (whose convolution counts the oracle tests pin to eq. inner /
outer-rot and to brute force), repack counts against a brute-force count of
rot-mask-add shifts over the oracle's slot map, the planner's choice against
brute force over the input block size, and a chain run at the planned block
size bit for bit against the oracle.
"""
import numpy as np
import pytest

from fenc_backends import BACKENDS, make, rng
from oracle import cnn_ref
from oracle import pyoracle as P
from paper_2606_16359_amd import fenc as F
from test_parity import SMALL, cmp

CONV_CASES = [
    dict(x=(2, 4, 8, 8), w=(4, 4, 3, 3), stride=2, pad=1, groups=1, S=2),
    dict(x=(2, 4, 8, 8), w=(4, 1, 3, 3), stride=1, pad=1, groups=4, S=2),
    dict(x=(2, 3, 8, 8), w=(5, 3, 3, 3), stride=1, pad=1, groups=1, S=1),
    dict(x=(16, 2, 8, 8), w=(5, 2, 5, 5), stride=1, pad=0, groups=1, S=1),
    dict(x=(1, 1, 12, 12), w=(6, 1, 5, 5), stride=1, pad=0, groups=1, S=1),
    dict(x=(2, 4, 8, 8), w=(6, 4, 1, 1), stride=1, pad=0, groups=1, S=1),
    dict(x=(4, 2, 16, 16), w=(4, 2, 3, 3), stride=1, pad=1, groups=1, S=4),
]


@pytest.fixture(scope="module")
def orc():
    return P.Oracle(*SMALL)


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_keyswitch_counts_match_runs(backend, case, orc):
    """fenc_conv2d_keyswitches (no build) equals the key switches the library
    performs and the oracle's rotation counts, in both hoisting schedules."""
    f = make(backend, *SMALL)
    r = rng(21)
    x, w = r.uniform(0, 1, case["x"]), r.normal(0, 0.1, case["w"])
    lay = f.plan_layout(*case["x"], case["w"][2], case["w"][0], case["S"])
    ct = f.encrypt(f.encode_fragment(x, lay), lay, 5)
    inner, outer, terms = f.conv2d_keyswitches(lay, case["w"][0], case["w"][2], case["stride"], case["pad"],
                                               case["groups"])
    ob = orc.encrypt_tensor(orc.fragment_layout(*case["x"], case["S"]), x, 5)
    f.set_plaintext_budget(0)   # the mask-basis form, whose scalar terms the count gives
    for hoist in (0, 1):
        f.set_hoisting(hoist)
        f.stats_reset()
        f.conv2d(ct, w, case["stride"], case["pad"], case["groups"])
        st = f.stats()
        assert (st["rot_inner"], st["rot_outer"], st["keyswitch"], st["smult"]) == (inner, outer, inner + outer, terms)
        _, cnt = orc.conv2d(ob, w, case["stride"], case["pad"], case["groups"], hoist=hoist)
        assert (cnt["inner_rot"], cnt["outer_rot"]) == (inner, outer)


def _brute_repack_shifts(o, Ls, Ld, shape):
    """Distinct (source ciphertext, shift != 0) over every element, from the
    oracle's own slot map: the rotations a rot-mask-add repack needs."""
    bs, c, h, w = shape
    ns = o.ns
    pairs = set()
    for b in range(bs):
        for ch in range(c):
            for y in range(h):
                for x in range(w):
                    (s_ct, s_sl) = o.element_slots(Ls, b, ch, y, x)[0]
                    for (_, d_sl) in o.element_slots(Ld, b, ch, y, x):
                        delta = (s_sl - d_sl) % ns
                        if delta:
                            pairs.add((s_ct, delta))
    return len(pairs)


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("shape,S,S2", [((2, 2, 8, 8), 1, 2), ((2, 2, 8, 8), 2, 1), ((1, 3, 8, 8), 2, 4),
                                        ((4, 1, 12, 12), 4, 2)])
def test_repack_keyswitch_counts_match_brute_force(backend, shape, S, S2, orc):
    """A block-size change S -> S2 (rot-mask-add into a fragment target):
    fenc_compress_keyswitches equals the library's run, the oracle's run and
    a brute-force count over the oracle's slot map; the repacked tensor
    decrypts to the input (one level, at the input's values)."""
    f = make(backend, *SMALL)
    x = rng(22).uniform(0, 1, shape)
    lay = f.plan_layout(*shape, 3, 2, S)
    tgt = f.plan_layout(*shape, 3, 2, S2)
    ct = f.encrypt(f.encode_fragment(x, lay), lay, 7)
    ks = f.compress_keyswitches(lay, tgt)
    f.set_hoisting(1)
    f.stats_reset()
    y = f.compress(ct, target=tgt)
    assert f.stats()["keyswitch"] == ks
    Ls, Ld = orc.fragment_layout(*shape, S), orc.fragment_layout(*shape, S2)
    assert ks == _brute_repack_shifts(orc, Ls, Ld, shape)
    yo, cnt = orc.compress(orc.encrypt_tensor(Ls, x, 7), target=Ld, hoist=1)
    assert cnt["ks"] == ks
    cmp(y, yo, f)
    assert y.lay.S == S2 and np.max(np.abs(f.decrypt(y) - x)) < 1e-4


def _walk(f, bs, shape, layers, S0):
    """(key switches, MAC terms) of a chain run at input block size S0
    without repacks, from the per-layer counting calls (brute force for the
    planner): convolutions, S = 1 pools (three rotations per ciphertext),
    activations (a relinearisation per ciphertext, two for degree 3), the
    final compression."""
    c, h, w = shape
    lay = f.plan_layout(bs, c, h, w, 1, 1, S0)
    ks = terms = 0
    for ly in layers:
        if ly["kind"] == "conv":
            i, o, t = f.conv2d_keyswitches(lay, ly["cout"], ly["k"], ly.get("stride", 1), ly.get("pad", 0),
                                           ly.get("groups", 1))
            ks, terms = ks + i + o, terms + t
            lay = f.conv2d_layout(lay, ly["cout"], ly["k"], ly.get("stride", 1), ly.get("pad", 0), ly.get("groups", 1))
        elif ly["kind"] == "act":
            ks += lay.n_ct() * (2 if ly.get("k", 2) >= 3 else 1)
        elif ly["kind"] == "pool":
            if lay.S == 1:
                ks += 3 * lay.n_ct()
            lay = f.avgpool2_layout(lay)
        elif ly["kind"] == "compress":
            ks += f.compress_keyswitches(lay)
    return ks, terms


def _cost(ks, terms):
    return ks + terms / 16.0


def test_planner_minimises_chain_cost_over_input_block_sizes():
    """At the LeNet, CIFAR and MobileNet benchmark parameters (host-only
    planning): the planner's choice minimises key switches + MAC terms / 16
    over input block sizes, the chain counted layer by layer; allowing
    repacks never raises it.  MobileNet blocks take S = 8, 4, 4 (the key
    switches fall, the MAC terms stay); LeNet keeps S = 2, where S = 4 would
    save key switches but replicate its single input channel four times per
    ciphertext and quadruple the masked MAC terms."""
    from paper_2606_16359_amd import workloads as W
    f = make("emu", *W.PARAMS["lenet"])
    S, ks, terms = f.plan_network(64, (1, 28, 28), W.LENET_LAYERS, 0)
    walks = {}
    for S0 in (1, 2, 4, 8, 16):
        try:
            walks[S0] = _walk(f, 64, (1, 28, 28), W.LENET_LAYERS, S0)
        except F.FencError:   # block size not admissible for this chain
            pass
    assert (ks, terms) == walks[S[0]]
    assert _cost(ks, terms) == min(_cost(*v) for v in walks.values())
    assert S[0] == 2 and walks[4][0] < walks[2][0] and walks[4][1] > 3 * walks[2][1]
    assert _cost(*f.plan_network(64, (1, 28, 28), W.LENET_LAYERS, 1)[1:]) <= _cost(ks, terms)
    g = make("emu", *W.PARAMS["cifar"])
    chosen = []
    for b in range(3):
        layers = W.mobilenet_layers(b)
        S, ks, terms = g.plan_network(64, W.MOBILENET_INPUTS[b], layers, 0)
        walks = {}
        for S0 in (1, 2, 4, 8, 16):
            try:
                walks[S0] = _walk(g, 64, W.MOBILENET_INPUTS[b], layers, S0)
            except F.FencError:
                pass
        assert (ks, terms) == walks[S[0]]
        assert _cost(ks, terms) == min(_cost(*v) for v in walks.values())
        chosen.append(S[0])
    assert chosen == [8, 4, 4]


@pytest.mark.parametrize("backend", BACKENDS)
def test_planned_chain_bit_exact_with_predicted_key_switches(backend, orc):
    """A LeNet-shaped chain at N = 2^10 encoded at the planner's input block
    size: every layer equals the oracle word for word, the library performs
    exactly the key switches the planner predicted (convolutions, pools,
    compression), the oracle's counts agree, and the output decrypts to the
    float64 network."""
    f = make(backend, *SMALL)
    f.set_hoisting(1)
    r = rng(23)
    x = r.uniform(0, 1, (4, 1, 14, 14))
    w1, w2 = r.normal(0, 0.1, (3, 1, 3, 3)), r.normal(0, 0.1, (4, 3, 3, 3))
    layers = [dict(kind="conv", cout=3, k=3), dict(kind="act"), dict(kind="pool"),
              dict(kind="conv", cout=4, k=3), dict(kind="act"), dict(kind="pool"), dict(kind="compress")]
    S, ks, _ = f.plan_network(4, (1, 14, 14), layers, 0)
    lay = f.plan_layout(4, 1, 14, 14, 3, 3, S[0])
    Lo = orc.fragment_layout(4, 1, 14, 14, S[0])
    fb, ob = f.encrypt(f.encode_fragment(x, lay), lay, 3), orc.encrypt_tensor(Lo, x, 3)
    f.stats_reset()
    steps = [(lambda c: f.conv2d(c, w1), lambda b: orc.conv2d(b, w1, hoist=1)),
             (f.poly_act, orc.square), (f.avgpool2, lambda b: orc.avgpool2(b, 1)),
             (lambda c: f.conv2d(c, w2), lambda b: orc.conv2d(b, w2, hoist=1)),
             (f.poly_act, orc.square), (f.avgpool2, lambda b: orc.avgpool2(b, 1)),
             (f.compress, lambda b: orc.compress(b, hoist=1))]
    orc_ks = 0
    for i, (fl, ol) in enumerate(steps):
        assert fb.lay.S == S[i]
        fb = fl(fb)
        ob, cnt = ol(ob)
        cmp(fb, ob, f)
        orc_ks += cnt["ks"]
    assert f.stats()["keyswitch"] == ks == orc_ks
    ref = cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(x, w1))), w2)))
    assert np.max(np.abs(f.decrypt(fb).reshape(ref.shape) - ref)) < 1e-4
