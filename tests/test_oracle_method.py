"""Pins of the oracle's method layer (fragment layout, planner, HE layers).

Expected values come from the paper's printed numbers (optimal-S table,
Fig. 2x2 toy, Theorem 1 worked example, slot-utilisation examples) or from a
float64 numpy CNN, never from the oracle itself.
"""
import json
import os

import numpy as np
import pytest

from oracle import pyoracle as P
from oracle import cnn_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_optimal_s_table_rotation_counts():
    """Every #Rot entry of the block-size table (N = 2^15, 32x32 maps, alpha = 16)."""
    g = load_golden("optimal_s_table.json")
    for row in g["rows"]:
        for S, rot in zip(row["S"], row["rot"]):
            assert P.rot_total_formula(row["BS"], row["Nin"], row["Nout"], row["K"], S, g["alpha"]) == rot
        o = P.Oracle(15, 2, 50, 1, 50, 2, 40, 1) if row is g["rows"][0] else o
        lay = o.plan_layout(row["BS"], row["Nin"], 32, 32, row["K"], row["Nout"])
        best = min(zip(row["rot"], row["S"]))[1]
        assert lay["S"] == best == row["best_S"]


def test_fig_2x2_toy_rotation_counts():
    """1x16x4x4 input, conv (16,16,3), BS=1, 16-slot ciphertexts: S=2 optimal."""
    g = load_golden("fig_2x2_toy.json")
    got = [P.rot_total_formula(1, 16, 16, 3, S, g["alpha"]) for S in g["S"]]
    assert got == g["rot"]
    assert g["S"][int(np.argmin(got))] == g["optimal_S"]
    S = 2   # inner and outer balanced at the optimum
    inner = 1 / g["alpha"] * (np.ceil(3 / S) ** 2 - 1) * 16
    outer = 1 / g["alpha"] * (g["alpha"] * S * S / 1 - 1) * 16
    assert inner == outer == g["inner_outer_at_optimum"]


def test_theorem1_worked_example():
    """Conv(128,32,9) on (8,128,32,32) at N=2^15: S* = 3.57, best block size 4."""
    assert abs(P.optimal_S(9, 128, 32, 16, 8) - 3.57) < 0.005


def test_slot_utilisation_example():
    """4x4 single-channel map in 4-slot ciphertexts: S=2 gives 4 full cts, S=4 gives 16."""
    o = P.Oracle(3, 2, 30, 1, 30, 2, 20, 1)   # N = 8 -> 4 slots
    assert o.ns == 4
    l2 = o.fragment_layout(1, 1, 4, 4, 2)
    l4 = o.fragment_layout(1, 1, 4, 4, 4)
    n = lambda L: L["nbg"] * L["ncg"] * L["S"] ** 2
    assert n(l2) == 4 and n(l4) == 16
    # equ. (opt): S <= sqrt(BS*N_in/alpha) = sqrt(1*1/(4/16)) = 2 -> the planner keeps S = 2
    assert o.plan_layout(1, 1, 4, 4, 3, 1)["S"] == 2


def all_slots(o, L):
    seen = {}
    for b in range(L["bs"]):
        for c in range(L["c"]):
            for h in range(L["h"]):
                for w in range(L["w"]):
                    seen[(b, c, h, w)] = o.element_slots(L, b, c, h, w)
    return seen


def test_slot_map_row_major_and_pixel_wise_special_cases():
    o = P.Oracle(9, 2, 30, 1, 30, 2, 20, 1)   # 256 slots
    # S = 1, BS = 1: row-major, channel after channel (CHET / Orion style)
    L = o.fragment_layout(1, 4, 8, 8, 1)
    for (b, c, h, w), sl in all_slots(o, L).items():
        assert sl[0] == (c // L["cpc"], (c % L["cpc"]) * 64 + h * 8 + w)
    # S = M: every ciphertext holds one pixel position of all channels and images (CryptoNets)
    L = o.fragment_layout(4, 8, 8, 8, 8)
    for (b, c, h, w), sl in all_slots(o, L).items():
        ct, slot = sl[0]
        assert ct == (c // L["cpc"]) * 64 + h * 8 + w and slot == (c % L["cpc"]) * 4 + b


@pytest.mark.parametrize("shape,S", [((3, 5, 28, 28), 2), ((64, 1, 28, 28), 2), ((2, 16, 16, 16), 4),
                                     ((1, 1, 28, 28), 1)])
def test_slot_map_is_injective(shape, S):
    o = P.Oracle(13, 2, 30, 1, 30, 2, 20, 1)
    L = o.fragment_layout(*shape, S)
    used = set()
    for sl in all_slots(o, L).values():
        for p in sl:
            assert p not in used and 0 <= p[1] < o.ns
            used.add(p)


def test_planner_choices_for_the_benchmark_shapes():
    o13 = P.Oracle(13, 4, 40, 1, 40, 4, 30, 1)
    L = o13.plan_layout(1, 1, 28, 28, 5, 6)
    assert (L["S"], L["cpc"], L["rep"], L["M"]) == (1, 4, 1, 32)          # replicated channel
    o15 = P.Oracle(15, 2, 50, 1, 50, 2, 40, 1)
    L = o15.plan_layout(64, 1, 28, 28, 5, 6)
    assert (L["S"], L["cpc"], L["bsg"]) == (2, 1, 64)                     # 4 fragment cts
    o16 = P.Oracle(16, 2, 50, 1, 50, 2, 40, 1)
    L = o16.plan_layout(256, 16, 32, 32, 3, 16)
    assert (L["S"], L["cpc"], L["bsg"]) == (4, 2, 256)
    assert L["nbg"] * L["ncg"] * L["S"] ** 2 == 128


# ---------------------------------------------------------------- encrypted layers

def small_oracle(nq=8, logN=10):
    return P.Oracle(logN, nq, 50, 3, 50, 3, 40, 17)   # special primes >= limbs per digit


def rand_x(shape, seed):
    return np.random.default_rng(seed).uniform(0, 1, shape)


def rand_w(shape, seed):
    return np.random.default_rng(seed).normal(0, 0.1, shape)


@pytest.mark.parametrize("case", [
    dict(x=(4, 1, 14, 14), w=(3, 1, 3, 3), stride=1, pad=0, groups=1, S=2),   # C'=2, replicated
    dict(x=(2, 3, 8, 8), w=(4, 3, 3, 3), stride=1, pad=1, groups=1, S=1),     # same padding, masks
    dict(x=(2, 4, 8, 8), w=(4, 4, 3, 3), stride=2, pad=1, groups=1, S=2),     # stride by discard
    dict(x=(2, 4, 8, 8), w=(4, 1, 3, 3), stride=1, pad=1, groups=4, S=2),     # depthwise
    dict(x=(16, 2, 8, 8), w=(5, 2, 5, 5), stride=1, pad=0, groups=1, S=1),    # C'=1, no masks
])
@pytest.mark.parametrize("budget", [1 << 30, 0])
@pytest.mark.parametrize("hoist", [0, 1])
def test_conv2d_decrypts_to_float64_conv(case, hoist, budget):
    o = small_oracle()
    x, w = rand_x(case["x"], 1), rand_w(case["w"], 2)
    L = o.fragment_layout(*case["x"], case["S"])
    b = o.encrypt_tensor(L, x, seed=4)
    y, cnt = o.conv2d(b, w, case["stride"], case["pad"], case["groups"], pt_budget=budget, hoist=hoist)
    got = o.decrypt_tensor(y)
    want = cnn_ref.conv2d(x, w, case["stride"], case["pad"], case["groups"])
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) < 1e-4
    if hoist:
        # the same rotations; each combined diagonal ciphertext moves down once instead of every copy
        _, c0 = o.conv2d(b, w, case["stride"], case["pad"], case["groups"], pt_budget=budget, hoist=0)
        assert (cnt["inner_rot"], cnt["outer_rot"], cnt["ks"]) == (c0["inner_rot"], c0["outer_rot"], c0["ks"])
        n_diag = L["c"] if L["rep"] else L["cpc"]    # diagonals per output ciphertext
        assert cnt["moddown"] <= c0["moddown"] - c0["inner_rot"] + len(y.data()) * n_diag


def test_conv2d_rotation_counts_match_formula_when_kernel_exceeds_block():
    """K > S with full ciphertexts: measured inner/outer rotations equal eq. (inner)/(outer-rot)."""
    o = small_oracle(nq=3, logN=10)    # 512 slots, M = 8 -> alpha = 8
    for (bs, cin, cout, k, S) in [(4, 8, 8, 3, 2), (1, 8, 16, 3, 1), (8, 4, 4, 5, 2)]:
        L = o.fragment_layout(bs, cin, 8, 8, S)
        x, w = rand_x((bs, cin, 8, 8), 3), rand_w((cout, cin, k, k), 4)
        b = o.encrypt_tensor(L, x, seed=1)
        _, cnt = o.conv2d(b, w, 1, k // 2, 1)
        alpha = o.ns / 64
        n_in = bs * cin / alpha
        assert cnt["inner_rot"] == n_in * (np.ceil(k / S) ** 2 - 1)
        assert cnt["outer_rot"] == max(bs * cout / alpha * (alpha * S * S / bs - 1), 0)
        assert cnt["inner_rot"] + cnt["outer_rot"] == P.rot_total_formula(bs, cin, cout, k, S, alpha)


def test_avgpool_square_compress_fc_decrypt_to_float64():
    o = small_oracle()
    x = rand_x((4, 1, 14, 14), 5)
    w1, w2 = rand_w((3, 1, 3, 3), 6), rand_w((4, 3, 3, 3), 7)
    f1, f2 = rand_w((8, 16), 8), rand_w((4, 8), 9)
    L = o.fragment_layout(4, 1, 14, 14, 2)
    b = o.encrypt_tensor(L, x, seed=2)
    b, _ = o.conv2d(b, w1)
    b, _ = o.square(b)
    b, _ = o.avgpool2(b)          # fragment sum
    ref = cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(x, w1)))
    assert np.max(np.abs(o.decrypt_tensor(b) - ref)) < 1e-4
    b, _ = o.conv2d(b, w2)
    b, _ = o.square(b)
    b, cnt = o.avgpool2(b)        # S = 1: hoisted rotations
    assert b.layout()["dil"] == 2 and cnt["other_rot"] > 0
    ref = cnn_ref.avgpool2(cnn_ref.square(cnn_ref.conv2d(ref, w2)))
    assert np.max(np.abs(o.decrypt_tensor(b) - ref)) < 1e-4
    nin = len(b.layout())
    b, cnt = o.compress(b)
    L = b.layout()
    assert L["kind"] == 1 and L["nbg"] == 1 and sorted(set(L["pos"])) == sorted(L["pos"])
    assert np.max(np.abs(o.decrypt_tensor(b).reshape(ref.shape) - ref)) < 1e-4
    b, _ = o.fc(b, f1)
    b, cnt = o.fc(b, f2)
    ref = cnn_ref.fc(cnn_ref.fc(ref, f1), f2)
    assert np.max(np.abs(o.decrypt_tensor(b) - ref)) < 1e-4


def test_compress_bottleneck_example():
    """8 -> 2 -> 8 bottleneck: four 25%-utilised ciphertexts merge into one dense one."""
    o = P.Oracle(6, 3, 50, 1, 50, 3, 40, 3)    # 32 slots
    L = o.fragment_layout(1, 2, 4, 4, 2)       # 2 channels in cts of 8 channel positions
    assert L["nbg"] * L["ncg"] * L["S"] ** 2 == 4
    distinct = 2 * 4 * 4 / (4 * o.ns)
    assert distinct == 0.25
    x = rand_x((1, 2, 4, 4), 1)
    b = o.encrypt_tensor(L, x, seed=3)
    c, cnt = o.compress(b)
    assert len(c.data()) == 1 and c.layout()["nfeat"] == o.ns
    assert np.max(np.abs(o.decrypt_tensor(c).reshape(x.shape) - x)) < 1e-6
    assert c.layout()["level"] == L["level"] - 1     # one level, like one PMult


def test_poly_act_quadratic_with_unit_leading_coefficient_is_the_square():
    """p(x) = x^2 takes exactly the x^2 path (same integer k, same residues)."""
    o = small_oracle()
    x = rand_x((4, 2, 8, 8), 11) - 0.5
    L = o.fragment_layout(4, 2, 8, 8, 2)
    b = o.encrypt_tensor(L, x, seed=5)
    sq, _ = o.square(b)
    pa, cnt = o.poly_act(b, [0.0, 0.0, 1.0])
    assert np.array_equal(sq.data(), pa.data())
    assert sq.layout()["scale"] == pa.layout()["scale"] and cnt["relin"] == len(b.data())


@pytest.mark.parametrize("coeffs", [
    [0.25, -1.5],                            # affine
    [0.1471, 0.5, 0.1196],                   # a x^2 + b x + c, ReLU-shaped
    [-0.3, 0.0, -2.0],                       # negative leading coefficient
    [0.02, 0.5, 0.2, -0.04],                 # cubic
    [0.0, 0.0, 0.0, 1.0],                    # x^3 alone
])
def test_poly_act_decrypts_to_the_polynomial(coeffs):
    o = small_oracle()
    x = 2.0 * rand_x((4, 2, 8, 8), 12) - 1.0
    L = o.fragment_layout(4, 2, 8, 8, 2)
    b = o.encrypt_tensor(L, x, seed=6)
    y, cnt = o.poly_act(b, coeffs)
    deg = len(coeffs) - 1
    Ly = y.layout()
    assert Ly["level"] == L["level"] - (2 if deg == 3 else 1)
    assert abs(np.log2(Ly["scale"]) - np.log2(2.0 ** 40)) < 0.02      # within 1.4% of Delta
    assert cnt["relin"] == len(b.data()) * {1: 0, 2: 1, 3: 2}[deg]
    ref = np.polynomial.polynomial.polyval(x, coeffs)
    assert np.max(np.abs(o.decrypt_tensor(y) - ref)) < 1e-5


def test_avgpool_rotation_sum_in_the_extended_basis():
    """S = 1 average pooling: the three rotations summed before one ModDown decrypt
    to the same mean as the per-rotation form, with one ModDown per ciphertext."""
    o = small_oracle()
    x = rand_x((4, 2, 8, 8), 13)
    L = o.fragment_layout(4, 2, 8, 8, 1)
    b = o.encrypt_tensor(L, x, seed=8)
    y0, c0 = o.avgpool2(b, hoist=0)
    y1, c1 = o.avgpool2(b, hoist=1)
    want = cnn_ref.avgpool2(x)
    for y in (y0, y1):
        assert np.max(np.abs(o.decrypt_tensor(y) - want)) < 1e-6
    assert (c0["moddown"], c1["moddown"]) == (3 * len(b.data()), len(b.data()))


def _border_rotations(L, h, w, k, stride, pad, n_groups):
    """Pixel-level count of the inner rotations a K <= S convolution needs: the
    distinct (input fragment, nonzero block offset) pairs that carry at least
    one valid input pixel to a valid output pixel, times the ciphertexts that
    share a fragment position (channel and batch groups)."""
    S, So = L["S"], L["S"] // stride
    ho, wo = (h + 2 * pad - k) // stride + 1, (w + 2 * pad - k) // stride + 1
    need = set()
    for y in range(ho):
        for x in range(wo):
            for di in range(k):
                for dj in range(k):
                    iy, ix = y * stride + di - pad, x * stride + dj - pad
                    if not (0 <= iy < h and 0 <= ix < w):
                        continue
                    off = (iy // S - y // So, ix // S - x // So)
                    if off != (0, 0):
                        need.add((iy % S, ix % S, off))
    return len(need) * n_groups


@pytest.mark.parametrize("case", [
    dict(x=(2, 2, 8, 8), k=3, S=4, stride=1, pad=1),     # same padding, borders on both sides
    dict(x=(2, 2, 8, 8), k=3, S=4, stride=2, pad=1),     # stride 2 keeps 4 of 16 fragments
    dict(x=(1, 3, 12, 12), k=3, S=4, stride=1, pad=0),   # valid conv, one-sided borders
    dict(x=(2, 1, 8, 8), k=2, S=2, stride=1, pad=0),     # K = S
    dict(x=(4, 2, 8, 8), k=1, S=2, stride=1, pad=0),     # 1x1: no rotation at all
])
def test_conv2d_border_rotations_match_brute_force_when_block_covers_kernel(case):
    """K <= S: eq. (total-rot) counts no inner rotation (the optimal-S table's
    convention); the convolution performs exactly the border rotations found
    by enumerating pixels."""
    o = small_oracle(nq=3, logN=10)
    bs, cin, h, w = case["x"]
    k, S = case["k"], case["S"]
    L = o.fragment_layout(bs, cin, h, w, S)
    b = o.encrypt_tensor(L, rand_x(case["x"], 3), seed=1)
    wt = rand_w((2, cin, k, k), 4)
    y, cnt = o.conv2d(b, wt, case["stride"], case["pad"], 1)
    want = _border_rotations(L, h, w, k, case["stride"], case["pad"], L["nbg"] * L["ncg"])
    assert cnt["inner_rot"] == want
    alpha = o.ns / L["M"] ** 2
    outer_only = bs / alpha * max(alpha * S * S / bs - 1, 0) * 2
    assert P.rot_total_formula(bs, cin, 2, k, S, alpha) == outer_only      # the formula has no inner term
    got = o.decrypt_tensor(y)
    ref = cnn_ref.conv2d(rand_x(case["x"], 3), wt, case["stride"], case["pad"], 1)
    assert np.max(np.abs(got - ref)) < 1e-4


# ---------------------------------------------------------------- Arch-aware Ct Compression

def test_fused_compression_bottleneck_adds_no_level_and_packs_densely():
    """Bottleneck 8 -> 2 -> 8 (Arch-aware Ct Compression, Fig. compression):
    the 1x1 reduction writes its two channels straight into the dense layout
    of the reduced tensor (the two channels repeated in every group of two of
    the eight channel positions), at the level the reduction alone would
    leave (no additional multiplicative depth: the masks multiply the weights'
    plaintexts and share their rescale), with no rotation beyond the
    reduction's own outer rotations.  The expansion layer then needs one outer
    rotation per output ciphertext instead of seven."""
    o = small_oracle(nq=6)                       # N = 2^10: 512 slots
    x = rand_x((4, 8, 4, 4), 21)                 # 8 channels x 16 pixels x 4 images: one full ciphertext
    w1, w2 = rand_w((2, 8, 1, 1), 22), rand_w((8, 2, 1, 1), 23)
    L = o.fragment_layout(4, 8, 4, 4, 1)
    assert (L["cpc"], L["ncg"], L["nbg"]) == (8, 1, 1)
    b = o.encrypt_tensor(L, x, seed=2)
    nat, cn = o.conv2d(b, w1, hoist=1)           # natural output: 2 of 8 positions used
    dense_layout = o.fragment_layout(4, 2, 4, 4, 1)
    assert dense_layout["rep"] == 1 and dense_layout["cpc"] == 8
    fused, cf = o.conv2d(b, w1, hoist=1, target=dense_layout)
    assert fused.layout()["level"] == nat.layout()["level"] == L["level"] - 1
    assert fused.layout()["rep"] == 1 and len(fused.data()) == 1
    assert cf["outer_rot"] == cn["outer_rot"] == 7 and cf["rescale"] == 1
    ref = cnn_ref.conv2d(x, w1)
    assert np.max(np.abs(o.decrypt_tensor(fused) - ref)) < 1e-4
    # every replica holds the value: decrypt the raw slots of the ciphertext
    o2 = o.decrypt_slots(fused)[0]
    for rep in range(4):
        for ch in range(2):
            for img in range(4):
                base = ((rep * 2 + ch) * 16) * 4 + img   # pixel (0, 0)
                assert abs(o2[base] - ref[img, ch, 0, 0]) < 1e-4
    y_nat, c_nat = o.conv2d(nat, w2, hoist=1)
    y_den, c_den = o.conv2d(fused, w2, hoist=1)
    assert (c_nat["outer_rot"], c_den["outer_rot"]) == (7, 1)
    ref2 = cnn_ref.conv2d(ref, w2)
    assert np.max(np.abs(o.decrypt_tensor(y_den) - ref2)) < 1e-4
    assert np.max(np.abs(o.decrypt_tensor(y_nat) - ref2)) < 1e-4


@pytest.mark.parametrize("hoist", [0, 1])
def test_compression_into_fragment_and_vector_targets(hoist):
    """Standalone rot-mask-add into an explicit target: decode(compress(x)) is
    x in the target layout; the masks take one level (no preceding product to
    share a scale with)."""
    o = small_oracle(nq=6)
    x = rand_x((4, 2, 4, 4), 31)
    L = o.fragment_layout(4, 2, 4, 4, 2)         # S = 2: 4 fragment cts, 2 of 32 positions per block used
    b = o.encrypt_tensor(L, x, seed=3)
    for S_t in (1, 2, 4):
        T = o.fragment_layout(4, 2, 4, 4, S_t)
        c, cnt = o.compress(b, target=T, hoist=hoist)
        Lc = c.layout()
        assert (Lc["S"], Lc["rep"], Lc["level"]) == (S_t, T["rep"], L["level"] - 1)
        assert np.max(np.abs(o.decrypt_tensor(c) - x)) < 1e-6
    v, _ = o.compress(b, hoist=hoist)            # default: the first-fit vector
    assert v.layout()["kind"] == 1 and np.max(np.abs(o.decrypt_tensor(v).reshape(x.shape) - x)) < 1e-6


def test_fused_convolution_into_other_block_size_and_vector_layouts():
    """The fused repack also changes the block size (S = 2 -> 1) and writes a
    flattened FC vector, each at the convolution's own level.  A block-size
    change moves every pixel row by its own shift, so it costs many rotations
    (here 114 against the layer's 4 outer rotations)."""
    o = small_oracle(nq=4)
    x = rand_x((8, 2, 8, 8), 41)
    w = rand_w((2, 2, 3, 3), 42)
    ref = cnn_ref.conv2d(x, w, 1, 1)
    L = o.fragment_layout(8, 2, 8, 8, 2)
    b = o.encrypt_tensor(L, x, seed=4)
    y, c = o.conv2d(b, w, 1, 1, 1, hoist=1, target=o.fragment_layout(8, 2, 8, 8, 1))
    assert (y.layout()["S"], y.layout()["level"]) == (1, L["level"] - 1)
    assert np.max(np.abs(o.decrypt_tensor(y) - ref)) < 1e-4
    # S = 1 (one channel per ciphertext, 8 images) into a vector whose feature
    # positions are rotated by five: the moves share a single shift
    L = o.fragment_layout(8, 2, 8, 8, 1)
    b = o.encrypt_tensor(L, x, seed=4)
    w1 = rand_w((1, 2, 3, 3), 43)
    vt = dict(o.fragment_layout(8, 1, 8, 8, 1), kind=1, d=o.ns // 8, nfeat=64, pos=[(f + 5) % 64 for f in range(64)])
    y, c = o.conv2d(b, w1, 1, 1, 1, hoist=1, target=vt)
    assert y.layout()["kind"] == 1 and y.layout()["pos"] == vt["pos"] and c["outer_rot"] == 1
    assert np.max(np.abs(o.decrypt_tensor(y).reshape(8, 1, 8, 8) - cnn_ref.conv2d(x, w1, 1, 1))) < 1e-4


def test_bias_is_added_at_the_output_scale():
    o = small_oracle(nq=6)
    x = rand_x((2, 3, 8, 8), 51)
    w, bias = rand_w((4, 3, 3, 3), 52), np.array([0.5, -0.25, 0.125, 1.0])
    L = o.fragment_layout(2, 3, 8, 8, 2)
    b = o.encrypt_tensor(L, x, seed=5)
    y, _ = o.conv2d(b, w, 1, 1, 1, hoist=1, bias=bias)
    ref = cnn_ref.conv2d(x, w, 1, 1) + bias[None, :, None, None]
    assert np.max(np.abs(o.decrypt_tensor(y) - ref)) < 1e-4
    v, _ = o.compress(y)
    fw, fb = rand_w((5, 256), 53), np.linspace(-1, 1, 5)
    z, _ = o.fc(v, fw, bias=fb)
    assert np.max(np.abs(o.decrypt_tensor(z).reshape(2, 5) - (ref.reshape(2, -1) @ fw.T + fb))) < 1e-4


def test_conv2d_output_subset_equals_the_full_output():
    """Sampled outputs (their input cone only) are the full layer's outputs,
    with and without a bias, under both plaintext forms."""
    o = small_oracle(nq=6)
    x, w = rand_x((4, 4, 8, 8), 61), rand_w((4, 4, 3, 3), 62)
    b = o.encrypt_tensor(o.fragment_layout(4, 4, 8, 8, 2), x, seed=6)
    for budget, bias in [(1 << 30, None), (0, np.arange(4.0))]:
        full, c = o.conv2d(b, w, 1, 1, 1, pt_budget=budget, hoist=1, bias=bias)
        sub, cs = o.conv2d(b, w, 1, 1, 1, pt_budget=budget, hoist=1, bias=bias, outputs=[3, 0])
        assert np.array_equal(sub, full.data()[[3, 0]])
        assert cs["inner_rot"] < c["inner_rot"]


@pytest.mark.parametrize("n1", [1, 2, 4, 16])
@pytest.mark.parametrize("k", [1, 3])
def test_conv2d_bsgs_outer_rotations_counts_and_decryption(k, n1):
    """Outer rotations by baby-step giant-step (Motivation, HE multi-channel
    convolution).  16 channels on 4x4 maps at N = 2^10 (S = 1, m = 4, one image)
    are replicated twice per ciphertext, so C' = 16 diagonals, shifted by
    s = m^2 = 16 slots each.  With baby step n1 an output takes ceil(16/n1) - 1
    giant-step rotations; the input takes one hoisted rotation per distinct
    nonzero shift (kernel shift + i s, i < n1).  Every form decrypts to the
    float64 convolution."""
    o = small_oracle(nq=3, logN=10)
    L = o.fragment_layout(1, 16, 4, 4, 1)
    assert (L["cpc"], L["rep"], L["m"], L["bsg"]) == (32, 1, 4, 1)
    x, w = rand_x((1, 16, 4, 4), 31), rand_w((16, 16, k, k), 32)
    b = o.encrypt_tensor(L, x, seed=3)
    y, cnt = o.conv2d(b, w, 1, k // 2, 1, baby=n1)
    assert cnt["outer_rot"] == -(-16 // n1) - 1
    shifts = {(a * 4 + c + 16 * i) % o.ns for a in range(-(k // 2), k // 2 + 1)
              for c in range(-(k // 2), k // 2 + 1) for i in range(n1)}
    assert cnt["inner_rot"] == len(shifts - {0})
    ref = cnn_ref.conv2d(x, w, 1, k // 2)
    assert np.max(np.abs(o.decrypt_tensor(y) - ref)) < 1e-4


def test_token_fragment_layout_places_features_by_fragment():
    """Token embeddings split into S fragments (Discussions, extensibility to
    Transformers): feature e of token t lies in fragment e mod S at position
    e div S, so a ciphertext holds E/S features of S times more tokens than
    full-embedding packing."""
    o = small_oracle(nq=3, logN=10)
    for n, E, S in [(8, 48, 1), (8, 48, 4), (16, 40, 8), (4, 200, 2)]:
        L = o.token_layout(n, E, S)
        per = -(-E // S)
        d0 = 1 << (per - 1).bit_length()
        assert L["kind"] == 2 and L["d"] * L["bsg"] == o.ns and L["d"] >= min(d0, o.ns)
        assert L["ncg"] == -(-per // L["d"]) and L["nbg"] == -(-n // L["bsg"])
        seen = set()
        for t in range(n):
            for e in range(E):
                (ct, sl), = o.element_slots(L, t, e, 0, 0)
                p = e // S
                assert ct == ((t // L["bsg"]) * S + e % S) * L["ncg"] + p // L["d"]
                assert sl == (p % L["d"]) * L["bsg"] + t % L["bsg"]
                seen.add((ct, sl))
        assert len(seen) == n * E


def test_token_fc_with_one_fragment_is_the_vector_fc():
    """With S = 1 the token layout is the FC vector layout (identity positions):
    the token-fragment linear layer gives the vector FC's words."""
    o = small_oracle(nq=3, logN=10)
    x, w = rand_x((8, 24), 41), rand_w((20, 24), 42)
    Lt = o.token_layout(8, 24, 1)
    Lv = dict(Lt)
    Lv.update(kind=1, pos=list(range(24)))
    yt, ct = o.fc(o.encrypt_tensor(Lt, x.reshape(8, 24, 1, 1), 5), w)
    yv, cv = o.fc(o.encrypt_tensor(Lv, x.reshape(8, 24, 1, 1), 5), w)
    assert np.array_equal(yt.data(), yv.data())
    assert (ct["other_rot"], ct["ks"]) == (cv["other_rot"], cv["ks"])


@pytest.mark.parametrize("n,E,E2,S", [(8, 48, 32, 4), (16, 64, 64, 8), (8, 24, 96, 2), (4, 32, 160, 1)])
def test_token_fc_decrypts_and_counts_rotations(n, E, E2, S):
    """A linear layer E -> E2 (with bias) on token fragments decrypts to
    x W^T + b within 1e-4, also where an output fragment spans several
    ciphertexts; per token group it takes S k_in (n1 - 1) baby-step and
    S k_out (n2 - 1) giant-step rotations, n1 n2 = d."""
    o = small_oracle(nq=3, logN=10)
    x, w, b = rand_x((n, E), 43), rand_w((E2, E), 44), rand_w((E2,), 45)
    L = o.token_layout(n, E, S)
    y, cnt = o.fc(o.encrypt_tensor(L, x.reshape(n, E, 1, 1), 6), w, bias=b)
    Ly = y.layout()
    assert (Ly["kind"], Ly["S"], Ly["bsg"]) == (2, S, L["bsg"]) and Ly["level"] == L["level"] - 1
    got = o.decrypt_tensor(y).reshape(n, E2)
    assert np.max(np.abs(got - (x @ w.T + b))) < 1e-4
    # brute force over the layout: the live diagonals of block (input ct a,
    # output ct o) are (j - i) mod d for used positions j of a and i of o; an
    # input takes a baby rotation per nonzero kd mod n1 it feeds, an output a
    # giant rotation per nonzero kd div n1 it receives
    d, kin, kout = L["d"], L["ncg"], Ly["ncg"]
    e = (d - 1).bit_length()
    n1 = 1 << ((e + 1) // 2)
    used = lambda k, s, F: [j for j in range(d) if (k * d + j) * S + s < F]
    babies, giants = 0, {}
    for s in range(S):
        for k in range(kin):
            b = set()
            for s2 in range(S):
                for k2 in range(kout):
                    kds = {(j - i) % d for j in used(k, s, E) for i in used(k2, s2, E2)}
                    b |= {kd % n1 for kd in kds}
                    giants.setdefault((s2, k2), set()).update(kd // n1 for kd in kds)
            babies += len(b - {0})
    assert cnt["other_rot"] == L["nbg"] * (babies + sum(len(g - {0}) for g in giants.values()))
    assert babies <= S * kin * (n1 - 1)


def test_token_fc_output_subset_equals_the_full_layer():
    """The oracle's token linear layer restricted to listed output
    ciphertexts (only the baby steps they use) gives those ciphertexts of the
    full layer word for word, bias included, in the listed order."""
    o = small_oracle(nq=3, logN=10)
    n, E, E2, S = 8, 48, 160, 2   # 2 fragments of 2 chunks each: 4 output cts
    x, w, b = rand_x((n, E), 46), rand_w((E2, E), 47), rand_w((E2,), 48)
    ob = o.encrypt_tensor(o.token_layout(n, E, S), x.reshape(n, E, 1, 1), 6)
    full, _ = o.fc(ob, w, bias=b)
    pick = [2, 0, full.layout()["S"] * full.layout()["ncg"] - 1]
    sub, _ = o.fc(ob, w, bias=b, outputs=pick)
    assert np.array_equal(sub, full.data()[pick])
