"""Token-fragment packing and the linear layer on it (the paper's extension to
Transformers, Discussions): the library against the oracle, word for word.

The oracle's token layout and linear layer are pinned in
test_oracle_method.py (slot map by brute force, S = 1 equal to the vector FC,
decryption to x W^T + b, rotation counts by brute force over the layout).
"""
import numpy as np
import pytest

from fenc_backends import BACKENDS, make, rng
from oracle import pyoracle as P
from test_parity import SMALL, cmp


@pytest.fixture(scope="module")
def orc():
    return P.Oracle(*SMALL)


def _same_layout(f, lay, L):
    assert (lay.kind, lay.S, lay.bs_g, lay.d, lay.n_bg, lay.n_cg, lay.level) == \
        (L["kind"], L["S"], L["bsg"], L["d"], L["nbg"], L["ncg"], L["level"])


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("n,E,S", [(8, 48, 4), (16, 40, 8), (4, 200, 2), (8, 24, 1), (3, 5, 4)])
def test_token_layout_and_encryption_match_the_oracle(backend, n, E, S, orc):
    """fenc_plan_tokens gives the oracle's token layout (fragment e mod S,
    position e div S, several ciphertexts per fragment when E/S exceeds the
    slots per group), the same slot of every element, and the same ciphertext
    words for the same seed; decryption returns the input."""
    f = make(backend, *SMALL)
    lay, L = f.plan_tokens(n, E, S), orc.token_layout(n, E, S)
    _same_layout(f, lay, L)
    for t in range(n):
        for e in range(E):
            assert f.layout_slot(lay, t, e, 0, 0) == orc.element_slots(L, t, e, 0, 0)[0]
    x = rng(61).uniform(-1, 1, (n, E, 1, 1))
    ct = f.encrypt(f.encode_fragment(x, lay), lay, 9)
    cmp(ct, orc.encrypt_tensor(L, x, 9), f)
    assert np.max(np.abs(f.decrypt(ct) - x)) < 1e-6


@pytest.mark.parametrize("backend", BACKENDS)
@pytest.mark.parametrize("n,E,E2,S", [(8, 48, 32, 4), (16, 64, 64, 8), (8, 24, 96, 2), (4, 32, 160, 1),
                                      (8, 40, 24, 4)])
@pytest.mark.parametrize("hoist", [1, 0])
def test_token_fc_bit_exact(backend, n, E, E2, S, hoist, orc):
    """A linear layer E -> E2 with a bias on token fragments: the library's
    words equal the oracle's, with its rotation count (baby steps hoisted per
    input ciphertext, giant steps per output ciphertext); output fragments
    that span several ciphertexts and a ragged last chunk included."""
    f = make(backend, *SMALL)
    f.set_hoisting(hoist)
    r = rng(62)
    x, w, b = r.uniform(-1, 1, (n, E, 1, 1)), r.normal(0, 0.1, (E2, E)), r.normal(0, 0.1, E2)
    lay, L = f.plan_tokens(n, E, S), orc.token_layout(n, E, S)
    ct, ob = f.encrypt(f.encode_fragment(x, lay), lay, 4), orc.encrypt_tensor(L, x, 4)
    f.stats_reset()
    y = f.fc(ct, w, bias=b)
    yo, cnt = orc.fc(ob, w, bias=b)
    _same_layout(f, y.lay, yo.layout())
    cmp(y, yo, f)
    st = f.stats()
    assert (st["rot_other"], st["pmult"]) == (cnt["other_rot"], cnt["pmult"])
    got = f.decrypt(y).reshape(n, E2)
    assert np.max(np.abs(got - (x.reshape(n, E) @ w.T + b))) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_token_fc_with_dead_blocks_bit_exact(backend, orc):
    """Weights with whole zero blocks (a fragment of the output reads only one
    fragment of the input, some outputs have no live diagonal at giant step 0,
    one output feature is all zero): only live diagonals are multiplied, and
    outputs with nothing to sum are zero ciphertexts, as in the oracle."""
    f = make(backend, *SMALL)
    n, E, E2, S = 8, 32, 16, 4
    r = rng(63)
    x = r.uniform(-1, 1, (n, E, 1, 1))
    w = r.normal(0, 0.1, (E2, E))
    w[np.arange(E2)[:, None] % S != (np.arange(E)[None, :] + 1) % S] = 0.0
    w[5] = 0.0
    w[:, 4:] *= np.arange(E)[4:] % 7 != 0
    lay, L = f.plan_tokens(n, E, S), orc.token_layout(n, E, S)
    y = f.fc(f.encrypt(f.encode_fragment(x, lay), lay, 2), w)
    yo, _ = orc.fc(orc.encrypt_tensor(L, x, 2), w)
    cmp(y, yo, f)
    assert np.max(np.abs(f.decrypt(y).reshape(n, E2) - x.reshape(n, E) @ w.T)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_token_ffn_chain_bit_exact(backend, orc):
    """A Transformer feed-forward block on token fragments, E -> 4E -> E with
    biases and a square activation between: every step equals the oracle word
    for word and the output decrypts to the float64 block."""
    f = make(backend, *SMALL)
    n, E, S = 8, 16, 4
    r = rng(64)
    x = r.uniform(-1, 1, (n, E, 1, 1))
    w1, b1 = r.normal(0, 0.2, (4 * E, E)), r.normal(0, 0.1, 4 * E)
    w2, b2 = r.normal(0, 0.2, (E, 4 * E)), r.normal(0, 0.1, E)
    lay, L = f.plan_tokens(n, E, S), orc.token_layout(n, E, S)
    y, yo = f.encrypt(f.encode_fragment(x, lay), lay, 8), orc.encrypt_tensor(L, x, 8)
    for fl, ol in [(lambda c: f.fc(c, w1, bias=b1), lambda b: orc.fc(b, w1, bias=b1)),
                   (f.poly_act, orc.square),
                   (lambda c: f.fc(c, w2, bias=b2), lambda b: orc.fc(b, w2, bias=b2))]:
        y, (yo, _) = fl(y), ol(yo)
        cmp(y, yo, f)
    h = x.reshape(n, E) @ w1.T + b1
    ref = (h * h) @ w2.T + b2
    assert np.max(np.abs(f.decrypt(y).reshape(n, E) - ref)) < 1e-4


@pytest.mark.parametrize("backend", BACKENDS)
def test_token_ffn_cubic_per_op_equals_batched_and_oracle(backend, orc):
    """The feed-forward chain with a cubic activation between (two levels:
    the second tensor product forms u = k3 x' + k2' itself): the per-op form
    (every operation of every ciphertext launched separately) and the batched
    form give the oracle's words at every step."""
    from paper_2606_16359_amd import fenc as F
    f = make(backend, 10, 8, 50, 3, 50, 3, 40, 17)
    o = P.Oracle(10, 8, 50, 3, 50, 3, 40, 17)
    n, E, S = 8, 16, 2
    r = rng(65)
    x = r.uniform(-1, 1, (n, E, 1, 1))
    w1, w2 = r.normal(0, 0.2, (2 * E, E)), r.normal(0, 0.2, (E, 2 * E))
    cubic = (0.1, 0.5, 0.25, -0.02)
    lay, L = f.plan_tokens(n, E, S), o.token_layout(n, E, S)
    yo = o.encrypt_tensor(L, x, 8)
    yo, _ = o.fc(yo, w1)
    yo, _ = o.poly_act(yo, cubic)
    yo, _ = o.fc(yo, w2)
    for mode in (F.FENC_MODE_BATCHED, F.FENC_MODE_PER_OP):
        f.set_mode(mode)
        y = f.fc(f.poly_act(f.fc(f.encrypt(f.encode_fragment(x, lay), lay, 8), w1), cubic), w2)
        cmp(y, yo, f)
