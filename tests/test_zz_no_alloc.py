"""The rescale that allocates nothing (static device scratch) against
fenc_rescale, through the C ABI: two calls in a row (the second with a
smaller batch) give the same residues, the context's device bytes do not
move, and the refusals (no tables for the level yet, a batch larger than
the scratch) are errors, not allocations."""
import numpy as np
import pytest

from fenc_backends import BACKENDS, make, rng
from paper_2606_16359_amd import fenc as F
from paper_2606_16359_amd import workloads as W


@pytest.mark.parametrize("backend", BACKENDS)
def test_rescale_noalloc_matches_rescale_on_two_calls(backend):
    f = make(backend, *W.PARAMS["lenet"])     # N = 2^15, 20 limbs: 10.5 MB of scratch per ciphertext
    x = rng(5).uniform(0, 1, (128, 1, 28, 28))
    lay_big = f.plan_layout(64, 1, 28, 28, 5, 6, 2)       # 4 ciphertexts
    lay_small = f.plan_layout(16, 1, 28, 28, 5, 6, 1)     # 1 ciphertext
    lay_huge = f.plan_layout(128, 1, 28, 28, 5, 6, 2)     # 8 ciphertexts: 84 MB of scratch
    assert (lay_big.n_ct(), lay_small.n_ct(), lay_huge.n_ct()) == (4, 1, 8)
    big = f.encrypt(f.encode_fragment(x[:64], lay_big), lay_big, 4)
    small = f.encrypt(f.encode_fragment(x[:16], lay_small), lay_small, 7)
    huge = f.encrypt(f.encode_fragment(x, lay_huge), lay_huge, 8)
    ref_big = f.export(f.rescale(big))        # also builds the tables of this level
    ref_small = f.export(f.rescale(small))
    before = f.device_bytes()
    got_big = f.rescale_noalloc(big)
    assert got_big.lay.level == lay_big.level - 1
    assert np.array_equal(f.export(got_big), ref_big)
    got_small = f.rescale_noalloc(small)      # second call, smaller batch, same scratch
    assert np.array_equal(f.export(got_small), ref_small)
    assert np.array_equal(f.export(f.rescale_noalloc(big)), ref_big)
    assert f.device_bytes() == before
    with pytest.raises(F.FencError) as e:
        f.rescale_noalloc(huge)
    assert e.value.code == -1 and "scratch" in str(e.value)
    with pytest.raises(F.FencError) as e:     # level 18 has no tables yet: refused, not built
        f.rescale_noalloc(got_big)
    assert e.value.code == -1 and "level" in str(e.value)
