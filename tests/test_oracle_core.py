"""Pins of the oracle's CKKS core against definitions independent of it.

Each check uses Python integers, numpy or a closed form, never the oracle's own
routines, as the expected value.
"""
import numpy as np
import pytest

from oracle import pyoracle as P

M64 = (1 << 64) - 1


def py_is_prime(n):
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47]
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            t = int(a[i]) * int(b[j])
            if i + j < n:
                out[i + j] += t
            else:
                out[i + j - n] -= t
    return [x % q for x in out]


def test_miller_rabin_against_trial_division():
    lib = P.lib()
    for n in range(0, 5000):
        trial = n >= 2 and all(n % p for p in range(2, int(n ** 0.5) + 1))
        assert bool(lib.orc_is_prime(n)) == trial, n
    for n in [(1 << 61) - 1, (1 << 31) - 1, 3215031751, 341550071728321, 18446744073709551557]:
        assert bool(lib.orc_is_prime(n)) == py_is_prime(n)


@pytest.mark.parametrize("logN,bits", [(6, 30), (13, 40), (15, 50)])
def test_primes_are_largest_ntt_friendly(logN, bits):
    o = P.Oracle(logN, 3, bits, 2, bits, 2, 20, 1)
    ps = o.primes()
    twoN = 2 << logN
    assert all(p % twoN == 1 and p < (1 << bits) and py_is_prime(p) for p in ps)
    assert ps == sorted(ps, reverse=True) and len(set(ps)) == len(ps)
    # nothing NTT-friendly and prime was skipped above the smallest chosen prime
    c = ((1 << bits) - 2) // twoN * twoN + 1
    while c > ps[-1]:
        assert (c in ps) == py_is_prime(c), c
        c -= twoN
    for p, psi in zip(ps, o.psi()):
        assert pow(psi, 1 << logN, p) == p - 1


@pytest.mark.parametrize("logN", [4, 5, 6])
def test_polymul_matches_schoolbook(logN):
    o = P.Oracle(logN, 2, 30, 1, 30, 2, 20, 3)
    rng = np.random.default_rng(logN)
    for pidx, q in enumerate(o.primes()):
        a = rng.integers(0, q, o.N, dtype=np.uint64)
        b = rng.integers(0, q, o.N, dtype=np.uint64)
        assert [int(x) for x in o.polymul(pidx, a, b)] == negacyclic(a, b, q)
        assert [int(x) for x in o.polymul(pidx, a, b, schoolbook=True)] == negacyclic(a, b, q)


def test_ntt_is_evaluation_at_odd_powers(orc_small):
    o = orc_small
    q, psi = o.primes()[0], o.psi()[0]
    rng = np.random.default_rng(5)
    a = rng.integers(0, q, o.N, dtype=np.uint64)
    A = o.ntt(0, a)
    for j in range(o.N):
        want = sum(int(a[i]) * pow(psi, (2 * j + 1) * i, q) for i in range(o.N)) % q
        assert int(A[j]) == want
    assert np.array_equal(o.ntt(0, A, inverse=True), a)


def test_splitmix_counter_generator_matches_definition():
    """SplitMix64 (Steele-Lea-Flood 2014): state += gamma; output = mix(state)."""
    g = 0x9E3779B97F4A7C15

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)

    for seed, tag in [(0, 0), (7, 1 << 56), (12345, (2 << 56) | (5 << 24) | 3)]:
        state = mix(seed ^ ((tag * 0xD1B54A32D192ED03) & M64))
        for i in range(8):
            state = (state + g) & M64
            assert P.lib().orc_rng(seed, tag, i) == mix(state)


def test_sampler_distributions():
    lib = P.lib()
    t = np.array([lib.orc_ternary(3, 1 << 56, i) for i in range(30000)])
    assert set(t.tolist()) == {-1, 0, 1}
    assert np.all(np.abs(np.bincount(t + 1) / len(t) - 1 / 3) < 0.015)
    e = np.array([lib.orc_gauss(3, 3 << 56, i) for i in range(60000)])
    assert np.abs(e).max() <= 19
    assert abs(e.mean()) < 0.05
    assert abs(e.std() - 3.2) < 0.05
    cdt = np.zeros(19, np.uint64)
    lib.orc_gauss_cdt(cdt)
    rho = np.exp(-np.arange(20) ** 2 / (2 * 3.2 ** 2))
    Z = rho[0] + 2 * rho[1:].sum()
    cdf = (rho[0] + 2 * np.concatenate([[0], np.cumsum(rho[1:19])])) / Z
    assert np.all(np.abs(cdt.astype(np.float64) / 2.0 ** 63 - cdf) < 1e-13)
    q = (1 << 50) - 27
    u = np.array([lib.orc_uniform(9, 4 << 56, i, q) for i in range(20000)], dtype=np.float64)
    assert u.max() < q and abs(u.mean() / q - 0.5) < 0.01


@pytest.mark.parametrize("logN", [3, 4, 5, 6])
def test_encoder_fft_equals_direct_definition(logN):
    o = P.Oracle(logN, 2, 30, 1, 30, 2, 20, 3)
    rng = np.random.default_rng(logN)
    re, im = rng.normal(size=o.ns), rng.normal(size=o.ns)
    for scale in (2.0 ** 20, 2.0 ** 40, 1234567.891):
        assert np.array_equal(o.encode_int(re, im, scale), o.encode_int(re, im, scale, direct=True))


def test_encoder_direct_sum_against_numpy_definition(orc_small):
    o = orc_small
    rng = np.random.default_rng(1)
    z = rng.normal(size=o.ns) + 1j * rng.normal(size=o.ns)
    m = o.encode_int(z.real, z.imag, 2.0 ** 30).astype(np.float64)
    zeta = np.exp(1j * np.pi / o.N)
    roots = zeta ** np.array([pow(5, j, 2 * o.N) for j in range(o.ns)])
    got = np.array([np.polyval(m[::-1], r) for r in roots]) / 2.0 ** 30
    assert np.max(np.abs(got - z)) < 1e-6


def test_constant_vector_encodes_to_constant_polynomial(orc_small):
    o = orc_small
    m = o.encode_int(np.full(o.ns, 0.375), None, 2.0 ** 20)
    assert m[0] == round(0.375 * 2 ** 20) and not np.any(m[1:])


def test_decode_inverts_encode(orc_small):
    o = orc_small
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, o.ns)
    pt = o.encode(x, None, 2.0 ** 20, level=0)
    assert np.max(np.abs(o.decode(pt[0], 2.0 ** 20).real - x)) < o.N / 2.0 ** 20


def centered(v, q):
    v = np.asarray(v, dtype=object)
    return np.array([int(x) - q if int(x) > q // 2 else int(x) for x in v], dtype=object)


def test_encrypt_decrypt_noise_is_the_sampled_error(orc_small):
    o = orc_small
    rng = np.random.default_rng(3)
    level = o.L
    qs = o.primes()
    pt = np.array([rng.integers(0, q, o.N, dtype=np.uint64) for q in qs[:level + 1]])
    ct = o.encrypt(pt, level, 2.0 ** 20, seed=99, ct_index=4)
    m = o.decrypt(ct)
    e = [int(P.lib().orc_gauss(99, (5 << 56) | (4 << 16), i)) for i in range(o.N)]
    for l in range(level + 1):
        d = centered((m[l].astype(object) - pt[l].astype(object)) % qs[l], qs[l])
        assert list(d) == e


def test_automorphism_composes_and_matches_evaluation_permutation(orc_small):
    o = orc_small
    q, psi = o.primes()[1], o.psi()[1]
    rng = np.random.default_rng(4)
    a = rng.integers(0, q, o.N, dtype=np.uint64)
    g, h = o.galois(3), o.galois(5)
    gh = g * h % (2 * o.N)
    assert np.array_equal(o.automorph(1, o.automorph(1, a, h), g), o.automorph(1, a, gh))
    assert gh == o.galois(8)
    # sigma_g(a)(psi^(2j+1)) = a(psi^((2j+1) g)): a permutation of the evaluations
    A, B = o.ntt(1, a), o.ntt(1, o.automorph(1, a, g))
    for j in range(o.N):
        jj = (((2 * j + 1) * g) % (2 * o.N) - 1) // 2
        assert B[j] == A[jj]


def crt(residues, primes):
    Q = 1
    for p in primes:
        Q *= p
    x = 0
    for r, p in zip(residues, primes):
        Mi = Q // p
        x += int(r) * Mi * pow(Mi, -1, p)
    return x % Q, Q


def test_mod_down_rescale_divides_by_P_times_q_l(orc_small):
    """ModDown by P q_l (the relinearisation's ModDown merged with the rescale):
    D x + y over Q_l U P gives x - v on Q_{l-1} with |v| <= K + 1 for
    |y| < D/2 (fast base conversion of K + 1 centred terms), and exactly x
    for y = 0; checked against the integers themselves."""
    o = orc_small
    qs = o.primes()
    level = 2
    basis = list(range(level + 1)) + [o.nq + k for k in range(o.np)]
    D = qs[level]
    for k in range(o.np):
        D *= qs[o.nq + k]
    rng = np.random.default_rng(7)
    x = [int(v) - (1 << 59) for v in rng.integers(0, 1 << 60, o.N, dtype=np.uint64)]
    y = [int(v) - (1 << 19) for v in rng.integers(0, 1 << 20, o.N, dtype=np.uint64)]
    a = np.array([[(D * xi + yi) % qs[t] for xi, yi in zip(x, y)] for t in basis], dtype=np.uint64)
    got = o.mod_down_rescale(a, level)
    assert got.shape == (level, o.N)
    zero_y = np.array([[(D * xi) % qs[t] for xi in x] for t in basis], dtype=np.uint64)
    assert np.array_equal(o.mod_down_rescale(zero_y, level),
                          np.array([[xi % qs[i] for xi in x] for i in range(level)], dtype=np.uint64))
    vs = set()
    for c in range(o.N):
        cands = [v for v in range(-o.np - 1, o.np + 2) if all(int(got[i][c]) == (x[c] - v) % qs[i]
                                                               for i in range(level))]
        assert cands, c
        vs.add(cands[0])
    assert len(vs) > 1   # the conversion's error term is exercised, not always zero


def test_mod_up_is_centred_digit_lift_plus_small_multiple(orc_small):
    o = orc_small
    qs = o.primes()
    level = o.L
    rng = np.random.default_rng(5)
    d = np.array([rng.integers(0, q, o.N, dtype=np.uint64) for q in qs[:level + 1]])
    ext = o.mod_up(d, level)
    basis = list(range(level + 1)) + [o.nq + k for k in range(o.np)]
    for j in range(ext.shape[0]):
        dig = list(range(j * o.alpha, min((j + 1) * o.alpha, level + 1)))
        for c in range(0, o.N, 7):
            a, Qj = crt([d[i][c] for i in dig], [qs[i] for i in dig])
            if a > Qj // 2:
                a -= Qj        # centred representative of the digit
            us = set()
            for li, t in enumerate(basis):
                diff = (int(ext[j][li][c]) - a) % qs[t]
                if t in dig:          # the digit's own limbs are copied unchanged
                    assert diff == 0
                    continue
                found = [u for u in range(-len(dig), len(dig) + 1) if (u * Qj) % qs[t] == diff]
                assert found, (j, c, t)
                us.add(found[0])
            assert len(us) == 1     # one integer a + u*Qj, |u| <= |D_j|, in every prime


def test_mod_down_divides_by_P(orc_small):
    o = orc_small
    qs = o.primes()
    level = 2
    basis = list(range(level + 1)) + [o.nq + k for k in range(o.np)]
    P_ = 1
    for k in range(o.np):
        P_ *= qs[o.nq + k]
    rng = np.random.default_rng(6)
    x = [int(v) for v in rng.integers(0, 1 << 60, o.N, dtype=np.uint64)]
    y = [int(v) for v in rng.integers(0, 1 << 20, o.N, dtype=np.uint64)]
    a = np.array([[(P_ * xi + yi) % qs[t] for xi, yi in zip(x, y)] for t in basis], dtype=np.uint64)
    got = o.mod_down(a, level)
    zero_y = np.array([[(P_ * xi) % qs[t] for xi in x] for t in basis], dtype=np.uint64)
    assert np.array_equal(o.mod_down(zero_y, level),
                          np.array([[xi % qs[i] for xi in x] for i in range(level + 1)], dtype=np.uint64))
    for i in range(level + 1):
        for c in range(o.N):
            # y < P/2 so its P-part converts to y + v P with |v| <= K, i.e. result x - v
            cands = [(x[c] - v) % qs[i] for v in range(-o.np, o.np + 1)]
            assert int(got[i][c]) in cands


def test_rescale_rounds_the_crt_integer(orc_small):
    o = orc_small
    qs = o.primes()
    level = o.L
    rng = np.random.default_rng(7)
    ct = np.array([[rng.integers(0, q, o.N, dtype=np.uint64) for q in qs[:level + 1]] for _ in range(2)])
    out = o.rescale(ct)
    ql = qs[level]
    for p in range(2):
        for c in range(0, o.N, 5):
            X, Q = crt([ct[p][i][c] for i in range(level + 1)], qs[:level + 1])
            if X > Q // 2:
                X -= Q
            r = (2 * X + ql) // (2 * ql)     # round to nearest (q odd: no ties)
            for i in range(level):
                assert int(out[p][i][c]) == r % qs[i]


def test_rotation_decrypts_to_rolled_slots():
    o = P.Oracle(7, 4, 40, 2, 41, 2, 30, 21)
    rng = np.random.default_rng(8)
    z = rng.uniform(-1, 1, o.ns)
    pt = o.encode(z, None, 2.0 ** 30)
    ct = o.encrypt(pt, o.L, 2.0 ** 30, seed=5)
    shifts = [1, 5, o.ns - 3, 17]
    rots = o.rotate(ct, shifts)
    for r, rc in zip(shifts, rots):
        got = o.decode(o.decrypt(rc)[0]).real
        assert np.max(np.abs(got - np.roll(z, -r))) < 1e-5
    # lazy sum: z0 + sum_r Rot(z_r, r) with one ModDown
    s = o.rotate_sum(ct, np.stack([ct, ct]), [1, 2])
    got = o.decode(o.decrypt(s)[0]).real
    assert np.max(np.abs(got - (z + np.roll(z, -1) + np.roll(z, -2)))) < 1e-5
    # key switching keeps the decryption: decrypt(rot) == sigma_g(decrypt(ct)) up to small noise
    g = o.galois(5)
    m, mr = o.decrypt(ct), o.decrypt(rots[1])
    q0 = o.primes()[0]
    diff = centered((mr[0].astype(object) - o.automorph(0, m[0], g).astype(object)) % q0, q0)
    assert max(abs(int(v)) for v in diff) < 2 ** 12


def test_square_relin_decrypts_to_square():
    o = P.Oracle(7, 4, 40, 2, 41, 2, 30, 22)
    rng = np.random.default_rng(9)
    z = rng.uniform(-1, 1, o.ns)
    ct = o.encrypt(o.encode(z, None, 2.0 ** 30), o.L, 2.0 ** 30, seed=6)
    sq = o.rescale(o.square_relin(ct))     # k = 1 through the C entry point
    got = o.decode(o.decrypt(sq)[0], 2.0 ** 60 / o.primes()[o.L]).real
    assert np.max(np.abs(got - z * z)) < 1e-4


def test_switch_key_structure(orc_small):
    """b_j + a_j s = e_j + P * [j-th digit indicator] * s' (mod each prime)."""
    o = orc_small
    qs = o.primes()
    s = o.secret()
    g = o.galois(1)
    key = o.switch_key(g)
    P_ = 1
    for k in range(o.np):
        P_ *= qs[o.nq + k]
    for j in range(key.shape[0]):
        e = [int(P.lib().orc_gauss(11, (3 << 56) | (g << 24) | (j << 16), i)) for i in range(o.N)]
        for t, q in enumerate(qs):
            sp = np.array([int(v) % q for v in s], dtype=np.uint64)
            bs_ = negacyclic(key[j][1][t], sp, q)
            lhs = [(int(b) + v) % q for b, v in zip(key[j][0][t], bs_)]
            sg = o.automorph(t, sp, g)
            indicator = 1 if (t < o.nq and j * o.alpha <= t < (j + 1) * o.alpha) else 0
            rhs = [(ei + indicator * (P_ % q) * int(sv)) % q for ei, sv in zip(e, sg)]
            assert lhs == rhs


def test_extended_basis_rotation_moves_down_to_the_rotation():
    """ModDown(KIP + P sigma(c0), KIP) is the rotated ciphertext word for word, and
    ModDown(P x) = x: the identity that lets a linear combination of rotated
    copies be taken before the single ModDown."""
    o = P.Oracle(10, 6, 50, 2, 50, 3, 40, 5)
    r = np.random.default_rng(3)
    z = r.uniform(-1, 1, o.ns)
    level = 5
    ct = o.encrypt(o.encode(z, None, 2.0 ** 40, level), level, 2.0 ** 40, 7)
    shifts = [1, 5, 200]
    assert np.array_equal(o.pq_roundtrip(ct, shifts), o.rotate(ct, shifts))
    assert np.array_equal(o.pq_roundtrip(ct, lift=True), ct)


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _rng(seed, tag, i):
    key = _mix(seed ^ ((tag * 0xD1B54A32D192ED03) & M64))
    return _mix((key + (i + 1) * 0x9E3779B97F4A7C15) & M64)


def test_sampler_words_are_the_stated_functions_of_the_stream():
    """Bit for bit: uniform mod q = (word 2i << 64 | word 2i+1) mod q (the first
    word is the high half), ternary = floor(3 r / 2^64) - 1, Gaussian = sign bit
    63 and the count of table entries <= the low 63 bits."""
    lib = P.lib()
    cdt = np.zeros(19, np.uint64)
    lib.orc_gauss_cdt(cdt)
    for seed, tag in [(0, 0), (9, 4 << 56), (3, (2 << 56) | (7 << 24) | (1 << 16) | 5)]:
        for q in [(1 << 50) - 27, 1125899904679937, 268369921]:
            for i in [0, 1, 2, 17, 1000, 65535]:
                hi, lo = _rng(seed, tag, 2 * i), _rng(seed, tag, 2 * i + 1)
                assert lib.orc_uniform(seed, tag, i, q) == ((hi << 64) | lo) % q
                assert lib.orc_uniform(seed, tag, i, q) != ((lo << 64) | hi) % q or hi == lo
        for i in range(200):
            r = _rng(seed, tag, i)
            assert lib.orc_ternary(seed, tag, i) == ((3 * r) >> 64) - 1
            mag = sum(1 for t in cdt if (r & ((1 << 63) - 1)) >= int(t))
            assert lib.orc_gauss(seed, tag, i) == (-mag if r >> 63 else mag)


def test_full_size_product_against_schoolbook_coefficients():
    """N = 2^16 with a 50-bit prime: sampled coefficients of the NTT product
    equal the negacyclic schoolbook sum computed with Python integers."""
    o = P.Oracle(16, 2, 50, 1, 50, 2, 40, 1)
    q = o.primes()[0]
    N = o.N
    rng = np.random.default_rng(16)
    a = rng.integers(0, q, N, dtype=np.uint64)
    b = rng.integers(0, q, N, dtype=np.uint64)
    c = o.polymul(0, a, b)
    al, bl = [int(v) for v in a], [int(v) for v in b]
    for k in [0, 1, 2, N // 2, N - 2, N - 1] + [int(v) for v in rng.integers(0, N, 26)]:
        # c_k = sum_{i<=k} a_i b_{k-i} - sum_{i>k} a_i b_{N+k-i}
        pos = sum(x * y for x, y in zip(al[:k + 1], reversed(bl[:k + 1])))
        neg = sum(x * y for x, y in zip(al[k + 1:], reversed(bl[k + 1:])))
        assert int(c[k]) == (pos - neg) % q, k
