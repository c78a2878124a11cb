"""Pins for the oracle's CKKS: the homomorphic properties the paper relies on
(Eq. 6-9, Sec. II-A.2), rotation identities and error bounds."""
import hashlib

import numpy as np
import pytest

from oracle import ckks, params, ring

SEED = hashlib.sha256(b"csrmf-2509.03024").digest()


@pytest.fixture(scope="module")
def ctx():
    prm = params.config_tiny()
    c = ckks.Context(prm, SEED)
    c.keygen(rot_steps=[1, 2, 3, 5, -4, 16], conj=True)
    return c


def _vec(seed, n, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def test_encode_decode_roundtrip(ctx):
    z = _vec(0, ctx.N // 2)
    m = ctx.encode(z, 2.0 ** 40)
    assert np.max(np.abs(ctx.decode(m, 2.0 ** 40) - z)) < 1e-9


def test_encode_matches_direct_definition():
    prm = params.config_tiny()
    c = ckks.Context(prm, SEED)
    N = 64
    c.N = N
    z = _vec(1, N // 2)
    S = 2.0 ** 30
    m = c.encode(z, S)
    zeta = [np.exp(1j * np.pi * pow(5, j, 2 * N) / N) for j in range(N // 2)]
    direct = [np.rint(S * 2 / N * sum(z[j] * zeta[j] ** (-n) for j in range(N // 2)).real) for n in range(N)]
    assert np.array_equal(m, np.array(direct, np.int64))


def test_scalar_encodes_as_constant_polynomial(ctx):
    S = 2.0 ** 30
    m = np.zeros(ctx.N, np.int64)
    m[0] = int(np.rint(0.7 * S))
    assert np.allclose(ctx.decode(m, S), 0.7, atol=1e-9)


def test_encrypt_decrypt(ctx):
    z = _vec(2, ctx.N // 2, 0, 5)
    ct = ctx.encrypt(z)
    assert ct.level == ctx.prm.L
    err = np.max(np.abs(ctx.decrypt(ct) - z))
    assert err < 1e-6


def test_homomorphic_add_and_plain_ops(ctx):
    a, b = _vec(3, ctx.N // 2), _vec(4, ctx.N // 2)
    ca, cb = ctx.encrypt(a), ctx.encrypt(b)
    assert np.max(np.abs(ctx.decrypt(ctx.add(ca, cb)) - (a + b))) < 1e-6          # Eq. 6
    assert np.max(np.abs(ctx.decrypt(ctx.sub(ca, cb)) - (a - b))) < 1e-6
    assert np.max(np.abs(ctx.decrypt(ctx.add_plain(ca, ctx.encode(b, ca.scale))) - (a + b))) < 1e-6  # Eq. 8
    qL = float(ctx.prm.q[-1])
    pm = ctx.encode(b, qL)
    prod = ctx.rescale(ctx.mul_plain(ca, pm, qL))                                    # Eq. 9
    assert prod.scale == ca.scale * qL / qL
    assert np.max(np.abs(ctx.decrypt(prod) - a * b)) < 1e-6


def test_hmult_relin_rescale(ctx):
    a, b = _vec(5, ctx.N // 2), _vec(6, ctx.N // 2)
    ca, cb = ctx.encrypt(a), ctx.encrypt(b)
    cab = ctx.hmult(ca, cb)                                                           # Eq. 7
    assert cab.level == ctx.prm.L - 1
    assert cab.scale == (2.0 ** 40 * 2.0 ** 40) / float(ctx.prm.q[-1])
    assert np.max(np.abs(ctx.decrypt(cab) - a * b)) < 1e-6
    c3 = ctx.hmult(cab, ca)
    assert np.max(np.abs(ctx.decrypt(c3) - a * a * b)) < 1e-5


def test_scale_mismatch_rejected(ctx):
    a = ctx.encrypt(_vec(7, 8), scale=2.0 ** 40)
    b = ctx.encrypt(_vec(8, 8), scale=2.0 ** 39)
    with pytest.raises(ckks.ScaleMismatch):
        ctx.add(a, b)


@pytest.mark.parametrize("r", [1, 2, 5, -4, 16])
def test_rotation(ctx, r):
    z = _vec(9 + r, ctx.N // 2)
    ct = ctx.encrypt(z)
    out = ctx.decrypt(ctx.rotate(ct, r))
    assert np.max(np.abs(out - np.roll(z, -r))) < 1e-6


def test_rotation_composition_and_conjugation(ctx):
    z = _vec(20, ctx.N // 2)
    ct = ctx.encrypt(z)
    r12 = ctx.rotate(ctx.rotate(ct, 1), 2)
    assert np.max(np.abs(ctx.decrypt(r12) - np.roll(z, -3))) < 1e-6
    assert np.max(np.abs(ctx.decrypt(ctx.conjugate(ct)) - z)) < 1e-6   # real slots


def test_hoisted_equals_rotate_bit_for_bit(ctx):
    """With centred ModUp digits the extension commutes with tau_g (tau_g
    permutes coefficients and negates some; the centred conversion of -x is
    exactly minus that of x for odd moduli), so hoisted and plain rotations
    give the same ciphertext."""
    z = _vec(21, ctx.N // 2)
    ct = ctx.encrypt(z)
    hs = ctx.hoisted_rotations(ct, [1, 3, 5])
    for r, h in hs.items():
        assert np.max(np.abs(ctx.decrypt(h) - np.roll(z, -r))) < 1e-6
        plain = ctx.rotate(ct, r)
        assert np.array_equal(plain.c0, h.c0) and np.array_equal(plain.c1, h.c1)


def test_key_switch_relation(ctx):
    """KS_{s'->s}(d) = (u0, u1) with u0 + u1*s ~ d*s' (small error), the defining property."""
    prm = ctx.prm
    lv = prm.L
    qm = prm.q
    idx = list(range(lv + 1))
    rng = np.random.default_rng(1)
    d = np.stack([rng.integers(0, q, ctx.N, dtype=np.uint64) for q in qm])
    s2 = ctx.mul(ctx.s[idx], ctx.s[idx], idx)
    u0, u1 = ctx.key_switch(d, ctx.relin_key, lv)
    lhs = ring.polyadd(u0, ctx.mul(u1, ctx.s[idx], idx), qm)
    rhs = ctx.mul(d, s2, idx)
    diff = ring.polysub(lhs, rhs, qm)[0].astype(object)
    q0 = qm[0]
    mag = max(min(int(v), q0 - int(v)) for v in diff)
    assert mag < 2 ** 30   # dnum * N * |e| * q_digit / P + rounding, far below q_0
