"""Pins for the oracle's bootstrapping (oracle.bootstrap), each against what the
mathematics fixes rather than against the oracle itself:

* the periodic and constant encodings against the encoder's definition,
  m_n = round(Delta (2/N) Re sum_j z_j zeta_j^-n), written out with numpy;
* the diagonals of CoeffToSlot and SlotToCoeff against the matrices they stand
  for (the embedding restricted to Z[X^(N/2n)], built with numpy's exp and
  inverted with numpy.linalg), and that matrix against the encoder's decode;
* ModRaise: the raised ciphertext decrypts over the whole chain (CRT) to the
  level-0 plaintext plus q_0 times small integers;
* SubSum: the decryption is N/2n times the coefficients at multiples of N/2n;
* the series and EvalMod against the same recipe in plain complex numbers and
  against 2 i sin(2^r theta); the arcsine term against 2 i (s + s^3/6);
* the whole bootstrap (slow: minutes) decrypts to its input within 1e-3."""
import math
import os

import numpy as np
import pytest

from oracle import bootstrap as bs
from oracle import ckks, params, rns
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _small_ctx(N=64):
    c = ckks.Context(params.config_tiny(), workloads.CRYPTO_SEED)
    c.N = N
    return c


def _direct_encode(N, zfull, scale):
    zeta = np.exp(1j * np.pi * np.array([pow(5, j, 2 * N) for j in range(N // 2)]) / N)
    return np.array([np.rint(scale * 2 / N * np.sum(zfull * zeta ** (-n)).real) for n in range(N)])


def _u0(n):
    """U0[j, i] = xi_j^i, xi_j = exp(i pi 5^j / 2n): slot j of a polynomial in Y = X^(N/2n)."""
    xi = np.exp(1j * np.pi * np.array([pow(5, j, 4 * n) for j in range(n)]) / (2 * n))
    return xi[:, None] ** np.arange(n)[None, :]


def _complex_decode(ctx, m, scale):
    N = ctx.N
    B = np.zeros(2 * N, dtype=np.complex128)
    B[:N] = np.asarray(m, dtype=np.float64)
    G = np.fft.ifft(B) * (2 * N)
    return G[ctx.slot_positions()] / scale


def _decrypt_complex(ctx, ct):
    return _complex_decode(ctx, ctx.decrypt_int(ct), ct.scale)


# ----------------------------------------------------------------- encodings
@pytest.mark.parametrize("P", [1, 2, 4, 8, 32])
def test_periodic_encoding_is_the_encoders_definition(P):
    N = 64
    rng = np.random.default_rng(P)
    z = rng.uniform(-1, 1, P) + 1j * rng.uniform(-1, 1, P)
    S = 2.0 ** 30
    got = bs.encode_periodic(N, [(v.real, v.imag) for v in z], S)
    want = _direct_encode(N, np.tile(z, N // 2 // P), S)
    assert np.max(np.abs(got - want)) <= 1
    assert np.mean(got == want) > 0.95
    # only multiples of N/2P are non-zero
    mask = np.ones(N, bool)
    mask[:: N // (2 * P)] = False
    assert not np.any(got[mask])


def test_periodic_encoding_of_real_values_matches_the_ckks_encoder():
    c = _small_ctx()
    z = np.random.default_rng(9).uniform(-1, 1, 8)
    got = bs.encode_periodic(c.N, [(v, 0.0) for v in z], 2.0 ** 30)
    assert np.max(np.abs(got - c.encode(np.tile(z, 4), 2.0 ** 30))) <= 1


def test_constant_encoding():
    N = 64
    S = 2.0 ** 30
    for cst in [(0.7, 0.0), (0.0, -0.3), (0.25, 0.5)]:
        got = bs.encode_const(N, cst, S)
        want = _direct_encode(N, np.full(N // 2, complex(*cst)), S)
        assert np.array_equal(got, want.astype(np.int64))


# --------------------------------------------------------------- the matrices
@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_u0_is_the_embedding_of_the_subring(n):
    c = _small_ctx()
    N = c.N
    t = np.random.default_rng(n).integers(-1000, 1000, 2 * n)
    m = np.zeros(N, np.int64)
    m[:: N // (2 * n)] = t
    slots = c.decode(m, 1.0)[:n]
    assert np.allclose(slots, (_u0(n) @ (t[:n] + 1j * t[n:])).real, atol=1e-6)


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_coeff_to_slot_diagonals(n):
    rng = np.random.default_rng(10 + n)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    D1, D2 = bs.cts_diagonals(n)
    out = np.zeros(2 * n, complex)
    for d in range(n):
        for j in range(2 * n):
            xv = x[(j + d) % n]
            out[j] += complex(*D1[d][j]) * xv + complex(*D2[d][j]) * np.conj(xv)
    w = np.linalg.inv(_u0(n)) @ x
    assert np.allclose(out, np.concatenate([w.real, w.imag]), atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_conjugate_map_has_the_conjugate_diagonals(n):
    """What lets CoeffToSlot be A + conj(A): D2_d = conj(D1_d), exactly."""
    D1, D2 = bs.cts_diagonals(n)
    for d in range(n):
        for (r1, i1), (r2, i2) in zip(D1[d], D2[d]):
            assert r2 == r1 and i2 == -i1


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_slot_to_coeff_diagonals(n):
    rng = np.random.default_rng(20 + n)
    D = rng.uniform(-1, 1, 2 * n) + 1j * rng.uniform(-1, 1, 2 * n)
    out = np.zeros(2 * n, complex)
    for d, diag in enumerate(bs.stc_diagonals(n)):
        for j in range(2 * n):
            out[j] += complex(*diag[j]) * D[(j + d) % (2 * n)]
    want = _u0(n) @ (-1j * D[:n] + D[n:])
    assert np.allclose(out, np.tile(want, 2), atol=1e-12)


def test_more_slots_than_a_quarter_ring_are_refused(tiny):
    """The linear maps use 2n-periodic vectors, which must fit the N/2 slots."""
    ct = tiny.encrypt(np.zeros(tiny.N // 2), level=0)
    with pytest.raises(AssertionError):
        bs.bootstrap(tiny, ct, bs.BootConfig(n=tiny.N // 2, r=0, d=1, pre_bits=0))


def test_levels_and_rotation_steps():
    assert bs.levels_used(bs.BootConfig(n=4, r=9, d=11, pre_bits=12)) == 17
    assert bs.levels_used(bs.BootConfig(n=1, r=0, d=1, pre_bits=0)) == 4
    assert bs.levels_used(bs.BootConfig(n=4, r=8, d=16, pre_bits=15, arcsine=True)) == 18
    assert bs.rotation_steps(4096, 4) == [1, 2, 3, 4, 5, 6, 7, 8, 16, 32, 64, 128, 256, 512, 1024]
    assert bs.rotation_steps(64, 16) == list(range(1, 32))
    assert bs.raise_scale(64, 97, 4, 3) == (64.0 * 97.0 * 8.0) / (4.0 * math.pi * 4.0)
    # baby-step giant-step split: B = 2^ceil(log2(count)/2), B * G >= count
    assert [bs.bsgs_split(c) for c in (1, 2, 4, 8, 16, 32, 64)] == \
        [(1, 1), (2, 1), (2, 2), (4, 2), (4, 4), (8, 4), (8, 8)]


# ----------------------------------------------------------------- the steps
@pytest.fixture(scope="module")
def tiny():
    c = ckks.Context(params.config_tiny(), workloads.CRYPTO_SEED)
    c.keygen(rot_steps=[256, 512, 1024], conj=True)
    return c


def test_mod_raise_adds_multiples_of_q0(tiny):
    c = tiny
    z = np.random.default_rng(3).uniform(-1, 1, c.N // 2)
    ct = c.encrypt(z, level=0)
    m0 = c.decrypt_int(ct)
    up = bs.mod_raise(c, ct, ct.scale)
    assert up.level == c.prm.L
    qm = c.qmods(c.prm.L)
    idx = list(range(c.prm.L + 1))
    c1s = c.mul(up.c1, c.s[idx], idx)
    rows = np.stack([(up.c0[i].astype(object) + c1s[i].astype(object)) % q
                     for i, q in enumerate(qm)]).astype(np.uint64)
    t = rns.crt(rows, qm)
    Q = math.prod(qm)
    t = np.array([v - Q if v > Q // 2 else v for v in t], dtype=object)
    q0 = c.prm.q[0]
    diff = t - m0.astype(object)
    assert all(int(v) % q0 == 0 for v in diff)
    I = np.array([int(v) // q0 for v in diff])
    assert np.any(I != 0) and np.max(np.abs(I)) < 6 * math.sqrt(c.N / 18) + 2


def test_sub_sum_is_the_trace(tiny):
    c = tiny
    n = 256
    z = np.random.default_rng(4).uniform(-1, 1, c.N // 2)
    ct = c.encrypt(z)
    m = c.decrypt_int(ct)
    out = bs.sub_sum(c, ct, n)
    got = c.decrypt_int(out)
    step = c.N // (2 * n)
    want = np.zeros(c.N, np.int64)
    want[::step] = step * m[::step]
    assert np.max(np.abs(got - want)) < 2 ** 24         # key-switching noise only
    assert np.max(np.abs(want)) > 2 ** 36


@pytest.fixture(scope="module")
def tiny2():
    c = ckks.Context(params.config_tiny_two_epochs(), workloads.CRYPTO_SEED)
    c.keygen(rot_steps=[1, 2, 3, 4, 5, 6, 7], conj=True)
    return c


def test_exp_series_and_eval_mod(tiny2):
    c = tiny2
    theta = np.random.default_rng(5).uniform(-0.8, 0.8, c.N // 2)
    ct = c.encrypt(theta)
    S = c.prm.scale
    e = bs.exp_series(c, ct, 7, S)
    series = sum((1j * theta) ** k / math.factorial(k) for k in range(8))
    assert np.max(np.abs(_decrypt_complex(c, e) - series)) < 1e-6
    d = bs.eval_mod(c, ct, 7, 2, S)
    want = series ** 4 - np.conj(series ** 4)
    got = _decrypt_complex(c, d)
    assert np.max(np.abs(got - want)) < 1e-5
    assert np.max(np.abs(got - 2j * np.sin(4 * theta))) < 1e-4


def test_arcsine_term(tiny2):
    c = tiny2
    sv = np.random.default_rng(8).uniform(-0.3, 0.3, c.N // 2)
    ct = c.encrypt(sv)
    S = c.prm.scale
    D = c.rescale(c.mul_plain(ct, bs.encode_const(c.N, (0.0, 2.0), S), S))    # 2 i s
    out = bs.arcsine_term(c, D)
    assert out.level == D.level - 2 and abs(out.scale / D.scale - 1) < 1e-12
    got = _decrypt_complex(c, out)
    assert np.max(np.abs(got - 2j * (sv + sv ** 3 / 6))) < 1e-6
    assert np.max(np.abs(got - 2j * np.arcsin(sv))) < 2 * (np.arcsin(0.3) - 0.3 - 0.3 ** 3 / 6) + 1e-6


def test_coeff_to_slot_and_slot_to_coeff_values(tiny2):
    c = tiny2
    n = 4
    x = np.random.default_rng(6).uniform(-1, 1, n)
    # the map runs after ModRaise, at a scale near q_l q_{l-1}: raise it by 2^35
    ct = c.mul_int(c.encrypt(np.tile(x, c.N // 2 // n)), 1 << 35)
    out = bs.coeff_to_slot(c, ct, n, c.prm.scale)
    assert out.level == c.prm.L - 2
    w = np.linalg.inv(_u0(n)) @ x
    got = c.decrypt(out)
    assert np.max(np.abs(got - np.tile(np.concatenate([w.real, w.imag]), c.N // 4 // n))) < 1e-6

    D = np.random.default_rng(7).uniform(-1, 1, 2 * n)
    ct = c.encrypt(np.tile(D, c.N // 4 // n))
    out = bs.slot_to_coeff(c, ct, n, 1.0, c.prm.scale)
    want = (_u0(n) @ (-1j * D[:n] + D[n:])).real
    assert np.max(np.abs(c.decrypt(out) - np.tile(want, c.N // 2 // n))) < 1e-6


# ------------------------------------------------------------ end to end
def test_golden_records_an_accurate_bootstrap():
    """The committed digests come from a bootstrap whose own decryption was
    within 1e-3 of its inputs (written by make_boot_n12.py from the oracle)."""
    from tests.golden import make_boot_n12 as gold
    _, meta = gold.read(os.path.join(HERE, "golden", "boot_n12.txt"))
    assert 0 < meta["max_abs_error"] < 1e-3
    assert 0 < meta["edge_max_abs_error"] < 1e-3
    assert 0 < meta["arcsine_max_abs_error"] < 1e-3


@pytest.mark.slow
def test_bootstrap_end_to_end():
    from tests.golden import make_boot_n12 as gold
    prm = gold.chain()
    c = ckks.Context(prm, workloads.CRYPTO_SEED)
    cfg = gold.config()
    bs.keygen_for(c, cfg)
    z = gold.values(0, prm.N)
    out = bs.bootstrap(c, c.encrypt(z, level=0), cfg)
    assert out.level == prm.L - bs.levels_used(cfg)
    assert abs(out.scale / prm.scale - 1) < 1e-9
    assert np.max(np.abs(c.decrypt(out) - z)) < 1e-3
