"""Pins for the oracle's primitives: primes, ChaCha20, samplers, modular arithmetic,
negacyclic products, CRT, basis conversion, rescale, ModDown."""
import os
import random
import shutil
import subprocess

import numpy as np
import pytest
import sympy

from oracle import chacha, sampling, params, ring, rns
from oracle.modarith import mulmod, addmod, submod

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ primes
@pytest.mark.parametrize("bits,logN,count", [(60, 12, 2), (40, 12, 3), (60, 16, 4), (40, 16, 24), (40, 15, 16)])
def test_ntt_primes_are_the_largest(bits, logN, count):
    N = 1 << logN
    ps = params.ntt_primes(bits, N, count)
    assert ps == sorted(ps, reverse=True)
    for p in ps:
        assert sympy.isprime(p) and p % (2 * N) == 1 and p < 2 ** bits
    # no prime = 1 mod 2N was skipped between 2^bits and the last one
    q = (1 << bits) - 2 * N + 1
    expect = []
    while q >= ps[-1]:
        if sympy.isprime(q):
            expect.append(q)
        q -= 2 * N
    assert expect == ps


def test_tiny_chain_values():
    prm = params.config_tiny()
    # (this chain is re-derived above; these are the values that derivation gives)
    assert prm.q[0] == 1152921504606830593 and prm.p == [1152921504606748673]
    assert [2 ** 40 - q for q in prm.q[1:]] == [147455, 237567, 368639]


@pytest.mark.parametrize("q,logN", [(1152921504606830593, 12), (1099511480321, 12), (1099511390209, 13)])
def test_primitive_root(q, logN):
    N = 1 << logN
    if (q - 1) % (2 * N):
        pytest.skip("not NTT friendly for this N")
    psi = params.primitive_2n_root(q, N)
    assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1
    assert sympy.n_order(psi, q) == 2 * N


# ------------------------------------------------------------------ ChaCha20
def _golden_chacha():
    lines = [l.strip() for l in open(os.path.join(GOLD, "chacha20_rfc8439.txt")) if l.strip() and not l.startswith("#")]
    block = bytes.fromhex(lines[0])
    qr_in, qr_out = lines[1].split("->")
    return block, [int(x, 16) for x in qr_in.split()], [int(x, 16) for x in qr_out.split()]


def test_chacha_quarter_round_rfc():
    _, qi, qo = _golden_chacha()
    assert list(chacha.quarter_round(*qi)) == qo


def test_chacha_block_rfc():
    block, _, _ = _golden_chacha()
    key = bytes(range(32))
    nonce = np.frombuffer(bytes.fromhex("000000090000004a00000000"), "<u4")
    out = chacha.blocks(key, np.array([1], np.uint32), nonce).astype("<u4").tobytes()
    assert out == block


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not available")
def test_chacha_stream_matches_openssl():
    key = bytes(random.Random(7).getrandbits(8) for _ in range(32))
    purpose, obj, limb = 4, 123457, 9
    n = 64 * 37
    ours = chacha.keystream_bytes(key, (purpose, obj, limb), n)
    iv = (0).to_bytes(4, "little") + purpose.to_bytes(4, "little") + obj.to_bytes(4, "little") + limb.to_bytes(4, "little")
    ref = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
                         input=bytes(n), capture_output=True, check=True).stdout
    assert ours == ref
    w = chacha.words_u64(key, purpose, obj, limb, n // 8)
    assert w.astype("<u8").tobytes() == ref


# ------------------------------------------------------------------ samplers
def test_samplers_distribution():
    key = bytes(32)
    N = 1 << 18
    t = sampling.ternary(key, 1, 0, N)
    assert set(np.unique(t)) <= {-1, 0, 1}
    freq = np.bincount(t + 1) / N
    assert np.all(np.abs(freq - 1 / 3) < 5 * np.sqrt(2 / 9 / N))
    e = sampling.cbd21(key, 3, 0, N)
    assert e.min() >= -21 and e.max() <= 21
    assert abs(e.mean()) < 5 * np.sqrt(10.5 / N)
    assert abs(e.var() - 10.5) < 5 * 10.5 * np.sqrt(2 / N)


def test_uniform_sampler_definition():
    key = bytes(range(32))
    q = 1099511480321
    u = sampling.uniform_mod(key, 2, 5, 3, 64, q)
    w = chacha.words_u64(key, 2, 5, 3, 128)
    ref = [((int(w[2 * n]) << 64) + int(w[2 * n + 1])) % q for n in range(64)]
    assert [int(x) for x in u] == ref


def test_ternary_and_cbd_definitions():
    key = bytes(range(1, 33))
    w = chacha.words_u64(key, 6, 2, 0, 100)
    t = sampling.ternary(key, 6, 2, 100)
    assert [int(x) for x in t] == [int(v) % 3 - 1 for v in w]
    w = chacha.words_u64(key, 7, 2, 0, 100)
    e = sampling.cbd21(key, 7, 2, 100)
    ref = [bin(int(v) & (2 ** 21 - 1)).count("1") - bin((int(v) >> 21) & (2 ** 21 - 1)).count("1") for v in w]
    assert [int(x) for x in e] == ref


# ------------------------------------------------------------------ modular arithmetic
@pytest.mark.parametrize("q", [1152921504606830593, 1152921504595968001, 1099511480321, 1099467194369, 97])
def test_mulmod_against_python_ints(q):
    rng = random.Random(q)
    xs = [rng.randrange(q) for _ in range(3000)] + [0, 1, q - 1, q - 2, q // 2, q // 2 + 1]
    ys = [rng.randrange(q) for _ in range(3000)] + [q - 1, q - 1, q - 1, q - 2, q - 1, q // 2]
    a = np.array(xs, np.uint64)
    b = np.array(ys, np.uint64)
    assert [int(v) for v in mulmod(a, b, q)] == [x * y % q for x, y in zip(xs, ys)]
    assert [int(v) for v in addmod(a, b, q)] == [(x + y) % q for x, y in zip(xs, ys)]
    assert [int(v) for v in submod(a, b, q)] == [(x - y) % q for x, y in zip(xs, ys)]


# ------------------------------------------------------------------ negacyclic product
def schoolbook_negacyclic(a, b, q):
    """Exact negacyclic product by Kronecker substitution in Python big integers."""
    N = len(a)
    w = 2 * q.bit_length() + N.bit_length() + 2
    A = sum(int(x) << (w * i) for i, x in enumerate(a))
    B = sum(int(x) << (w * i) for i, x in enumerate(b))
    C = A * B
    mask = (1 << w) - 1
    c = [(C >> (w * i)) & mask for i in range(2 * N - 1)] + [0]
    return [(c[i] - c[i + N]) % q for i in range(N)]


@pytest.mark.parametrize("logN", [3, 6, 10, 12])
def test_ntt_product_equals_schoolbook(logN):
    N = 1 << logN
    rng = random.Random(logN)
    for q in (params.ntt_primes(60, N, 1)[0], params.ntt_primes(40, N, 1)[0]):
        psi = params.primitive_2n_root(q, N)
        a = [rng.randrange(q) for _ in range(N)]
        b = [rng.randrange(q) for _ in range(N)]
        got = ring.polymul(np.array([a], np.uint64), np.array([b], np.uint64), [q], [psi])[0]
        assert [int(x) for x in got] == schoolbook_negacyclic(a, b, q)


def test_ntt_is_evaluation_at_odd_powers():
    N, q = 16, params.ntt_primes(40, 16, 1)[0]
    psi = params.primitive_2n_root(q, N)
    a = np.array(random.Random(1).sample(range(q), N), np.uint64)
    A = ring.ntt(a, q, psi)
    for t in range(N):
        x = pow(psi, 2 * t + 1, q)
        assert int(A[t]) == sum(int(a[n]) * pow(x, n, q) for n in range(N)) % q
    assert np.array_equal(ring.intt(A, q, psi), a)


def test_automorphism_composition_and_identity():
    N = 64
    q = params.ntt_primes(40, N, 1)[0]
    a = np.array([random.Random(3).randrange(q) for _ in range(N)], np.uint64)[None]
    g, h = 5, 25
    ab = ring.apply_automorphism(ring.apply_automorphism(a, g, [q]), h, [q])
    assert np.array_equal(ab, ring.apply_automorphism(a, g * h % (2 * N), [q]))
    assert np.array_equal(ring.apply_automorphism(a, pow(5, N // 2, 2 * N), [q]), a)
    # tau_g is a ring homomorphism: tau(a*b) = tau(a)*tau(b)
    psi = params.primitive_2n_root(q, N)
    b = np.array([random.Random(4).randrange(q) for _ in range(N)], np.uint64)[None]
    lhs = ring.apply_automorphism(ring.polymul(a, b, [q], [psi]), g, [q])
    rhs = ring.polymul(ring.apply_automorphism(a, g, [q]), ring.apply_automorphism(b, g, [q]), [q], [psi])
    assert np.array_equal(lhs, rhs)


# ------------------------------------------------------------------ RNS
def _rand_rns(mods, N, seed):
    rng = random.Random(seed)
    Q = rns.prod(mods)
    xs = [rng.randrange(Q) for _ in range(N)]
    return xs, np.array([[x % q for x in xs] for q in mods], np.uint64)


def test_crt_roundtrip():
    prm = params.config_tiny()
    xs, rows = _rand_rns(prm.q, 32, 1)
    assert list(rns.crt(rows, prm.q)) == xs


def test_basis_conversion_overflow_bound():
    prm = params.config_tiny()
    src = prm.q[1:4]
    dst = [prm.q[0]] + prm.p
    xs, rows = _rand_rns(src, 64, 2)
    conv = rns.basis_convert(rows, src, dst)
    B = rns.prod(src)
    for n, x in enumerate(xs):
        ok = False
        for e in range(len(src)):
            if all(int(conv[k][n]) == (x + e * B) % c for k, c in enumerate(dst)):
                ok = True
        assert ok


def test_rescale_is_rounded_division():
    prm = params.config_tiny()
    xs, rows = _rand_rns(prm.q, 64, 3)
    out = rns.rescale(rows, prm.q)
    ql = prm.q[-1]
    Qm = rns.prod(prm.q[:-1])
    for n, x in enumerate(xs):
        y = ((x + ql // 2) // ql) % Qm
        assert [int(out[i][n]) for i in range(len(prm.q) - 1)] == [y % q for q in prm.q[:-1]]


def test_mod_down_close_to_division_by_P():
    prm = params.config_kernel_batch()
    qm = prm.q[:5]
    pm = prm.p
    mods = qm + pm
    xs, rows = _rand_rns(mods, 32, 4)
    out = rns.mod_down(rows, qm, pm)
    P = rns.prod(pm)
    Q = rns.prod(qm)
    rec = rns.crt(out, qm)
    for n, x in enumerate(xs):
        diff = (int(rec[n]) - x // P) % Q
        diff = diff - Q if diff > Q // 2 else diff
        assert abs(diff) <= len(pm)


def test_mod_up_digit():
    prm = params.config_tiny()
    qm = prm.q
    xs, rows = _rand_rns(qm, 16, 5)
    D = [1, 2]
    ext = rns.mod_up(rows, qm, D, prm.p)
    QD = qm[1] * qm[2]
    mods = qm + prm.p
    for n, x in enumerate(xs):
        xd = x % QD
        xc = xd - QD if 2 * xd > QD else xd          # centred representative
        cands = [[(xc + e * QD) % m for m in mods] for e in range(-(len(D) // 2) - 1, len(D) // 2 + 2)]
        assert [int(ext[i][n]) for i in range(len(mods))] in cands


def test_mod_up_extension_is_centred():
    """The extended digit, read as an integer through the CRT over all limbs,
    is x_c + e*Q_D with x_c the centred representative of the digit and
    |e| <= |D|/2 + 1; over many coefficients its mean is ~0 relative to Q_D
    (the uncentred conversion averages Q_D/2 or more)."""
    prm = params.config_tiny()
    qm = prm.q
    xs, rows = _rand_rns(qm, 400, 9)
    D = [0, 1]
    ext = rns.mod_up(rows, qm, D, prm.p)
    mods = qm + prm.p
    M = rns.prod(mods)
    QD = qm[0] * qm[1]
    rec = rns.crt(ext, mods)
    vals = []
    for n, x in enumerate(xs):
        v = int(rec[n])
        v = v - M if v > M // 2 else v
        xd = x % QD
        xc = xd - QD if 2 * xd > QD else xd
        e, r = divmod(v - xc, QD)
        assert r == 0 and abs(e) <= len(D) // 2 + 1
        vals.append(v / QD)
    assert abs(sum(vals) / len(vals)) < 0.15
