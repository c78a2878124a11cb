"""GPU parity of the CKKS primitives: every ciphertext the HIP library produces
is compared residue by residue (coefficient form) with the CPU oracle's, from
the same seed and the same integer plaintexts."""
import numpy as np
import pytest

from oracle import ckks, params, ring
import workloads
from tests.gpu_util import to_device_u64, from_device_u64, brev

pytestmark = pytest.mark.gpu

SEED = workloads.CRYPTO_SEED
STEPS = [1, 2, 3, -4, 5, 16]


@pytest.fixture(scope="module")
def pair():
    import torch
    assert torch.cuda.is_available()
    import paper_2509_03024_amd as pk
    lib = pk.Context(pk.tiny_params(), SEED)
    lib.keygen(STEPS, conj=True)
    orc = ckks.Context(params.config_tiny(), SEED)
    orc.keygen(rot_steps=STEPS, conj=True)
    yield lib, orc
    lib.close()


def _enc_pair(lib, orc, seed, level=None, scale=2.0 ** 40, lo=-1.0, hi=1.0):
    level = orc.prm.L if level is None else level
    z = np.random.default_rng(seed).uniform(lo, hi, orc.N // 2)
    m = orc.encode(z, scale)
    return lib.encrypt_int(m, level, scale), orc.encrypt_int(m, level, scale), z


def _same(lib, h, oct_):
    got, lvl, scale = lib.export_ct(h)
    assert lvl == oct_.level
    assert scale == oct_.scale
    assert np.array_equal(got[0], oct_.c0), "c0 differs"
    assert np.array_equal(got[1], oct_.c1), "c1 differs"


def test_chain_matches_oracle(pair):
    lib, orc = pair
    assert lib.moduli == orc.moduli


@pytest.mark.parametrize("logN", [12, 15, 16])
def test_forward_ntt_is_evaluation_in_bit_reversed_order(logN):
    """Every split of the butterfly stages between the two passes (6 to 9
    stages each) gives the oracle's transform, and the inverse undoes it."""
    import paper_2509_03024_amd as pk
    prm = {12: params.config_tiny, 15: params.config_mf_n15, 16: params.config_kernel_batch}[logN]()
    lp = {12: pk.tiny_params(), 15: pk.mf_n15_params(), 16: pk.kernel_batch_params()}[logN]
    lib = pk.Context(lp, SEED)
    N = 1 << logN
    mods = prm.moduli
    limbs = [0, 1, len(prm.q) - 1, len(mods) - 1]
    x = workloads.random_residues([mods[i] for i in limbs], N, 2, seed=logN)   # [2][4][N]
    perm = np.array([brev(i, logN) for i in range(N)])
    want = np.array([[ring.ntt(x[b, r], mods[li], prm.psi[li])[perm] for r, li in enumerate(limbs)]
                     for b in range(2)])
    splits = [s for s in range(6, 10) if 6 <= logN - s <= 9]
    assert lib.schedule()["ntt_split"] == logN // 2
    for split in splits:
        lib.set_schedule(0, 0, 0, split)
        t = to_device_u64(x.reshape(-1, N))
        lib.ntt_rows(t.data_ptr(), 8, limbs, inverse=False)
        y = from_device_u64(t).reshape(2, 4, N)
        for b in range(2):
            for r, li in enumerate(limbs):
                assert np.array_equal(y[b, r], want[b, r]), (split, b, li)
        lib.ntt_rows(t.data_ptr(), 8, limbs, inverse=True)
        assert np.array_equal(from_device_u64(t).reshape(2, 4, N), x), split
    with pytest.raises(RuntimeError):
        lib.set_schedule(0, 0, 0, logN - 5)       # a row pass of 5 stages
    lib.close()


def test_keys_match(pair):
    lib, orc = pair
    assert np.array_equal(lib.export_key(0), orc.s)
    pk_ = lib.export_key(1)
    assert np.array_equal(pk_[0], orc.pk[0]) and np.array_equal(pk_[1], orc.pk[1])
    rk = lib.export_key(2)
    for j, b, a in orc.relin_key:
        assert np.array_equal(rk[j, 0], b) and np.array_equal(rk[j, 1], a)
    g = ckks.galois_for_step(-4, orc.N)
    gk = lib.export_key(3, g)
    for j, b, a in orc.rot_keys[g]:
        assert np.array_equal(gk[j, 0], b) and np.array_equal(gk[j, 1], a)


def test_encrypt_decrypt(pair):
    lib, orc = pair
    h, o, z = _enc_pair(lib, orc, 1)
    _same(lib, h, o)
    assert np.array_equal(lib.decrypt_int(h), orc.decrypt_int(o))
    assert np.max(np.abs(lib.decrypt(h) - z)) < 1e-6
    h2, o2, z2 = _enc_pair(lib, orc, 2, level=1)
    _same(lib, h2, o2)


def test_add_sub_plain_ops(pair):
    lib, orc = pair
    ha, oa, za = _enc_pair(lib, orc, 3)
    hb, ob, zb = _enc_pair(lib, orc, 4, level=2)
    _same(lib, lib.add(ha, hb), orc.add(oa, ob))
    _same(lib, lib.sub(ha, hb), orc.sub(oa, ob))
    m = orc.encode(zb, float(orc.prm.q[-1]))
    _same(lib, lib.mul_plain(ha, m, float(orc.prm.q[-1])), orc.mul_plain(oa, m, float(orc.prm.q[-1])))
    _same(lib, lib.add_plain(ha, m), orc.add_plain(oa, m))
    _same(lib, lib.mul_int(ha, -12345), orc.mul_int(oa, -12345))


def test_hmult_relin_rescale(pair):
    lib, orc = pair
    ha, oa, za = _enc_pair(lib, orc, 5)
    hb, ob, zb = _enc_pair(lib, orc, 6)
    d0, d1, d2, sc = orc.tensor(oa, ob)
    _same(lib, lib.mul_relin(ha, hb), orc.relinearize(d0, d1, d2, sc))
    hp = lib.hmult(ha, hb)
    op = orc.hmult(oa, ob)
    _same(lib, hp, op)
    _same(lib, lib.rescale(lib.mul_relin(ha, hb)), op)
    _same(lib, lib.hmult(hp, ha), orc.hmult(op, oa))
    assert np.max(np.abs(lib.decrypt(hp) - za * zb)) < 1e-6


@pytest.mark.parametrize("r", [1, 2, 3, -4, 5, 16])
def test_rotation(pair, r):
    lib, orc = pair
    h, o, z = _enc_pair(lib, orc, 10 + r)
    _same(lib, lib.rotate(h, r), orc.rotate(o, r))


def test_rotate_add_batch(pair):
    """acc + Rot(a, r) with the addition fused into the key switch equals the
    oracle's rotation followed by its addition; also with acc = a, with an
    accumulator above a's level, and for r = 0 (a plain addition)."""
    lib, orc = pair
    hs = [_enc_pair(lib, orc, 60 + i) for i in range(3)]
    acc = [_enc_pair(lib, orc, 70 + i) for i in range(3)]
    a = [h for h, _, _ in hs]
    out = lib.rotate_add_batch(a, [h for h, _, _ in acc], 3)
    for (h, o, _), (ha, oa, _), ho in zip(hs, acc, out):
        _same(lib, ho, orc.add(oa, orc.rotate(o, 3)))
    out = lib.rotate_add_batch(a, a, 5)
    for (h, o, _), ho in zip(hs, out):
        _same(lib, ho, orc.add(o, orc.rotate(o, 5)))
    hl, ol, _ = _enc_pair(lib, orc, 80, level=1)
    (ho,) = lib.rotate_add_batch([hl], [hs[0][0]], 1)
    _same(lib, ho, orc.add(hs[0][1], orc.rotate(ol, 1)))
    (ho,) = lib.rotate_add_batch([a[1]], [a[2]], 0)
    _same(lib, ho, orc.add(hs[2][1], hs[1][1]))


def test_rotation_lower_level_and_conjugate(pair):
    lib, orc = pair
    h, o, z = _enc_pair(lib, orc, 30, level=1)
    _same(lib, lib.rotate(h, 3), orc.rotate(o, 3))
    _same(lib, lib.conjugate(h), orc.conjugate(o))


def test_hoisted_rotations(pair):
    lib, orc = pair
    h, o, z = _enc_pair(lib, orc, 31)
    hs = lib.rotate_hoisted(h, [1, 2, 5, 16])
    os_ = orc.hoisted_rotations(o, [1, 2, 5, 16])
    for hh, r in zip(hs, [1, 2, 5, 16]):
        _same(lib, hh, os_[r])


def test_batched_equals_single(pair):
    lib, orc = pair
    hs = [_enc_pair(lib, orc, 40 + i) for i in range(4)]
    a = [h for h, _, _ in hs]
    b = a[1:] + a[:1]
    prods = lib.hmult_batch(a, b)
    for i in range(4):
        _same(lib, prods[i], orc.hmult(hs[i][1], hs[(i + 1) % 4][1]))
    rots = lib.rotate_batch(prods, 2)
    for i in range(4):
        _same(lib, rots[i], orc.rotate(orc.hmult(hs[i][1], hs[(i + 1) % 4][1]), 2))
    sums = lib.add_batch(a, b)
    diffs = lib.add_batch(a, b, subtract=True)
    for i in range(4):
        _same(lib, sums[i], orc.add(hs[i][1], hs[(i + 1) % 4][1]))
        _same(lib, diffs[i], orc.sub(hs[i][1], hs[(i + 1) % 4][1]))
    conj = lib.conjugate_batch(a)
    for i in range(4):
        _same(lib, conj[i], orc.conjugate(hs[i][1]))


def test_autotune_installs_its_choice(pair):
    """The tuner keeps the schedule its report names (transform schedules
    ranked again on batched rotations, the context having rotation keys), and
    results under it keep the oracle's bits."""
    lib, orc = pair
    rep = lib.autotune()
    s = lib.schedule()
    assert (s["ntt_chunk_rows"], s["ntt_cached_mid"], s["ntt_split"], s["modup_chunk"]) == \
        (rep["chosen"], rep["cached_mid"], rep["ntt_split"], rep["modup_chunk"])
    ranked = [k for k in rep if k.startswith("rotation ")]
    assert 1 <= len(ranked) <= 4
    assert list(rep["chosen_by_rotation"]) == [s["ntt_split"], s["ntt_chunk_rows"], s["ntt_cached_mid"]]
    h, o, _ = _enc_pair(lib, orc, 60)
    _same(lib, lib.rotate(h, 3), orc.rotate(o, 3))
    lib.set_schedule(0, 0, 0)


def test_import_export_roundtrip(pair):
    lib, orc = pair
    h, o, z = _enc_pair(lib, orc, 50)
    got, lvl, sc = lib.export_ct(h)
    h2 = lib.import_ct(got, lvl, sc)
    _same(lib, h2, o)


def test_error_codes(pair):
    import paper_2509_03024_amd as pk
    lib, orc = pair
    h, o, z = _enc_pair(lib, orc, 60, level=0)
    with pytest.raises(pk.CsrmfError) as e:
        lib.rescale(h)
    assert e.value.name == "LEVEL"
    h2, o2, z2 = _enc_pair(lib, orc, 61)
    with pytest.raises(pk.CsrmfError) as e:
        lib.rotate(h2, 7)
    assert e.value.name == "KEY"
    h3 = lib.encrypt_int(orc.encode(z2, 2.0 ** 30), 3, 2.0 ** 30)
    orc.serial += 1
    with pytest.raises(pk.CsrmfError) as e:
        lib.add(h2, h3)
    assert e.value.name == "SCALE"
    with pytest.raises(pk.CsrmfError) as e:
        lib.export_ct(987654321)
    assert e.value.name == "INVAL"
