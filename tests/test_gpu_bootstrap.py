"""GPU parity of bootstrapping (csrmf_bootstrap).

N = 2^12 test chain (q_0 + 18 x 40-bit, 3 x 60-bit special, dnum 5): two
ciphertexts encrypted at level 0 are bootstrapped as one batch and one at a
time; each output is compared with the oracle's through the SHA-256 digests
that tests/golden/make_boot_n12.py wrote from the oracle alone, after checking
that the inputs themselves equal the oracle's.  At N = 2^16 (the MF chain,
dnum 7) the bootstrap's values are checked against its inputs."""
import os

import numpy as np
import pytest

import workloads
from tests.golden import make_boot_n12 as gold

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _digest_of(ctx, h):
    got, lvl, scale = ctx.export_ct(h)
    return lvl, scale, gold.digest(got[0], got[1])


@pytest.fixture(scope="module")
def n12():
    import paper_2509_03024_amd as pk
    golden, meta = gold.read(os.path.join(HERE, "golden", "boot_n12.txt"))
    ctx = pk.Context(pk.params(*gold.CHAIN), workloads.CRYPTO_SEED)
    cfg = pk.BootConfig(gold.N_SLOTS, gold.SQUARINGS, gold.DEGREE, gold.PRE_BITS)
    ctx.keygen(ctx.boot_rotation_steps(cfg), conj=True)
    cts = [ctx.encrypt(gold.values(i, ctx.N), level=0, scale=gold.SCALE) for i in range(gold.N_CT)]
    edge = ctx.encrypt(gold.edge_values(ctx.N), level=gold.EDGE_LEVEL, scale=gold.SCALE)   # serial 2
    asn = ctx.encrypt(gold.arcsine_values(ctx.N), level=0, scale=gold.SCALE)               # serial 3
    yield pk, ctx, cfg, cts + [edge, asn], golden
    ctx.close()


def test_inputs_equal_the_oracles(n12):
    pk, ctx, cfg, cts, golden = n12
    for i, h in enumerate(cts[:2]):
        assert _digest_of(ctx, h) == golden[("input", i)], f"input {i}"
    assert _digest_of(ctx, cts[2]) == golden[("edge_input", 0)]
    assert _digest_of(ctx, cts[3]) == golden[("arcsine_input", 0)]


def test_bootstrap_batch_matches_the_oracle(n12):
    pk, ctx, cfg, cts, golden = n12
    assert pk.boot_levels(cfg) == 17
    out = ctx.bootstrap(cts[:2], cfg)
    for i, h in enumerate(out):
        lvl, scale, dg = _digest_of(ctx, h)
        want = golden[("boot", i)]
        assert (lvl, scale) == want[:2], f"bootstrap {i}: level/scale"
        assert dg == want[2], f"bootstrap {i}: ciphertext differs from the oracle's"
        got = ctx.decrypt(h)
        assert np.max(np.abs(got - gold.values(i, ctx.N))) < 1e-3
    for h in out:
        ctx.free(h)


def test_bootstrap_of_one_ciphertext_matches_the_oracle(n12):
    pk, ctx, cfg, cts, golden = n12
    out = ctx.bootstrap([cts[1]], cfg)
    assert _digest_of(ctx, out[0]) == golden[("boot", 1)]
    ctx.free(out[0])


def test_bootstrap_one_slot_from_level_2_matches_the_oracle(n12):
    """n = 1 (CoeffToSlot without rotations, the longest SubSum), the input given
    at level 2 (the bootstrap drops it to level 0 itself)."""
    pk, ctx, cfg, cts, golden = n12
    out = ctx.bootstrap([cts[2]], pk.BootConfig(1, gold.SQUARINGS, gold.DEGREE, gold.PRE_BITS))
    assert _digest_of(ctx, out[0]) == golden[("edge_boot", 0)]
    assert np.max(np.abs(ctx.decrypt(out[0]) - gold.edge_values(ctx.N))) < 1e-3
    ctx.free(out[0])


def test_bootstrap_with_the_arcsine_term_matches_the_oracle(n12):
    """r = 8, degree 16, 2^15 pre-multiplication and the arcsine term: all 18
    levels of the chain, output at level 0."""
    pk, ctx, cfg, cts, golden = n12
    acfg = pk.BootConfig(gold.N_SLOTS, 8, 16, 15, 1)
    assert pk.boot_levels(acfg) == 18
    out = ctx.bootstrap([cts[3]], acfg)
    assert _digest_of(ctx, out[0]) == golden[("arcsine_boot", 0)]
    assert np.max(np.abs(ctx.decrypt(out[0]) - gold.arcsine_values(ctx.N))) < 1e-3
    ctx.free(out[0])


def test_bootstrap_argument_errors(n12):
    pk, ctx, cfg, cts, golden = n12
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap(cts, pk.BootConfig(3, gold.SQUARINGS, gold.DEGREE, gold.PRE_BITS))     # n not a power of 2
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap(cts[:1], pk.BootConfig(ctx.N // 2, 0, 1, 0))                          # n above N/4
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap(cts, pk.BootConfig(gold.N_SLOTS, 12, gold.DEGREE, gold.PRE_BITS))      # 20 levels > 18
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap(cts, pk.BootConfig(64, gold.SQUARINGS, gold.DEGREE, gold.PRE_BITS))    # keys for n = 64 absent
    other = ctx.mul_int(cts[0], 3)
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap([cts[1], other], cfg)                                                   # scales differ
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap([], cfg)                                                                # empty batch
    with pytest.raises(pk.CsrmfError):
        ctx.bootstrap(cts[:1], pk.BootConfig(gold.N_SLOTS, gold.SQUARINGS, gold.DEGREE, gold.PRE_BITS, 2))
    ctx.free(other)


def test_bootstrap_n16_values():
    """N = 2^16, MF chain (q_0 + 24 x 40-bit, dnum 7): n = 16 slots, r = 10 with
    a degree-16 series (|I| up to about 360 for the dense secret keeps the
    series' argument below 2.3), 2^15 pre-multiplication with the arcsine
    term, 20 levels; a batch of 4.  The error is the rescale noise at scale
    2^40 times about 2^(r+1) from the squarings and q_0 / (4 pi 2^55) sqrt(2n)
    from SlotToCoeff."""
    import paper_2509_03024_amd as pk
    ctx = pk.Context(pk.mf_n16_params(), workloads.CRYPTO_SEED)
    cfg = pk.BootConfig(16, 10, 16, 15, 1)
    ctx.keygen(ctx.boot_rotation_steps(cfg), conj=True)
    vals = [np.tile(np.random.default_rng(200 + i).uniform(-1, 1, 16), ctx.N // 32) for i in range(4)]
    cts = [ctx.encrypt(v, level=0, scale=2.0 ** 40) for v in vals]
    out = ctx.bootstrap(cts, cfg)
    for h, v in zip(out, vals):
        lvl, scale = ctx.info(h)[:2]
        assert lvl == ctx.L - pk.boot_levels(cfg) and abs(scale / 2.0 ** 40 - 1) < 1e-6
        assert np.max(np.abs(ctx.decrypt(h) - v)) < 2e-2
    ctx.close()
