"""Pins of the oracle's CKKS back end for the encrypted MF program
(oracle.program.CkksBackend), each against a fact fixed independently of it:

* the block mask I_p = tau_{g_p}(I_0) decodes to the indicator of slots
  pB .. pB+k-1, within the rounding bound of the encoder (N/2 units of the
  mask scale: each of the N integer coefficients is off by at most 1/2);
* the integer weights W follow round-half-even on hand-computed cases;
* mask_mul multiplies the slots by const + sum_m W_m * S_I * 1[block p_m]
  (decrypted, against the ideal indicator with the stated error bound);
* refresh returns a fresh top-level encryption of the same plaintext (the
  mask it adds for the key holder is removed again).
"""
import numpy as np
import pytest

from oracle import ckks, params, program
import workloads

K = 4


@pytest.fixture(scope="module")
def tiny():
    prm = params.config_tiny()
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    ctx.keygen()
    masks = program.block_masks(ctx, K)
    be = program.CkksBackend(ctx, masks)
    lay = program.make_layout(prm.N, K, 1, 1, np.array([0, 0]), np.array([], np.int64))
    be.set_block(lay.B)
    return ctx, be, lay


@pytest.mark.parametrize("scale", [program.S_I, program.S_IG])
@pytest.mark.parametrize("p", [0, 1, 37, 255])
def test_mask_decodes_to_the_block_indicator(tiny, p, scale):
    ctx, be, lay = tiny
    N, B = ctx.N, lay.B
    m = be._mask(p, scale)
    z = ctx.decode(np.array([int(v) for v in m], dtype=np.int64), scale)
    ind = np.zeros(N // 2)
    ind[p * B: p * B + K] = 1.0
    # rounding each coefficient by at most 1/2 moves a slot by at most N/2 units
    assert np.max(np.abs(z - ind)) <= (N / 2) / scale + 1e-9


def test_weight_rounding_hand_cases():
    # rint((w * target * q) / (s_src * mask_scale)), halves to even
    assert program.weight(0.5, 1.0, 5.0, 1.0, False, 1.0) == 2       # 2.5 -> 2
    assert program.weight(1.5, 1.0, 5.0, 1.0, False, 1.0) == 8       # 7.5 -> 8
    assert program.weight(-0.5, 1.0, 5.0, 1.0, False, 1.0) == -2     # -2.5 -> -2
    assert program.weight(1.0, 2.0 ** 40, 2.0 ** 40, 2.0 ** 30, False, 2.0 ** 40) == 1024
    assert program.weight(0.01, 2.0 ** 40, 2.0 ** 41, 2.0 ** 24, False, 2.0 ** 50) == 1342177   # 1342177.28
    assert program.weight(0.3, 7.0, 11.0, 13.0, True, 17.0) == 0.3  # exact weights pass through


def test_mask_mul_multiplies_slots_by_the_masked_weights(tiny):
    ctx, be, lay = tiny
    N, B = ctx.N, lay.B
    scale = 2.0 ** 30
    z = np.random.default_rng(2).uniform(-1, 1, N // 2)
    ct = ctx.encrypt(z, level=ctx.prm.L, scale=scale)
    const, terms = 1 << 22, [(2, 3), (5, -5)]
    out = be.mask_mul(ct, terms, scale * program.S_I, program.S_I, const=const)
    assert out.level == ct.level and out.scale == scale * program.S_I
    got = ctx.decode(ctx.decrypt_int(out), scale)
    mult = np.full(N // 2, float(const))
    for p, W in terms:
        mult[p * B: p * B + K] += W * program.S_I
    # mask rounding: at most (N/2) * (|3| + |-5|) per slot; ciphertext noise times the
    # mask's slot values (~1e8) is below 1e4 at scale 2^30
    err = np.abs(got - z * mult)
    assert np.max(err) < (N / 2) * 8 + 1e4
    assert np.min(np.abs(mult[2 * B: 2 * B + K])) > 1e7 and np.min(np.abs(mult[5 * B: 5 * B + K])) > 1e7


def test_refresh_reencrypts_the_same_plaintext(tiny):
    ctx, be, lay = tiny
    z = np.random.default_rng(3).uniform(-1, 1, ctx.N // 2)
    ct = ctx.encrypt(z, level=1, scale=2.0 ** 40)
    saved = ctx.serial
    fresh = be.refresh(ct, 7)
    assert ctx.serial == saved                      # refresh uses its own serial numbers
    assert fresh.level == ctx.prm.L and fresh.scale == ct.scale
    # the mask (|coefficients| up to 2^50) is gone: the difference is encryption noise
    d = ctx.decrypt_int(fresh) - ctx.decrypt_int(ct)
    assert np.max(np.abs(d)) < 2 ** 12
    assert np.max(np.abs(ctx.decrypt(fresh) - z)) < 1e-6
