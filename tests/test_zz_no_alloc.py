"""The allocation-free rotation (csrmf_rotate_noalloc) against csrmf_rotate,
through the C ABI: bit-identical outputs on two calls in a row into the same
output ciphertext, the second with a smaller input (a lower level); a
rotation whose scratch exceeds the static buffer is refused."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _same(ctx, h1, h2):
    a, l1, s1 = ctx.export_ct(h1)
    b, l2, s2 = ctx.export_ct(h2)
    assert (l1, s1) == (l2, s2)
    assert np.array_equal(a, b)


def test_noalloc_rotation_equals_rotate_on_two_calls():
    import paper_2509_03024_amd as pk
    ctx = pk.Context(pk.mf_n15_params(), workloads.CRYPTO_SEED)
    ctx.keygen([1, 5])
    L = ctx.L
    rng = np.random.default_rng(21)
    big = ctx.encrypt(rng.uniform(-1, 1, ctx.N // 2), L, 2.0 ** 40)
    small = ctx.encrypt(rng.uniform(-1, 1, ctx.N // 2), 2, 2.0 ** 40)
    out = ctx.encrypt(np.zeros(4), L, 2.0 ** 40)          # the caller's output ciphertext
    ctx.rotate_noalloc(big, 5, out)
    _same(ctx, out, ctx.rotate(big, 5))
    ctx.rotate_noalloc(small, 1, out)                        # smaller input, same output buffer
    _same(ctx, out, ctx.rotate(small, 1))
    assert ctx.info(out)[0] == 2
    with pytest.raises(pk.CsrmfError) as e:
        ctx.rotate_noalloc(big, 1, big)
    assert e.value.name == "INVAL"
    ctx.close()


def test_noalloc_rejects_scratch_beyond_the_buffer():
    import paper_2509_03024_amd as pk
    ctx = pk.Context(pk.mf_n16_params(), workloads.CRYPTO_SEED)   # 7 digits of 4 limbs at N = 2^16
    ctx.keygen([1])
    a = ctx.encrypt(np.ones(4), ctx.L, 2.0 ** 40)
    out = ctx.encrypt(np.zeros(4), ctx.L, 2.0 ** 40)
    with pytest.raises(pk.CsrmfError) as e:
        ctx.rotate_noalloc(a, 1, out)
    assert e.value.name == "INVAL" and "MiB of scratch" in str(e.value)
    b = ctx.mod_drop(a, 12)                                  # 4 digits at level 12 fit
    ctx.rotate_noalloc(b, 1, out)
    _same(ctx, out, ctx.rotate(b, 1))
    ctx.close()
