"""GPU parity of key switching at N = 2^16 on the shapes the benchmark runs:
the kernel-batch chain (q_0 + 24 x 40-bit, 3 x 60-bit special, dnum 3, so
ModUp converts digits of 9, 9 and 7 limbs at the top level) and the MF chain
at N = 2^16 (4-limb digits, dnum 7).  Inputs are the benchmark's uniform
random residues; each output ciphertext is compared with the oracle's through
the SHA-256 digests that tests/golden/make_ks_n16.py wrote from the oracle
alone.  Batched calls process all 64 ciphertexts (two sampled outputs are
compared) under the benchmark's NTT schedule (2048 rows per pair of passes)."""
import os

import numpy as np
import pytest

import workloads
from tests.golden import make_ks_n16 as gold

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
N_CT = 64


def _load(ctx, i):
    x = workloads.random_residues(ctx.moduli[: ctx.L + 1], ctx.N, 2, seed=1000 + i)
    return ctx.import_ct(x, ctx.L, gold.SCALE)


def _check(ctx, h, want, what):
    got, lvl, scale = ctx.export_ct(h)
    assert (lvl, scale) == want[:2], what
    assert gold.digest(got[0], got[1]) == want[2], f"{what}: ciphertext differs from the oracle's"


@pytest.fixture(scope="module")
def kb():
    import paper_2509_03024_amd as pk
    golden = gold.read(os.path.join(HERE, "golden", "ks_kernel_batch_n16.txt"))
    ctx = pk.Context(pk.kernel_batch_params(), workloads.CRYPTO_SEED)
    ctx.keygen(sorted({gold.ROT_STEP, gold.ROTADD_STEP, *gold.HOIST_STEPS}), conj=True)
    ctx.set_ntt_schedule(2048)
    cts = [_load(ctx, i) for i in range(N_CT)]
    yield ctx, cts, golden
    ctx.close()


def test_hmult_batch_of_64(kb):
    ctx, cts, golden = kb
    prods = ctx.hmult_batch(cts, cts[1:] + cts[:1])
    for i in gold.SAMPLES:
        _check(ctx, prods[i], golden[("hmult", i)], f"HMult {i}")
    for h in prods:
        ctx.free(h)


def test_rotate_batch_of_64(kb):
    ctx, cts, golden = kb
    rots = ctx.rotate_batch(cts, gold.ROT_STEP)
    for i in gold.SAMPLES:
        _check(ctx, rots[i], golden[("rotate", i)], f"rotation {i}")
    for h in rots:
        ctx.free(h)


def test_conjugate_batch_of_64(kb):
    ctx, cts, golden = kb
    out = ctx.conjugate_batch(cts)
    for i in gold.SAMPLES:
        _check(ctx, out[i], golden[("conj", i)], f"conjugation {i}")
    for h in out:
        ctx.free(h)


def test_rotate_add_batch_of_64(kb):
    ctx, cts, golden = kb
    out = ctx.rotate_add_batch(cts, cts, gold.ROTADD_STEP)
    for i in gold.SAMPLES:
        _check(ctx, out[i], golden[("rotadd", i)], f"rotate-and-add {i}")
    for h in out:
        ctx.free(h)


def test_hoisted_fan_out(kb):
    ctx, cts, golden = kb
    out = ctx.rotate_hoisted(cts[gold.HOIST_SOURCE], list(gold.HOIST_STEPS))
    for h, r in zip(out, gold.HOIST_STEPS):
        _check(ctx, h, golden[("hoisted", r)], f"hoisted rotation by {r}")
        ctx.free(h)


def test_one_ciphertext_per_call_path(kb):
    """The plain path (one ciphertext per call, the whole-batch NTT schedule)."""
    ctx, cts, golden = kb
    ctx.set_ntt_schedule(0)
    try:
        i = gold.SAMPLES[1]
        h = ctx.rotate(cts[i], gold.ROT_STEP)
        _check(ctx, h, golden[("rotate", i)], "single rotation")
        ctx.free(h)
        h = ctx.hmult(cts[i], cts[i + 1])
        _check(ctx, h, golden[("hmult", i)], "single HMult")
        ctx.free(h)
    finally:
        ctx.set_ntt_schedule(2048)


def test_mf_chain_dnum7():
    import paper_2509_03024_amd as pk
    golden = gold.read(os.path.join(HERE, "golden", "ks_mf_n16.txt"))
    ctx = pk.Context(pk.mf_n16_params(), workloads.CRYPTO_SEED)
    ctx.keygen([gold.ROT_STEP])
    a, b = _load(ctx, 0), _load(ctx, 1)
    _check(ctx, ctx.hmult_batch([a], [b])[0], golden[("hmult", 0)], "HMult, dnum 7")
    _check(ctx, ctx.rotate(a, gold.ROT_STEP), golden[("rotate", 0)], "rotation, dnum 7")
    ctx.close()


@pytest.mark.parametrize("sched", [(2048, 1, 16, 7), (256, 1, 8, 9), (0, 0, 32, 8)])
def test_schedules_give_the_same_bits(kb, sched):
    """Cached or streamed NTT intermediates, NTT chunks, ModUp sub-batches and
    the split of the transform's stages between its passes change only the
    order and shape of the launches: the batched rotation and HMult of the 64
    ciphertexts keep the oracle's bits."""
    ctx, cts, golden = kb
    ctx.set_schedule(*sched)
    try:
        rots = ctx.rotate_batch(cts, gold.ROT_STEP)
        prods = ctx.hmult_batch(cts, cts[1:] + cts[:1])
        for i in gold.SAMPLES:
            _check(ctx, rots[i], golden[("rotate", i)], f"rotation {i} under {sched}")
            _check(ctx, prods[i], golden[("hmult", i)], f"HMult {i} under {sched}")
        for h in rots + prods:
            ctx.free(h)
    finally:
        ctx.set_schedule(2048, 0, 0)
