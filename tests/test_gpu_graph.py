"""HIP graphs of evaluation sequences: the batched key-switching step of the
benchmark (HMult of 64 ciphertexts, a rotate-and-sum chain and a
conjugation at N = 2^16) and one encrypted MF epoch are captured once and
launched; every launch gives the same ciphertexts as the same calls run
eagerly, also after eager work and synchronisations between launches."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CHAIN = [1, 2, 4, 1 << 14]


def _same(ctx, h1, h2):
    a, l1, s1 = ctx.export_ct(h1)
    b, l2, s2 = ctx.export_ct(h2)
    assert (l1, s1) == (l2, s2) and np.array_equal(a, b)


def _step(ctx, cts):
    prods = ctx.hmult_batch(cts, cts[1:] + cts[:1])
    cur, owned = list(cts), []
    for r in CHAIN:
        nxt = ctx.rotate_add_batch(cur, cur, r)
        for h in owned:
            ctx.free(h)
        cur = owned = nxt
    conj = ctx.conjugate_batch(cur)
    return prods, cur, conj


def test_key_switch_step_graph_equals_eager():
    import paper_2509_03024_amd as pk
    ctx = pk.Context(pk.kernel_batch_params(), workloads.CRYPTO_SEED)
    ctx.keygen(CHAIN, conj=True)
    ctx.set_schedule(2048, 0, 0)
    cts = []
    for i in range(64):
        x = workloads.random_residues(ctx.moduli[: ctx.L + 1], ctx.N, 2, seed=1000 + i)
        cts.append(ctx.import_ct(x, ctx.L, 2.0 ** 40))
    eager = _step(ctx, cts)
    ctx.sync()
    ctx.graph_begin()
    with pytest.raises(pk.CsrmfError) as e:          # waiting for the device cannot be captured
        ctx.export_ct(cts[0])
    assert e.value.name == "STATE"
    cap = _step(ctx, cts)
    g = ctx.graph_end()
    for rep in range(3):
        ctx.graph_launch(g)
        ctx.sync()
        for ge, gc in zip(eager, cap):
            for i in (0, 17, 63):
                _same(ctx, ge[i], gc[i])
        # eager work between launches (its own allocations and syncs)
        h = ctx.rotate(cts[rep], 1)
        ctx.export_ct(h)
        ctx.free(h)
    ctx.graph_destroy(g)
    ctx.close()


def test_mf_epoch_graph_equals_eager():
    import paper_2509_03024_amd as pk
    csr = workloads.tiny_ratings()
    U0, V0 = workloads.init_factors(32, 64, 4)

    def run(capture):
        ctx = pk.Context(pk.tiny_params(k=4, lr=0.01, lam=0.02, rule=1), workloads.CRYPTO_SEED)
        ctx.keygen([])
        m = pk.MF(ctx)
        m.encrypt_csr_rows(32, 64, csr.row_ptr, csr.col_idx, csr.values)
        m.init_factors(U0, V0)
        ctx.sync()
        if capture:
            ctx.graph_begin()
            m.epochs(1)
            g = ctx.graph_end()
            ctx.graph_launch(g)
            ctx.sync()
        else:
            m.epochs(1)
        out = [ctx.export_ct(h) for w in (1, 2, 5) for h in m.handles(w)]
        return ctx, out

    ce, e = run(False)
    cg, c = run(True)
    for (a, la, sa), (b, lb, sb) in zip(e, c):
        assert (la, sa) == (lb, sb) and np.array_equal(a, b)
    ce.close()
    cg.close()
