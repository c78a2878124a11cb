"""Serving loop on the GPU (N = 2^12 chain, k = 4): PREDICT and UPDATE results
against plaintext arithmetic, a row cut into two chunks, and the same request
giving bit-identical result ciphertexts alone and inside a mix of other
requests (continuous batching changes only how launches are grouped)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

LR, LAM, K = 0.05, 0.02, 4


def _params():
    """N = 2^12, q_0 + 5 x 40-bit, 2 x 60-bit special primes, dnum 3: an UPDATE uses 4 levels."""
    import paper_2509_03024_amd as pk
    return pk.params(12, 60, 5, 40, 2, 60, 3, 40, k=K, lr=LR, lam=LAM, rule=2)


def _server(n_users=32, n_items=600, sigma=0.1):
    import paper_2509_03024_amd as pk
    U0, V0 = workloads.init_factors(n_users, n_items, K, seed=5, sigma=sigma)
    ctx = pk.Context(_params(), workloads.CRYPTO_SEED)
    ctx.keygen([])
    srv = pk.Server(ctx, U0, V0, hbm_budget_bytes=8e9, max_batch=32)
    return ctx, srv, U0, V0


def _row(rng, n_items, d):
    items = np.sort(rng.choice(n_items, size=d, replace=False)).astype(np.int32)
    return items, np.rint(np.clip(rng.normal(3.5, 1.1, d), 1, 5))


def test_predict_and_update_values():
    ctx, srv, U0, V0 = _server()
    rng = np.random.default_rng(3)
    B = 8
    items, r = _row(rng, 600, 40)
    rid = srv.submit(srv.PREDICT, 3, items)
    st, res, lat = srv.poll(rid, wait=True)
    assert st == 2 and len(res) == 1 and lat > 0
    z = ctx.decrypt(res[0])
    assert np.max(np.abs(z[np.arange(40) * B] - V0[items] @ U0[3])) < 1e-4
    # UPDATE on a row longer than D = 256 blocks: two chunks
    items, r = _row(rng, 600, 300)
    rid = srv.submit(srv.UPDATE, 7, items, r, client_serial=11)
    st, res, lat = srv.poll(rid, wait=True)
    assert st == 2 and len(res) == 1
    u = U0[7]
    e = r - V0[items] @ u
    want = (1 - LR * LAM) * u + (LR / len(items)) * (e[:, None] * V0[items]).sum(0)
    assert np.max(np.abs(ctx.decrypt(res[0])[:K] - want)) < 1e-4
    srv.close()
    ctx.close()


def test_result_identical_alone_and_in_a_mix():
    rng = np.random.default_rng(9)
    x_items, x_r = _row(rng, 600, 120)
    y_items, _ = _row(rng, 600, 30)
    others = [(_row(rng, 600, int(rng.integers(5, 200))), int(rng.integers(0, 32)), int(rng.integers(0, 2)))
              for _ in range(12)]

    ctx_a, srv_a, _, _ = _server()
    xa = srv_a.submit(srv_a.UPDATE, 5, x_items, x_r, client_serial=77)
    ya = srv_a.submit(srv_a.PREDICT, 9, y_items, client_serial=78)
    ra = srv_a.poll(xa, wait=True)[1] + srv_a.poll(ya, wait=True)[1]

    ctx_b, srv_b, _, _ = _server()
    ids = []
    for n, ((it, rr), user, op) in enumerate(others[:6]):
        ids.append(srv_b.submit(op, user, it, rr if op else None, client_serial=1000 + n))
    xb = srv_b.submit(srv_b.UPDATE, 5, x_items, x_r, client_serial=77)
    for n, ((it, rr), user, op) in enumerate(others[6:]):
        ids.append(srv_b.submit(op, user, it, rr if op else None, client_serial=2000 + n))
    yb = srv_b.submit(srv_b.PREDICT, 9, y_items, client_serial=78)
    rb = srv_b.poll(xb, wait=True)[1] + srv_b.poll(yb, wait=True)[1]
    for i in ids:
        assert srv_b.poll(i, wait=True)[0] == 2
    assert srv_b.stats()["max_batch"] > 1, "the mix was never batched"
    for ha, hb in zip(ra, rb):
        ea, la, sa = ctx_a.export_ct(ha)
        eb, lb, sb = ctx_b.export_ct(hb)
        assert la == lb and sa == sb and np.array_equal(ea, eb)
    for s, c in ((srv_a, ctx_a), (srv_b, ctx_b)):
        s.close()
        c.close()


def test_admission_rejects_oversized_request():
    import paper_2509_03024_amd as pk
    U0, V0 = workloads.init_factors(32, 64, K, seed=5)
    ctx = pk.Context(_params(), workloads.CRYPTO_SEED)
    ctx.keygen([])
    srv = pk.Server(ctx, U0, V0, hbm_budget_bytes=1e6, max_batch=4)   # below one request's footprint
    with pytest.raises(pk.CsrmfError) as e:
        srv.submit(srv.PREDICT, 0, np.arange(10, dtype=np.int32))
    assert e.value.name == "NOMEM"
    with pytest.raises(pk.CsrmfError):
        srv.submit(srv.PREDICT, 0, np.array([3, 2], dtype=np.int32))   # unsorted row
    srv.close()
    ctx.close()
