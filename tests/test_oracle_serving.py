"""Pins of the oracle's serving requests (oracle.serving) against plaintext
arithmetic: a PREDICT decrypts to <u_i, v_j> for every item of the row, an
UPDATE to one rule-R2 gradient step of u_i with the items fixed,
    u' = (1 - lr*lambda) u + (lr/d) sum_j (r_j - <u, v_j>) v_j,
within 1e-4, including a row cut into two chunks (k = 16 at N = 2^12, so a
chunk holds D = 64 items).""" 
import numpy as np
import pytest

from oracle import ckks, params, serving
import workloads

K, LR, LAM = 16, 0.05, 0.02
N_USERS, N_ITEMS = 32, 100


def serving_params():
    """N = 2^12, q_0 + 5 x 40-bit, 2 x 60-bit special primes, dnum 3: an UPDATE uses 4 levels."""
    return params.make_params(12, 60, 5, 40, 2, 60, 3, 40, name="serve")


def serving_rotations(st_like_B, kp, D, G):
    steps = set()
    q = 1
    while q < st_like_B:
        steps.add(q)
        q *= 2
    steps.add(-kp)
    steps.update(b * st_like_B for b in range(1, G))
    steps.update(g * G * st_like_B for g in range(1, D // G))
    q = st_like_B
    while q < st_like_B * D:
        steps.add(q)
        q *= 2
    return sorted(steps)


def table_plaintexts(ctx, F, D, B, k, scale=2.0 ** 40):
    n_tab = -(-F.shape[0] // D)
    Z = np.zeros((n_tab, ctx.N // 2))
    for e in range(F.shape[0]):
        a, b = divmod(e, D)
        Z[a, b * B: b * B + k] = F[e]
    return [ctx.encode(z, scale) for z in Z]


def rating_plaintexts(ctx, ratings, D, B, k, scale=2.0 ** 40):
    out = []
    for s in range(0, len(ratings), D):
        z = np.zeros(ctx.N // 2)
        for t, r in enumerate(ratings[s:s + D]):
            z[t * B: t * B + k] = r
        out.append(ctx.encode(z, scale))
    return out


def make_state(U0, V0, k=K, lr=LR, lam=LAM):
    """Oracle context with the serving keys and the resident tables (serial
    numbers 0, 1, .. for the U tables, then the V tables)."""
    prm = serving_params()
    ctx = ckks.Context(prm, workloads.CRYPTO_SEED)
    kp = 1
    while kp < k:
        kp *= 2
    B = 2 * kp
    D = ctx.N // (2 * B)
    G = 1 << (((D.bit_length() - 1) + 1) // 2)
    ctx.keygen(rot_steps=serving_rotations(B, kp, D, G))
    ut = table_plaintexts(ctx, U0, D, B, k)
    vt = table_plaintexts(ctx, V0, D, B, k)
    ind = np.zeros(ctx.N // 2)
    ind[:k] = 1.0
    mask = ctx.encode(ind, 2.0 ** 30)
    utab = [ctx.encrypt_int(m, prm.L, 2.0 ** 40) for m in ut]
    vtab = [ctx.encrypt_int(m, prm.L, 2.0 ** 40) for m in vt]
    st = serving.ServingState(ctx, k, utab, vtab, mask, lr, lam)
    return ctx, st, (ut, vt, mask)


@pytest.fixture(scope="module")
def state():
    U0, V0 = workloads.init_factors(N_USERS, N_ITEMS, K, seed=5)
    ctx, st, _ = make_state(U0, V0)
    return ctx, st, U0, V0


def test_layout_of_the_serving_chain(state):
    ctx, st, U0, V0 = state
    assert (st.B, st.D, st.G) == (32, 64, 8)


def test_predict_decrypts_to_dot_products(state):
    ctx, st, U0, V0 = state
    rng = np.random.default_rng(3)
    items = np.sort(rng.choice(N_ITEMS, size=20, replace=False))
    (S,) = st.predict(3, items)
    z = ctx.decrypt(S)
    assert np.max(np.abs(z[np.arange(20) * st.B] - V0[items] @ U0[3])) < 1e-4


def test_update_two_chunks_is_one_r2_step(state):
    ctx, st, U0, V0 = state
    rng = np.random.default_rng(4)
    items = np.sort(rng.choice(N_ITEMS, size=70, replace=False))        # two chunks of D = 64
    r = np.rint(np.clip(rng.normal(3.5, 1.1, 70), 1, 5))
    out = st.update(7, items, rating_plaintexts(ctx, r, st.D, st.B, K), client_serial=11)
    u = U0[7]
    e = r - V0[items] @ u
    want = (1 - LR * LAM) * u + (LR / len(items)) * (e[:, None] * V0[items]).sum(0)
    assert out.scale == 2.0 ** 40 or abs(out.scale / 2.0 ** 40 - 1) < 1e-9
    assert np.max(np.abs(ctx.decrypt(out)[:K] - want)) < 1e-4
