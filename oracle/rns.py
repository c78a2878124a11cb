"""RNS tools: CRT, fast basis conversion, ModUp, ModDown, rescale (oracle).

TEST INFRASTRUCTURE ONLY.

These follow full-RNS CKKS (Cheon-Han-Kim-Kim-Song, SAC 2018) and hybrid key
switching (Han-Ki, CT-RSA 2020); the paper itself only relies on a CKKS library
for them (Sec. IV-A).  Exact integer definitions used here:

* fast basis conversion from basis B to modulus c:
      Conv(x)_c = sum_{i in B} [x_i * (B/b_i)^-1]_{b_i} * (B/b_i)   (mod c)
  with no overflow correction, so Conv(x) = x + e*B for some 0 <= e < |B|;
* ModDown from Q_l u P to Q_l:
      out_i = (u_{q_i} - Conv_{P -> q_i}(u_P)) * P^-1   (mod q_i)
  with no +P/2 rounding;
* rescale at level l (round half up):
      h = floor(q_l / 2),  t = (c_l + h) mod q_l,
      c'_i = (c_i + h - t) * q_l^-1   (mod q_i),  i < l,
  which equals floor((x + h) / q_l) for the integer x the residues represent.
"""
import numpy as np

from .modarith import addmod, submod, mulmod


def prod(xs):
    r = 1
    for x in xs:
        r *= int(x)
    return r


def crt(rows, moduli):
    """Exact CRT reconstruction of an RNS polynomial -> object array of ints in [0, Q)."""
    Q = prod(moduli)
    acc = np.zeros(rows.shape[-1], dtype=object)
    for r, q in zip(rows, moduli):
        q = int(q)
        qhat = Q // q
        c = qhat * pow(qhat % q, -1, q)
        acc = acc + np.array([int(v) for v in r], dtype=object) * c
    return acc % Q


def basis_convert(x, src, dst, centered=False):
    """Conv_{src -> dst}(x) = sum_i y_i * (B/b_i) mod c with
    y_i = [x_i * (B/b_i)^-1]_{b_i}, for x of shape [len(src), N]; returns
    [len(dst), N].  centered: y_i taken in (-b_i/2, b_i/2] (y_i - b_i when
    2 y_i > b_i), so the result is x's centred representative mod B plus a
    multiple e*B with |e| <= len(src)/2 instead of x + e*B, 0 <= e < len(src)."""
    B = prod(src)
    ys = []
    for i, b in enumerate(src):
        b = int(b)
        bhat = B // b
        y = mulmod(x[i], np.uint64(pow(bhat % b, -1, b)), b).astype(object)
        if centered:
            y = np.array([int(v) - b if 2 * int(v) > b else int(v) for v in y], dtype=object)
        ys.append(y)
    out = []
    for c in dst:
        c = int(c)
        acc = np.zeros(x.shape[-1], dtype=np.uint64)
        for i, b in enumerate(src):
            bhat_c = (B // int(b)) % c
            y = np.array([int(v) % c for v in ys[i]], dtype=np.uint64)
            acc = addmod(acc, mulmod(y, np.uint64(bhat_c), c), c)
        out.append(acc)
    return np.stack(out)


def mod_up(d, qmods, digit, pmods):
    """Extend the digit limbs `digit` (indices into qmods) of d to all of Q_l u P.

    d has shape [l+1, N] (limbs q_0..q_l); the result has shape [l+1+alpha, N]
    in the order q_0..q_l, p_0..p_{alpha-1}.  Limbs inside the digit are copied;
    the others come from the centred conversion: the digit is taken as its
    centred representative mod Q_D (up to a small multiple of Q_D), so its
    mean is 0 and key-switching adds no key-dependent bias.
    """
    all_mods = list(qmods) + list(pmods)
    src = [qmods[i] for i in digit]
    tgt_idx = [t for t in range(len(all_mods)) if t not in digit]
    conv = basis_convert(d[digit], src, [all_mods[t] for t in tgt_idx], centered=True)
    out = np.empty((len(all_mods), d.shape[-1]), dtype=np.uint64)
    for i in digit:
        out[i] = d[i]
    for k, t in enumerate(tgt_idx):
        out[t] = conv[k]
    return out


def mod_down(u, qmods, pmods):
    """u over Q_l u P (shape [l+1+alpha, N]) -> approximately u / P over Q_l."""
    nq = len(qmods)
    uq = u[:nq]
    up = u[nq:]
    conv = basis_convert(up, pmods, qmods)
    P = prod(pmods)
    out = []
    for i, q in enumerate(qmods):
        q = int(q)
        pinv = np.uint64(pow(P % q, -1, q))
        out.append(mulmod(submod(uq[i], conv[i], q), pinv, q))
    return np.stack(out)


def rescale(c, qmods):
    """Divide by the top modulus q_l with rounding half up and drop limb l."""
    l = len(qmods) - 1
    ql = int(qmods[l])
    h = ql // 2
    t = addmod(c[l], np.uint64(h), ql)
    out = []
    for i in range(l):
        q = int(qmods[i])
        x = addmod(c[i], np.uint64(h % q), q)
        x = submod(x, t % np.uint64(q), q)
        out.append(mulmod(x, np.uint64(pow(ql % q, -1, q)), q))
    return np.stack(out)
