"""Integer-only samplers over ChaCha20 word streams (oracle; test infrastructure only).

The paper defers the secret and error distributions to its CKKS library.  The
readings used here are integer-only so that two implementations can agree bit
for bit:

* uniform residue mod q_i (one stream per limb): coefficient n is
  (w[2n] * 2^64 + w[2n+1]) mod q_i;
* ternary (secret s, encryption randomness v; limb field 0):
  coefficient n is (w[n] mod 3) - 1;
* centred binomial with 21 coin pairs (errors; limb field 0):
  popcount(w[n] & (2^21-1)) - popcount((w[n] >> 21) & (2^21-1)), variance 10.5.
"""
import numpy as np

from . import chacha, modarith


def uniform_mod(key, purpose, obj, limb, N, q):
    w = chacha.words_u64(key, purpose, obj, limb, 2 * N)
    hi = w[0::2]
    lo = w[1::2]
    q = int(q)
    # (hi * 2^64 + lo) mod q = ((hi mod q) * (2^64 mod q) + (lo mod q)) mod q
    qq = np.uint64(q)
    t = modarith.mulmod(hi % qq, np.uint64((1 << 64) % q), q)
    return modarith.addmod(t, lo % qq, q)


def ternary(key, purpose, obj, N):
    w = chacha.words_u64(key, purpose, obj, 0, N)
    return (w % np.uint64(3)).astype(np.int64) - 1


def _popcount(x):
    x = np.asarray(x, dtype=np.uint64)
    c = np.zeros(x.shape, dtype=np.int64)
    for b in range(64):
        c += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def cbd21(key, purpose, obj, N):
    w = chacha.words_u64(key, purpose, obj, 0, N)
    m = np.uint64((1 << 21) - 1)
    a = _popcount(w & m)
    b = _popcount((w >> np.uint64(21)) & m)
    return a - b
