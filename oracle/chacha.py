"""ChaCha20 block function (RFC 8439, Sec. 2.1-2.3) and the seeded word streams (oracle).

TEST INFRASTRUCTURE ONLY.

The paper does not say where its randomness comes from (it inherits the CKKS
library's).  Every random polynomial here is drawn from a ChaCha20 keystream:

* key     = the 32-byte master seed;
* nonce   = (purpose, object id, limb) as three little-endian u32 words;
* counter = 0, 1, 2, ... (one 64-byte block each);
* output  = the keystream read as little-endian u64 words, in order.

The blocks are computed with numpy uint32 arrays, many counters at once.
"""
import numpy as np

_CONST = np.array([0x61707865, 0x3320646E, 0x79622D32, 0x6B206574], dtype=np.uint32)


def _rotl(x, n):
    return (x << np.uint32(n)) | (x >> np.uint32(32 - n))


def _quarter(s, a, b, c, d):
    s[a] += s[b]; s[d] ^= s[a]; s[d] = _rotl(s[d], 16)
    s[c] += s[d]; s[b] ^= s[c]; s[b] = _rotl(s[b], 12)
    s[a] += s[b]; s[d] ^= s[a]; s[d] = _rotl(s[d], 8)
    s[c] += s[d]; s[b] ^= s[c]; s[b] = _rotl(s[b], 7)


def quarter_round(a, b, c, d):
    """The RFC 8439 quarter round on four u32 values (used by the tests)."""
    s = [np.array([v], dtype=np.uint32) for v in (a, b, c, d)]
    _quarter(s, 0, 1, 2, 3)
    return tuple(int(v[0]) for v in s)


def blocks(key: bytes, counters, nonce_words):
    """ChaCha20 blocks for an array of counters; returns uint32 array [n, 16]."""
    assert len(key) == 32
    counters = np.asarray(counters, dtype=np.uint32)
    n = counters.shape[0]
    kw = np.frombuffer(key, dtype="<u4").astype(np.uint32)
    init = []
    for i in range(4):
        init.append(np.full(n, _CONST[i], dtype=np.uint32))
    for i in range(8):
        init.append(np.full(n, kw[i], dtype=np.uint32))
    init.append(counters.copy())
    for i in range(3):
        init.append(np.full(n, np.uint32(nonce_words[i]), dtype=np.uint32))
    s = [x.copy() for x in init]
    with np.errstate(over="ignore"):
        for _ in range(10):
            _quarter(s, 0, 4, 8, 12)
            _quarter(s, 1, 5, 9, 13)
            _quarter(s, 2, 6, 10, 14)
            _quarter(s, 3, 7, 11, 15)
            _quarter(s, 0, 5, 10, 15)
            _quarter(s, 1, 6, 11, 12)
            _quarter(s, 2, 7, 8, 13)
            _quarter(s, 3, 4, 9, 14)
        out = np.stack([s[i] + init[i] for i in range(16)], axis=1)
    return out


def keystream_bytes(key: bytes, nonce_words, n_bytes: int, counter0: int = 0) -> bytes:
    nb = -(-n_bytes // 64)
    b = blocks(key, np.arange(counter0, counter0 + nb, dtype=np.uint64).astype(np.uint32), nonce_words)
    return b.astype("<u4").tobytes()[:n_bytes]


def words_u64(key: bytes, purpose: int, obj: int, limb: int, n_words: int):
    """The first n_words little-endian u64 words of stream (purpose, obj, limb)."""
    nb = -(-n_words // 8)
    b = blocks(key, np.arange(nb, dtype=np.uint64).astype(np.uint32), (purpose, obj, limb))
    w = b.astype("<u4").reshape(-1)
    lo = w[0::2].astype(np.uint64)
    hi = w[1::2].astype(np.uint64)
    return (lo | (hi << np.uint64(32)))[:n_words]


# stream purposes
P_SECRET = 1
P_PK_A = 2
P_PK_E = 3
P_KSK_A = 4
P_KSK_E = 5
P_ENC_V = 6
P_ENC_E0 = 7
P_ENC_E1 = 8
P_REFRESH_MASK = 9
P_REFRESH_ENC = 10
P_RANDOM_RESIDUES = 11
