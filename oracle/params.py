"""RNS-CKKS parameters: prime chains, primitive roots, gadget digits (oracle).

TEST INFRASTRUCTURE ONLY.

The paper runs CKKS (Sec. II-A.2; Sec. IV-A: degree 8192, 32-bit scale) through a
library and never states its modulus chain.  The chain used here is the
full-RNS CKKS one (Cheon-Han-Kim-Kim-Song, SAC 2018) with hybrid key switching
(Han-Ki, CT-RSA 2020):

* primes are NTT-friendly, q = 1 (mod 2N), taken as the largest ones strictly
  below 2^b, i.e. q = 2^b - j*2N + 1 for j = 1, 2, ... in descending order;
* the 60-bit list supplies q_0 and then the special primes p_0..p_{alpha-1};
* the 40-bit list supplies q_1 > q_2 > ... > q_L, so rescale at level l drops
  the smallest remaining scale prime q_l;
* key-switching digits are D_j = [j*g, min((j+1)*g, L+1)) with g = ceil((L+1)/dnum).
"""
from dataclasses import dataclass, field
from typing import List


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; the first 12 prime bases are exact below 3.3e24."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d = n - 1
    s = 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, N: int, count: int) -> List[int]:
    """The `count` largest primes q < 2^bits with q = 1 (mod 2N), descending."""
    out = []
    j = 1
    while len(out) < count:
        q = (1 << bits) - j * 2 * N + 1
        if q < (1 << (bits - 1)):
            raise ValueError("ran out of primes")
        if is_prime(q):
            out.append(q)
        j += 1
    return out


def _factor_small(n: int) -> List[int]:
    """Distinct prime factors of n by trial division plus Pollard rho (n < 2^64)."""
    fs = set()
    for p in range(2, 1000):
        while n % p == 0:
            fs.add(p)
            n //= p
    stack = [n] if n > 1 else []
    while stack:
        m = stack.pop()
        if m == 1:
            continue
        if is_prime(m):
            fs.add(m)
            continue
        c = 1
        while True:
            x = y = 2
            d = 1
            while d == 1:
                x = (x * x + c) % m
                y = (y * y + c) % m
                y = (y * y + c) % m
                d = _gcd(abs(x - y), m)
            if d != m:
                break
            c += 1
        stack += [d, m // d]
    return sorted(fs)


def _gcd(a, b):
    while b:
        a, b = b, a % b
    return a


def primitive_2n_root(q: int, N: int) -> int:
    """The smallest primitive 2N-th root of unity mod q.  Which root is used does
    not change any compared result (residues are compared in coefficient form)."""
    order = 2 * N
    assert (q - 1) % order == 0
    fac = _factor_small(q - 1)
    # generator of Z_q^*, then raise to (q-1)/2N; then scan for the smallest root
    g = 2
    while any(pow(g, (q - 1) // f, q) == 1 for f in fac):
        g += 1
    base = pow(g, (q - 1) // order, q)
    # all primitive 2N-th roots are base^k for odd k
    best = None
    x = base
    b2 = base * base % q
    for _ in range(N):
        if best is None or x < best:
            best = x
        x = x * b2 % q
    return best


@dataclass
class CkksParams:
    """One CKKS parameter set.  All lists are Python ints."""
    logN: int
    q: List[int]            # q_0 (60-bit) then q_1 > ... > q_L (scale primes)
    p: List[int]            # special primes
    dnum: int
    log2_scale: int
    name: str = ""
    psi: List[int] = field(default_factory=list)   # one 2N-th root per limb, Q then P

    @property
    def N(self):
        return 1 << self.logN

    @property
    def L(self):
        return len(self.q) - 1

    @property
    def alpha(self):
        return len(self.p)

    @property
    def moduli(self):
        """All limbs in global order: q_0..q_L, p_0..p_{alpha-1}."""
        return list(self.q) + list(self.p)

    @property
    def digit_size(self):
        return -(-(self.L + 1) // self.dnum)

    def digits(self, level: int):
        """Gadget digits restricted to limbs 0..level (empty digits dropped)."""
        g = self.digit_size
        out = []
        for j in range(self.dnum):
            lo = j * g
            hi = min((j + 1) * g, self.L + 1, level + 1)
            if lo < hi:
                out.append((j, list(range(lo, hi))))
        return out

    @property
    def scale(self):
        return float(2 ** self.log2_scale)


def make_params(logN, base_bits, n_scale, scale_bits, n_special, special_bits, dnum,
                log2_scale, name="") -> CkksParams:
    N = 1 << logN
    big = ntt_primes(base_bits, N, 1 + (n_special if special_bits == base_bits else 0))
    q0 = big[0]
    if special_bits == base_bits:
        p = big[1:1 + n_special]
    else:
        p = ntt_primes(special_bits, N, n_special)
    qs = ntt_primes(scale_bits, N, n_scale)
    prm = CkksParams(logN=logN, q=[q0] + qs, p=p, dnum=dnum, log2_scale=log2_scale, name=name)
    prm.psi = [primitive_2n_root(m, N) for m in prm.moduli]
    return prm


def config_tiny():
    """N = 2^12, q_0 60-bit + 3 x 40-bit, 1 x 60-bit special, one limb per digit, scale 2^40."""
    return make_params(12, 60, 3, 40, 1, 60, 4, 40, name="tiny")


def config_tiny_two_epochs():
    """N = 2^12, q_0 60-bit + 7 x 40-bit, 2 x 60-bit special, dnum 4 (2-limb digits,
    each below P ~ 2^120), scale 2^40: room for two MF epochs (3 + 4 levels), so a
    gather runs encrypted."""
    return make_params(12, 60, 7, 40, 2, 60, 4, 40, name="tiny2")


def config_kernel_batch():
    """N = 2^16, q_0 60-bit + 24 x 40-bit, 3 x 60-bit special, dnum = 3 (digits 9, 9, 7)."""
    return make_params(16, 60, 24, 40, 3, 60, 3, 40, name="kernel_batch")


def config_mf_n15():
    """N = 2^15, q_0 + 16 x 40-bit, 3 x 60-bit special, 4-limb digits (dnum = 5)."""
    return make_params(15, 60, 16, 40, 3, 60, 5, 40, name="mf_n15")


def config_mf_n16():
    """N = 2^16, q_0 + 24 x 40-bit, 3 x 60-bit special, 4-limb digits (dnum = 7)."""
    return make_params(16, 60, 24, 40, 3, 60, 7, 40, name="mf_n16")
