"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/csrmf.h declares, and the binding declares matching calls."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csrmf.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csrmf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_calls():
    names = declared()
    for n in ["csrmf_create", "csrmf_keygen", "csrmf_hmult", "csrmf_rotate", "csrmf_rescale", "csrmf_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2509_03024_amd as pk
    lib = ctypes.CDLL(pk.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_2509_03024_amd as pk
    missing = [n for n in declared() if n not in pk._SIGS]
    assert not missing, missing


def test_create_rejects_bad_params_without_gpu_work():
    import paper_2509_03024_amd as pk
    h = ctypes.c_void_p()
    bad = pk.params(9, 60, 3, 40, 1, 60, 4)          # N = 2^9 is below the supported range
    assert pk.lib.csrmf_create(ctypes.byref(bad), bytes(32), ctypes.byref(h)) == -1
    bad = pk.params(12, 61, 3, 40, 1, 61, 4)         # primes must be below 2^60
    assert pk.lib.csrmf_create(ctypes.byref(bad), bytes(32), ctypes.byref(h)) == -1
    assert b"log2N" not in pk.lib.csrmf_last_error(None)
    bad = pk.params(9, 60, 3, 40, 1, 60, 4)
    assert pk.lib.csrmf_create(ctypes.byref(bad), bytes(32), ctypes.byref(h)) == -1
    assert b"log2N must be in [12, 16]" in pk.lib.csrmf_last_error(None)    # the failed create's message
    assert pk.lib.csrmf_create(None, bytes(32), ctypes.byref(h)) == -1
    assert b"null argument" in pk.lib.csrmf_last_error(None)


def test_boot_levels_through_the_abi_match_the_oracle():
    """csrmf_boot_levels is host arithmetic: the library's level count of a
    bootstrap equals the oracle's for every degree, squaring count and flag,
    and an invalid configuration is refused."""
    import paper_2509_03024_amd as pk
    from oracle import bootstrap as bs
    for d in range(1, 19):
        for r in (0, 1, 8, 12):
            for asn in (0, 1):
                cfg = pk.BootConfig(4, r, d, 12, asn)
                want = bs.levels_used(bs.BootConfig(n=4, r=r, d=d, pre_bits=12, arcsine=bool(asn)))
                assert pk.boot_levels(cfg) == want, (d, r, asn)
    v = ctypes.c_int32()
    assert pk.lib.csrmf_boot_levels(ctypes.byref(pk.BootConfig(4, 9, 0, 12, 0)), ctypes.byref(v)) == -1
    assert pk.lib.csrmf_boot_levels(ctypes.byref(pk.BootConfig(4, 9, 11, 12, 2)), ctypes.byref(v)) == -1
