"""Python binding of libcsrmf (CKKS arithmetic for encrypted CSR matrix
factorisation on AMD Instinct MI355X).

Argument marshalling only: every homomorphic operation runs in the HIP
library.  The library must have been built (``python -m
paper_2509_03024_amd.build`` or ``__graft_entry__.build()``); importing this
module without it raises immediately.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsrmf.so")

CSRMF_OK = 0
ERRORS = {-1: "INVAL", -2: "NOMEM", -3: "LEVEL", -4: "SCALE", -5: "STATE", -6: "DEVICE", -7: "KEY"}


class CsrmfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"csrmf error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code
        self.name = ERRORS.get(code, "?")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python -m paper_2509_03024_amd.build)")

# One HIP runtime per process.  PyTorch ships its own libamdhip64 (soname
# libamdhip64.so.7, loaded under the file name libamdhip64.so); when it is
# loaded first, this library binds to it by soname.  Loaded the other way
# round, the process would hold two HIP runtimes and PyTorch's would see no
# device.  So PyTorch, when installed, is loaded before the library.
try:
    import torch  # noqa: F401
except ImportError:
    pass

lib = ctypes.CDLL(LIB_PATH)


class Params(ctypes.Structure):
    _fields_ = [("log2N", ctypes.c_int32), ("base_bits", ctypes.c_int32),
                ("n_scale_primes", ctypes.c_int32), ("scale_bits", ctypes.c_int32),
                ("n_special", ctypes.c_int32), ("special_bits", ctypes.c_int32),
                ("dnum", ctypes.c_int32), ("log2_scale", ctypes.c_int32),
                ("k", ctypes.c_int32), ("lr", ctypes.c_double), ("lam", ctypes.c_double),
                ("damp", ctypes.c_double), ("rule", ctypes.c_int32), ("refresh_mode", ctypes.c_int32),
                ("batch_pairs", ctypes.c_int32)]


class BootConfig(ctypes.Structure):
    """Bootstrapping parameters (csrmf_boot_config)."""
    _fields_ = [("n_slots", ctypes.c_int32), ("squarings", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("pre_bits", ctypes.c_int32), ("arcsine", ctypes.c_int32)]

_p = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "csrmf_create": [ctypes.POINTER(Params), ctypes.c_char_p, ctypes.POINTER(_p)],
    "csrmf_destroy": [_p],
    "csrmf_last_error": [_p],
    "csrmf_set_stream": [_p, _p],
    "csrmf_sync": [_p],
    "csrmf_get_chain": [_p, _i32p, _i32p, _u64p],
    "csrmf_keygen": [_p, _i32p, ctypes.c_int32, ctypes.c_int32],
    "csrmf_encrypt": [_p, _dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _u64p],
    "csrmf_encrypt_int": [_p, _i64p, ctypes.c_int32, ctypes.c_double, _u64p],
    "csrmf_decrypt_int": [_p, ctypes.c_uint64, _i64p],
    "csrmf_decrypt": [_p, ctypes.c_uint64, _dp, ctypes.c_int32],
    "csrmf_encode": [_p, _dp, ctypes.c_int32, ctypes.c_double, _i64p],
    "csrmf_decode": [_p, _i64p, ctypes.c_double, _dp, ctypes.c_int32],
    "csrmf_import_ct": [_p, _u64p, ctypes.c_int32, ctypes.c_double, _u64p],
    "csrmf_export_ct": [_p, ctypes.c_uint64, _u64p, _i32p, _dp],
    "csrmf_ct_info": [_p, ctypes.c_uint64, _i32p, _dp],
    "csrmf_free_ct": [_p, ctypes.c_uint64],
    "csrmf_export_key": [_p, ctypes.c_int32, ctypes.c_uint32, _u64p],
    "csrmf_add": [_p, ctypes.c_uint64, ctypes.c_uint64, _u64p],
    "csrmf_sub": [_p, ctypes.c_uint64, ctypes.c_uint64, _u64p],
    "csrmf_add_plain": [_p, ctypes.c_uint64, _i64p, _u64p],
    "csrmf_add_batch": [_p, _u64p, _u64p, ctypes.c_int32, ctypes.c_int32, _u64p],
    "csrmf_mul_plain": [_p, ctypes.c_uint64, _i64p, ctypes.c_double, _u64p],
    "csrmf_mul_int": [_p, ctypes.c_uint64, ctypes.c_int64, _u64p],
    "csrmf_hmult": [_p, ctypes.c_uint64, ctypes.c_uint64, _u64p],
    "csrmf_mul_relin": [_p, ctypes.c_uint64, ctypes.c_uint64, _u64p],
    "csrmf_rescale": [_p, ctypes.c_uint64, _u64p],
    "csrmf_mod_drop": [_p, ctypes.c_uint64, ctypes.c_int32, _u64p],
    "csrmf_rotate": [_p, ctypes.c_uint64, ctypes.c_int32, _u64p],
    "csrmf_conjugate": [_p, ctypes.c_uint64, _u64p],
    "csrmf_rotate_hoisted": [_p, ctypes.c_uint64, _i32p, ctypes.c_int32, _u64p],
    "csrmf_hmult_batch": [_p, _u64p, _u64p, ctypes.c_int32, _u64p],
    "csrmf_rotate_batch": [_p, _u64p, ctypes.c_int32, ctypes.c_int32, _u64p],
    "csrmf_rotate_add_batch": [_p, _u64p, _u64p, ctypes.c_int32, ctypes.c_int32, _u64p],
    "csrmf_conjugate_batch": [_p, _u64p, ctypes.c_int32, _u64p],
    "csrmf_boot_levels": [ctypes.POINTER(BootConfig), _i32p],
    "csrmf_boot_rotation_steps": [_p, ctypes.POINTER(BootConfig), _i32p, ctypes.c_int32, _i32p],
    "csrmf_bootstrap": [_p, ctypes.POINTER(BootConfig), _u64p, ctypes.c_int32, _u64p],
    "csrmf_ntt_rows": [_p, _p, ctypes.c_int32, _i32p, ctypes.c_int32, ctypes.c_int32],
    "csrmf_encrypt_csr_rows": [_p, ctypes.c_int32, ctypes.c_int32, _i64p, _i32p, _dp, _i32p],
    "csrmf_encrypt_csr_rows_int": [_p, ctypes.c_int32, ctypes.c_int32, _i64p, _i32p, _i64p, ctypes.c_int32, _i32p],
    "csrmf_init_factors": [_p, _dp, _dp],
    "csrmf_init_factors_int": [_p, _i64p, _i64p, _i64p, _i64p, _i64p, _i64p],
    "csrmf_mf_layout": [_p, _i32p, _i32p, _i32p, _i32p, _i32p],
    "csrmf_mf_epochs": [_p, ctypes.c_int32],
    "csrmf_predict": [_p],
    "csrmf_decrypt_factors": [_p, _dp, _dp],
    "csrmf_decrypt_predictions": [_p, _dp, ctypes.c_int32],
    "csrmf_mf_handles": [_p, ctypes.c_int32, _u64p, ctypes.c_int32, _i32p],
    "csrmf_mf_stats": [_p, _i32p, _i32p, ctypes.POINTER(ctypes.c_double)],
    "csrmf_mf_mac_counts": [_p, ctypes.POINTER(ctypes.c_int64)],
    "csrmf_autotune": [_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32],
    "csrmf_set_ntt_schedule": [_p, ctypes.c_int32],
    "csrmf_rotate_noalloc": [_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint64],
    "csrmf_set_baby_budget": [_p, ctypes.c_int32],
    "csrmf_set_schedule": [_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "csrmf_graph_begin": [_p],
    "csrmf_graph_end": [_p, _u64p],
    "csrmf_graph_launch": [_p, ctypes.c_uint64],
    "csrmf_graph_destroy": [_p, ctypes.c_uint64],
    "csrmf_get_schedule": [_p, _i32p, _i32p, _i32p, _i32p],
    "csrmf_counters": [_p, ctypes.POINTER(ctypes.c_int64)],
    "csrmf_protocol_ingest": [_p, ctypes.c_int32, ctypes.c_int32, _i64p, _i32p, _dp, _i32p],
    "csrmf_protocol_recommend": [_p, ctypes.c_int32, _dp],
    "csrmf_protocol_counters": [_p, _i64p, _i64p],
    "csrmf_server_create": [_p, ctypes.c_int32, ctypes.c_int32, _dp, _dp, ctypes.c_double, ctypes.c_int32,
                            ctypes.POINTER(_p)],
    "csrmf_server_submit": [_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _dp, ctypes.c_uint32, _u64p],
    "csrmf_server_create_int": [_p, ctypes.c_int32, ctypes.c_int32, _i64p, _i64p, _i64p, ctypes.c_double,
                                ctypes.c_int32, ctypes.POINTER(_p)],
    "csrmf_server_submit_int": [_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _i64p, ctypes.c_uint32,
                                _u64p],
    "csrmf_server_poll": [_p, ctypes.c_uint64, ctypes.c_int32, _i32p, _u64p, ctypes.c_int32, _i32p, _dp],
    "csrmf_server_stats": [_p, ctypes.c_char_p, ctypes.c_int32],
    "csrmf_server_destroy": [_p],
    "csrmf_profile_enable": [ctypes.c_int32],
    "csrmf_profile_report": [ctypes.c_char_p, ctypes.c_int32],
}

for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = None if _name in ("csrmf_destroy", "csrmf_server_destroy") else (
        ctypes.c_char_p if _name == "csrmf_last_error" else ctypes.c_int)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def params(log2N, base_bits, n_scale, scale_bits, n_special, special_bits, dnum, log2_scale=40,
           k=0, lr=0.0, lam=0.0, damp=0.0, rule=1, refresh_mode=0, batch_pairs=0):
    return Params(log2N, base_bits, n_scale, scale_bits, n_special, special_bits, dnum, log2_scale,
                  k, lr, lam, damp, rule, refresh_mode, batch_pairs)


class Context:
    """One libcsrmf context (one modulus chain, one key set, one stream)."""

    def __init__(self, prm: Params, seed: bytes):
        assert len(seed) == 32
        h = _p()
        rc = lib.csrmf_create(ctypes.byref(prm), seed, ctypes.byref(h))
        if rc != CSRMF_OK:
            raise CsrmfError(rc, lib.csrmf_last_error(None).decode())
        self.h = h
        self.prm = prm
        self.N = 1 << prm.log2N
        L = ctypes.c_int32()
        a = ctypes.c_int32()
        lib.csrmf_get_chain(self.h, ctypes.byref(L), ctypes.byref(a), None)
        self.L, self.alpha = L.value, a.value
        mods = np.zeros(self.L + 1 + self.alpha, np.uint64)
        lib.csrmf_get_chain(self.h, None, None, _ptr(mods, ctypes.c_uint64))
        self.moduli = [int(x) for x in mods]

    def close(self):
        if self.h:
            for srv in list(getattr(self, "_servers", [])):
                srv._detach()
            lib.csrmf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != CSRMF_OK:
            raise CsrmfError(rc, lib.csrmf_last_error(self.h).decode())

    # ---------------------------------------------------------------- keys
    def keygen(self, rot_steps=(), conj=False):
        st = np.asarray(list(rot_steps), np.int32)
        self._chk(lib.csrmf_keygen(self.h, _ptr(st, ctypes.c_int32), len(st), int(bool(conj))))

    def export_key(self, which, galois=0):
        nall = self.L + 1 + self.alpha
        if which == 0:
            shape = (nall, self.N)
        elif which == 1:
            shape = (2, self.L + 1, self.N)
        else:
            nd = -(-(self.L + 1) // ((self.L + 1 + self.prm.dnum - 1) // self.prm.dnum))
            shape = (nd, 2, nall, self.N)
        out = np.zeros(shape, np.uint64)
        self._chk(lib.csrmf_export_key(self.h, which, galois, _ptr(out, ctypes.c_uint64)))
        return out

    def sync(self):
        self._chk(lib.csrmf_sync(self.h))

    def set_stream(self, stream_ptr):
        self._chk(lib.csrmf_set_stream(self.h, _p(stream_ptr)))

    # ---------------------------------------------------------------- ciphertexts
    def encode(self, z, scale):
        z = np.ascontiguousarray(z, np.float64)
        m = np.zeros(self.N, np.int64)
        self._chk(lib.csrmf_encode(self.h, _ptr(z, ctypes.c_double), len(z), scale, _ptr(m, ctypes.c_int64)))
        return m

    def decode(self, m, scale, n=None):
        m = np.ascontiguousarray(m, np.int64)
        n = self.N // 2 if n is None else n
        z = np.zeros(n, np.float64)
        self._chk(lib.csrmf_decode(self.h, _ptr(m, ctypes.c_int64), scale, _ptr(z, ctypes.c_double), n))
        return z

    def encrypt(self, z, level=None, scale=None):
        z = np.ascontiguousarray(z, np.float64)
        level = self.L if level is None else level
        scale = float(2 ** self.prm.log2_scale) if scale is None else scale
        h = ctypes.c_uint64()
        self._chk(lib.csrmf_encrypt(self.h, _ptr(z, ctypes.c_double), len(z), level, scale, ctypes.byref(h)))
        return h.value

    def encrypt_int(self, m, level, scale):
        m = np.ascontiguousarray(m, np.int64)
        h = ctypes.c_uint64()
        self._chk(lib.csrmf_encrypt_int(self.h, _ptr(m, ctypes.c_int64), level, scale, ctypes.byref(h)))
        return h.value

    def decrypt_int(self, h):
        m = np.zeros(self.N, np.int64)
        self._chk(lib.csrmf_decrypt_int(self.h, h, _ptr(m, ctypes.c_int64)))
        return m

    def decrypt(self, h, n=None):
        n = self.N // 2 if n is None else n
        z = np.zeros(n, np.float64)
        self._chk(lib.csrmf_decrypt(self.h, h, _ptr(z, ctypes.c_double), n))
        return z

    def info(self, h):
        lv = ctypes.c_int32()
        sc = ctypes.c_double()
        self._chk(lib.csrmf_ct_info(self.h, h, ctypes.byref(lv), ctypes.byref(sc)))
        return lv.value, sc.value

    def export_ct(self, h):
        lv, _ = self.info(h)
        out = np.zeros((2, lv + 1, self.N), np.uint64)
        lvl = ctypes.c_int32()
        sc = ctypes.c_double()
        self._chk(lib.csrmf_export_ct(self.h, h, _ptr(out, ctypes.c_uint64), ctypes.byref(lvl), ctypes.byref(sc)))
        return out, lvl.value, sc.value

    def import_ct(self, coeffs, level, scale):
        c = np.ascontiguousarray(coeffs, np.uint64)
        h = ctypes.c_uint64()
        self._chk(lib.csrmf_import_ct(self.h, _ptr(c, ctypes.c_uint64), level, scale, ctypes.byref(h)))
        return h.value

    def free(self, h):
        self._chk(lib.csrmf_free_ct(self.h, h))

    def _unary(self, fn, *args):
        out = ctypes.c_uint64()
        self._chk(fn(self.h, *args, ctypes.byref(out)))
        return out.value

    def add(self, a, b):
        return self._unary(lib.csrmf_add, a, b)

    def sub(self, a, b):
        return self._unary(lib.csrmf_sub, a, b)

    def add_batch(self, a, b, subtract=False):
        a = np.asarray(a, np.uint64)
        b = np.asarray(b, np.uint64)
        out = np.zeros(len(a), np.uint64)
        self._chk(lib.csrmf_add_batch(self.h, _ptr(a, ctypes.c_uint64), _ptr(b, ctypes.c_uint64), len(a),
                                      int(bool(subtract)), _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def add_plain(self, a, m):
        m = np.ascontiguousarray(m, np.int64)
        return self._unary(lib.csrmf_add_plain, a, _ptr(m, ctypes.c_int64))

    def mul_plain(self, a, m, pt_scale):
        m = np.ascontiguousarray(m, np.int64)
        return self._unary(lib.csrmf_mul_plain, a, _ptr(m, ctypes.c_int64), pt_scale)

    def mul_int(self, a, w):
        return self._unary(lib.csrmf_mul_int, a, int(w))

    def hmult(self, a, b):
        return self._unary(lib.csrmf_hmult, a, b)

    def mul_relin(self, a, b):
        return self._unary(lib.csrmf_mul_relin, a, b)

    def rescale(self, a):
        return self._unary(lib.csrmf_rescale, a)

    def mod_drop(self, a, level):
        return self._unary(lib.csrmf_mod_drop, a, level)

    def rotate(self, a, r):
        return self._unary(lib.csrmf_rotate, a, r)

    def conjugate(self, a):
        return self._unary(lib.csrmf_conjugate, a)

    def rotate_noalloc(self, a, r, out):
        """Rotation of a by r written into the existing ciphertext `out`; no
        device allocation (the library's static scratch buffer)."""
        self._chk(lib.csrmf_rotate_noalloc(self.h, a, r, out))

    def graph_begin(self):
        """Capture the following evaluation calls into a HIP graph (see csrmf_graph_begin)."""
        self._chk(lib.csrmf_graph_begin(self.h))

    def graph_end(self):
        g = ctypes.c_uint64()
        self._chk(lib.csrmf_graph_end(self.h, ctypes.byref(g)))
        return g.value

    def graph_launch(self, g):
        self._chk(lib.csrmf_graph_launch(self.h, g))

    def graph_destroy(self, g):
        self._chk(lib.csrmf_graph_destroy(self.h, g))

    def set_schedule(self, ntt_chunk_rows=0, ntt_cached_mid=0, modup_chunk=0, ntt_split=0):
        """Fix this context's whole schedule (see csrmf_set_schedule)."""
        self._chk(lib.csrmf_set_schedule(self.h, int(ntt_chunk_rows), int(ntt_cached_mid), int(modup_chunk),
                                         int(ntt_split)))

    def schedule(self):
        a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._chk(lib.csrmf_get_schedule(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return {"ntt_chunk_rows": a.value, "ntt_cached_mid": b.value, "modup_chunk": c.value, "ntt_split": d.value}

    def counters(self):
        """{"key_switches": relinearisations and rotations enqueued so far}."""
        v = ctypes.c_int64()
        self._chk(lib.csrmf_counters(self.h, ctypes.byref(v)))
        return {"key_switches": v.value}

    def set_ntt_schedule(self, chunk_rows):
        """Fix this context's NTT schedule (rows per pair of passes; 0 = whole batch)."""
        self._chk(lib.csrmf_set_ntt_schedule(self.h, int(chunk_rows)))

    def rotate_hoisted(self, a, steps):
        st = np.asarray(list(steps), np.int32)
        out = np.zeros(len(st), np.uint64)
        self._chk(lib.csrmf_rotate_hoisted(self.h, a, _ptr(st, ctypes.c_int32), len(st), _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def hmult_batch(self, a, b):
        a = np.asarray(a, np.uint64)
        b = np.asarray(b, np.uint64)
        out = np.zeros(len(a), np.uint64)
        self._chk(lib.csrmf_hmult_batch(self.h, _ptr(a, ctypes.c_uint64), _ptr(b, ctypes.c_uint64), len(a),
                                        _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def rotate_batch(self, a, r):
        a = np.asarray(a, np.uint64)
        out = np.zeros(len(a), np.uint64)
        self._chk(lib.csrmf_rotate_batch(self.h, _ptr(a, ctypes.c_uint64), len(a), r, _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def rotate_add_batch(self, a, acc, r):
        """[acc[i] + Rot(a[i], r)], the addition fused into the key switch."""
        a = np.asarray(a, np.uint64)
        acc = np.asarray(acc, np.uint64)
        if len(acc) != len(a):
            raise ValueError("one accumulator per rotated ciphertext")
        out = np.zeros(len(a), np.uint64)
        self._chk(lib.csrmf_rotate_add_batch(self.h, _ptr(a, ctypes.c_uint64), _ptr(acc, ctypes.c_uint64), len(a), r,
                                             _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def conjugate_batch(self, a):
        a = np.asarray(a, np.uint64)
        out = np.zeros(len(a), np.uint64)
        self._chk(lib.csrmf_conjugate_batch(self.h, _ptr(a, ctypes.c_uint64), len(a), _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def boot_rotation_steps(self, cfg):
        """Rotation steps whose keys bootstrap(cfg) needs (plus conjugation)."""
        cnt = ctypes.c_int32()
        lib.csrmf_boot_rotation_steps(self.h, ctypes.byref(cfg), None, 0, ctypes.byref(cnt))
        st = np.zeros(max(cnt.value, 1), np.int32)
        self._chk(lib.csrmf_boot_rotation_steps(self.h, ctypes.byref(cfg), _ptr(st, ctypes.c_int32), len(st),
                                                ctypes.byref(cnt)))
        return [int(x) for x in st[: cnt.value]]

    def bootstrap(self, handles, cfg):
        """Bootstrap a batch of ciphertexts (one scale); new handles at level
        L - boot_levels(cfg)."""
        a = np.asarray(list(handles), np.uint64)
        out = np.zeros(len(a), np.uint64)
        self._chk(lib.csrmf_bootstrap(self.h, ctypes.byref(cfg), _ptr(a, ctypes.c_uint64), len(a),
                                      _ptr(out, ctypes.c_uint64)))
        return [int(x) for x in out]

    def autotune(self, rows=0):
        """Pick the fastest NTT schedule for this ring on `rows` limbs; returns the timings."""
        import json
        buf = ctypes.create_string_buffer(4096)
        self._chk(lib.csrmf_autotune(self.h, rows, buf, 4096))
        return json.loads(buf.value.decode())

    def ntt_rows(self, dev_ptr, n_rows, limb_idx, inverse=False):
        """In-place (I)NTT of rows at a device pointer (e.g. a torch tensor's data_ptr())."""
        idx = np.asarray(limb_idx, np.int32)
        self._chk(lib.csrmf_ntt_rows(self.h, _p(dev_ptr), n_rows, _ptr(idx, ctypes.c_int32), len(idx), int(inverse)))


class MF:
    """Encrypted CSR matrix factorisation on a Context (the calls of Alg. 1)."""

    def __init__(self, ctx: "Context"):
        self.ctx = ctx

    def encrypt_csr_rows(self, n_rows, n_cols, row_ptr, col_idx, values):
        rp = np.ascontiguousarray(row_ptr, np.int64)
        ci = np.ascontiguousarray(col_idx, np.int32)
        v = np.ascontiguousarray(values, np.float64)
        n = ctypes.c_int32()
        self.ctx._chk(lib.csrmf_encrypt_csr_rows(self.ctx.h, n_rows, n_cols, _ptr(rp, ctypes.c_int64),
                                                 _ptr(ci, ctypes.c_int32), _ptr(v, ctypes.c_double), ctypes.byref(n)))
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, len(ci)
        return n.value

    def encrypt_csr_rows_int(self, n_rows, n_cols, row_ptr, col_idx, plain):
        rp = np.ascontiguousarray(row_ptr, np.int64)
        ci = np.ascontiguousarray(col_idx, np.int32)
        pl = np.ascontiguousarray(plain, np.int64)
        n = ctypes.c_int32()
        self.ctx._chk(lib.csrmf_encrypt_csr_rows_int(self.ctx.h, n_rows, n_cols, _ptr(rp, ctypes.c_int64),
                                                     _ptr(ci, ctypes.c_int32), _ptr(pl, ctypes.c_int64),
                                                     pl.shape[0], ctypes.byref(n)))
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, len(ci)
        return n.value

    def layout(self):
        v = [ctypes.c_int32() for _ in range(5)]
        self.ctx._chk(lib.csrmf_mf_layout(self.ctx.h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["n_ct", "n_utab", "n_vtab", "D", "B"], [x.value for x in v]))

    def stats(self):
        e, r, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self.ctx._chk(lib.csrmf_mf_stats(self.ctx.h, ctypes.byref(e), ctypes.byref(r), ctypes.byref(s)))
        return {"epochs_done": e.value, "refreshes": r.value, "refresh_seconds": s.value}

    def mac_counts(self):
        """Masked-MAC work since init_factors (see csrmf_mf_mac_counts)."""
        v = (ctypes.c_int64 * 7)()
        self.ctx._chk(lib.csrmf_mf_mac_counts(self.ctx.h, v))
        keys = ["tasks", "groups", "terms", "const_terms", "task_rows", "group_rows", "term_rows"]
        return dict(zip(keys, list(v)))

    def init_factors(self, U0, V0):
        U = np.ascontiguousarray(U0, np.float64)
        V = np.ascontiguousarray(V0, np.float64)
        self.k = U.shape[1]
        self.ctx._chk(lib.csrmf_init_factors(self.ctx.h, _ptr(U, ctypes.c_double), _ptr(V, ctypes.c_double)))

    def init_factors_int(self, utab, vtab, ug, vg, mask_scatter, mask_gather, k):
        arrs = [np.ascontiguousarray(a, np.int64) for a in (utab, vtab, ug, vg, mask_scatter, mask_gather)]
        self.k = k
        self.ctx._chk(lib.csrmf_init_factors_int(self.ctx.h, *[_ptr(a, ctypes.c_int64) for a in arrs]))

    def epochs(self, n):
        self.ctx._chk(lib.csrmf_mf_epochs(self.ctx.h, n))

    def protocol_ingest(self, n_rows, n_cols, row_ptr, col_idx, values):
        """The protocol's initialization phase (users -> RS -> CSP -> RS); returns n_ct."""
        rp = np.ascontiguousarray(row_ptr, np.int64)
        ci = np.ascontiguousarray(col_idx, np.int32)
        v = np.ascontiguousarray(values, np.float64)
        n = ctypes.c_int32()
        self.ctx._chk(lib.csrmf_protocol_ingest(self.ctx.h, n_rows, n_cols, _ptr(rp, ctypes.c_int64),
                                                _ptr(ci, ctypes.c_int32), _ptr(v, ctypes.c_double), ctypes.byref(n)))
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, len(ci)
        return n.value

    def protocol_recommend(self, which=0):
        """The recommendation phase: the users' unmasked predictions (CSR order)."""
        out = np.zeros(self.nnz)
        self.ctx._chk(lib.csrmf_protocol_recommend(self.ctx.h, which, _ptr(out, ctypes.c_double)))
        return out

    CHANNELS = ["csp_to_users_pk", "csp_to_rs_keys", "users_to_rs", "rs_to_csp_masked", "csp_to_rs_ratings",
                "rs_to_csp_predictions", "csp_to_users_predictions", "rs_to_users_masks"]

    def protocol_counters(self):
        """{channel: (messages, bytes)} of the last protocol run."""
        msgs = np.zeros(8, np.int64)
        byts = np.zeros(8, np.int64)
        self.ctx._chk(lib.csrmf_protocol_counters(self.ctx.h, _ptr(msgs, ctypes.c_int64), _ptr(byts, ctypes.c_int64)))
        return {n: (int(a), int(b)) for n, a, b in zip(self.CHANNELS, msgs, byts)}

    def set_baby_budget(self, max_babies):
        """Block permutations keep at most max_babies baby rotations alive (memory bound)."""
        self.ctx._chk(lib.csrmf_set_baby_budget(self.ctx.h, int(max_babies)))

    def predict(self):
        self.ctx._chk(lib.csrmf_predict(self.ctx.h))

    def decrypt_factors(self):
        U = np.zeros((self.n_rows, self.k))
        V = np.zeros((self.n_cols, self.k))
        self.ctx._chk(lib.csrmf_decrypt_factors(self.ctx.h, _ptr(U, ctypes.c_double), _ptr(V, ctypes.c_double)))
        return U, V

    def decrypt_predictions(self, which=0):
        r = np.zeros(self.nnz)
        self.ctx._chk(lib.csrmf_decrypt_predictions(self.ctx.h, _ptr(r, ctypes.c_double), which))
        return r

    def handles(self, which):
        n = ctypes.c_int32()
        self.ctx._chk(lib.csrmf_mf_handles(self.ctx.h, which, None, 0, ctypes.byref(n)))
        out = np.zeros(max(1, n.value), np.uint64)
        self.ctx._chk(lib.csrmf_mf_handles(self.ctx.h, which, _ptr(out, ctypes.c_uint64), n.value, ctypes.byref(n)))
        return [int(x) for x in out[: n.value]]


class Server:
    """Request server (continuous batching) on a Context; see csrmf_server_*."""
    PREDICT, UPDATE = 0, 1

    def __init__(self, ctx: "Context", U, V, hbm_budget_bytes, max_batch=64, plain=None):
        """U, V: factor matrices (encoded by the library); or plain =
        (n_users, n_items, utab, vtab, mask_gather) integer plaintexts."""
        self.ctx = ctx
        h = _p()
        if plain is None:
            U = np.ascontiguousarray(U, np.float64)
            V = np.ascontiguousarray(V, np.float64)
            ctx._chk(lib.csrmf_server_create(ctx.h, U.shape[0], V.shape[0], _ptr(U, ctypes.c_double),
                                             _ptr(V, ctypes.c_double), float(hbm_budget_bytes), max_batch,
                                             ctypes.byref(h)))
        else:
            nu, nv, ut, vt, mg = plain
            ut, vt, mg = (np.ascontiguousarray(a, np.int64) for a in (ut, vt, mg))
            ctx._chk(lib.csrmf_server_create_int(ctx.h, nu, nv, _ptr(ut, ctypes.c_int64), _ptr(vt, ctypes.c_int64),
                                                 _ptr(mg, ctypes.c_int64), float(hbm_budget_bytes), max_batch,
                                                 ctypes.byref(h)))
        self.h = h
        if not hasattr(ctx, "_servers"):
            ctx._servers = []
        ctx._servers.append(self)

    def _detach(self):
        """The context is being destroyed; it stops and frees this server itself."""
        self.h = None

    def submit(self, op, user, items, ratings=None, client_serial=0, plain=None):
        """plain: an UPDATE's rating chunks encoded by the caller ([chunks][N] int64)."""
        it = np.ascontiguousarray(items, np.int32)
        rid = ctypes.c_uint64()
        if plain is not None:
            pl = np.ascontiguousarray(plain, np.int64)
            rc = lib.csrmf_server_submit_int(self.h, op, user, len(it), _ptr(it, ctypes.c_int32),
                                             _ptr(pl, ctypes.c_int64), client_serial, ctypes.byref(rid))
        else:
            r = None if ratings is None else np.ascontiguousarray(ratings, np.float64)
            rc = lib.csrmf_server_submit(self.h, op, user, len(it), _ptr(it, ctypes.c_int32),
                                         None if r is None else _ptr(r, ctypes.c_double), client_serial,
                                         ctypes.byref(rid))
        if rc != CSRMF_OK:
            raise CsrmfError(rc, lib.csrmf_last_error(None).decode())
        return rid.value

    def poll(self, rid, wait=False):
        """(status, [result handles], latency_s)."""
        st = ctypes.c_int32()
        n = ctypes.c_int32(0)
        lat = ctypes.c_double(0)
        out = np.zeros(16, np.uint64)
        rc = lib.csrmf_server_poll(self.h, rid, int(bool(wait)), ctypes.byref(st), _ptr(out, ctypes.c_uint64), 16,
                                   ctypes.byref(n), ctypes.byref(lat))
        if rc != CSRMF_OK:
            raise CsrmfError(rc, "request failed")
        return st.value, [int(x) for x in out[: n.value]], lat.value

    def stats(self):
        import json
        buf = ctypes.create_string_buffer(1024)
        lib.csrmf_server_stats(self.h, buf, 1024)
        return json.loads(buf.value.decode())

    def close(self):
        if self.h:
            lib.csrmf_server_destroy(self.h)
            self.h = None
            if self in getattr(self.ctx, "_servers", []):
                self.ctx._servers.remove(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on=True):
    lib.csrmf_profile_enable(int(bool(on)))


def profile_report():
    """{kernel: (launches, total_ms, algorithmic_bytes)} recorded since profile_enable()."""
    import json
    cap = 1 << 20
    while True:   # one call that fits: two calls could see reports of different lengths
        buf = ctypes.create_string_buffer(cap)
        n = lib.csrmf_profile_report(buf, cap)
        if n < cap:
            break
        cap = 2 * n
    return {k: (int(v[0]), float(v[1]), float(v[2])) for k, v in json.loads(buf.value.decode()).items()}


def boot_levels(cfg):
    """Levels one bootstrap with this configuration consumes."""
    v = ctypes.c_int32()
    rc = lib.csrmf_boot_levels(ctypes.byref(cfg), ctypes.byref(v))
    if rc != CSRMF_OK:
        raise CsrmfError(rc, "invalid bootstrapping configuration")
    return v.value


def boot_n12_params():
    """N = 2^12, q_0 60-bit + 18 x 40-bit, 3 x 60-bit special primes, dnum 5 (4-limb digits),
    scale 2^40: room for one bootstrap (17 levels at r = 9, d = 11) and one level after it."""
    return params(12, 60, 18, 40, 3, 60, 5, 40)


def tiny_params(k=4, lr=0.01, lam=0.02, rule=1):
    """N = 2^12, q_0 60-bit + 3 x 40-bit scale primes, 1 x 60-bit special prime, dnum 4, scale 2^40."""
    return params(12, 60, 3, 40, 1, 60, 4, 40, k=k, lr=lr, lam=lam, rule=rule)


def kernel_batch_params():
    """N = 2^16, q_0 60-bit + 24 x 40-bit, 3 x 60-bit special primes, dnum 3, scale 2^40."""
    return params(16, 60, 24, 40, 3, 60, 3, 40)


def mf_n15_params(k=10, lr=0.01, lam=0.02, rule=2, refresh_mode=0):
    """N = 2^15, q_0 60-bit + 16 x 40-bit, 3 x 60-bit special primes, dnum 5 (4-limb digits)."""
    return params(15, 60, 16, 40, 3, 60, 5, 40, k=k, lr=lr, lam=lam, rule=rule, refresh_mode=refresh_mode)


def mf_n16_params(k=16, lr=0.01, lam=0.02, rule=2, refresh_mode=0):
    """N = 2^16, q_0 60-bit + 24 x 40-bit, 3 x 60-bit special primes, dnum 7 (4-limb digits)."""
    return params(16, 60, 24, 40, 3, 60, 7, 40, k=k, lr=lr, lam=lam, rule=rule, refresh_mode=refresh_mode)
