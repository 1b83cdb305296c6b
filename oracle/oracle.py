"""ctypes + numpy wrapper of the C oracle (test infrastructure only).

Blocks are numpy uint8 arrays of shape (count, B): row j is block j.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class _Field(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int), ("poly", ctypes.c_uint),
                ("q", ctypes.c_int), ("order", ctypes.c_int),
                ("exp", ctypes.c_uint8 * 256), ("log", ctypes.c_int * 256),
                ("mul", (ctypes.c_uint8 * 256) * 256)]


def load():
    """Loads oracle/librs_oracle.so, building it first if it is absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    P = ctypes.POINTER
    u8p = P(ctypes.c_uint8)
    ip = P(ctypes.c_int)
    fp = P(_Field)
    lib.rso_field_init.argtypes = [fp, ctypes.c_int, ctypes.c_uint]
    lib.rso_mul.argtypes = [fp, ctypes.c_uint8, ctypes.c_uint8]
    lib.rso_mul.restype = ctypes.c_uint8
    lib.rso_alpha_pow.argtypes = [fp, ctypes.c_long]
    lib.rso_alpha_pow.restype = ctypes.c_uint8
    lib.rso_genpoly.argtypes = [fp, ctypes.c_int, u8p]
    lib.rso_encode.argtypes = [fp, ctypes.c_int, ctypes.c_int, u8p, u8p,
                               ctypes.c_size_t]
    lib.rso_position.argtypes = [ctypes.c_int] * 3
    lib.rso_vandermonde.argtypes = [fp, ctypes.c_int, ctypes.c_int, ip,
                                    ctypes.c_int, u8p]
    lib.rso_invert.argtypes = [fp, ctypes.c_int, u8p, u8p]
    lib.rso_syndromes.argtypes = [fp, ctypes.c_int, ctypes.c_int, u8p, ip,
                                  ctypes.c_int, u8p]
    lib.rso_decode.argtypes = [fp, ctypes.c_int, ctypes.c_int, u8p,
                               ctypes.c_size_t, ip, ctypes.c_int]
    _LIB = lib
    return lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _ints(seq):
    arr = (ctypes.c_int * max(1, len(seq)))(*seq)
    return arr


class Field:
    """GF(2^w) built from the field polynomial `poly` with alpha = 2."""

    def __init__(self, w=8, poly=0x11D):
        lib = load()
        self._f = _Field()
        if lib.rso_field_init(ctypes.byref(self._f), w, poly) != 0:
            raise ValueError(f"poly {poly:#x} is not primitive of degree {w}")
        self.w, self.poly, self.q, self.order = w, poly, 1 << w, (1 << w) - 1

    @property
    def ref(self):
        return ctypes.byref(self._f)

    def exp_table(self):
        return np.frombuffer(bytes(self._f.exp), dtype=np.uint8)[:self.order].copy()

    def log_table(self):
        return np.array(self._f.log[:self.q], dtype=np.int64)

    def mul_table(self):
        t = np.frombuffer(bytes(self._f.mul), dtype=np.uint8).reshape(256, 256)
        return t[:self.q, :self.q].copy()

    def mul(self, a, b):
        return int(load().rso_mul(self.ref, a, b))

    def alpha_pow(self, e):
        return int(load().rso_alpha_pow(self.ref, e))


def genpoly(F, m):
    g = np.zeros(m + 1, dtype=np.uint8)
    if load().rso_genpoly(F.ref, m, _u8(g)) != 0:
        raise ValueError("bad m")
    return g


def encode(F, k, m, data):
    """data: (k, B) uint8 -> parity (m, B) uint8."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    assert data.ndim == 2 and data.shape[0] == k
    B = data.shape[1]
    parity = np.zeros((m, B), dtype=np.uint8)
    if load().rso_encode(F.ref, k, m, _u8(data), _u8(parity), B) != 0:
        raise ValueError("rso_encode rejected its arguments")
    return parity


def decode(F, k, m, blocks, erasures):
    """blocks: (k+m, B) uint8, rebuilt in place at the erased rows; returned."""
    assert blocks.dtype == np.uint8 and blocks.flags.c_contiguous
    assert blocks.shape[0] == k + m
    er = list(erasures)
    rc = load().rso_decode(F.ref, k, m, _u8(blocks), blocks.shape[1],
                           _ints(er), len(er))
    if rc != 0:
        raise ValueError("rso_decode rejected its arguments")
    return blocks


def syndromes(F, k, m, word, erasures):
    word = np.ascontiguousarray(word, dtype=np.uint8)
    er = list(erasures)
    S = np.zeros(max(1, len(er)), dtype=np.uint8)
    if load().rso_syndromes(F.ref, k, m, _u8(word), _ints(er), len(er), _u8(S)) != 0:
        raise ValueError("bad arguments")
    return S[:len(er)]


def vandermonde(F, k, m, erasures):
    er = list(erasures)
    t = len(er)
    V = np.zeros(max(1, t * t), dtype=np.uint8)
    if load().rso_vandermonde(F.ref, k, m, _ints(er), t, _u8(V)) != 0:
        raise ValueError("bad arguments")
    return V[:t * t].reshape(t, t)


def invert(F, A):
    A = np.ascontiguousarray(A, dtype=np.uint8)
    t = A.shape[0]
    out = np.zeros_like(A)
    if load().rso_invert(F.ref, t, _u8(A), _u8(out)) != 0:
        raise ValueError("singular")
    return out


def position(k, m, b):
    return int(load().rso_position(k, m, b))
