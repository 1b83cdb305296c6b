"""ctypes binding of librs_poly.so -- argument marshalling only.

Function names mirror the C ABI in include/rs_poly.h.  Every step of encode
and decode runs in the library's HIP kernels; PyTorch is only used by callers
for device memory and streams.  The library must have been built
(`python -m paper_1312_5155_amd.build`); there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librs_poly.so")

RS_OK = 0
RS_EINVAL = -1
RS_ERANGE = -2
RS_ETOOMANY = -3
RS_ENULL = -4
RS_EDEVICE = -5
RS_ENOMEM = -6
RS_EBUSY = -7
RS_POLY_FLAG_ALL_SURVIVORS = 1
RS_POLY_MAX_M = 8
RS_POLY_MAX_N = 255

_lib = None


class RsPolyError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load().rs_poly_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")


def load():
    """Loads the in-tree librs_poly.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1312_5155_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, u, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_size_t
    pp = ctypes.POINTER(ctypes.c_void_p)
    ip = ctypes.POINTER(ctypes.c_int)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.rs_poly_init.argtypes = [i, i, i, u, ctypes.POINTER(vp)]
    lib.rs_poly_free.argtypes = [vp]
    lib.rs_poly_free.restype = None
    lib.rs_poly_strerror.argtypes = [i]
    lib.rs_poly_strerror.restype = ctypes.c_char_p
    lib.rs_poly_generator.argtypes = [vp, u8p]
    lib.rs_poly_encode.argtypes = [vp, pp, pp, sz, vp]
    lib.rs_poly_decode.argtypes = [vp, pp, sz, ip, i, u, vp]
    lib.rs_poly_decode_plan.argtypes = [vp, ip, i, u, ip, ip, u8p]
    _lib = lib
    return lib


def check(rc, where):
    if rc != RS_OK:
        raise RsPolyError(rc, where)
    return rc


def _ptr(x):
    """Device pointer of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _ptr_array(items):
    arr = (ctypes.c_void_p * max(1, len(items)))()
    for j, x in enumerate(items):
        arr[j] = _ptr(x)
    return arr


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------- raw ABI --

def rs_poly_init(k, m, w=8, prim_poly=0x11D):
    h = ctypes.c_void_p()
    check(load().rs_poly_init(k, m, w, prim_poly, ctypes.byref(h)), "rs_poly_init")
    return h


def rs_poly_free(h):
    load().rs_poly_free(h)


def rs_poly_strerror(err):
    return load().rs_poly_strerror(err).decode()


def rs_poly_generator(h, m):
    g = (ctypes.c_uint8 * (m + 1))()
    check(load().rs_poly_generator(h, g), "rs_poly_generator")
    return list(g)


def rs_poly_encode(h, data, parity, block_bytes, stream=None):
    d, p = _ptr_array(data), _ptr_array(parity)
    return check(load().rs_poly_encode(h, d, p, block_bytes, _stream(stream)),
                 "rs_poly_encode")


def rs_poly_decode(h, blocks, block_bytes, erasures, flags=0, stream=None):
    b = _ptr_array(blocks)
    er = (ctypes.c_int * max(1, len(erasures)))(*erasures)
    return check(load().rs_poly_decode(h, b, block_bytes, er, len(erasures), flags,
                                       _stream(stream)), "rs_poly_decode")


def rs_poly_decode_plan(h, n, m, erasures, flags=0):
    """Returns (read_set, coeffs) with coeffs a t x m list of lists."""
    er = (ctypes.c_int * max(1, len(erasures)))(*erasures)
    rs = (ctypes.c_int * n)()
    nr = ctypes.c_int()
    co = (ctypes.c_uint8 * max(1, len(erasures) * m))()
    check(load().rs_poly_decode_plan(h, er, len(erasures), flags, rs, ctypes.byref(nr), co),
          "rs_poly_decode_plan")
    t = len(erasures)
    return list(rs[:nr.value]), [list(co[r * m:(r + 1) * m]) for r in range(t)]


# ------------------------------------------------------ convenience --

class Code:
    """An RS(k,m) code handle.  Blocks are uint8 device tensors (or ints)."""

    def __init__(self, k, m, w=8, prim_poly=0x11D):
        self.k, self.m, self.w, self.prim_poly = k, m, w, prim_poly
        self.n = k + m
        self._h = rs_poly_init(k, m, w, prim_poly)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None:
            rs_poly_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def generator(self):
        return rs_poly_generator(self._h, self.m)

    def encode(self, data, parity, block_bytes=None, stream=None):
        if block_bytes is None:
            block_bytes = data[0].numel()
        return rs_poly_encode(self._h, list(data), list(parity), block_bytes, stream)

    def decode(self, blocks, erasures, block_bytes=None, flags=0, stream=None):
        if block_bytes is None:
            block_bytes = next(b for b in blocks if b is not None).numel()
        return rs_poly_decode(self._h, list(blocks), block_bytes, list(erasures), flags, stream)

    def decode_plan(self, erasures, flags=0):
        return rs_poly_decode_plan(self._h, self.n, self.m, list(erasures), flags)
