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
RS_POLY_MATRIX_MAX_K = 32
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
    try:
        # When PyTorch provides device memory and streams, load its HIP
        # runtime first: the library then binds to the same (one) runtime.
        import torch  # noqa: F401
    except ImportError:
        pass
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
    lib.rs_poly_update.argtypes = [vp, pp, pp, sz, vp]
    lib.rs_poly_update_nibble.argtypes = [vp, pp, pp, sz, vp]
    lib.rs_poly_encode_bitmatrix.argtypes = [vp, pp, pp, sz, vp]
    lib.rs_poly_encode_matrix.argtypes = [vp, pp, pp, sz, vp]
    lib.rs_poly_bitmatrix_supported.argtypes = [i, i, i, u]
    lib.rs_poly_decode.argtypes = [vp, pp, sz, ip, i, u, vp]
    lib.rs_poly_decode_plan.argtypes = [vp, ip, i, u, ip, ip, u8p]
    lib.rs_poly_stream_probe.argtypes = [vp, sz, sz, i, i, i, sz, i, i, vp]
    sp = ctypes.POINTER(Stripe)
    lp = ctypes.POINTER(Launch)
    lib.rs_poly_batch_create.argtypes = [ctypes.POINTER(vp)]
    lib.rs_poly_batch_free.argtypes = [vp]
    lib.rs_poly_batch_free.restype = None
    lib.rs_poly_batch_encode.argtypes = [vp, sp, i, vp]
    lib.rs_poly_batch_decode.argtypes = [vp, sp, i, vp]
    lib.rs_poly_batch_update.argtypes = [vp, sp, i, vp]
    lib.rs_poly_encode_batch.argtypes = [vp, sp, i, vp]
    lib.rs_poly_batch_noalloc.argtypes = [i, sp, i, vp]
    lib.rs_poly_decode_batch.argtypes = [vp, sp, i, vp]
    lib.rs_poly_batch_reserve.argtypes = [vp, i, sz]
    lib.rs_poly_batch_get_launch.argtypes = [vp, i, i, lp]
    lib.rs_poly_batch_set_launch.argtypes = [vp, i, i, lp]
    lib.rs_poly_tune.argtypes = [vp, i, sp, i, vp, lp]
    rq = ctypes.POINTER(ServeRequest)
    cp = ctypes.POINTER(ServeCompletion)
    lib.rs_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
    lib.rs_serve_submit.argtypes = [vp, rq, ctypes.POINTER(ctypes.c_uint64)]
    lib.rs_serve_replay.argtypes = [vp, rq, ctypes.POINTER(ctypes.c_double), i]
    lib.rs_serve_poll.argtypes = [vp, cp, i, ip, i]
    lib.rs_serve_release.argtypes = [vp, ctypes.c_uint64]
    lib.rs_serve_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    lib.rs_serve_destroy.argtypes = [vp]
    lib.rs_serve_destroy.restype = None
    _lib = lib
    return lib


class ServeConfig(ctypes.Structure):
    """rs_serve_config_t."""
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("streams", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("auto_release", ctypes.c_int),
                ("max_block_bytes", ctypes.c_size_t)]


class ServeRequest(ctypes.Structure):
    """rs_serve_request_t."""
    _fields_ = [("op", ctypes.c_int), ("code", ctypes.c_void_p),
                ("blocks", ctypes.POINTER(ctypes.c_void_p)), ("block_bytes", ctypes.c_size_t),
                ("erasures", ctypes.POINTER(ctypes.c_int)), ("n_erasures", ctypes.c_int),
                ("flags", ctypes.c_uint), ("user_tag", ctypes.c_uint64)]


class ServeCompletion(ctypes.Structure):
    """rs_serve_completion_t."""
    _fields_ = [("ticket", ctypes.c_uint64), ("user_tag", ctypes.c_uint64),
                ("status", ctypes.c_int), ("n_out", ctypes.c_int),
                ("out", ctypes.c_void_p * RS_POLY_MAX_M),
                ("out_index", ctypes.c_int * RS_POLY_MAX_M),
                ("charge_bytes", ctypes.c_size_t), ("queue_us", ctypes.c_double),
                ("latency_us", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    """rs_serve_stats_t."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("user_bytes", ctypes.c_uint64),
                ("budget_in_use", ctypes.c_size_t), ("budget_peak", ctypes.c_size_t),
                ("peak_inflight_batches", ctypes.c_int), ("pending", ctypes.c_int),
                ("launch_host_us", ctypes.c_double), ("batch_device_us", ctypes.c_double),
                ("admit_host_us", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stripe(ctypes.Structure):
    """rs_poly_stripe_t."""
    _fields_ = [("code", ctypes.c_void_p),
                ("blocks", ctypes.POINTER(ctypes.c_void_p)),
                ("block_bytes", ctypes.c_size_t),
                ("erasures", ctypes.POINTER(ctypes.c_int)),
                ("n_erasures", ctypes.c_int),
                ("flags", ctypes.c_uint)]


class Launch(ctypes.Structure):
    """rs_poly_launch_t."""
    _fields_ = [("bytes_per_lane", ctypes.c_int), ("threads", ctypes.c_int),
                ("tile_bytes", ctypes.c_int), ("wgs_per_cu", ctypes.c_int),
                ("table_placement", ctypes.c_int), ("tile_order", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


RS_POLY_OP_ENCODE = 0
RS_POLY_OP_DECODE = 1
RS_POLY_OP_UPDATE = 2
RS_POLY_TABLES_PACKED = 0
RS_POLY_TABLES_NIBBLE = 1
RS_POLY_TABLES_BITMATRIX = 2
RS_POLY_TABLES_REGISTERS = 3


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


def rs_poly_encode_bitmatrix(h, data, parity, block_bytes, stream=None):
    d, p = _ptr_array(data), _ptr_array(parity)
    return check(load().rs_poly_encode_bitmatrix(h, d, p, block_bytes, _stream(stream)),
                 "rs_poly_encode_bitmatrix")


def rs_poly_encode_matrix(h, data, parity, block_bytes, stream=None):
    d, p = _ptr_array(data), _ptr_array(parity)
    return check(load().rs_poly_encode_matrix(h, d, p, block_bytes, _stream(stream)),
                 "rs_poly_encode_matrix")


def rs_poly_bitmatrix_supported(k, m, w=8, prim_poly=0x11D):
    return bool(load().rs_poly_bitmatrix_supported(k, m, w, prim_poly))


def rs_poly_update(h, delta, parity, block_bytes, stream=None):
    d, p = _ptr_array(delta), _ptr_array(parity)
    return check(load().rs_poly_update(h, d, p, block_bytes, _stream(stream)),
                 "rs_poly_update")


def rs_poly_update_nibble(h, delta, parity, block_bytes, stream=None):
    d, p = _ptr_array(delta), _ptr_array(parity)
    return check(load().rs_poly_update_nibble(h, d, p, block_bytes, _stream(stream)),
                 "rs_poly_update_nibble")


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


class StripeArray:
    """A prepared rs_poly_stripe_t array (and the host arrays it points to),
    reusable across batch calls.  Entries: (code, blocks, block_bytes) for
    encode and update (update: blocks 0..k-1 are delta blocks or None), plus
    (erasures, flags) for decode."""

    def __init__(self, entries):
        self.count = len(entries)
        self.arr = (Stripe * max(1, self.count))()
        self._keep = []
        for i, e in enumerate(entries):
            code, blocks, nbytes = e[0], e[1], e[2]
            er = list(e[3]) if len(e) > 3 and e[3] is not None else []
            flags = e[4] if len(e) > 4 else 0
            bl = _ptr_array(list(blocks))
            ea = (ctypes.c_int * max(1, len(er)))(*er)
            self._keep += [bl, ea]
            h = code.handle if isinstance(code, Code) else code
            self.arr[i] = Stripe(h, ctypes.cast(bl, ctypes.POINTER(ctypes.c_void_p)),
                                 nbytes, ctypes.cast(ea, ctypes.POINTER(ctypes.c_int)),
                                 len(er), flags)


def rs_poly_batch_create():
    b = ctypes.c_void_p()
    check(load().rs_poly_batch_create(ctypes.byref(b)), "rs_poly_batch_create")
    return b


def rs_poly_batch_free(b):
    load().rs_poly_batch_free(b)


def _stripes(stripes):
    return stripes if isinstance(stripes, StripeArray) else StripeArray(stripes)


def rs_poly_batch_encode(b, stripes, stream=None):
    sa = _stripes(stripes)
    return check(load().rs_poly_batch_encode(b, sa.arr, sa.count, _stream(stream)),
                 "rs_poly_batch_encode")


def rs_poly_batch_decode(b, stripes, stream=None):
    sa = _stripes(stripes)
    return check(load().rs_poly_batch_decode(b, sa.arr, sa.count, _stream(stream)),
                 "rs_poly_batch_decode")


def rs_poly_encode_batch(b, stripes, stream=None):
    sa = _stripes(stripes)
    return check(load().rs_poly_encode_batch(b, sa.arr, sa.count, _stream(stream)),
                 "rs_poly_encode_batch")


def rs_poly_decode_batch(b, stripes, stream=None):
    sa = _stripes(stripes)
    return check(load().rs_poly_decode_batch(b, sa.arr, sa.count, _stream(stream)),
                 "rs_poly_decode_batch")


def rs_poly_batch_noalloc(op, stripes, stream=None):
    sa = _stripes(stripes)
    return check(load().rs_poly_batch_noalloc(op, sa.arr, sa.count, _stream(stream)),
                 "rs_poly_batch_noalloc")


def rs_poly_stream_probe(base, stripe_stride, block_stride, stripes, n_in, n_out, block_bytes,
                         tile_bytes=65536, tile_order=0, stream=None):
    return check(load().rs_poly_stream_probe(_ptr(base), stripe_stride, block_stride, stripes,
                                             n_in, n_out, block_bytes, tile_bytes, tile_order,
                                             _stream(stream)), "rs_poly_stream_probe")


def rs_poly_batch_update(b, stripes, stream=None):
    sa = _stripes(stripes)
    return check(load().rs_poly_batch_update(b, sa.arr, sa.count, _stream(stream)),
                 "rs_poly_batch_update")


def rs_poly_batch_get_launch(b, op, wide):
    c = Launch()
    check(load().rs_poly_batch_get_launch(b, op, wide, ctypes.byref(c)),
          "rs_poly_batch_get_launch")
    return c


def rs_poly_batch_set_launch(b, op, wide, cfg):
    if isinstance(cfg, dict):
        cfg = Launch(**cfg)
    return check(load().rs_poly_batch_set_launch(b, op, wide, ctypes.byref(cfg)),
                 "rs_poly_batch_set_launch")


def rs_poly_tune(b, op, stripes, stream=None):
    sa = _stripes(stripes)
    best = Launch()
    check(load().rs_poly_tune(b, op, sa.arr, sa.count, _stream(stream), ctypes.byref(best)),
          "rs_poly_tune")
    return best


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

    def encode_bitmatrix(self, data, parity, block_bytes=None, stream=None):
        """The same parity as encode, from the bit-sliced XOR-only kernel
        (codes for which rs_poly_bitmatrix_supported is true)."""
        if block_bytes is None:
            block_bytes = data[0].numel()
        return rs_poly_encode_bitmatrix(self._h, list(data), list(parity), block_bytes, stream)

    def encode_matrix(self, data, parity, block_bytes=None, stream=None):
        """The same parity as encode, from the generator-matrix kernel
        (codes with k <= 32)."""
        if block_bytes is None:
            block_bytes = data[0].numel()
        return rs_poly_encode_matrix(self._h, list(data), list(parity), block_bytes, stream)

    def update(self, delta, parity, block_bytes=None, stream=None):
        """parity ^= encode(delta) in place; None entries of delta are
        unchanged blocks."""
        if block_bytes is None:
            block_bytes = parity[0].numel()
        return rs_poly_update(self._h, list(delta), list(parity), block_bytes, stream)

    def update_nibble(self, delta, parity, block_bytes=None, stream=None):
        """The same update with register-held split-nibble products (1 or 2
        changed blocks, changed * m <= 8, 16-byte-aligned blocks)."""
        if block_bytes is None:
            block_bytes = parity[0].numel()
        return rs_poly_update_nibble(self._h, list(delta), list(parity), block_bytes, stream)

    def decode(self, blocks, erasures, block_bytes=None, flags=0, stream=None):
        if block_bytes is None:
            block_bytes = next(b for b in blocks if b is not None).numel()
        return rs_poly_decode(self._h, list(blocks), block_bytes, list(erasures), flags, stream)

    def decode_plan(self, erasures, flags=0):
        return rs_poly_decode_plan(self._h, self.n, self.m, list(erasures), flags)


class Batch:
    """A batch object: one persistent, graph-replayed launch per call."""

    def __init__(self):
        self._b = rs_poly_batch_create()

    @property
    def handle(self):
        return self._b

    def close(self):
        if self._b is not None:
            rs_poly_batch_free(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def encode(self, stripes, stream=None):
        return rs_poly_batch_encode(self._b, stripes, stream)

    def decode(self, stripes, stream=None):
        return rs_poly_batch_decode(self._b, stripes, stream)

    def update(self, stripes, stream=None):
        return rs_poly_batch_update(self._b, stripes, stream)

    def reserve(self, max_stripes, max_block_bytes):
        return check(load().rs_poly_batch_reserve(self._b, max_stripes, max_block_bytes),
                     "rs_poly_batch_reserve")

    def get_launch(self, op, wide=0):
        return rs_poly_batch_get_launch(self._b, op, wide)

    def set_launch(self, op, wide, cfg):
        return rs_poly_batch_set_launch(self._b, op, wide, cfg)

    def tune(self, op, stripes, stream=None):
        return rs_poly_tune(self._b, op, stripes, stream)


class RequestArray:
    """A prepared rs_serve_request_t array.  Entries are dicts with keys op,
    code, blocks, block_bytes and, for decode, erasures (and flags); tag
    defaults to the entry's index."""

    def __init__(self, entries):
        self.count = len(entries)
        self.arr = (ServeRequest * max(1, self.count))()
        self._keep = []
        for i, e in enumerate(entries):
            bl = _ptr_array(list(e["blocks"]))
            er = list(e.get("erasures") or [])
            ea = (ctypes.c_int * max(1, len(er)))(*er)
            self._keep += [bl, ea]
            code = e["code"]
            h = code.handle if isinstance(code, Code) else code
            self.arr[i] = ServeRequest(e["op"], h, ctypes.cast(bl, ctypes.POINTER(ctypes.c_void_p)),
                                       e["block_bytes"],
                                       ctypes.cast(ea, ctypes.POINTER(ctypes.c_int)), len(er),
                                       e.get("flags", 0), e.get("tag", i))


class Serve:
    """The continuous-batching serving engine (rs_serve_*)."""

    def __init__(self, hbm_budget_bytes, streams=4, max_batch=64, auto_release=True,
                 max_block_bytes=0):
        cfg = ServeConfig(hbm_budget_bytes, streams, max_batch, 1 if auto_release else 0,
                          max_block_bytes)
        self._s = ctypes.c_void_p()
        check(load().rs_serve_create(ctypes.byref(cfg), ctypes.byref(self._s)),
              "rs_serve_create")
        self._keep = []

    def submit(self, entry):
        ra = RequestArray([entry])
        t = ctypes.c_uint64()
        check(load().rs_serve_submit(self._s, ra.arr, ctypes.byref(t)), "rs_serve_submit")
        return t.value

    def replay(self, entries, arrival_us):
        ra = entries if isinstance(entries, RequestArray) else RequestArray(entries)
        times = (ctypes.c_double * max(1, ra.count))(*arrival_us)
        self._keep.append((ra, times))
        check(load().rs_serve_replay(self._s, ra.arr, times, ra.count), "rs_serve_replay")

    def poll(self, max_n=256, timeout_us=0):
        """Up to max_n completions (copies), waiting up to timeout_us."""
        if getattr(self, "_pbuf_n", 0) < max_n:
            self._pbuf = (ServeCompletion * max_n)()
            self._pbuf_n = max_n
        buf = self._pbuf
        n = ctypes.c_int()
        check(load().rs_serve_poll(self._s, buf, max_n, ctypes.byref(n), timeout_us),
              "rs_serve_poll")
        out = []
        for i in range(n.value):
            c = ServeCompletion()
            ctypes.pointer(c)[0] = buf[i]
            out.append(c)
        return out

    def release(self, ticket):
        check(load().rs_serve_release(self._s, ticket), "rs_serve_release")

    def stats(self):
        st = ServeStats()
        check(load().rs_serve_stats(self._s, ctypes.byref(st)), "rs_serve_stats")
        return st.as_dict()

    def close(self):
        if self._s is not None:
            load().rs_serve_destroy(self._s)
            self._s = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
