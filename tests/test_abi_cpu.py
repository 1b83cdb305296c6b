"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, validates its arguments before touching the device, and its host-side
decode plan (the per-pattern coefficients) rebuilds erased blocks when
applied on the CPU to remainders computed by the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(rs_[a-z_0-9]+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = declared_functions()
    assert "rs_poly_init" in names and "rs_poly_decode" in names
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("k,m,w,poly,err", [
    (0, 4, 8, 0x11D, B.RS_EINVAL),
    (10, 0, 8, 0x11D, B.RS_EINVAL),
    (10, 9, 8, 0x11D, B.RS_EINVAL),       # m above RS_POLY_MAX_M
    (250, 6, 8, 0x11D, B.RS_EINVAL),      # n = 256 > 2^8 - 1
    (12, 4, 4, 0x13, B.RS_EINVAL),        # n = 16 > 2^4 - 1
    (10, 4, 6, 0x43, B.RS_EINVAL),        # w not in {4, 8}
    (10, 4, 8, 0x11B, B.RS_EINVAL),       # irreducible, x not primitive
    (10, 4, 8, 0x1D, B.RS_EINVAL),        # degree != w
    (10, 4, 4, 0x11D, B.RS_EINVAL),
])
def test_init_rejects(k, m, w, poly, err):
    h = ctypes.c_void_p()
    assert B.load().rs_poly_init(k, m, w, poly, ctypes.byref(h)) == err
    assert not h.value


def test_init_null_out():
    assert B.load().rs_poly_init(10, 4, 8, 0x11D, None) == B.RS_ENULL


def test_strerror_covers_codes():
    for c in range(0, -8, -1):
        assert B.rs_poly_strerror(c) != "unknown status"
    assert B.rs_poly_strerror(-99) == "unknown status"


def test_generator_matches_paper_and_oracle(golden_example):
    code = B.Code(4, 3)
    assert code.generator() == golden_example["genpoly_m3"]   # Sec. 3.1
    F = oracle.Field(8, 0x11D)
    for m in range(1, 9):
        assert B.Code(10, m).generator() == oracle.genpoly(F, m).tolist()
    F4 = oracle.Field(4, 0x13)
    assert B.Code(4, 3, 4, 0x13).generator() == oracle.genpoly(F4, 3).tolist()


def test_validation_happens_before_any_device_call():
    # These return errors (or no-op success) without a GPU in the container.
    lib = B.load()
    code = B.Code(10, 4)
    h = code.handle
    ptrs = (ctypes.c_void_p * 14)(*([0x1000] * 14))
    def dec(er, flags=0, blocks=ptrs, nbytes=4096):
        arr = (ctypes.c_int * max(1, len(er)))(*er)
        return lib.rs_poly_decode(h, blocks, nbytes, arr, len(er), flags, None)
    assert dec([0, 1, 2, 3, 4]) == B.RS_ETOOMANY
    assert dec([0, 0]) == B.RS_ERANGE
    assert dec([14]) == B.RS_ERANGE
    assert dec([-1]) == B.RS_ERANGE
    assert dec([1], flags=2) == B.RS_EINVAL
    assert dec([]) == B.RS_OK                      # t = 0: no-op
    assert dec([3], blocks=None) == B.RS_ENULL
    assert lib.rs_poly_decode(h, ptrs, 4096, None, 2, 0, None) == B.RS_ENULL
    assert lib.rs_poly_decode(None, ptrs, 4096, None, 0, 0, None) == B.RS_ENULL
    assert lib.rs_poly_decode(h, ptrs, 4096, None, -1, 0, None) == B.RS_EINVAL
    # an erased block's pointer is required; an unread survivor's is not
    holes = (ctypes.c_void_p * 14)(*([0x1000] * 14))
    holes[5] = None
    assert dec([5], blocks=holes) == B.RS_ENULL
    holes2 = (ctypes.c_void_p * 14)(*([0x1000] * 14))
    holes2[9] = None        # data block 9, unread when only data block 2 is lost
    assert dec([2], blocks=holes2, nbytes=0) == B.RS_OK
    assert dec([2], blocks=holes2, flags=B.RS_POLY_FLAG_ALL_SURVIVORS, nbytes=0) == B.RS_ENULL
    d = (ctypes.c_void_p * 10)(*([0x1000] * 10))
    p = (ctypes.c_void_p * 4)(*([0x2000] * 4))
    assert lib.rs_poly_encode(h, d, p, 0, None) == B.RS_OK   # empty: no-op
    assert lib.rs_poly_encode(h, None, p, 16, None) == B.RS_ENULL
    p[2] = None
    assert lib.rs_poly_encode(h, d, p, 16, None) == B.RS_ENULL
    # bit-matrix encode: k <= 32, 16-byte aligned pointers
    p3 = (ctypes.c_void_p * 4)(*([0x2000] * 4))
    enc_bm = lib.rs_poly_encode_bitmatrix
    assert enc_bm(h, d, p3, 0, None) == B.RS_OK                    # empty: no-op
    assert enc_bm(h, None, p3, 16, None) == B.RS_ENULL
    assert enc_bm(None, d, p3, 16, None) == B.RS_ENULL
    d_odd = (ctypes.c_void_p * 10)(*([0x1000] * 9 + [0x1008]))
    assert enc_bm(h, d_odd, p3, 16, None) == B.RS_EINVAL            # 8-byte aligned
    h33b = B.Code(33, 4)
    d33b = (ctypes.c_void_p * 33)(*([0x1000] * 33))
    assert enc_bm(h33b.handle, d33b, p3, 16, None) == B.RS_EINVAL   # k = 33 > 32
    assert lib.rs_poly_bitmatrix_supported(10, 4, 8, 0x11D) == 1   # compiled in
    assert lib.rs_poly_bitmatrix_supported(32, 8, 8, 0x11D) == 1
    assert lib.rs_poly_bitmatrix_supported(9, 3, 8, 0x11D) == 1    # run-time rows
    assert lib.rs_poly_bitmatrix_supported(10, 4, 8, 0x12B) == 1
    assert lib.rs_poly_bitmatrix_supported(4, 3, 4, 0x13) == 1
    assert lib.rs_poly_bitmatrix_supported(33, 4, 8, 0x11D) == 0   # k > 32
    assert lib.rs_poly_bitmatrix_supported(10, 4, 8, 0x11B) == 0   # not a code
    assert lib.rs_poly_bitmatrix_supported(12, 4, 4, 0x13) == 0
    # generator-matrix encode: k <= 32
    enc_mx = lib.rs_poly_encode_matrix
    h6 = B.Code(6, 3)
    d6 = (ctypes.c_void_p * 6)(*([0x1000] * 6))
    p6 = (ctypes.c_void_p * 3)(*([0x2000] * 3))
    assert enc_mx(h6.handle, d6, p6, 0, None) == B.RS_OK            # empty: no-op
    assert enc_mx(h6.handle, None, p6, 16, None) == B.RS_ENULL
    p6[1] = None
    assert enc_mx(h6.handle, d6, p6, 16, None) == B.RS_ENULL
    h33 = B.Code(33, 4)
    d33 = (ctypes.c_void_p * 33)(*([0x1000] * 33))
    assert enc_mx(h33.handle, d33, p3, 16, None) == B.RS_EINVAL      # k = 33 > 32
    assert enc_mx(h, d, p3, 0, None) == B.RS_OK                      # k = 10: wide form
    # update: NULL delta entries are unchanged blocks; parity is required
    nod = (ctypes.c_void_p * 10)()
    p2 = (ctypes.c_void_p * 4)(*([0x2000] * 4))
    assert lib.rs_poly_update(h, nod, p2, 4096, None) == B.RS_OK   # nothing changed
    assert lib.rs_poly_update(h, d, p2, 0, None) == B.RS_OK        # empty
    assert lib.rs_poly_update(h, None, p2, 16, None) == B.RS_ENULL
    assert lib.rs_poly_update(h, d, None, 16, None) == B.RS_ENULL
    assert lib.rs_poly_update(None, d, p2, 16, None) == B.RS_ENULL
    assert lib.rs_poly_update(h, nod, p, 16, None) == B.RS_ENULL   # p[2] is NULL


def test_nibble_update_validates_before_any_device_call():
    # No GPU here: every case below must return before a HIP call.
    lib = B.load()
    upd = lib.rs_poly_update_nibble
    code = B.Code(10, 4)          # kept alive: the handle is freed with it
    h = code.handle
    p4 = (ctypes.c_void_p * 4)(*([0x2000] * 4))
    one = (ctypes.c_void_p * 10)(*([None] * 9 + [0x1000]))
    two = (ctypes.c_void_p * 10)(*([0x1000, None, None, 0x3000] + [None] * 6))
    three = (ctypes.c_void_p * 10)(*([0x1000, 0x1010, 0x1020] + [None] * 7))
    nod = (ctypes.c_void_p * 10)()
    assert upd(h, nod, p4, 4096, None) == B.RS_OK        # nothing changed
    assert upd(h, one, p4, 0, None) == B.RS_OK           # empty
    assert upd(h, two, p4, 0, None) == B.RS_OK           # 2 x 4 = 8 products
    assert upd(h, three, p4, 16, None) == B.RS_EINVAL    # 3 changed blocks
    assert upd(None, one, p4, 16, None) == B.RS_ENULL
    assert upd(h, None, p4, 16, None) == B.RS_ENULL
    assert upd(h, one, None, 16, None) == B.RS_ENULL
    p4[1] = None
    assert upd(h, one, p4, 16, None) == B.RS_ENULL
    p4[1] = 0x2008                                        # 8-byte aligned parity
    assert upd(h, one, p4, 16, None) == B.RS_EINVAL
    p4[1] = 0x2000
    one[9] = 0x1004                                       # 4-byte aligned delta
    assert upd(h, one, p4, 16, None) == B.RS_EINVAL
    # RS(6,6): one changed block gives 6 products, two give 12 > 8
    code6 = B.Code(6, 6)
    h6 = code6.handle
    p6 = (ctypes.c_void_p * 6)(*([0x2000] * 6))
    d1 = (ctypes.c_void_p * 6)(*([0x1000] + [None] * 5))
    d2 = (ctypes.c_void_p * 6)(*([0x1000, 0x1000] + [None] * 4))
    assert upd(h6, d1, p6, 0, None) == B.RS_OK
    assert upd(h6, d2, p6, 16, None) == B.RS_EINVAL


def test_boundary_names_of_the_batch_calls():
    # rs_poly_encode_batch / rs_poly_decode_batch are the batch calls under
    # op-first names; they validate exactly as rs_poly_batch_encode/decode.
    lib = B.load()
    for name in ("rs_poly_encode_batch", "rs_poly_decode_batch"):
        fn = getattr(lib, name)
        assert fn(None, None, 0, None) == B.RS_ENULL          # no batch object


def test_noalloc_batch_validates_before_any_device_call():
    lib = B.load()
    code = B.Code(10, 4)
    one = B.StripeArray([(code, [0x1000] * 14, 4096)])
    assert lib.rs_poly_batch_noalloc(7, one.arr, 1, None) == B.RS_EINVAL     # unknown op
    assert lib.rs_poly_batch_noalloc(-1, one.arr, 1, None) == B.RS_EINVAL
    assert lib.rs_poly_batch_noalloc(B.RS_POLY_OP_ENCODE, one.arr, -1, None) == B.RS_EINVAL
    assert lib.rs_poly_batch_noalloc(B.RS_POLY_OP_DECODE, None, 2, None) == B.RS_ENULL
    assert lib.rs_poly_batch_noalloc(B.RS_POLY_OP_UPDATE, None, 0, None) == B.RS_OK
    # the advertised scratch size is the sum of its regions
    assert (64 << 10) + 2 * (512 << 10) + 2 * 4 * (128 << 10) == 2162688


def test_stream_probe_validates_before_any_device_call():
    lib = B.load()
    probe = lib.rs_poly_stream_probe
    base = ctypes.c_void_p(0x100000)
    MiB = 1 << 20
    ok = dict(ss=14 * MiB, bs=MiB, st=4, ni=10, no=4, bb=MiB, tb=65536, to=0)

    def call(base=base, **kw):
        a = {**ok, **kw}
        return probe(base, a["ss"], a["bs"], a["st"], a["ni"], a["no"], a["bb"], a["tb"], a["to"],
                     None)

    assert call(base=None) == B.RS_ENULL
    assert call(st=0) == B.RS_OK                             # nothing to stream
    assert call(bb=0) == B.RS_OK
    assert call(base=ctypes.c_void_p(0x100008)) == B.RS_EINVAL   # 8-byte aligned
    assert call(ni=0, no=0) == B.RS_EINVAL                    # nothing read or written
    assert call(ni=-1) == B.RS_EINVAL
    assert call(no=-1) == B.RS_EINVAL
    assert call(no=9) == B.RS_EINVAL
    assert call(st=-1) == B.RS_EINVAL
    assert call(bb=MiB + 16) == B.RS_EINVAL                   # block over its stride
    assert call(bb=1000) == B.RS_EINVAL                       # not a multiple of 16
    assert call(ss=13 * MiB) == B.RS_EINVAL                   # stripe holds 14 blocks
    assert call(tb=2048) == B.RS_EINVAL
    assert call(tb=65537) == B.RS_EINVAL
    assert call(to=2) == B.RS_EINVAL


def apply_plan_on_cpu(F, k, m, full, erasures, flags, code):
    """Rebuilds the erased rows of `full` with the library's plan: remainder
    of the received word (unread and erased rows zeroed) by the oracle, then
    lost_e = sum_l C[e][l] r_l with the oracle's product table."""
    read, C = code.decode_plan(erasures, flags)
    recv = np.zeros_like(full)
    recv[read] = full[read]
    r = oracle.encode(F, k, m, recv[:k]) ^ recv[k:]
    mul = F.mul_table()
    out = {}
    for e, row in zip(erasures, C):
        acc = np.zeros(full.shape[1], dtype=np.uint8)
        for l in range(m):
            acc ^= mul[row[l], r[l]]
        out[e] = acc
    return read, out


@pytest.mark.parametrize("flags", [0, B.RS_POLY_FLAG_ALL_SURVIVORS])
def test_decode_plan_every_pattern_rs63(flags):
    F = oracle.Field(8, 0x11D)
    k, m = 6, 3
    code = B.Code(k, m)
    data = workloads.random_bytes(21, (k, 257))
    full = np.concatenate([data, oracle.encode(F, k, m, data)])
    for er in workloads.all_patterns(k + m, m)[1:]:
        er = list(reversed(er))
        read, out = apply_plan_on_cpu(F, k, m, full, er, flags, code)
        assert read == sorted(read) and not set(read) & set(er)
        assert len(read) == (k + m - len(er) if flags else k)
        for e, v in out.items():
            assert np.array_equal(v, full[e]), (er, e)


def test_decode_reads_the_lowest_degree_survivors():
    # Default read set: the k survivors of lowest degree (p_i at degree i,
    # d_j at degree m + j), found here by brute force over the pattern.
    for k, m in [(10, 4), (6, 3), (2, 4), (32, 8)]:
        code = B.Code(k, m)
        rng = workloads.meta_rng(77 + k)
        for _ in range(30):
            er = workloads.random_erasures(rng, k + m, int(rng.integers(1, m + 1)))
            degree = {b: (b - k if b >= k else m + b) for b in range(k + m)}
            surv = sorted((b for b in range(k + m) if b not in er), key=degree.get)
            read, _ = code.decode_plan(er, 0)
            assert read == sorted(surv[:k]), (k, m, er)
            read_all, _ = code.decode_plan(er, B.RS_POLY_FLAG_ALL_SURVIVORS)
            assert read_all == sorted(surv), (k, m, er)


@pytest.mark.parametrize("k,m,w,poly", [(10, 4, 8, 0x11D), (12, 4, 8, 0x11D),
                                        (32, 8, 8, 0x11D), (5, 7, 8, 0x11D),
                                        (4, 3, 4, 0x13), (9, 5, 4, 0x19)])
def test_decode_plan_random_patterns(k, m, w, poly):
    F = oracle.Field(w, poly)
    code = B.Code(k, m, w, poly)
    rng = workloads.meta_rng(k * 1000 + m)
    data = workloads.random_bytes(k + m, (k, 300)) & ((1 << w) - 1)
    full = np.concatenate([data, oracle.encode(F, k, m, data)])
    for _ in range(40):
        t = int(rng.integers(1, m + 1))
        er = workloads.random_erasures(rng, k + m, t)
        for flags in (0, B.RS_POLY_FLAG_ALL_SURVIVORS):
            _, out = apply_plan_on_cpu(F, k, m, full, er, flags, code)
            for e, v in out.items():
                assert np.array_equal(v, full[e]), (er, e, flags)


def test_ctypes_structs_match_the_c_header(tmp_path):
    # The binding's struct layouts against what a C compiler makes of
    # include/rs_poly.h.
    import subprocess
    src = tmp_path / "sizes.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "rs_poly.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(rs_poly_stripe_t), sizeof(rs_poly_launch_t),
         sizeof(rs_serve_config_t), sizeof(rs_serve_request_t),
         sizeof(rs_serve_completion_t), sizeof(rs_serve_stats_t));
  printf("%zu %zu %zu %zu\\n", offsetof(rs_serve_completion_t, out),
         offsetof(rs_serve_completion_t, charge_bytes), offsetof(rs_serve_request_t, user_tag),
         offsetof(rs_serve_config_t, max_block_bytes));
  return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True,
                           check=True).stdout.split("\n")
    want = [int(x) for x in lines[0].split()]
    got = [ctypes.sizeof(t) for t in (B.Stripe, B.Launch, B.ServeConfig, B.ServeRequest,
                                      B.ServeCompletion, B.ServeStats)]
    assert got == want
    offs = [int(x) for x in lines[1].split()]
    assert offs == [B.ServeCompletion.out.offset, B.ServeCompletion.charge_bytes.offset,
                    B.ServeRequest.user_tag.offset, B.ServeConfig.max_block_bytes.offset]
