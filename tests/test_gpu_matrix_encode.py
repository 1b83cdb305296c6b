"""GPU parity of the generator-matrix encode (Sec. 6: p = sum_j P[:, j] d_j,
one packed lookup per data block; codes with k <= 8 in one LDS row set, up
to k = 32 in the wide form) against the oracle, byte for byte, through the C
ABI: ragged sizes, misaligned blocks with guard bytes, m > 4 and GF(2^4)
codes, and agreement with the LFSR encode on large aligned blocks (the 16-
and 8-byte-per-lane kernels with several rounds per lane)."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CODES = [(1, 1, 8, 0x11D), (3, 2, 8, 0x11D), (6, 3, 8, 0x11D), (8, 4, 8, 0x11D),
         (5, 6, 8, 0x11D), (8, 8, 8, 0x11D), (4, 3, 4, 0x13),
         # wide form
         (9, 3, 8, 0x11D), (10, 4, 8, 0x11D), (12, 4, 8, 0x11D), (17, 6, 8, 0x11D),
         (32, 8, 8, 0x11D), (32, 2, 8, 0x11D), (25, 5, 8, 0x11D), (10, 3, 4, 0x13)]
SIZES = [1, 15, 16, 17, 1000, 4097, 65539]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def matrix_encode(code, data_np, offset=0):
    k, Bn = data_np.shape
    m = code.m
    stride = Bn + 64
    dbuf = torch.zeros(k * stride + offset + 64, dtype=torch.uint8, device="cuda")
    pbuf = torch.full((m * stride + offset + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    for j in range(k):
        dbuf[offset + j * stride: offset + j * stride + Bn] = torch.from_numpy(
            np.ascontiguousarray(data_np[j])).cuda()
    dptr = [dbuf.data_ptr() + offset + j * stride for j in range(k)]
    pptr = [pbuf.data_ptr() + offset + i * stride for i in range(m)]
    code.encode_matrix(dptr, pptr, Bn)
    torch.cuda.synchronize()
    host = pbuf.cpu().numpy()
    par = np.stack([host[offset + i * stride: offset + i * stride + Bn] for i in range(m)])
    guards = all((host[offset + i * stride + Bn: offset + (i + 1) * stride] == 0xA5).all()
                 for i in range(m))
    return par, guards


@pytest.mark.parametrize("k,m,w,poly", CODES)
def test_matrix_encode_matches_oracle(k, m, w, poly):
    code = B.Code(k, m, w, poly)
    F = oracle.Field(w, poly)
    for i, Bn in enumerate(SIZES):
        say(f"matrix encode RS({k},{m}) w={w} B={Bn}")
        data = workloads.random_bytes(300 + 17 * k + m + i, (k, Bn)) & ((1 << w) - 1)
        for offset in (0, 5):
            par, guards = matrix_encode(code, data, offset)
            assert np.array_equal(par, oracle.encode(F, k, m, data)), (k, m, Bn, offset)
            assert guards, (k, m, Bn, offset)


@pytest.mark.parametrize("k,m,Bn", [(8, 4, (32 << 20) + 7), (6, 3, (8 << 20) + 48),
                                    (10, 4, (16 << 20) + 7), (32, 8, (16 << 20) + 32)])
def test_matrix_encode_equals_lfsr_encode_large(k, m, Bn):
    # Blocks on a 256-byte-padded stride, so every block is 16-byte aligned
    # and the wide-load kernels run (several rounds per lane), with a ragged
    # length; the parity equals the LFSR encode's and matches the oracle on
    # column windows at both ends and in the middle.
    say(f"matrix vs LFSR encode RS({k},{m}) B={Bn}")
    code = B.Code(k, m)
    stride = (Bn + 255) // 256 * 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(5) + k)
    data = torch.randint(0, 256, (k, stride), dtype=torch.uint8, device="cuda", generator=gen)
    p1 = torch.zeros((m, stride), dtype=torch.uint8, device="cuda")
    p2 = torch.full((m, stride), 0x3C, dtype=torch.uint8, device="cuda")
    assert data[1].data_ptr() % 16 == 0 and p2[1].data_ptr() % 16 == 0
    code.encode([data[j] for j in range(k)], [p1[i] for i in range(m)], Bn)
    code.encode_matrix([data[j] for j in range(k)], [p2[i] for i in range(m)], Bn)
    torch.cuda.synchronize()
    assert torch.equal(p1[:, :Bn], p2[:, :Bn])
    assert (p2[:, Bn:] == 0x3C).all()                 # nothing past the blocks
    F = oracle.Field(8, 0x11D)
    for c0 in (0, Bn // 2 - 777, Bn - 70001):
        w = (c0, c0 + 70001)
        want = oracle.encode(F, k, m, data[:, w[0]:w[1]].cpu().numpy())
        assert np.array_equal(p2[:, w[0]:w[1]].cpu().numpy(), want), (k, m, c0)
