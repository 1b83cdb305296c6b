"""Blocks larger than 2 GiB: the kernels address columns with 32-bit
offsets, so the library splits such blocks into column ranges (plain and
batched path).  The results are checked against the oracle on column
windows around the split point and at both ends, and the batched, plain,
decode and update paths against each other on the whole blocks."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K, M = 3, 2
NB = (1 << 31) + 4096 + 17          # over 2 GiB, ragged tail
NBP = (NB + 255) // 256 * 256       # row stride: 16-byte aligned rows
WINDOWS = [(0, 1 << 16), ((1 << 31) - (1 << 15), (1 << 31) + (1 << 15)), (NB - (1 << 16), NB)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stripe():
    # k data blocks, m parity blocks and m more for the batched result
    rows = torch.zeros((K + 2 * M, NBP), dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(9))
    for j in range(K):
        rows[j, :NB] = torch.randint(0, 256, (NB,), dtype=torch.uint8, device="cuda",
                                     generator=gen)
    yield rows
    del rows
    torch.cuda.empty_cache()


def check_windows(rows, parity_rows):
    F = oracle.Field(8, 0x11D)
    for lo, hi in WINDOWS:
        d = rows[:K, lo:hi].cpu().numpy()
        p = rows[parity_rows, lo:hi].cpu().numpy()
        assert np.array_equal(p, oracle.encode(F, K, M, d)), (lo, hi)


def test_encode_over_2GiB_plain_and_batched(stripe):
    say(f"encode RS({K},{M}) blocks of {NB} bytes")
    code = B.Code(K, M)
    ptr = [stripe[b].data_ptr() for b in range(K + 2 * M)]
    code.encode(ptr[:K], ptr[K:K + M], NB)
    torch.cuda.synchronize()
    check_windows(stripe, list(range(K, K + M)))
    bt = B.Batch()
    bt.encode([(code, ptr[:K] + ptr[K + M:], NB)])
    torch.cuda.synchronize()
    assert torch.equal(stripe[K:K + M, :NB], stripe[K + M:, :NB])


def test_decode_and_update_over_2GiB(stripe):
    say("decode and update over 2 GiB")
    code = B.Code(K, M)
    ptr = [stripe[b].data_ptr() for b in range(K + M)]
    lost = [1, K]                      # a data block and a parity block
    saved = stripe[lost, :NB].clone()
    stripe[lost, :NB] = 0x5A
    code.decode(ptr, lost, NB)
    torch.cuda.synchronize()
    assert torch.equal(stripe[lost, :NB], saved)
    del saved
    # update block 2 by a delta, batched; then check windows of the new data
    delta = torch.randint(0, 256, (NB,), dtype=torch.uint8, device="cuda")
    bt = B.Batch()
    bt.update([(code, [None, None, delta.data_ptr()] + ptr[K:], NB)])
    stripe[2, :NB] ^= delta
    torch.cuda.synchronize()
    check_windows(stripe, list(range(K, K + M)))


def test_bitmatrix_encode_over_2GiB():
    # The bit-sliced encode splits blocks over 2 GiB the same way, plain and
    # batched; both equal the LFSR encode, and windows match the oracle.
    k, m = 6, 3
    say(f"bit-matrix encode RS({k},{m}) blocks of {NB} bytes")
    rows = torch.zeros((k + 3 * m, NBP), dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(10))
    for j in range(k):
        rows[j, :NB] = torch.randint(0, 256, (NB,), dtype=torch.uint8, device="cuda",
                                     generator=gen)
    code = B.Code(k, m)
    ptr = [rows[b].data_ptr() for b in range(k + 3 * m)]
    code.encode(ptr[:k], ptr[k:k + m], NB)
    code.encode_bitmatrix(ptr[:k], ptr[k + m:k + 2 * m], NB)
    bt = B.Batch()
    bt.set_launch(B.RS_POLY_OP_ENCODE, 0,
                  {"bytes_per_lane": 16, "threads": 512, "tile_bytes": 16384, "wgs_per_cu": 2,
                   "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": 0})
    bt.encode([(code, ptr[:k] + ptr[k + 2 * m:], NB)])
    torch.cuda.synchronize()
    assert torch.equal(rows[k:k + m, :NB], rows[k + m:k + 2 * m, :NB])
    assert torch.equal(rows[k:k + m, :NB], rows[k + 2 * m:, :NB])
    F = oracle.Field(8, 0x11D)
    for lo, hi in WINDOWS:
        d = rows[:k, lo:hi].cpu().numpy()
        assert np.array_equal(rows[k + m:k + 2 * m, lo:hi].cpu().numpy(), oracle.encode(F, k, m, d))
    del rows
    torch.cuda.empty_cache()


def test_nibble_update_over_2GiB():
    # The split-nibble update walks blocks of any size in one launch (64-bit
    # chunk indices): 2 changed blocks of RS(3,2) with blocks over 2 GiB.  The
    # result equals the LDS update of the same delta from the same parity,
    # and on windows the parity change equals the oracle's encoding of the
    # delta.
    k, m = 3, 2
    say(f"nibble update RS({k},{m}) blocks of {NB} bytes")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(11))
    delta = torch.zeros((k, NBP), dtype=torch.uint8, device="cuda")
    for j in (0, 2):
        delta[j, :NB] = torch.randint(0, 256, (NB,), dtype=torch.uint8, device="cuda",
                                      generator=gen)
    par = torch.randint(0, 256, (2 * m, NBP), dtype=torch.uint8, device="cuda", generator=gen)
    par[m:] = par[:m]
    before = {w: par[:m, w[0]:w[1]].cpu().numpy() for w in WINDOWS}
    code = B.Code(k, m)
    dptr = [delta[0].data_ptr(), None, delta[2].data_ptr()]
    code.update_nibble(dptr, [par[i].data_ptr() for i in range(m)], NB)
    code.update(dptr, [par[m + i].data_ptr() for i in range(m)], NB)
    torch.cuda.synchronize()
    assert torch.equal(par[:m, :NB], par[m:, :NB])
    assert torch.equal(par[:m, NB:], par[m:, NB:])     # bytes past the blocks untouched
    F = oracle.Field(8, 0x11D)
    for w in WINDOWS:
        d = delta[:, w[0]:w[1]].cpu().numpy()
        want = before[w] ^ oracle.encode(F, k, m, d)
        assert np.array_equal(par[:m, w[0]:w[1]].cpu().numpy(), want), w
    del delta, par
    torch.cuda.empty_cache()
