"""GPU parity of the bit-sliced (XOR-only) encode against the oracle, byte
for byte, through the C ABI: every code whose XOR network is compiled in
and codes that take their matrices at run time (other k and m, another
GF(2^8) polynomial, GF(2^4)), sizes that span several 2048-column wave
chunks with ragged tails (bytes past the blocks left untouched), and
agreement with the LFSR encode at full workload sizes."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BUILT_IN = [(6, 3), (10, 4), (12, 4), (32, 8)]
# (k, m, w, poly): codes whose matrices the kernel takes at run time
RUNTIME = [(9, 4, 8, 0x11D), (1, 1, 8, 0x11D), (5, 8, 8, 0x11D), (20, 6, 8, 0x11D),
           (32, 7, 8, 0x11D), (3, 2, 8, 0x11D), (10, 4, 8, 0x12B), (16, 5, 8, 0x187),
           (4, 3, 4, 0x13), (9, 5, 4, 0x13), (13, 2, 4, 0x19)]
SIZES = [1, 15, 16, 17, 1000, 2047, 2048, 2049, 4096 + 100, 3 * 65536 + 5]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bitmatrix_encode(code, data_np):
    """Encodes rows of data_np with the bit-matrix kernel; rows sit at a
    256-byte stride with guard bytes after each block.  Returns parity and
    whether every guard byte kept its fill value."""
    k, Bn = data_np.shape
    m = code.m
    stride = (Bn + 255) // 256 * 256 + 256
    dbuf = torch.zeros(k * stride, dtype=torch.uint8, device="cuda")
    pbuf = torch.full((m * stride,), 0xA5, dtype=torch.uint8, device="cuda")
    for j in range(k):
        dbuf[j * stride: j * stride + Bn] = torch.from_numpy(np.ascontiguousarray(data_np[j])).cuda()
    dptr = [dbuf.data_ptr() + j * stride for j in range(k)]
    pptr = [pbuf.data_ptr() + i * stride for i in range(m)]
    code.encode_bitmatrix(dptr, pptr, Bn)
    torch.cuda.synchronize()
    host = pbuf.cpu().numpy().reshape(m, stride)
    return host[:, :Bn], bool((host[:, Bn:] == 0xA5).all())


def test_supported_codes():
    for k, m in BUILT_IN:
        assert B.rs_poly_bitmatrix_supported(k, m)
    for k, m, w, poly in RUNTIME:
        assert B.rs_poly_bitmatrix_supported(k, m, w, poly)
    assert not B.rs_poly_bitmatrix_supported(33, 4)


@pytest.mark.parametrize("k,m,w,poly", RUNTIME)
def test_runtime_bitmatrix_encode_matches_oracle(k, m, w, poly):
    code = B.Code(k, m, w, poly)
    F = oracle.Field(w, poly)
    for i, Bn in enumerate(SIZES):
        say(f"bit-matrix (run-time rows) RS({k},{m}) GF(2^{w}) poly {poly:#x} B={Bn}")
        data = workloads.random_bytes(3000 * k + 7 * m + i, (k, Bn)) & ((1 << w) - 1)
        par, guards = bitmatrix_encode(code, data)
        assert np.array_equal(par, oracle.encode(F, k, m, data)), (k, m, w, Bn)
        assert guards, (k, m, w, Bn)


@pytest.mark.parametrize("k,m", BUILT_IN)
def test_bitmatrix_encode_matches_oracle(k, m):
    code = B.Code(k, m)
    F = oracle.Field(8, 0x11D)
    for i, Bn in enumerate(SIZES):
        say(f"bit-matrix RS({k},{m}) B={Bn}")
        data = workloads.random_bytes(1000 * k + i, (k, Bn))
        par, guards = bitmatrix_encode(code, data)
        assert np.array_equal(par, oracle.encode(F, k, m, data)), (k, m, Bn)
        assert guards, (k, m, Bn)


def test_bitmatrix_unit_data_gives_generator_columns():
    # Unit data in one block gives that block's generator-matrix column
    # x^(m+j) mod g(x); all-zero data gives zero parity.
    k, m = 10, 4
    code = B.Code(k, m)
    F = oracle.Field(8, 0x11D)
    Bn = 4096
    data = np.zeros((k, Bn), dtype=np.uint8)
    for j in range(k):
        data[j, 64 * j + 3] = 1
    par, _ = bitmatrix_encode(code, data)
    assert np.array_equal(par, oracle.encode(F, k, m, data))
    assert not par[:, np.setdiff1d(np.arange(Bn), 64 * np.arange(k) + 3)].any()


@pytest.mark.parametrize("k,m,Bn", [(10, 4, 64 << 20), (32, 8, (16 << 20) + 48),
                                    (16, 4, (32 << 20) + 48)])
def test_bitmatrix_full_size_agrees_with_lfsr_encode(k, m, Bn):
    say(f"bit-matrix vs LFSR RS({k},{m}) B={Bn}")
    code = B.Code(k, m)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(k))
    data = torch.randint(0, 256, (k, Bn), dtype=torch.uint8, device="cuda", generator=gen)
    p1 = torch.zeros((m, Bn), dtype=torch.uint8, device="cuda")
    p2 = torch.full((m, Bn), 0x5A, dtype=torch.uint8, device="cuda")
    code.encode([data[j] for j in range(k)], [p1[i] for i in range(m)], Bn)
    code.encode_bitmatrix([data[j] for j in range(k)], [p2[i] for i in range(m)], Bn)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2)
    F = oracle.Field(8, 0x11D)
    for lo in (0, Bn // 2 - 1000, Bn - 3000):
        d = data[:, lo:lo + 3000].cpu().numpy()
        assert np.array_equal(p2[:, lo:lo + 3000].cpu().numpy(), oracle.encode(F, k, m, d))


def batch_encode(stripes_np, codes, launch):
    """Batched encode of the given stripes (one (k, B) array each) with the
    launch shape `launch`; returns each stripe's parity."""
    bufs, ents = [], []
    for data, code in zip(stripes_np, codes):
        k, Bn = data.shape
        stride = (Bn + 255) // 256 * 256
        t = torch.zeros((k + code.m) * stride, dtype=torch.uint8, device="cuda")
        for j in range(k):
            t[j * stride: j * stride + Bn] = torch.from_numpy(np.ascontiguousarray(data[j])).cuda()
        t[k * stride:] = 0xA5
        bufs.append((t, stride))
        ents.append((code, [t.data_ptr() + b * stride for b in range(k + code.m)], Bn))
    bt = B.Batch()
    bt.set_launch(B.RS_POLY_OP_ENCODE, 1 if codes[0].m > 4 else 0, launch)
    bt.encode(B.StripeArray(ents))
    torch.cuda.synchronize()
    out = []
    for (t, stride), data, code in zip(bufs, stripes_np, codes):
        k, Bn = data.shape
        host = t.cpu().numpy()
        out.append(np.stack([host[(k + i) * stride:(k + i) * stride + Bn] for i in range(code.m)]))
    return out


@pytest.mark.parametrize("k,m", [(10, 4), (32, 8), (6, 3)])
@pytest.mark.parametrize("threads,tile,order", [(256, 8192, 0), (1024, 65536, 1), (512, 16384, 0)])
def test_batched_bitmatrix_matches_oracle(k, m, threads, tile, order):
    say(f"batched bit-matrix RS({k},{m}) threads={threads} tile={tile} order={order}")
    F = oracle.Field(8, 0x11D)
    sizes = [1, 4095, 2048, 70001, 1 << 16, 3 * 2048 + 17, 200000]
    data = [workloads.random_bytes(77 * k + i, (k, n)) for i, n in enumerate(sizes)]
    codes = [B.Code(k, m)] * len(sizes)
    # (bytes_per_lane only shapes the table fallback; it must still be valid)
    bpl = 4 if threads == 1024 else 16 if m <= 4 else 8
    launch = {"bytes_per_lane": bpl, "threads": threads, "tile_bytes": tile,
              "wgs_per_cu": 2, "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": order}
    for par, d in zip(batch_encode(data, codes, launch), data):
        assert np.array_equal(par, oracle.encode(F, k, m, d))


@pytest.mark.parametrize("k,m,w,poly", [(9, 4, 8, 0x11D), (20, 6, 8, 0x11D), (7, 3, 4, 0x13)])
def test_batched_runtime_bitmatrix_matches_oracle(k, m, w, poly):
    say(f"batched bit-matrix (run-time rows) RS({k},{m}) GF(2^{w})")
    F = oracle.Field(w, poly)
    sizes = [1, 4095, 2048, 70001, 3 * 2048 + 17, 200000]
    data = [workloads.random_bytes(91 * k + i, (k, n)) & ((1 << w) - 1)
            for i, n in enumerate(sizes)]
    codes = [B.Code(k, m, w, poly)] * len(sizes)
    launch = {"bytes_per_lane": 16 if m <= 4 else 8, "threads": 512, "tile_bytes": 16384,
              "wgs_per_cu": 2, "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": 1}
    for par, d in zip(batch_encode(data, codes, launch), data):
        assert np.array_equal(par, oracle.encode(F, k, m, d))


def test_batched_bitmatrix_mixed_codes_fall_back_to_tables():
    # Two codes in one width: the call runs the packed tables; same bytes.
    F = oracle.Field(8, 0x11D)
    specs = [(10, 4, 5000), (12, 4, 7000), (10, 4, 4096), (9, 4, 3000)]
    data = [workloads.random_bytes(5 + i, (k, n)) for i, (k, _, n) in enumerate(specs)]
    codes = [B.Code(k, m) for k, m, _ in specs]
    launch = {"bytes_per_lane": 16, "threads": 512, "tile_bytes": 16384, "wgs_per_cu": 2,
              "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": 0}
    for par, d, (k, m, _) in zip(batch_encode(data, codes, launch), data, specs):
        assert np.array_equal(par, oracle.encode(F, k, m, d))


def test_batched_bitmatrix_full_bench_workload():
    # The bench's batched comparison run: 256 RS(10,4) stripes of 1 MiB blocks
    # in the bench's bit-sliced launch shape; every parity byte equals the
    # LFSR batch's, and sampled stripes match the oracle.
    say("batched bit-matrix RS(10,4) 256 x 1 MiB")
    k, m, S, nb = 10, 4, 256, 1 << 20
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(1))
    buf = torch.zeros((S, k + 2 * m, nb), dtype=torch.uint8, device="cuda")
    buf[:, :k] = torch.randint(0, 256, (S, k, nb), dtype=torch.uint8, device="cuda",
                               generator=gen)
    code = B.Code(k, m)
    lfsr = B.StripeArray([(code, [buf[s, b].data_ptr() for b in range(k + m)], nb)
                          for s in range(S)])
    bits = B.StripeArray([(code, [buf[s, b].data_ptr() for b in range(k)] +
                           [buf[s, k + m + i].data_ptr() for i in range(m)], nb)
                          for s in range(S)])
    bt = B.Batch()
    bt.encode(lfsr)
    bt.set_launch(B.RS_POLY_OP_ENCODE, 0,
                  {"bytes_per_lane": 16, "threads": 256, "tile_bytes": 8192, "wgs_per_cu": 2,
                   "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": 0})
    bt.encode(bits)
    torch.cuda.synchronize()
    assert torch.equal(buf[:, k:k + m], buf[:, k + m:])
    F = oracle.Field(8, 0x11D)
    for s in (0, 97, 255):
        d = buf[s, :k, :65536].cpu().numpy()
        assert np.array_equal(buf[s, k + m:, :65536].cpu().numpy(), oracle.encode(F, k, m, d))
    del buf
    torch.cuda.empty_cache()
