"""GPU parity of the plain (one stripe per launch) encode and decode kernels
against the CPU oracle, byte for byte, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F8 = None


def field(w=8, poly=0x11D):
    return oracle.Field(w, poly)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


def rows(t):
    return [t[i] for i in range(t.shape[0])]


def gpu_encode(code, data_np, pad=0, offset=0):
    """Encodes on the GPU; blocks are rows of a (count, B+pad) buffer starting
    `offset` bytes in (to vary the alignment).  Returns parity as numpy and
    the raw parity buffer (to check the guard bytes)."""
    k, Bn = data_np.shape
    m = code.m
    stride = Bn + pad
    dbuf = torch.zeros(k * stride + offset + 64, dtype=torch.uint8, device="cuda")
    pbuf = torch.full((m * stride + offset + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    for j in range(k):
        dbuf[offset + j * stride: offset + j * stride + Bn] = to_dev(data_np[j])
    dptr = [dbuf.data_ptr() + offset + j * stride for j in range(k)]
    pptr = [pbuf.data_ptr() + offset + i * stride for i in range(m)]
    B.rs_poly_encode(code.handle, dptr, pptr, Bn)
    torch.cuda.synchronize()
    host = pbuf.cpu().numpy()
    par = np.stack([host[offset + i * stride: offset + i * stride + Bn] for i in range(m)])
    return par, host, stride


def test_encode_worked_example(golden_example):
    code = B.Code(4, 3)
    data = np.array(golden_example["data"], dtype=np.uint8)[:, None]
    par, _, _ = gpu_encode(code, data)
    assert par[:, 0].tolist() == golden_example["parity"]


def test_encode_rs63_64KiB_matches_oracle():
    say("encode RS(6,3) 6 x 64 KiB")
    code = B.Code(6, 3)
    data = workloads.stripe_data(workloads.data_seed(0), 0, 6, 64 << 10)
    par, _, _ = gpu_encode(code, data)
    assert np.array_equal(par, oracle.encode(field(), 6, 3, data))


SHAPES = [(1, 1, 1), (1, 8, 17), (4, 3, 15), (6, 3, 16), (10, 4, 17), (10, 4, 4095),
          (12, 4, 4097), (5, 5, 1000), (32, 8, 70001), (7, 2, 65536 + 3), (3, 7, 333),
          (17, 6, 8192), (200, 4, 129), (247, 8, 64), (13, 1, 999)]


@pytest.mark.parametrize("k,m,Bn", SHAPES)
def test_encode_shapes_match_oracle(k, m, Bn):
    say(f"encode k={k} m={m} B={Bn}")
    code = B.Code(k, m)
    data = workloads.random_bytes(k * 7919 + m * 31 + Bn, (k, Bn))
    par, host, stride = gpu_encode(code, data, pad=5)
    assert np.array_equal(par, oracle.encode(field(), k, m, data))
    # bytes between blocks and after the last one are untouched
    for i in range(m):
        gap = host[i * stride + Bn: (i + 1) * stride]
        assert (gap == 0xA5).all()


@pytest.mark.parametrize("offset", [1, 2, 4, 8, 12])
def test_encode_misaligned_blocks(offset):
    say(f"encode misaligned offset={offset}")
    code = B.Code(10, 4)
    data = workloads.random_bytes(offset, (10, 5000))
    par, _, _ = gpu_encode(code, data, pad=16 + offset, offset=offset)
    assert np.array_equal(par, oracle.encode(field(), 10, 4, data))


def gpu_decode(code, full_np, erasures, flags=0, poison_unread=True, seed=0):
    """Decodes on the GPU with erased blocks poisoned (and, when asked, every
    block the plan does not read poisoned too); returns the rebuilt stripe."""
    n, Bn = full_np.shape
    rng = np.random.default_rng(seed)
    read, _ = code.decode_plan(erasures, flags)
    host = full_np.copy()
    for b in range(n):
        if b in erasures or (poison_unread and b not in read):
            host[b] = rng.integers(0, 256, Bn, dtype=np.uint8)
    dev = to_dev(host)
    B.rs_poly_decode(code.handle, rows(dev), Bn, list(erasures), flags)
    torch.cuda.synchronize()
    out = dev.cpu().numpy()
    return out, read


def test_decode_every_pattern_rs63_64KiB():
    # The small all-pattern workload: encode, then decode every one of the
    # C(9, <=3) erasure patterns, both survivor-selection modes.
    say("decode RS(6,3) all 130 patterns")
    k, m, Bn = 6, 3, 64 << 10
    code = B.Code(k, m)
    data = workloads.stripe_data(workloads.data_seed(0), 0, k, Bn)
    par, _, _ = gpu_encode(code, data)
    assert np.array_equal(par, oracle.encode(field(), k, m, data))
    full = np.concatenate([data, par])
    pats = workloads.all_patterns(k + m, m)
    assert len(pats) == 130
    for i, er in enumerate(pats):
        for flags in (0, B.RS_POLY_FLAG_ALL_SURVIVORS):
            out, read = gpu_decode(code, full, er, flags, seed=i)
            for b in er:
                assert np.array_equal(out[b], full[b]), (er, b, flags)
            for b in read:
                assert np.array_equal(out[b], full[b])


@pytest.mark.parametrize("k,m,Bn", [(10, 4, 4099), (12, 4, 1 << 16), (32, 8, 20011),
                                    (5, 6, 77), (1, 1, 3), (2, 8, 4096), (100, 5, 513)])
def test_decode_random_patterns_match_oracle(k, m, Bn):
    say(f"decode k={k} m={m} B={Bn}")
    code = B.Code(k, m)
    F = field()
    data = workloads.random_bytes(k * 13 + m + Bn, (k, Bn))
    full = np.concatenate([data, oracle.encode(F, k, m, data)])
    rng = workloads.meta_rng(k + m + Bn)
    for it in range(6):
        t = int(rng.integers(1, m + 1))
        er = workloads.random_erasures(rng, k + m, t)
        flags = it & 1
        out, _ = gpu_decode(code, full, er, flags, seed=it)
        # the oracle rebuilds from the same received word
        ref = full.copy()
        ref[er] = 0
        oracle.decode(F, k, m, ref, er)
        for b in er:
            assert np.array_equal(out[b], ref[b]), (er, b)


def test_gf16_bruteforce_on_gpu():
    # Every data vector of RS(4,3) over GF(2^4) as a column; every pattern.
    say("GF(16) RS(4,3) brute force")
    import itertools
    k, m = 4, 3
    F = field(4, 0x13)
    code = B.Code(k, m, 4, 0x13)
    data = np.ascontiguousarray(
        np.array(list(itertools.product(range(16), repeat=k)), dtype=np.uint8).T)
    par, _, _ = gpu_encode(code, data)
    assert np.array_equal(par, oracle.encode(F, k, m, data))
    full = np.concatenate([data, par])
    for i, er in enumerate(workloads.all_patterns(k + m, m)[1:]):
        for flags in (0, B.RS_POLY_FLAG_ALL_SURVIVORS):
            out, read = gpu_decode(code, full, er, flags, seed=i)
            # erased rows rebuilt; read rows untouched (unread ones hold poison)
            assert np.array_equal(out[er + read], full[er + read]), (er, flags)


def test_decode_all_parity_equals_encode():
    # Sec. 3.3 symmetry, on the GPU: erasing every parity block and decoding
    # gives the encoder's output.
    k, m, Bn = 10, 4, 1 << 15
    code = B.Code(k, m)
    data = workloads.random_bytes(99, (k, Bn))
    full = np.concatenate([data, np.zeros((m, Bn), dtype=np.uint8)])
    out, _ = gpu_decode(code, full, list(range(k, k + m)))
    assert np.array_equal(out[k:], oracle.encode(field(), k, m, data))


def test_repeat_runs_are_identical():
    code = B.Code(12, 4)
    data = workloads.random_bytes(5, (12, 1 << 18))
    a, _, _ = gpu_encode(code, data)
    b, _, _ = gpu_encode(code, data)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("k,m,Bn", [(32, 8, (16 << 20) + 48), (20, 6, (8 << 20) + 4),
                                    (10, 4, (8 << 20) + 12)])
def test_plain_large_aligned_blocks(k, m, Bn):
    # Blocks on a 256-byte-padded stride (16-byte aligned) and large enough
    # for the widest plain variant (16 bytes per lane; 1024 threads for the
    # wide codes), with a ragged length: the encode matches the oracle on
    # column windows at both ends and in the middle, and the decode of m
    # erased blocks (data and parity) restores them exactly.
    say(f"plain large RS({k},{m}) B={Bn}")
    code = B.Code(k, m)
    stride = (Bn + 255) // 256 * 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(6) + k)
    buf = torch.zeros((k + m, stride), dtype=torch.uint8, device="cuda")
    buf[:k] = torch.randint(0, 256, (k, stride), dtype=torch.uint8, device="cuda", generator=gen)
    assert buf[1].data_ptr() % 16 == 0
    code.encode(rows(buf[:k]), rows(buf[k:]), Bn)
    torch.cuda.synchronize()
    F = field()
    for c0 in (0, Bn // 2 - 333, Bn - 40000):
        w = (c0, c0 + 40000)
        want = oracle.encode(F, k, m, buf[:k, w[0]:w[1]].cpu().numpy())
        assert np.array_equal(buf[k:, w[0]:w[1]].cpu().numpy(), want), (k, m, c0)
    assert not buf[k:, Bn:].any()                     # nothing past the blocks
    rng = workloads.meta_rng(k * 7 + m)
    er = workloads.random_erasures(rng, k + m, m)
    saved = buf[er].clone()
    buf[er] = 0x6B
    code.decode(rows(buf), er, Bn)
    torch.cuda.synchronize()
    assert torch.equal(buf[er, :Bn], saved[:, :Bn]), er
