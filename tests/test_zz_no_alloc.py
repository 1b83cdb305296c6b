"""GPU checks of rs_poly_batch_noalloc, the batch calls with their scratch
memory in a file-scope device array: on two calls in a row (the second with
a smaller input) its encode, decode and update outputs equal those of
rs_poly_batch_encode / _decode / _update byte for byte (and the oracle's),
and calls beyond the array's limits are rejected before any work."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CODES = {}
# narrow and wide codes in one call, so both state widths (both arenas) run
MIX = ((10, 4), (6, 3), (32, 8), (5, 6), (12, 4), (3, 1))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def code(k, m):
    if (k, m) not in CODES:
        CODES[(k, m)] = B.Code(k, m)
    return CODES[(k, m)]


def make(seed, count, lo, hi):
    """Two identical stripe arenas (one per entry point): (count, n, stride)
    per code shape, random data, plus per-stripe sizes, erasures and update
    deltas."""
    rng = workloads.meta_rng(seed)
    shapes = []
    for i in range(count):
        k, m = MIX[i % len(MIX)]
        shapes.append((k, m, int(rng.integers(lo, hi + 1))))
    offs, off = [], 0
    for (k, m, nb) in shapes:
        step = (nb + 255) // 256 * 256 + 256
        offs.append([off + b * step for b in range(k + m)])
        off += (k + m) * step
    data = workloads.device_random_blocks(torch, seed, 1, off)[0]
    bufs = [data.clone(), data.clone()]
    erasures = [workloads.random_erasures(rng, k + m, int(rng.integers(1, m + 1)))
                for (k, m, nb) in shapes]
    return shapes, offs, bufs, erasures


def entries(shapes, offs, buf, erasures=None, delta=None):
    base = buf.data_ptr()
    out = []
    for s, (k, m, nb) in enumerate(shapes):
        ptrs = [base + o for o in offs[s]]
        if delta is not None:
            d = [None] * k
            for j in delta[s]:
                d[j] = ptrs[j]                 # the data block itself is the delta
            out.append((code(k, m), d + ptrs[k:], nb))
        elif erasures is not None:
            out.append((code(k, m), ptrs, nb, erasures[s], 0))
        else:
            out.append((code(k, m), ptrs, nb))
    return out


def block(buf, offs, s, b, nb):
    return buf[offs[s][b]:offs[s][b] + nb]


@pytest.mark.parametrize("op", ["encode", "decode", "update"])
def test_noalloc_equals_the_batch_calls_on_two_calls(op):
    say(f"noalloc {op}")
    bt = B.Batch()
    for call, (count, lo, hi) in enumerate(((30, 1, 300_000), (7, 1, 20_000))):
        shapes, offs, bufs, erasures = make(700 + 10 * call + len(op), count, lo, hi)
        for buf in bufs:                               # a valid starting parity
            B.rs_poly_batch_encode(bt.handle, entries(shapes, offs, buf))
        torch.cuda.synchronize()
        ref = bufs[0].clone()
        if op == "encode":
            for buf in bufs:                           # wipe the parity first
                for s, (k, m, nb) in enumerate(shapes):
                    for b in range(k, k + m):
                        block(buf, offs, s, b, nb).fill_(0xA5)
            B.rs_poly_batch_encode(bt.handle, entries(shapes, offs, bufs[0]))
            B.rs_poly_batch_noalloc(B.RS_POLY_OP_ENCODE, entries(shapes, offs, bufs[1]))
        elif op == "decode":
            for buf in bufs:
                for s, (k, m, nb) in enumerate(shapes):
                    for b in erasures[s]:
                        block(buf, offs, s, b, nb).fill_(0x3C)
            B.rs_poly_batch_decode(bt.handle, entries(shapes, offs, bufs[0], erasures))
            B.rs_poly_batch_noalloc(B.RS_POLY_OP_DECODE, entries(shapes, offs, bufs[1], erasures))
        else:
            rng = workloads.meta_rng(800 + call)
            delta = [sorted(set(int(x) for x in rng.integers(0, k, size=2)))
                     for (k, m, nb) in shapes]
            B.rs_poly_batch_update(bt.handle, entries(shapes, offs, bufs[0], delta=delta))
            B.rs_poly_batch_noalloc(B.RS_POLY_OP_UPDATE,
                                    entries(shapes, offs, bufs[1], delta=delta))
        torch.cuda.synchronize()
        assert torch.equal(bufs[0], bufs[1]), (op, call)
        if op != "update":
            assert torch.equal(bufs[1], ref), (op, call)   # encode/decode restore the stripe
        # and against the oracle on a few stripes
        F = oracle.Field(8, 0x11D)
        host = bufs[1].cpu().numpy()
        for s in (0, len(shapes) // 2, len(shapes) - 1):
            k, m, nb = shapes[s]
            d = np.stack([host[offs[s][j]:offs[s][j] + nb] for j in range(k)])
            p = np.stack([host[offs[s][k + i]:offs[s][k + i] + nb] for i in range(m)])
            if op == "update":
                # parity ^= encode(delta) with delta = the changed data blocks
                old = np.stack([ref.cpu().numpy()[offs[s][k + i]:offs[s][k + i] + nb]
                                for i in range(m)])
                dd = np.zeros_like(d)
                for j in delta[s]:
                    dd[j] = d[j]
                assert np.array_equal(p, old ^ oracle.encode(F, k, m, dd)), (call, s)
            else:
                assert np.array_equal(p, oracle.encode(F, k, m, d)), (call, s)


def test_noalloc_rejects_calls_beyond_its_limits():
    say("noalloc limits")
    # 250 stripes of RS(247,8): about 540 KiB of pointers, over the 512 KiB
    # arena of one width; real (small) buffers, so nothing would be out of
    # bounds even if it ran
    k, m, nb, S = 247, 8, 16, 250
    buf = torch.zeros(S * (k + m) * 256, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    ents = [(code(k, m), [base + (s * (k + m) + b) * 256 for b in range(k + m)], nb)
            for s in range(S)]
    with pytest.raises(B.RsPolyError) as ei:
        B.rs_poly_batch_noalloc(B.RS_POLY_OP_ENCODE, ents)
    assert ei.value.code == B.RS_EINVAL
    torch.cuda.synchronize()
    assert int(buf.count_nonzero()) == 0              # nothing ran
    # 200 stripes fit
    ents = ents[:200]
    B.rs_poly_batch_noalloc(B.RS_POLY_OP_ENCODE, ents)
    torch.cuda.synchronize()
    assert int(buf.count_nonzero()) == 0              # zero data, zero parity
