"""A seeded random sweep over every entry point: random codes (both fields,
k up to 40, m up to 8), block sizes with ragged tails and pointer offsets,
erasure patterns and changed-block sets.  Each case runs the plain encode,
decode (both survivor modes), update, generator-matrix encode, bit-sliced
encode and split-nibble update where they apply, and all cases together run
through one batched encode, decode and update; every result is compared
byte for byte with the oracle (or, for decode, the original blocks)."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_CASES = 40
FIELDS = {8: 0x11D, 4: 0x13}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Case:
    """One random stripe: data, the oracle's parity, and device rows on a
    stride that keeps every block at `offset` bytes past a 256-byte
    boundary, with guard bytes after each block."""

    def __init__(self, rng, idx):
        self.w = 4 if rng.random() < 0.15 else 8
        self.poly = FIELDS[self.w]
        n_max = (1 << self.w) - 1
        self.m = int(rng.integers(1, 9))
        self.k = int(rng.integers(1, min(40, n_max - self.m) + 1))
        self.n = self.k + self.m
        self.nb = int(rng.choice([int(rng.integers(1, 64)), int(rng.integers(64, 5000)),
                                  int(rng.integers(5000, 70000))]))
        self.offset = int(rng.choice([0, 0, 16, 1, 3, 4, 8]))
        self.F = oracle.Field(self.w, self.poly)
        self.code = B.Code(self.k, self.m, self.w, self.poly)
        mask = (1 << self.w) - 1
        self.data = workloads.random_bytes(7000 + idx, (self.k, self.nb)) & mask
        self.parity = oracle.encode(self.F, self.k, self.m, self.data)
        self.full = np.concatenate([self.data, self.parity])
        self.stride = (self.nb + self.offset + 255) // 256 * 256 + 256
        t = int(rng.integers(1, self.m + 1))
        self.erasures = workloads.random_erasures(rng, self.n, t)
        self.flags = int(rng.integers(0, 2))
        c = int(rng.integers(0, self.k + 1))
        self.changed = sorted(rng.choice(self.k, size=c, replace=False).tolist())
        fresh = workloads.random_bytes(8000 + idx, (self.k, self.nb)) & mask
        self.delta = np.zeros_like(self.data)
        for j in self.changed:
            self.delta[j] = self.data[j] ^ fresh[j]
        self.new_parity = oracle.encode(self.F, self.k, self.m, self.data ^ self.delta)

    def aligned(self):
        return self.offset % 16 == 0

    def buffer(self, rows, fill=0xA5):
        buf = torch.full((rows * self.stride,), fill, dtype=torch.uint8, device="cuda")
        return buf

    def ptrs(self, buf, rows):
        base = buf.data_ptr() + self.offset
        return [base + r * self.stride for r in range(rows)]

    def put(self, buf, r, arr):
        o = self.offset + r * self.stride
        buf[o:o + self.nb] = torch.from_numpy(np.ascontiguousarray(arr)).cuda()

    def get(self, host, r):
        o = self.offset + r * self.stride
        return host[o:o + self.nb]

    def guards_ok(self, host, rows, fill=0xA5):
        for r in range(rows):
            o = self.offset + r * self.stride
            if not (host[o + self.nb:o + self.stride - self.offset] == fill).all():
                return False
        return True


def make_cases():
    rng = workloads.meta_rng(4242)
    return [Case(rng, i) for i in range(N_CASES)]


@pytest.fixture(scope="module")
def cases():
    return make_cases()


def run_encode(case, fn):
    dbuf = case.buffer(case.k)
    for j in range(case.k):
        case.put(dbuf, j, case.data[j])
    pbuf = case.buffer(case.m)
    fn(case.code.handle, case.ptrs(dbuf, case.k), case.ptrs(pbuf, case.m), case.nb)
    torch.cuda.synchronize()
    host = pbuf.cpu().numpy()
    got = np.stack([case.get(host, i) for i in range(case.m)])
    return got, case.guards_ok(host, case.m)


def test_plain_encoders(cases):
    for i, c in enumerate(cases):
        say(f"case {i}: RS({c.k},{c.m}) GF(2^{c.w}) B={c.nb} offset={c.offset}")
        got, ok = run_encode(c, B.rs_poly_encode)
        assert np.array_equal(got, c.parity) and ok, i
        if c.k <= B.RS_POLY_MATRIX_MAX_K:
            got, ok = run_encode(c, B.rs_poly_encode_matrix)
            assert np.array_equal(got, c.parity) and ok, i
        if c.aligned() and B.rs_poly_bitmatrix_supported(c.k, c.m, c.w, c.poly):
            got, ok = run_encode(c, B.rs_poly_encode_bitmatrix)
            assert np.array_equal(got, c.parity) and ok, i


def test_plain_decode(cases):
    for i, c in enumerate(cases):
        say(f"case {i}: decode {c.erasures} flags={c.flags}")
        buf = c.buffer(c.n)
        for b in range(c.n):
            c.put(buf, b, c.full[b])
        for b in c.erasures:
            c.put(buf, b, np.full(c.nb, 0x3C, dtype=np.uint8))
        B.rs_poly_decode(c.code.handle, c.ptrs(buf, c.n), c.nb, c.erasures, c.flags)
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        for b in c.erasures:
            assert np.array_equal(c.get(host, b), c.full[b]), (i, b)
        assert c.guards_ok(host, c.n), i


def run_update(c, fn):
    dbuf = c.buffer(c.k, fill=0)
    for j in c.changed:
        c.put(dbuf, j, c.delta[j])
    pbuf = c.buffer(c.m)
    for i2 in range(c.m):
        c.put(pbuf, i2, c.parity[i2])
    dp = c.ptrs(dbuf, c.k)
    fn(c.code.handle, [dp[j] if j in c.changed else None for j in range(c.k)],
       c.ptrs(pbuf, c.m), c.nb)
    torch.cuda.synchronize()
    host = pbuf.cpu().numpy()
    return np.stack([c.get(host, i2) for i2 in range(c.m)]), c.guards_ok(host, c.m)


def test_plain_updates(cases):
    for i, c in enumerate(cases):
        say(f"case {i}: update changed={c.changed}")
        got, ok = run_update(c, B.rs_poly_update)
        assert np.array_equal(got, c.new_parity) and ok, i
        n = len(c.changed)
        if c.aligned() and 1 <= n <= 2 and n * c.m <= 8:
            got, ok = run_update(c, B.rs_poly_update_nibble)
            assert np.array_equal(got, c.new_parity) and ok, i


def test_batched_all_cases(cases):
    # The batch path needs 16-byte-aligned blocks: the aligned cases, plus
    # the others moved to offset 0, in one call per op.
    for c in cases:
        if not c.aligned():
            c.offset = 0
    say(f"batched: {len(cases)} stripes")
    bufs = []
    for c in cases:
        buf = c.buffer(c.n)
        for j in range(c.k):
            c.put(buf, j, c.data[j])
        bufs.append(buf)
    bt = B.Batch()
    bt.encode([(c.code, c.ptrs(buf, c.n), c.nb) for c, buf in zip(cases, bufs)])
    torch.cuda.synchronize()
    for i, (c, buf) in enumerate(zip(cases, bufs)):
        host = buf.cpu().numpy()
        got = np.stack([c.get(host, c.k + r) for r in range(c.m)])
        assert np.array_equal(got, c.parity), i
        assert c.guards_ok(host, c.n), i
    for c, buf in zip(cases, bufs):
        for b in c.erasures:
            c.put(buf, b, np.full(c.nb, 0x3C, dtype=np.uint8))
    bt.decode([(c.code, c.ptrs(buf, c.n), c.nb, c.erasures, c.flags)
               for c, buf in zip(cases, bufs)])
    torch.cuda.synchronize()
    for i, (c, buf) in enumerate(zip(cases, bufs)):
        host = buf.cpu().numpy()
        for b in range(c.n):
            assert np.array_equal(c.get(host, b), c.full[b]), (i, b)
    # updates, in each placement (REGISTERS falls back to the table forms
    # for the widths where a stripe changes more than 2 blocks)
    for placement in (B.RS_POLY_TABLES_REGISTERS, B.RS_POLY_TABLES_PACKED):
        bt2 = B.Batch()
        for w in (0, 1):
            cfg = bt2.get_launch(B.RS_POLY_OP_UPDATE, w).as_dict()
            bt2.set_launch(B.RS_POLY_OP_UPDATE, w, dict(cfg, table_placement=placement))
        dbufs = []
        ents = []
        for c, buf in zip(cases, bufs):
            db = c.buffer(c.k, fill=0)
            for j in c.changed:
                c.put(db, j, c.delta[j])
            dbufs.append(db)
            dp = c.ptrs(db, c.k)
            ents.append((c.code, [dp[j] if j in c.changed else None for j in range(c.k)] +
                         c.ptrs(buf, c.n)[c.k:], c.nb))
        bt2.update(ents)
        torch.cuda.synchronize()
        for i, (c, buf) in enumerate(zip(cases, bufs)):
            host = buf.cpu().numpy()
            got = np.stack([c.get(host, c.k + r) for r in range(c.m)])
            assert np.array_equal(got, c.new_parity), (i, placement)
        # the same deltas again bring the parity back
        bt2.update(ents)
        torch.cuda.synchronize()
        for i, (c, buf) in enumerate(zip(cases, bufs)):
            host = buf.cpu().numpy()
            got = np.stack([c.get(host, c.k + r) for r in range(c.m)])
            assert np.array_equal(got, c.parity), (i, placement)
