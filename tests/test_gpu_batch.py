"""GPU parity of the batched (persistent, graph-replayed) encode and decode
against the CPU oracle and the plain one-stripe-per-launch path."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELD = {}


def field(w=8, poly=0x11D):
    if (w, poly) not in FIELD:
        FIELD[(w, poly)] = oracle.Field(w, poly)
    return FIELD[(w, poly)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Arena:
    """Device memory for many stripes: every block 256-byte aligned."""

    def __init__(self, shapes):
        self.offsets = []
        off = 0
        for (k, m, nbytes) in shapes:
            blocks = []
            step = (nbytes + 255) // 256 * 256
            for _ in range(k + m):
                blocks.append(off)
                off += max(step, 256)
            self.offsets.append(blocks)
        self.buf = torch.zeros(max(off, 256), dtype=torch.uint8, device="cuda")
        self.base = self.buf.data_ptr()
        self.shapes = shapes

    def ptrs(self, s):
        return [self.base + o for o in self.offsets[s]]

    def block(self, s, b):
        nbytes = self.shapes[s][2]
        o = self.offsets[s][b]
        return self.buf[o:o + nbytes]


def mixed_shapes(seed, count, codes, lo, hi):
    rng = workloads.meta_rng(seed)
    sizes = workloads.log_uniform_sizes(rng, count, lo, hi)
    picks = rng.integers(0, len(codes), size=count)
    return [(codes[c][0], codes[c][1], int(b)) for c, b in zip(picks, sizes)]


def fill_data(arena, seed):
    """Random data blocks on the device; returns host copies."""
    host = []
    for s, (k, m, nbytes) in enumerate(arena.shapes):
        d = workloads.stripe_data(seed, s, k, nbytes)
        for j in range(k):
            arena.block(s, j).copy_(torch.from_numpy(d[j]))
        host.append(d)
    return host


CODES = {}


def code(k, m):
    if (k, m) not in CODES:
        CODES[(k, m)] = B.Code(k, m)
    return CODES[(k, m)]


def encode_entries(arena):
    return [(code(k, m), arena.ptrs(s), nbytes) for s, (k, m, nbytes) in enumerate(arena.shapes)]


def check_encoded(arena, host, which=None):
    for s in (range(len(arena.shapes)) if which is None else which):
        k, m, nbytes = arena.shapes[s]
        want = oracle.encode(field(), k, m, host[s])
        for i in range(m):
            got = arena.block(s, k + i).cpu().numpy()
            assert np.array_equal(got, want[i]), (s, k, m, nbytes, i)


SMALL_CODES = ((6, 3), (10, 4), (12, 4), (32, 8), (5, 6), (3, 1))


def test_batch_encode_mixed_matches_oracle():
    say("batch encode mixed 48 stripes")
    shapes = mixed_shapes(1, 48, SMALL_CODES, 1, 300_000)
    shapes += [(10, 4, 0), (6, 3, 16), (12, 4, 17)]
    arena = Arena(shapes)
    host = fill_data(arena, 11)
    bt = B.Batch()
    bt.encode(encode_entries(arena))
    torch.cuda.synchronize()
    check_encoded(arena, host)


def test_batch_decode_mixed_matches_oracle():
    say("batch decode mixed 40 stripes")
    shapes = mixed_shapes(2, 40, SMALL_CODES, 1, 200_000)
    arena = Arena(shapes)
    host = fill_data(arena, 12)
    bt = B.Batch()
    bt.encode(encode_entries(arena))
    torch.cuda.synchronize()
    full = [arena.buf.cpu().numpy()]
    rng = workloads.meta_rng(99)
    entries, lost = [], []
    for s, (k, m, nbytes) in enumerate(shapes):
        t = int(rng.integers(0, m + 1))
        er = workloads.random_erasures(rng, k + m, t)
        flags = int(rng.integers(0, 2))
        for b in er:
            arena.block(s, b).fill_(0xEE)   # poison what must be rebuilt
        entries.append((code(k, m), arena.ptrs(s), nbytes, er, flags))
        lost.append(er)
    bt.decode(entries)
    torch.cuda.synchronize()
    after = arena.buf.cpu().numpy()
    for s, er in enumerate(lost):
        for b in er:
            o = arena.offsets[s][b]
            nb = shapes[s][2]
            assert np.array_equal(after[o:o + nb], full[0][o:o + nb]), (s, shapes[s], er)


def test_batch_equals_plain_path():
    say("batch vs plain")
    shapes = mixed_shapes(3, 24, ((10, 4), (6, 3), (32, 8)), 4096, 100_000)
    a1, a2 = Arena(shapes), Arena(shapes)
    fill_data(a1, 5)
    a2.buf.copy_(a1.buf)
    B.Batch().encode(encode_entries(a1))
    for s, (k, m, nbytes) in enumerate(shapes):
        p = a2.ptrs(s)
        code(k, m).encode(p[:k], p[k:], nbytes)
    torch.cuda.synchronize()
    assert torch.equal(a1.buf, a2.buf)


def test_graph_replays_with_new_descriptors():
    # Same batch object, several calls: new data, then a different stripe
    # set; every replay of the captured graph must be right.
    say("graph replays")
    bt = B.Batch()
    for it in range(4):
        shapes = mixed_shapes(10 + (it // 2), 20, SMALL_CODES[:3], 1000, 80_000)
        arena = Arena(shapes)
        host = fill_data(arena, 100 + it)
        bt.encode(encode_entries(arena))
        torch.cuda.synchronize()
        check_encoded(arena, host)


@pytest.mark.parametrize("bpl", [4, 8, 16])
@pytest.mark.parametrize("threads", [256, 768, 1024])
@pytest.mark.parametrize("placement", [B.RS_POLY_TABLES_PACKED, B.RS_POLY_TABLES_NIBBLE])
@pytest.mark.parametrize("order", [0, 1])
def test_every_launch_shape(bpl, threads, placement, order):
    say(f"launch shape bpl={bpl} threads={threads} placement={placement} order={order}")
    shapes = mixed_shapes(7, 12, ((10, 4), (6, 3), (32, 8), (5, 6)), 1, 70_000)
    arena = Arena(shapes)
    host = fill_data(arena, 21)
    bt = B.Batch()
    for wide in (0, 1):
        # register-bound workgroup limit of the narrow 16-byte-per-lane variants
        th = min(threads, 512) if bpl == 16 and not wide else threads
        cfg = dict(bytes_per_lane=bpl, threads=th, tile_bytes=4096 * (1 + wide),
                   wgs_per_cu=1 + wide, table_placement=placement, tile_order=order)
        bt.set_launch(B.RS_POLY_OP_ENCODE, wide, cfg)
        bt.set_launch(B.RS_POLY_OP_DECODE, wide, cfg)
        bt.set_launch(B.RS_POLY_OP_UPDATE, wide, cfg)
    bt.encode(encode_entries(arena))
    torch.cuda.synchronize()
    check_encoded(arena, host)
    before = arena.buf.clone()
    entries = []
    for s, (k, m, nbytes) in enumerate(shapes):
        er = list(range(min(m, k + m)))[::-1]   # first m blocks: data first
        for b in er:
            arena.block(s, b).fill_(0x11)
        entries.append((code(k, m), arena.ptrs(s), nbytes, er, 0))
    bt.decode(entries)
    torch.cuda.synchronize()
    assert torch.equal(arena.buf, before)
    # delta-parity update in both forms: two changed blocks (generator-matrix
    # form) and every data block (LFSR form for k > 8); the delta of block j
    # is block j itself, so the parity becomes old ^ encode(changed blocks)
    for every in (False, True):
        old = [[arena.block(s, k + i).cpu().numpy() for i in range(m)]
               for s, (k, m, nbytes) in enumerate(shapes)]
        ents, changed = [], []
        for s, (k, m, nbytes) in enumerate(shapes):
            ch = list(range(k)) if every else sorted({0, k - 1})
            ptrs = arena.ptrs(s)
            ents.append((code(k, m), [ptrs[j] if j in ch else None for j in range(k)] + ptrs[k:],
                         nbytes))
            changed.append(ch)
        bt.update(ents)
        torch.cuda.synchronize()
        for s, (k, m, nbytes) in enumerate(shapes):
            dd = np.zeros_like(host[s])
            dd[changed[s]] = host[s][changed[s]]
            want = oracle.encode(field(), k, m, dd)
            for i in range(m):
                got = arena.block(s, k + i).cpu().numpy()
                assert np.array_equal(got, old[s][i] ^ want[i]), (every, s, i)


def test_set_launch_validation():
    bt = B.Batch()
    bad = [dict(bytes_per_lane=3, threads=256, tile_bytes=4096, wgs_per_cu=1),
           dict(bytes_per_lane=4, threads=256, tile_bytes=4096, wgs_per_cu=1,
                table_placement=3),     # register split-nibble: updates only
           dict(bytes_per_lane=4, threads=256, tile_bytes=4096, wgs_per_cu=1,
                table_placement=4),
           dict(bytes_per_lane=4, threads=256, tile_bytes=4096, wgs_per_cu=1,
                tile_order=2),
           dict(bytes_per_lane=16, threads=300, tile_bytes=4096, wgs_per_cu=1),
           dict(bytes_per_lane=16, threads=256, tile_bytes=4000, wgs_per_cu=1),
           dict(bytes_per_lane=16, threads=256, tile_bytes=4096, wgs_per_cu=3)]
    for cfg in bad:
        with pytest.raises(B.RsPolyError):
            bt.set_launch(B.RS_POLY_OP_ENCODE, 0, cfg)
    with pytest.raises(B.RsPolyError):
        bt.set_launch(B.RS_POLY_OP_DECODE, 0, dict(bytes_per_lane=16, threads=1024,
                                                  tile_bytes=4096, wgs_per_cu=2))
    # the bit-sliced placement is an encode kernel only
    bt.set_launch(B.RS_POLY_OP_ENCODE, 0, dict(bytes_per_lane=16, threads=512, tile_bytes=4096,
                                              wgs_per_cu=2,
                                              table_placement=B.RS_POLY_TABLES_BITMATRIX))
    for op in (B.RS_POLY_OP_DECODE, B.RS_POLY_OP_UPDATE):
        with pytest.raises(B.RsPolyError):
            bt.set_launch(op, 0, dict(bytes_per_lane=16, threads=512, tile_bytes=4096,
                                      wgs_per_cu=2, table_placement=B.RS_POLY_TABLES_BITMATRIX))
    # the register split-nibble placement is an update kernel only
    for w in (0, 1):
        bt.set_launch(B.RS_POLY_OP_UPDATE, w, dict(bytes_per_lane=4, threads=1024,
                                                  tile_bytes=16384, wgs_per_cu=2,
                                                  table_placement=B.RS_POLY_TABLES_REGISTERS))
    with pytest.raises(B.RsPolyError):
        bt.set_launch(B.RS_POLY_OP_DECODE, 0, dict(bytes_per_lane=4, threads=512,
                                                  tile_bytes=4096, wgs_per_cu=2,
                                                  table_placement=B.RS_POLY_TABLES_REGISTERS))
    # narrow codes at 16 bytes per lane take at most 512 threads; wide codes
    # (m > 4) run every width with up to 1024, 768 included
    with pytest.raises(B.RsPolyError):
        bt.set_launch(B.RS_POLY_OP_ENCODE, 0, dict(bytes_per_lane=16, threads=1024,
                                                  tile_bytes=4096, wgs_per_cu=1))
    for op in (B.RS_POLY_OP_ENCODE, B.RS_POLY_OP_DECODE, B.RS_POLY_OP_UPDATE):
        for bpl in (4, 8, 16):
            for th in (256, 512, 768, 1024):
                bt.set_launch(op, 1, dict(bytes_per_lane=bpl, threads=th, tile_bytes=4096,
                                          wgs_per_cu=1))
    with pytest.raises(B.RsPolyError):
        bt.set_launch(B.RS_POLY_OP_DECODE, 1, dict(bytes_per_lane=8, threads=640,
                                                  tile_bytes=4096, wgs_per_cu=1))


def test_batch_rejects_bad_input_without_running():
    bt = B.Batch()
    arena = Arena([(10, 4, 4096), (10, 4, 4096)])
    fill_data(arena, 1)
    before = arena.buf.clone()
    good = (code(10, 4), arena.ptrs(0), 4096)
    p = arena.ptrs(1)
    p[3] += 4   # misaligned
    with pytest.raises(B.RsPolyError) as ei:
        bt.encode([good, (code(10, 4), p, 4096)])
    assert ei.value.code == B.RS_EINVAL
    with pytest.raises(B.RsPolyError) as ei:
        bt.decode([(code(10, 4), arena.ptrs(0), 4096, [1, 1], 0)])
    assert ei.value.code == B.RS_ERANGE
    with pytest.raises(B.RsPolyError) as ei:
        bt.decode([(code(10, 4), arena.ptrs(0), 4096, [0, 1, 2, 3, 4], 0)])
    assert ei.value.code == B.RS_ETOOMANY
    torch.cuda.synchronize()
    assert torch.equal(arena.buf, before)


def test_autotuner_picks_a_valid_shape_and_stays_exact(tmp_path, monkeypatch):
    say("autotuner")
    monkeypatch.setenv("RS_POLY_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    shapes = [(10, 4, 1 << 18)] * 8
    arena = Arena(shapes)
    host = fill_data(arena, 3)
    bt = B.Batch()
    best = bt.tune(B.RS_POLY_OP_ENCODE, encode_entries(arena))
    assert best.bytes_per_lane in (4, 8, 16) and best.threads in (256, 512, 1024)
    assert bt.get_launch(B.RS_POLY_OP_ENCODE, 0).as_dict() == best.as_dict()
    text = (tmp_path / "tune.jsonl").read_text()
    assert '"op": 0' in text and '"bytes_per_lane"' in text and '"table_placement"' in text
    arena.buf[:] = 0
    fill_data(arena, 4)
    host = [workloads.stripe_data(4, s, 10, 1 << 18) for s in range(8)]
    bt2 = B.Batch()
    best2 = bt2.tune(B.RS_POLY_OP_ENCODE, encode_entries(arena))   # cache hit
    assert best2.as_dict() == best.as_dict()
    bt2.encode(encode_entries(arena))
    torch.cuda.synchronize()
    check_encoded(arena, host)


# ------------------------------------------------- full-size workloads --

def full_size_arena(stripes, k, m, nbytes, seed):
    """(stripes, k+m, nbytes) device tensor with random data rows."""
    buf = torch.empty((stripes, k + m, nbytes), dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    for s in range(stripes):
        buf[s, :k] = torch.randint(0, 256, (k, nbytes), dtype=torch.uint8, device="cuda",
                                   generator=gen)
    return buf


def check_stripe_against_oracle(buf, s, k, m, cols=None):
    """The oracle re-encodes data (a column window, or all) of stripe s."""
    d = buf[s, :k] if cols is None else buf[s, :k, cols[0]:cols[1]]
    p = buf[s, k:] if cols is None else buf[s, k:, cols[0]:cols[1]]
    want = oracle.encode(field(), k, m, d.cpu().numpy())
    assert np.array_equal(p.cpu().numpy(), want), (s, cols)


def oracle_windows(buf, k, m, nbytes, window, seed):
    """Checks a seeded `window`-column window of every stripe's parity
    against the oracle (the last stripe's window ends at the block's end)."""
    S = buf.shape[0]
    rng = workloads.meta_rng(seed)
    for s in range(S):
        if s == S - 1:
            c0 = nbytes - window
        else:
            c0 = int(rng.integers(0, nbytes - window + 1))
        check_stripe_against_oracle(buf, s, k, m, (c0, c0 + window))


def test_full_size_rs104_256x1MiB_batched():
    # 256 stripes x 10 x 1 MiB: the launch configuration the benchmark times.
    say("full size RS(10,4) 256 x 1 MiB")
    k, m, nbytes, S = 10, 4, 1 << 20, 256
    buf = full_size_arena(S, k, m, nbytes, workloads.data_seed(1))
    c = code(k, m)
    ents = [(c, [buf[s, b].data_ptr() for b in range(k + m)], nbytes) for s in range(S)]
    bt = B.Batch()
    bt.encode(ents)
    torch.cuda.synchronize()
    for s in (0, 1, 127, 254, 255):
        check_stripe_against_oracle(buf, s, k, m)
    # a 64 KiB window of every stripe against the oracle
    oracle_windows(buf, k, m, nbytes, 64 << 10, workloads.meta_seed(1) + 11)
    # decode with 1..4 uniformly random erased blocks per stripe
    rng = workloads.meta_rng(workloads.meta_seed(1))
    ref = buf.clone()
    dents = []
    for s in range(S):
        t = int(rng.integers(1, m + 1))
        er = workloads.random_erasures(rng, k + m, t)
        buf[s, er] = 0xC3
        dents.append((c, [buf[s, b].data_ptr() for b in range(k + m)], nbytes, er, 0))
    bt.decode(dents)
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)


def test_full_size_mixed_4096_uneven():
    # 4096 stripes, block size log-uniform in [4 KiB, 4 MiB], codes RS(6,3),
    # RS(10,4), RS(12,4); one persistent launch each for encode and decode.
    say("full size mixed 4096 stripes")
    cfg = workloads.CONFIGS["mixed_4096_uneven"]
    shapes = mixed_shapes(workloads.meta_seed(2), cfg["stripes"], cfg["codes"],
                          cfg["min_bytes"], cfg["max_bytes"])
    arena = Arena(shapes)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(2))
    arena.buf[:] = torch.randint(0, 256, arena.buf.shape, dtype=torch.uint8, device="cuda",
                                 generator=gen)
    bt = B.Batch()
    bt.encode(encode_entries(arena))
    torch.cuda.synchronize()
    rng = workloads.meta_rng(5)
    for s in list(rng.choice(len(shapes), size=12, replace=False)) + [0, len(shapes) - 1]:
        k, m, nbytes = shapes[s]
        d = np.stack([arena.block(s, j).cpu().numpy() for j in range(k)])
        want = oracle.encode(field(), k, m, d)
        for i in range(m):
            assert np.array_equal(arena.block(s, k + i).cpu().numpy(), want[i]), (s, i)
    # and a seeded window of up to 4 KiB of every stripe (gathered on the
    # device, copied to the host once)
    wins = []
    for s, (k, m, nbytes) in enumerate(shapes):
        w = min(nbytes, 4096)
        c0 = int(rng.integers(0, nbytes - w + 1))
        wins.append(torch.stack([arena.block(s, b)[c0:c0 + w] for b in range(k + m)]))
    flat = torch.cat([x.flatten() for x in wins]).cpu().numpy()
    host = np.split(flat, np.cumsum([x.numel() for x in wins])[:-1])
    for s, (k, m, nbytes) in enumerate(shapes):
        rows = host[s].reshape(k + m, -1)
        assert np.array_equal(oracle.encode(field(), k, m, rows[:k]), rows[k:]), s
    ref = arena.buf.clone()
    ents = []
    for s, (k, m, nbytes) in enumerate(shapes):
        t = int(rng.integers(1, m + 1))
        er = workloads.random_erasures(rng, k + m, t)
        for b in er:
            arena.block(s, b).fill_(0x3C)
        ents.append((code(k, m), arena.ptrs(s), nbytes, er, 0))
    bt.decode(ents)
    torch.cuda.synchronize()
    assert torch.equal(arena.buf, ref)


def test_full_size_rs328_64x16MiB():
    # RS(32,8), 64 stripes x 32 x 16 MiB (the benchmark's headline workload, in
    # its launch configuration); decode with 8 erased blocks in every stripe.
    say("full size RS(32,8) 64 x 16 MiB")
    k, m, nbytes, S = 32, 8, 16 << 20, 64
    buf = full_size_arena(S, k, m, nbytes, workloads.data_seed(4))
    c = code(k, m)
    ents = [(c, [buf[s, b].data_ptr() for b in range(k + m)], nbytes) for s in range(S)]
    bt = B.Batch()
    bt.encode(ents)
    torch.cuda.synchronize()
    # a seeded 64 KiB window of every stripe's parity against the oracle
    oracle_windows(buf, k, m, nbytes, 64 << 10, workloads.meta_seed(4) + 11)
    rng = workloads.meta_rng(workloads.meta_seed(4))
    patterns = [workloads.random_erasures(rng, k + m, m) for _ in range(S)]
    # the lost blocks of every stripe, kept on the device (8 GiB), then wiped
    saved = torch.stack([buf[s, patterns[s]] for s in range(S)])
    dents = []
    for s in range(S):
        buf[s, patterns[s]] = 0x77
        dents.append((c, [buf[s, b].data_ptr() for b in range(k + m)], nbytes, patterns[s], 0))
    bt.decode(dents)
    torch.cuda.synchronize()
    for s in range(S):
        assert torch.equal(buf[s, patterns[s]], saved[s]), s
