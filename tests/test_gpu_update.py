"""GPU parity of the delta-parity update (the update property of Sec. 3.2):
after an update with delta = new data XOR old data, the parity equals the
oracle's encoding of the new data, byte for byte, on the plain and the
batched path.  The starting parity is the oracle's encoding of the old
data, so no GPU encode is involved."""
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


class UpdateCase:
    """Old and new data of one stripe (host), the oracle's parity of the old
    data, and device buffers for the delta blocks and the parity.  Blocks
    are rows of buffers with a `pad`-byte gap (guard bytes) starting
    `offset` bytes in."""

    def __init__(self, k, m, nbytes, changed, seed, w=8, poly=0x11D, offset=0, pad=64):
        self.k, self.m, self.n, self.changed = k, m, nbytes, sorted(changed)
        mask = (1 << w) - 1
        self.F = field(w, poly)
        self.old = workloads.random_bytes(seed, (k, nbytes)) & mask
        self.new = self.old.copy()
        fresh = workloads.random_bytes(seed + 1, (k, nbytes)) & mask
        for j in self.changed:
            self.new[j] = fresh[j]
        self.parity0 = oracle.encode(self.F, k, m, self.old)
        self.stride = nbytes + pad
        self.offset = offset
        self.dbuf = torch.zeros(k * self.stride + offset + 64, dtype=torch.uint8, device="cuda")
        self.pbuf = torch.full((m * self.stride + offset + 64,), 0xA5, dtype=torch.uint8,
                               device="cuda")
        for j in self.changed:
            o = offset + j * self.stride
            self.dbuf[o:o + nbytes] = torch.from_numpy(self.old[j] ^ self.new[j])
        for i in range(m):
            o = offset + i * self.stride
            self.pbuf[o:o + nbytes] = torch.from_numpy(self.parity0[i])

    def delta_ptrs(self):
        base = self.dbuf.data_ptr() + self.offset
        return [base + j * self.stride if j in self.changed else None for j in range(self.k)]

    def parity_ptrs(self):
        base = self.pbuf.data_ptr() + self.offset
        return [base + i * self.stride for i in range(self.m)]

    def parity(self):
        host = self.pbuf.cpu().numpy()
        rows = [host[self.offset + i * self.stride: self.offset + i * self.stride + self.n]
                for i in range(self.m)]
        return np.stack(rows), host

    def check(self, want=None):
        got, host = self.parity()
        want = oracle.encode(self.F, self.k, self.m, self.new) if want is None else want
        assert np.array_equal(got, want), (self.k, self.m, self.n, self.changed)
        # guard bytes between and around the parity blocks are untouched
        for i in range(self.m):
            end = self.offset + i * self.stride + self.n
            assert (host[end:end + (self.stride - self.n)] == 0xA5).all()
        assert (host[:self.offset] == 0xA5).all()


PLAIN = [(10, 4, 100003, [0]), (10, 4, 100003, [9]), (10, 4, 65536, [3, 7]),
         (10, 4, 4097, list(range(10))), (6, 3, 17, [5]), (6, 3, 65536, [0, 2, 4]),
         (12, 4, 8191, [11]), (32, 8, 70001, [0, 31]), (32, 8, 8192, [12]),
         (5, 6, 1000, [1, 2]), (1, 1, 1, [0]), (13, 1, 999, [12]), (3, 7, 333, [0]),
         (247, 8, 64, [100, 246]), (200, 4, 129, [0, 1, 2, 3, 4, 199])]


@pytest.mark.parametrize("k,m,nbytes,changed", PLAIN)
def test_update_matches_oracle_encode_of_new_data(k, m, nbytes, changed):
    say(f"update k={k} m={m} B={nbytes} changed={changed}")
    case = UpdateCase(k, m, nbytes, changed, seed=k * 131 + m * 17 + nbytes)
    code = B.Code(k, m)
    B.rs_poly_update(code.handle, case.delta_ptrs(), case.parity_ptrs(), nbytes)
    torch.cuda.synchronize()
    case.check()


@pytest.mark.parametrize("offset", [1, 2, 4, 8])
def test_update_misaligned_blocks(offset):
    say(f"update misaligned offset={offset}")
    case = UpdateCase(10, 4, 20001, [2, 6], seed=900 + offset, offset=offset, pad=3)
    code = B.Code(10, 4)
    code.update(case.delta_ptrs(), case.parity_ptrs(), 20001)
    torch.cuda.synchronize()
    case.check()


def test_update_twice_restores_parity():
    say("update twice")
    case = UpdateCase(10, 4, 1 << 16, [1, 8], seed=41)
    code = B.Code(10, 4)
    for _ in range(2):
        code.update(case.delta_ptrs(), case.parity_ptrs(), 1 << 16)
    torch.cuda.synchronize()
    case.check(want=case.parity0)


def test_update_with_no_changed_block_is_a_noop():
    case = UpdateCase(10, 4, 4096, [], seed=42)
    code = B.Code(10, 4)
    code.update(case.delta_ptrs(), case.parity_ptrs(), 4096)
    torch.cuda.synchronize()
    case.check(want=case.parity0)


def test_update_gf16():
    say("update GF(2^4)")
    for (k, m, changed) in ((4, 3, [0]), (9, 5, [3, 8]), (12, 3, [11])):
        case = UpdateCase(k, m, 777, changed, seed=k * 7 + m, w=4, poly=0x13)
        code = B.Code(k, m, 4, 0x13)
        code.update(case.delta_ptrs(), case.parity_ptrs(), 777)
        torch.cuda.synchronize()
        case.check()


def test_update_sequence_tracks_the_data():
    # Several rounds of random changes: the parity always equals the
    # encoding of the current data.
    say("update sequence")
    k, m, nbytes = 12, 4, 50000
    F = field()
    rng = workloads.meta_rng(4242)
    data = workloads.random_bytes(4243, (k, nbytes))
    parity = torch.from_numpy(oracle.encode(F, k, m, data)).cuda()
    dbuf = torch.zeros((k, nbytes), dtype=torch.uint8, device="cuda")
    code = B.Code(k, m)
    for r in range(6):
        changed = sorted(rng.choice(k, size=int(rng.integers(1, 4)), replace=False).tolist())
        fresh = workloads.random_bytes(5000 + r, (k, nbytes))
        new = data.copy()
        for j in changed:
            new[j] = fresh[j]
            dbuf[j] = torch.from_numpy(data[j] ^ new[j])
        code.update([dbuf[j] if j in changed else None for j in range(k)],
                    [parity[i] for i in range(m)], nbytes)
        data = new
    torch.cuda.synchronize()
    assert np.array_equal(parity.cpu().numpy(), oracle.encode(F, k, m, data))


# ------------------------------------------------------------- batched --

def batch_cases(seed, count, codes, lo, hi, max_changed=None):
    rng = workloads.meta_rng(seed)
    sizes = workloads.log_uniform_sizes(rng, count, lo, hi)
    cases = []
    for s in range(count):
        k, m = codes[int(rng.integers(0, len(codes)))]
        n_changed = int(rng.integers(0, min(k, max_changed or k) + 1))
        changed = rng.choice(k, size=n_changed, replace=False).tolist()
        # 256-byte aligned rows (the batch path needs 16-byte alignment)
        cases.append(UpdateCase(k, m, int(sizes[s]), changed, seed=seed * 1000 + s,
                                pad=(-int(sizes[s])) % 256 + 256))
    return cases


CODES = {}


def code(k, m):
    if (k, m) not in CODES:
        CODES[(k, m)] = B.Code(k, m)
    return CODES[(k, m)]


def entries(cases):
    return [(code(c.k, c.m), c.delta_ptrs() + c.parity_ptrs(), c.n) for c in cases]


def test_batch_update_mixed_matches_oracle():
    say("batch update mixed 40 stripes")
    cases = batch_cases(61, 40, ((6, 3), (10, 4), (12, 4), (32, 8), (5, 6), (3, 1)),
                        1, 300000)
    bt = B.Batch()
    bt.update(entries(cases))
    torch.cuda.synchronize()
    for c in cases:
        c.check()


@pytest.mark.parametrize("placement", [B.RS_POLY_TABLES_PACKED, B.RS_POLY_TABLES_NIBBLE,
                                       B.RS_POLY_TABLES_REGISTERS])
def test_batch_update_table_placements(placement):
    # (with REGISTERS most of these stripes change more than 2 blocks, so the
    # call falls back to the table forms)
    say(f"batch update placement={placement}")
    cases = batch_cases(65, 16, ((10, 4), (32, 8), (6, 3)), 1, 200000)
    bt = B.Batch()
    for wide in (0, 1):
        cfg = bt.get_launch(B.RS_POLY_OP_UPDATE, wide).as_dict()
        bt.set_launch(B.RS_POLY_OP_UPDATE, wide, dict(cfg, table_placement=placement))
    bt.update(entries(cases))
    torch.cuda.synchronize()
    for c in cases:
        c.check()


def set_update_placement(bt, placement, threads=None, tile=None):
    for wide in (0, 1):
        cfg = bt.get_launch(B.RS_POLY_OP_UPDATE, wide).as_dict()
        cfg["table_placement"] = placement
        if threads:
            cfg.update(bytes_per_lane=4, threads=threads)
        if tile:
            cfg["tile_bytes"] = tile
        bt.set_launch(B.RS_POLY_OP_UPDATE, wide, cfg)


@pytest.mark.parametrize("threads,tile,order", [(None, None, 0), (1024, 65536, 1),
                                                (256, 4096, 0), (512, 16384, 1)])
def test_batch_update_register_nibble_form(threads, tile, order):
    # every stripe changes at most 2 blocks (1 for the wide codes, so that
    # changed * m <= 8): both widths take the register split-nibble kernel;
    # uneven sizes (ragged tails, blocks under 16 bytes), stripes with no
    # changed block, m from 1 to 8
    say(f"batch update, register split-nibble form, threads={threads} tile={tile}")
    narrow = batch_cases(67, 30, ((6, 3), (10, 4), (12, 4), (3, 1), (5, 2)), 1, 300000,
                         max_changed=2)
    wide = batch_cases(68, 12, ((32, 8), (5, 6), (20, 5), (4, 7)), 1, 300000, max_changed=1)
    cases = narrow + wide
    bt = B.Batch()
    set_update_placement(bt, B.RS_POLY_TABLES_REGISTERS, threads, tile)
    for w in (0, 1):
        cfg = bt.get_launch(B.RS_POLY_OP_UPDATE, w).as_dict()
        bt.set_launch(B.RS_POLY_OP_UPDATE, w, dict(cfg, tile_order=order))
    bt.update(entries(cases))
    torch.cuda.synchronize()
    for c in cases:
        c.check()
    # and again: the same deltas restore the starting parity
    bt.update(entries(cases))
    torch.cuda.synchronize()
    for c in cases:
        c.check(want=c.parity0)


def test_batch_update_register_form_equals_matrix_form():
    say("batch update: register split-nibble form vs matrix form")
    cases = batch_cases(69, 16, ((10, 4), (6, 3), (32, 8)), 4096, 1 << 20, max_changed=1)
    twins = batch_cases(69, 16, ((10, 4), (6, 3), (32, 8)), 4096, 1 << 20, max_changed=1)
    bt = B.Batch()
    set_update_placement(bt, B.RS_POLY_TABLES_REGISTERS)
    bt.update(entries(cases))
    B.Batch().update(entries(twins))
    torch.cuda.synchronize()
    for a, b in zip(cases, twins):
        assert np.array_equal(a.parity()[0], b.parity()[0])
        a.check()


def test_batch_update_matrix_form_matches_oracle():
    # at most 8 changed blocks per stripe: every width takes the
    # generator-matrix form (one lookup per changed block)
    say("batch update, matrix form")
    cases = batch_cases(66, 40, ((6, 3), (10, 4), (12, 4), (32, 8), (5, 6), (3, 1)),
                        1, 300000, max_changed=8)
    bt = B.Batch()
    bt.update(entries(cases))
    torch.cuda.synchronize()
    for c in cases:
        c.check()


def test_plain_update_both_forms_at_the_boundary():
    # 8 changed blocks (matrix form) and 9 (LFSR form) of RS(32,8) and
    # RS(12,4), as the plain path chooses them
    say("plain update, 8 and 9 changed blocks")
    for k, m in ((32, 8), (12, 4)):
        for n in (8, 9):
            changed = list(range(0, k, max(1, k // n)))[:n]
            assert len(set(changed)) == n and max(changed) < k
            case = UpdateCase(k, m, 30001, changed, seed=k * 10 + n)
            B.Code(k, m).update(case.delta_ptrs(), case.parity_ptrs(), 30001)
            torch.cuda.synchronize()
            case.check()


@pytest.mark.parametrize("k,m,changed", [(10, 4, [2, 7]), (32, 8, [0, 13, 31]),
                                         (12, 4, list(range(12)))])
def test_plain_update_large_aligned_blocks(k, m, changed):
    # 4 MiB + 48-byte blocks on a 256-byte stride: 16-byte aligned, so the
    # widest-load kernels run, with several rounds per lane (matrix form for
    # up to 8 changed blocks, LFSR form for all 12)
    nbytes = (4 << 20) + 48
    say(f"plain update RS({k},{m}) B={nbytes} changed={len(changed)}")
    case = UpdateCase(k, m, nbytes, changed, seed=900 + k, pad=256 - 48)
    assert case.stride % 16 == 0 and case.dbuf.data_ptr() % 16 == 0
    B.Code(k, m).update(case.delta_ptrs(), case.parity_ptrs(), nbytes)
    torch.cuda.synchronize()
    case.check()


def test_batch_update_equals_plain_update():
    say("batch update vs plain")
    cases = batch_cases(62, 12, ((10, 4), (32, 8)), 4096, 1 << 20)
    twins = batch_cases(62, 12, ((10, 4), (32, 8)), 4096, 1 << 20)
    B.Batch().update(entries(cases))
    for c in twins:
        code(c.k, c.m).update(c.delta_ptrs(), c.parity_ptrs(), c.n)
    torch.cuda.synchronize()
    for a, b in zip(cases, twins):
        assert np.array_equal(a.parity()[0], b.parity()[0])


def test_batch_update_tune_leaves_parity_unchanged(tmp_path, monkeypatch):
    say("batch update autotuner")
    monkeypatch.setenv("RS_POLY_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    cases = batch_cases(63, 6, ((10, 4),), 1 << 16, 1 << 18)
    bt = B.Batch()
    best = bt.tune(B.RS_POLY_OP_UPDATE, entries(cases))
    torch.cuda.synchronize()
    assert best.bytes_per_lane in (4, 8, 16)
    assert '"op": 2' in (tmp_path / "tune.jsonl").read_text()
    for c in cases:
        c.check(want=c.parity0)
    bt.update(entries(cases))
    torch.cuda.synchronize()
    for c in cases:
        c.check()


def test_batch_update_rejects_bad_input():
    cases = batch_cases(64, 2, ((10, 4),), 4096, 8192)
    bt = B.Batch()
    ents = entries(cases)
    bad = [(ents[0][0], ents[0][1][:10] + [None] + ents[0][1][11:], ents[0][2])]
    with pytest.raises(B.RsPolyError) as ei:
        bt.update(bad + ents[1:])
    assert ei.value.code == B.RS_ENULL
    odd = list(ents[0][1])
    odd[10] += 1                     # parity not 16-byte aligned
    with pytest.raises(B.RsPolyError) as ei:
        bt.update([(ents[0][0], odd, ents[0][2])])
    assert ei.value.code == B.RS_EINVAL
    torch.cuda.synchronize()
    for c in cases:
        c.check(want=c.parity0)      # nothing ran


@pytest.mark.parametrize("placement", [B.RS_POLY_TABLES_PACKED, B.RS_POLY_TABLES_REGISTERS])
def test_full_size_rs104_256x1MiB_batch_update(placement):
    # One changed block per stripe of the 256 x 10 x 1 MiB workload (matrix
    # form, or register split-nibble form); the oracle checks a column
    # window of sampled stripes.
    say(f"full size batch update RS(10,4) 256 x 1 MiB placement={placement}")
    k, m, nbytes, S = 10, 4, 1 << 20, 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(1) + 77)
    old = torch.randint(0, 256, (S, k, nbytes), dtype=torch.uint8, device="cuda", generator=gen)
    par = torch.empty((S, m, nbytes), dtype=torch.uint8, device="cuda")
    c = code(k, m)
    bt = B.Batch()
    bt.encode([(c, [old[s, j].data_ptr() for j in range(k)] +
                [par[s, i].data_ptr() for i in range(m)], nbytes) for s in range(S)])
    rng = workloads.meta_rng(workloads.meta_seed(1) + 77)
    changed = rng.integers(0, k, size=S)
    delta = torch.randint(0, 256, (S, nbytes), dtype=torch.uint8, device="cuda", generator=gen)
    ents = []
    for s in range(S):
        ptrs = [None] * k + [par[s, i].data_ptr() for i in range(m)]
        ptrs[int(changed[s])] = delta[s].data_ptr()
        ents.append((c, ptrs, nbytes))
    set_update_placement(bt, placement)
    bt.update(ents)
    torch.cuda.synchronize()
    F = field()
    for s in (0, 1, 100, 255):
        lo, hi = (s * 4099) % (nbytes - 65536), (s * 4099) % (nbytes - 65536) + 65536
        d = old[s, :, lo:hi].cpu().numpy().copy()
        d[int(changed[s])] ^= delta[s, lo:hi].cpu().numpy()
        assert np.array_equal(par[s, :, lo:hi].cpu().numpy(), oracle.encode(F, k, m, d)), s


# Register-held split-nibble update (rs_poly_update_nibble): the same parity
# as the LDS-table kernels, for 1 or 2 changed blocks with changed * m <= 8.
# Block strides are multiples of 16 so every block is 16-byte aligned; the
# sizes cover a tail-only block (B < 16), one chunk plus a tail, several
# grid strides with a ragged tail, and m above 4.
NIBBLE = [(10, 4, 100003, [3]), (10, 4, 100003, [0, 9]), (10, 4, 15, [5]), (10, 4, 17, [1, 2]),
          (10, 4, 16, [7]), (6, 6, 65551, [2]), (32, 8, 70001, [31]), (3, 7, 333, [1]),
          (6, 3, 8191, [1, 4]), (12, 2, 4097, [0, 11]), (8, 1, 1000, [3, 5]), (1, 1, 1, [0]),
          (13, 1, 999, [12]), (247, 8, 4112, [100])]


def _aligned_pad(nbytes, extra=16):
    return (-nbytes) % 16 + extra


@pytest.mark.parametrize("k,m,nbytes,changed", NIBBLE)
def test_nibble_update_matches_oracle(k, m, nbytes, changed):
    say(f"nibble update k={k} m={m} B={nbytes} changed={changed}")
    case = UpdateCase(k, m, nbytes, changed, seed=k * 37 + m * 5 + nbytes,
                      pad=_aligned_pad(nbytes))
    assert case.stride % 16 == 0
    B.Code(k, m).update_nibble(case.delta_ptrs(), case.parity_ptrs(), nbytes)
    torch.cuda.synchronize()
    case.check()


def test_nibble_update_gf16():
    say("nibble update GF(2^4)")
    for (k, m, changed) in ((4, 3, [0]), (9, 5, [3]), (12, 3, [0, 11]), (7, 4, [2, 6])):
        case = UpdateCase(k, m, 777, changed, seed=k * 11 + m, w=4, poly=0x13,
                          pad=_aligned_pad(777))
        B.Code(k, m, 4, 0x13).update_nibble(case.delta_ptrs(), case.parity_ptrs(), 777)
        torch.cuda.synchronize()
        case.check()


def test_nibble_update_twice_restores_parity():
    say("nibble update twice")
    case = UpdateCase(10, 4, 1 << 16, [1, 8], seed=43)
    code = B.Code(10, 4)
    for _ in range(2):
        code.update_nibble(case.delta_ptrs(), case.parity_ptrs(), 1 << 16)
    torch.cuda.synchronize()
    case.check(want=case.parity0)


@pytest.mark.parametrize("k,m,changed", [(10, 4, [2, 7]), (10, 4, [9]), (32, 8, [0])])
def test_nibble_update_large_blocks_equal_the_lds_update(k, m, changed):
    # 4 MiB + 48-byte blocks: many grid-stride rounds; the result equals the
    # oracle's encoding of the new data and, byte for byte, what the
    # LDS-table update makes of the same delta from the same parity
    nbytes = (4 << 20) + 48
    say(f"nibble update large RS({k},{m}) changed={changed}")
    case = UpdateCase(k, m, nbytes, changed, seed=700 + k + len(changed), pad=256 - 48)
    ref = case.pbuf.clone()
    code = B.Code(k, m)
    code.update_nibble(case.delta_ptrs(), case.parity_ptrs(), nbytes)
    base = ref.data_ptr() + case.offset
    code.update(case.delta_ptrs(), [base + i * case.stride for i in range(m)], nbytes)
    torch.cuda.synchronize()
    assert torch.equal(case.pbuf, ref)
    case.check()


def test_nibble_update_rejects_beyond_its_limits():
    case = UpdateCase(10, 4, 4096, [0, 1, 2], seed=44)
    code = B.Code(10, 4)
    with pytest.raises(B.RsPolyError) as ei:
        code.update_nibble(case.delta_ptrs(), case.parity_ptrs(), 4096)
    assert ei.value.code == B.RS_EINVAL
    torch.cuda.synchronize()
    case.check(want=case.parity0)     # nothing was touched
