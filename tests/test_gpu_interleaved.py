"""GPU parity of the interleaved-layout kernels (m > 4 at 16 bytes per lane,
the library's choice for 16-byte-aligned blocks of 4 MiB and more) for every
m from 5 to 8, over both fields: encode against the oracle on column windows
at both ends and in the middle of ragged blocks, decode of m erasures that
include the top data blocks (whose LFSR steps the kernel skips) and parity
blocks, and the LFSR-form update (more than 8 changed blocks) against the
oracle's encode of the new data."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = {8: 0x11D, 4: 0x13}
WINDOW = 24000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rows(t):
    return [t[i] for i in range(t.shape[0])]


def windows(Bn):
    return [(0, WINDOW), (Bn // 2 - 777, Bn // 2 - 777 + WINDOW), (Bn - WINDOW, Bn)]


CASES = [(3, 5, 8), (13, 6, 8), (9, 7, 8), (32, 8, 8), (21, 8, 8), (6, 6, 4), (7, 8, 4)]


@pytest.mark.parametrize("k,m,w", CASES)
def test_interleaved_encode_decode_update(k, m, w):
    Bn = (4 << 20) + 36
    say(f"interleaved RS({k},{m}) GF(2^{w}) B={Bn}")
    F = oracle.Field(w, FIELDS[w])
    code = B.Code(k, m, w, FIELDS[w])
    mask = (1 << w) - 1
    stride = (Bn + 255) // 256 * 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.data_seed(7) + 100 * k + 10 * m + w)
    buf = torch.zeros((k + m, stride), dtype=torch.uint8, device="cuda")
    buf[:k, :Bn] = torch.randint(0, mask + 1, (k, Bn), dtype=torch.uint8, device="cuda",
                                 generator=gen)
    assert buf[1].data_ptr() % 16 == 0
    code.encode(rows(buf[:k]), rows(buf[k:]), Bn)
    torch.cuda.synchronize()
    for c0, c1 in windows(Bn):
        want = oracle.encode(F, k, m, buf[:k, c0:c1].cpu().numpy())
        assert np.array_equal(buf[k:, c0:c1].cpu().numpy(), want), (k, m, w, c0)
    assert not buf[k:, Bn:].any()

    # m erasures: the top data block (and the one below it when k > 1), the
    # lowest parity block, the rest drawn at random
    er = {k - 1, k}
    if k > 1:
        er.add(k - 2)
    rng = workloads.meta_rng(31 * k + m + w)
    while len(er) < m:
        er.add(int(rng.integers(0, k + m)))
    er = sorted(er)
    for flags in (0, B.RS_POLY_FLAG_ALL_SURVIVORS):
        saved = buf[er].clone()
        buf[er] = 0x5A
        code.decode(rows(buf), er, Bn, flags)
        torch.cuda.synchronize()
        assert torch.equal(buf[er, :Bn], saved[:, :Bn]), (er, flags)

    # LFSR-form update: every data block but the top one changes (more than
    # 8 blocks when k > 9; fewer run the matrix form, also checked)
    changed = list(range(k - 1)) if k > 1 else [0]
    delta = torch.zeros((k, stride), dtype=torch.uint8, device="cuda")
    delta[changed, :Bn] = torch.randint(0, mask + 1, (len(changed), Bn), dtype=torch.uint8,
                                        device="cuda", generator=gen)
    code.update([delta[j] if j in changed else None for j in range(k)], rows(buf[k:]), Bn)
    torch.cuda.synchronize()
    new_data = buf[:k] ^ delta
    for c0, c1 in windows(Bn):
        want = oracle.encode(F, k, m, new_data[:, c0:c1].cpu().numpy())
        assert np.array_equal(buf[k:, c0:c1].cpu().numpy(), want), ("update", k, m, w, c0)
