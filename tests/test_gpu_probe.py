"""GPU checks of the streaming probe (the achievable-bandwidth measurement
beside the codec kernels) and of the op-first names of the batch calls."""
import sys

import pytest

import workloads
from paper_1312_5155_amd import binding as B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("S,n_in,n_out,nb,tile", [
    (3, 10, 4, 3 * 4096 + 48, 4096),     # ragged last tile
    (2, 32, 8, 65536, 8192),
    (1, 1, 1, 16, 4096),
    (4, 9, 2, 1 << 20, 65536),
    (5, 3, 3, 1000 * 16, 4096),          # not a multiple of a wave's 2 KiB
    (2, 7, 0, 65536 + 32, 8192),         # reads only
    (3, 0, 5, 3 * 4096 + 48, 4096),      # writes only (zeros)
])
@pytest.mark.parametrize("order", [0, 1])
def test_stream_probe_writes_the_xor_of_its_inputs(S, n_in, n_out, nb, tile, order):
    say(f"probe S={S} in={n_in} out={n_out} B={nb} order={order}")
    bs = (nb + 255) // 256 * 256 + 256          # guard bytes after every block
    ss = (n_in + n_out) * bs + 256
    buf = workloads.device_random_blocks(torch, 91 + n_in, 1, S * ss)[0]
    ref = buf.clone()
    B.rs_poly_stream_probe(buf.data_ptr(), ss, bs, S, n_in, n_out, nb, tile, order)
    torch.cuda.synchronize()
    v, r = buf.view(S, ss), ref.view(S, ss)
    for s in range(S):
        x = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        for b in range(n_in):
            x ^= r[s, b * bs:b * bs + nb]
        for o in range(n_out):
            c0 = (n_in + o) * bs
            assert torch.equal(v[s, c0:c0 + nb], x), (s, o)
            # nothing past the block's end is written
            assert torch.equal(v[s, c0 + nb:c0 + bs], r[s, c0 + nb:c0 + bs])
        assert torch.equal(v[s, :n_in * bs], r[s, :n_in * bs])       # inputs untouched
        assert torch.equal(v[s, (n_in + n_out) * bs:], r[s, (n_in + n_out) * bs:])


def test_op_first_batch_names_match_the_batch_calls():
    say("rs_poly_encode_batch / rs_poly_decode_batch")
    k, m, nb, S = 10, 4, 65536 + 32, 6
    code = B.Code(k, m)
    buf = torch.zeros((2, S, k + m, nb), dtype=torch.uint8, device="cuda")
    buf[:, :, :k] = workloads.device_random_blocks(torch, 93, S * k, nb).view(S, k, nb)
    ents = [[(code, [buf[c, s, b].data_ptr() for b in range(k + m)], nb) for s in range(S)]
            for c in range(2)]
    bt = B.Batch()
    B.rs_poly_batch_encode(bt.handle, ents[0])
    B.rs_poly_encode_batch(bt.handle, ents[1])
    torch.cuda.synchronize()
    assert torch.equal(buf[0], buf[1])
    rng = workloads.meta_rng(94)
    ref = buf[1].clone()
    dents = []
    for s in range(S):
        er = workloads.random_erasures(rng, k + m, int(rng.integers(1, m + 1)))
        buf[1, s, er] = 0
        dents.append((code, [buf[1, s, b].data_ptr() for b in range(k + m)], nb, er, 0))
    B.rs_poly_decode_batch(bt.handle, dents)
    torch.cuda.synchronize()
    assert torch.equal(buf[1], ref)
