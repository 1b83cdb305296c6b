"""Resident stripe sets for the serving engine and request building.

Serving requests read caller-resident device data: encodes read k data
blocks, degraded reads (decodes) read the surviving blocks of an encoded
stripe.  `ResidentSets` holds `n_sets` stripes of n blocks x max_block bytes
in one device tensor, filled with seeded random data and encoded once with
the batch API, so any prefix of B bytes of every block is a valid stripe
(byte columns are independent codewords).  Requests of a trace use the first
block_bytes of the set they name.
"""
import torch

from . import binding as B


class ResidentSets:
    def __init__(self, code, n_sets, max_block_bytes, seed, device="cuda"):
        self.code = code
        self.k, self.m, self.n = code.k, code.m, code.n
        self.stride = (max_block_bytes + 255) // 256 * 256
        self.buf = torch.empty((n_sets, self.n, self.stride), dtype=torch.uint8, device=device)
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        for s in range(n_sets):
            self.buf[s, :self.k] = torch.randint(0, 256, (self.k, self.stride), dtype=torch.uint8,
                                                 device=device, generator=gen)
        batch = B.Batch()
        batch.encode([(code, self.ptrs(s), self.stride) for s in range(n_sets)])
        torch.cuda.synchronize()
        batch.close()

    def ptrs(self, s):
        return [self.buf[s, b].data_ptr() for b in range(self.n)]

    def entries(self, trace):
        """Serving request entries (see binding.RequestArray) of a trace made
        by workloads.serving_trace."""
        out = []
        for i, r in enumerate(trace):
            e = {"op": r["op"], "code": self.code, "blocks": self.ptrs(r["set"]),
                 "block_bytes": r["block_bytes"], "tag": i}
            if r["op"] == B.RS_POLY_OP_DECODE:
                e["erasures"] = r["erasures"]
            out.append(e)
        return out
