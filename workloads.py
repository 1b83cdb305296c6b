"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers: stripe bytes, erasure patterns, block
sizes, codes and arrival times.  It holds none of the coding arithmetic, so
both the CPU oracle and the GPU library can take their inputs from it without
sharing any code.

The paper's workload is random bytes generated in memory before timing
(Sec. 5.1); every draw below is a pure function of its seed so that any
stripe or block can be regenerated on its own.
"""
import math

import numpy as np

# Base seed of the synthetic workloads; config i uses BASE_SEED + i for data
# bytes and BASE_SEED + i + 1000 for sizes, codes, erasures and arrivals.
BASE_SEED = 0x13125155

# The five workload shapes: small all-pattern check, RS(10,4) 256 x 1 MiB,
# 4096 mixed uneven stripes, a serving mix, and the wide RS(32,8) code.
CONFIGS = {
    "rs63_allpatterns": dict(index=0, k=6, m=3, stripes=1, block_bytes=64 << 10),
    "rs104_256x1MiB": dict(index=1, k=10, m=4, stripes=256, block_bytes=1 << 20),
    "mixed_4096_uneven": dict(index=2, stripes=4096, codes=((6, 3), (10, 4), (12, 4)),
                              min_bytes=4 << 10, max_bytes=4 << 20),
    "serving_rs104": dict(index=3, k=10, m=4, min_request=64 << 10,
                          max_request=64 << 20, encode_frac=0.7,
                          hbm_budget=64 << 30),
    "rs328_64x16MiB": dict(index=4, k=32, m=8, stripes=64, block_bytes=16 << 20),
}


def data_seed(cfg_index):
    return BASE_SEED + cfg_index


def meta_seed(cfg_index):
    return BASE_SEED + cfg_index + 1000


def block_bytes_rng(seed, stripe, block, nbytes):
    """Uniform random bytes of one block, addressed by (seed, stripe, block)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stripe, block])))
    return np.frombuffer(rng.bytes(nbytes), dtype=np.uint8).copy()


def stripe_data(seed, stripe, k, nbytes):
    """(k, nbytes) uint8 data blocks of one stripe."""
    out = np.empty((k, nbytes), dtype=np.uint8)
    for j in range(k):
        out[j] = block_bytes_rng(seed, stripe, j, nbytes)
    return out


def random_bytes(seed, shape):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(np.prod(shape))
    return np.frombuffer(rng.bytes(n), dtype=np.uint8).reshape(shape).copy()


def meta_rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_erasures(rng, n, t):
    """A uniform t-subset of the n API block indices, in random order."""
    return [int(x) for x in rng.choice(n, size=t, replace=False)]


def log_uniform_sizes(rng, count, lo, hi):
    """floor(exp(U[ln lo, ln hi])) bytes: not rounded, so tails occur."""
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.minimum(np.floor(np.exp(u)).astype(np.int64), hi)


def poisson_arrivals(rng, rate_per_s, count):
    """Arrival times in seconds of a Poisson process of the given rate."""
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


def all_patterns(n, max_t):
    """Every erasure list of size 0..max_t over n blocks (sorted indices)."""
    from itertools import combinations
    out = []
    for t in range(max_t + 1):
        out.extend(list(c) for c in combinations(range(n), t))
    return out


def device_random_blocks(torch, seed, count, nbytes, device="cuda"):
    """count x nbytes uniform random bytes drawn on the device by torch's
    seeded generator (fast for multi-GiB stripes); returns a uint8 tensor."""
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return torch.randint(0, 256, (count, nbytes), dtype=torch.uint8,
                         device=device, generator=gen)


def serving_trace(seed, count, k, m, min_request, max_request, encode_frac, rate_per_s,
                  n_sets):
    """Request mix of the serving workload: op (encode with probability
    encode_frac, else a degraded-read decode), data size S log-uniform in
    [min_request, max_request] (block size ceil(S/k)), which resident set it
    uses, 1..m erased blocks for decodes, and Poisson arrival times in
    microseconds (all zero when rate_per_s is None: a backlog)."""
    rng = meta_rng(seed)
    sizes = log_uniform_sizes(rng, count, min_request, max_request)
    ops = (rng.random(count) >= encode_frac).astype(int)   # 0 encode, 1 decode
    sets = rng.integers(0, n_sets, size=count)
    out = []
    for i in range(count):
        s = int(sizes[i])
        er = []
        if ops[i] == 1:
            er = random_erasures(rng, k + m, int(rng.integers(1, m + 1)))
        out.append({"op": int(ops[i]), "data_bytes": s, "block_bytes": -(-s // k),
                    "set": int(sets[i]), "erasures": er})
    if rate_per_s is None:
        times = np.zeros(count)
    else:
        times = poisson_arrivals(rng, rate_per_s, count) * 1e6
    return out, times
