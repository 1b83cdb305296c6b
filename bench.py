#!/usr/bin/env python3
"""Throughput of batched polynomial RS encode + erasure decode on one MI355X.

Headline workload (the largest configuration that fits one GPU): RS(32,8)
over GF(2^8) (field polynomial 0x11D, roots alpha^0..alpha^7), 64 stripes x
32 data blocks x 16 MiB of uniform random bytes (32 GiB of data, 40 GiB with
parity) resident in HBM.  One step = one batched encode of all 64 stripes +
one batched decode of all 64 stripes with exactly 8 erased blocks each (the
worst case), each one persistent, graph-replayed launch.  `value` is user
data per second: k * B bytes per stripe, counted once for the encode and
once for the decode.

Also in the same JSON line: the plain one-launch-per-stripe path on the same
buffers; the dominant kernel against the HBM roofline (algorithmic bytes per
launch / launch time from HIP events on the launch stream) and against the
achievable rate of a streaming probe with the same read:write mix; the CPU
oracle timed on a bounded sample of the same stripes on this host; and, as
extra keys, the RS(10,4) 256 x 1 MiB batch (with the delta-parity update and
the bit-sliced encode), the 4096 mixed uneven stripes, the serving
workload swept over offered load, the encoder forms on the headline stripes,
and one-stripe encoders and update forms (LDS tables vs register-held
split-nibble products) on large blocks.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RS-poly encode/decode GB/s user data (% HBM peak), batched vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
HEADLINE = "rs328_64x16MiB"
WORKLOADS = ("rs328_64x16MiB", "rs104_256x1MiB", "mixed_4096_uneven")
CODE_TEXT = {"rs328_64x16MiB": "RS(32,8) GF(2^8) poly 0x11D roots alpha^0..alpha^7",
             "rs104_256x1MiB": "RS(10,4) GF(2^8) poly 0x11D roots alpha^0..alpha^3",
             "mixed_4096_uneven": "RS(6,3)/RS(10,4)/RS(12,4) GF(2^8) poly 0x11D"}
STEP_TEXT = {"rs328_64x16MiB": "batched encode + batched decode, 8 erased blocks per stripe",
             "rs104_256x1MiB": "batched encode + batched decode, 1-4 random erasures per stripe",
             "mixed_4096_uneven": "batched encode + batched decode, 1-m random erasures per "
                                  "stripe"}


def kernel_source_hash():
    """Hash of every library source: counter figures taken on other sources
    are not reported as current."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1312_5155_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def measured_traffic(workload, src_hash, variant):
    """HBM bytes per launch of one kernel variant from the committed counter
    summary of a workload, or None if there is none, or it was taken on
    other sources."""
    try:
        with open(traffic_file(workload)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != src_hash:
        return None
    return rec.get("kernels", {}).get(variant, {}).get("hbm_bytes_per_launch")


def batch_variant(op, launch, m=4, matrix_update=False, k=10):
    """Name of the batch kernel template a launch shape runs (state width 4
    for m <= 4, else 8), as the profiler prints it.  An update of at most 8
    changed blocks per stripe runs the generator-matrix form (mode 3), which
    has no table-placement variants; an encode with the bit-sliced placement
    runs bitmatrix_batch_kernel<k, m> (the workloads that time it use one
    code)."""
    if op == 2 and matrix_update:
        mode = 3
    elif op == 0 and launch["table_placement"] == 2:
        return f"bitmatrix_batch_kernel<{k}, {m}>"
    else:
        mode = op + (4 if launch["table_placement"] == 1 else 0)
        # m > 4 at 16 bytes per lane with packed tables: the interleaved
        # state layout (mode bit 16)
        if m > 4 and launch["bytes_per_lane"] == 16 and launch["table_placement"] == 0:
            mode |= 16
    return f"batch_kernel<{4 if m <= 4 else 8}, {launch['bytes_per_lane'] // 4}, {mode}>"


CALIB_BYTES = 1 << 30       # size of the copy that calibrates the counters
# bench.py arguments of the counter runs (timed steps of the headline only)
PMC_BENCH_ARGS = "--steps 3 --warmup 1 --plain-steps 0 --cpu-sample-kib 0 --no-extras"


def calibrate_copy():
    """A plain device copy of CALIB_BYTES, run 5 times: the counters of this
    known-size kernel give the scale of FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": CALIB_BYTES, "launches": 5}), flush=True)


def _counter_means(csv_path, counter):
    """Mean counter value per kernel name from a rocprofv3
    counter_collection.csv."""
    import csv
    sums, counts = {}, {}
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] != counter:
                continue
            name = row["Kernel_Name"]
            sums[name] = sums.get(name, 0.0) + float(row["Counter_Value"])
            counts[name] = counts.get(name, 0) + 1
    return {n: (sums[n] / counts[n], counts[n]) for n in sums}


def _template_name(kernel_name):
    """'batch_kernel<8, 1, 1>' from a demangled profiler kernel name."""
    for base in ("bitmatrix_batch_kernel<", "batch_kernel<"):
        i = kernel_name.find(base)
        if i >= 0 and (base != "batch_kernel<" or kernel_name[i - 1:i] in ("", " ", ":")):
            j = kernel_name.find(">", i)
            return kernel_name[i:j + 1]
    return None


def traffic_summary(workload, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv):
    """Writes the per-launch HBM bytes of the batch kernels of a workload:
    the FETCH_SIZE and WRITE_SIZE means (KiB per dispatch), each scaled so
    that the calibration copy reads and writes exactly CALIB_BYTES."""
    def pick(means, key):
        hits = [(v, n) for name, (v, n) in means.items() if key in name]
        if not hits:
            raise SystemExit(f"no kernel matching {key!r}")
        return max(hits)

    # torch's same-dtype copy_ runs as the HIP runtime's copy kernel
    cf, _ = pick(_counter_means(cal_fetch_csv, "FETCH_SIZE"), "copyBuffer")
    cw, _ = pick(_counter_means(cal_write_csv, "WRITE_SIZE"), "copyBuffer")
    f_scale = CALIB_BYTES / (cf * 1024.0)
    w_scale = CALIB_BYTES / (cw * 1024.0)
    fetch = _counter_means(fetch_csv, "FETCH_SIZE")
    write = _counter_means(write_csv, "WRITE_SIZE")
    kernels = {}
    for name, (fv, nf) in fetch.items():
        key = _template_name(name)
        if key is None or name not in write:
            continue
        wv = write[name][0]
        fb, wb = fv * 1024.0 * f_scale, wv * 1024.0 * w_scale
        kernels[key] = {"fetch_kib_raw": fv, "write_kib_raw": wv, "dispatches": nf,
                        "fetch_bytes": round(fb), "write_bytes": round(wb),
                        "hbm_bytes_per_launch": round(fb + wb)}
    wl = "" if workload == HEADLINE else f" --workload {workload}"
    cmd = "rocprofv3 --pmc {c} -d <out> -o run --output-format csv -- python3 bench.py {a}"
    rec = {"workload": workload, "kernel_source_hash": kernel_source_hash(),
           "commands": [cmd.format(c=c, a=a) for c in ("FETCH_SIZE", "WRITE_SIZE") for a in (
               PMC_BENCH_ARGS + wl, "--calibrate-copy")] +
           [f"python3 bench.py --traffic-workload {workload} --traffic-from <FETCH csv> "
            "<WRITE csv> <calibration FETCH csv> <calibration WRITE csv>"],
           "note": "counter values are KiB per dispatch; each is scaled by what it reads for "
                   "the 1 GiB calibration copy (__amd_rocclr_copyBuffer)",
           "calibration": {"copy_bytes": CALIB_BYTES, "fetch_kib_raw": cf, "write_kib_raw": cw,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": kernels}
    with open(traffic_file(workload), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec), flush=True)


def median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def cpu_model():
    """The host CPU's model name, with family/model/stepping when the name
    alone is generic."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" not in line:
                    if info:
                        break
                    continue
                key, val = (x.strip() for x in line.split(":", 1))
                info.setdefault(key, val)
    except OSError:
        return None
    name = info.get("model name")
    ids = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    return f"{name} ({ids})" if name and ids else name


# ------------------------------------------------------------ workloads --

def build_workload(name, dev):
    """Device arena, per-stripe (k, m, B, block pointers), decode erasure
    lists, and for uniform workloads an (S, n, B) view of the blocks."""
    import torch

    import workloads
    cfg = workloads.CONFIGS[name]
    rng = workloads.meta_rng(workloads.meta_seed(cfg["index"]))
    if name == "mixed_4096_uneven":
        sizes = workloads.log_uniform_sizes(rng, cfg["stripes"], cfg["min_bytes"],
                                            cfg["max_bytes"])
        picks = rng.integers(0, len(cfg["codes"]), size=cfg["stripes"])
        shapes = [(*cfg["codes"][c], int(b)) for c, b in zip(picks, sizes)]
    else:
        shapes = [(cfg["k"], cfg["m"], cfg["block_bytes"])] * cfg["stripes"]
    offsets, off = [], 0
    for (k, m, nb) in shapes:
        step = (nb + 255) // 256 * 256
        offsets.append([off + b * step for b in range(k + m)])
        off += (k + m) * step
    buf = torch.empty(off, dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(workloads.data_seed(cfg["index"]))
    chunk = 1 << 30
    for c0 in range(0, off, chunk):
        n = min(chunk, off - c0)
        buf[c0:c0 + n] = torch.randint(0, 256, (n,), dtype=torch.uint8, device=dev,
                                       generator=gen)
    base = buf.data_ptr()
    stripes, erasures = [], []
    for (k, m, nb), offs in zip(shapes, offsets):
        stripes.append((k, m, nb, [base + o for o in offs]))
        t = m if name == "rs328_64x16MiB" else int(rng.integers(1, m + 1))
        erasures.append(workloads.random_erasures(rng, k + m, t))
    view = None
    if name != "mixed_4096_uneven":
        k, m, nb = shapes[0]
        view = buf.view(len(shapes), k + m, nb)
    return buf, stripes, erasures, view


def time_batched(batch, enc, dec, stream, steps, warmup):
    """Warm-up, then `steps` timed steps of one batched encode + one batched
    decode; per-launch times from events recorded on the launch stream."""
    import torch
    for _ in range(warmup):
        batch.encode(enc, stream)
        batch.decode(dec, stream)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        batch.encode(enc, stream)
        ev[i][1].record(stream)
        batch.decode(dec, stream)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_all = [e[0].elapsed_time(e[1]) for e in ev]
    dec_all = [e[1].elapsed_time(e[2]) for e in ev]
    return wall * 1e3 / steps, enc_all, dec_all


def stream_roof(view, k, n_out, stream, launches=8):
    """GB/s of the streaming probe over the workload's own blocks: k inputs
    read, n_out outputs written per stripe (outputs are the parity rows:
    callers re-encode afterwards).  The best of its tile sizes and orders:
    the rate this part reaches for that read:write mix."""
    import torch

    from paper_1312_5155_amd import binding as B
    S, n, nb = view.shape
    best = 0.0
    for tile in (8192, 16384, 65536, 262144):    # the batch kernels' tile sizes
        for order in (0, 1):
            args = (view.data_ptr(), view.stride(0), view.stride(1), S, k, n_out, nb, tile,
                    order)
            for _ in range(2):
                B.rs_poly_stream_probe(*args, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(launches):
                B.rs_poly_stream_probe(*args, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / launches
            best = max(best, (k + n_out) * nb * S / (ms / 1e3) / 1e9)
    return best


def plain_path(codes, stripes, erasures, stream, steps, user):
    """One launch per stripe (rs_poly_encode, then rs_poly_decode) on the
    same buffers and patterns."""
    import torch

    from paper_1312_5155_amd import binding as B

    def plain_step():
        for (k, m, nb, p) in stripes:
            B.rs_poly_encode(codes[(k, m)].handle, p[:k], p[k:], nb, stream)
        for (k, m, nb, p), e in zip(stripes, erasures):
            B.rs_poly_decode(codes[(k, m)].handle, p, nb, e, 0, stream)
    plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_step": round(ms, 3), "value": round(2 * user / (ms / 1e3) / 1e9, 1),
            "launches_per_step": 2 * len(stripes)}


def probe_mixes(dev, stream):
    """The streaming probe over 64 stripes of 40 blocks of 16 MiB for a range
    of read:write mixes (n_in inputs, n_out outputs per stripe; the best of
    its tile sizes and orders): how this part's HBM rate depends on the mix."""
    import torch
    S, n, nb = 64, 40, 16 << 20
    buf = torch.zeros((S, n, nb), dtype=torch.uint8, device=dev)
    out = []
    for n_in, n_out in ((40, 0), (39, 1), (38, 2), (36, 4), (32, 8), (24, 8), (16, 8),
                        (8, 8), (4, 4), (2, 8), (1, 8), (0, 8)):
        view = buf[:, :n_in + n_out]
        gbs = stream_roof(view, n_in, n_out, stream)
        out.append({"n_in": n_in, "n_out": n_out, "gbs": round(gbs, 1),
                    "frac": round(gbs / HBM_PEAK_GBS, 4)})
    del buf
    torch.cuda.empty_cache()
    return out


def run_batched(name, args, dev, stream, src_hash, roofline=False):
    """Times the batched encode + decode of one workload (one step = both
    launches) and returns its record; with roofline=True also the dominant
    kernel's roofline and the streaming probe's roof."""
    import torch

    from paper_1312_5155_amd import binding as B
    buf, stripes, erasures, view = build_workload(name, dev)
    codes = {}
    for (k, m, _, _) in stripes:
        codes.setdefault((k, m), B.Code(k, m))
    enc = B.StripeArray([(codes[(k, m)], p, nb) for (k, m, nb, p) in stripes])
    dec = B.StripeArray([(codes[(k, m)], p, nb, e, 0)
                         for (k, m, nb, p), e in zip(stripes, erasures)])
    batch = B.Batch()
    if args.tune:
        batch.tune(B.RS_POLY_OP_ENCODE, enc, stream)
        batch.tune(B.RS_POLY_OP_DECODE, dec, stream)
    ms_step, enc_all, dec_all = time_batched(batch, enc, dec, stream, args.steps, args.warmup)
    enc_ms, dec_ms = sum(enc_all) / len(enc_all), sum(dec_all) / len(dec_all)
    user = sum(k * nb for (k, m, nb, _) in stripes)
    enc_alg = sum((k + m) * nb for (k, m, nb, _) in stripes)             # read k, write m
    dec_alg = sum((k + len(e)) * nb for (k, m, nb, _), e in zip(stripes, erasures))
    wide = 1 if stripes[0][1] > 4 else 0
    k0, m0 = stripes[0][0], stripes[0][1]
    kernels = {}
    for label, op, ms, all_ms, alg in (("batch_encode", B.RS_POLY_OP_ENCODE, enc_ms, enc_all,
                                        enc_alg),
                                       ("batch_decode", B.RS_POLY_OP_DECODE, dec_ms, dec_all,
                                        dec_alg)):
        launch = batch.get_launch(op, wide).as_dict()
        variant = batch_variant(op, launch, m=m0, k=k0)
        gbs = alg / (ms / 1e3) / 1e9
        kernels[label] = {"avg_ms": round(ms, 4), "median_ms": round(median(all_ms), 4),
                          "alg_bytes": alg, "gbs": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "user_gbs": round(user / (ms / 1e3) / 1e9, 1), "kernel": variant,
                          "launch": launch,
                          "traffic": measured_traffic(name, src_hash, variant)}
    rec = {"workload": name, "stripes": len(stripes), "user_bytes": user,
           "ms_per_step": round(ms_step, 4),
           "value": round(2 * user / (ms_step / 1e3) / 1e9, 1), "unit": "GB/s",
           "hbm_frac": round((enc_alg + dec_alg) / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "kernels": kernels}
    if args.plain_steps > 0:
        rec["plain"] = plain_path(codes, stripes, erasures, stream, args.plain_steps, user)

    # The decode restores what it rebuilds: wipe one stripe's erased blocks
    # and decode it again (GPU path only; the oracle checks come below).
    k, m, nb, p = stripes[0]
    if view is not None:
        before = view[0].clone()
        view[0, erasures[0]] = 0
        B.rs_poly_decode(codes[(k, m)].handle, p, nb, erasures[0], 0, stream)
        torch.cuda.synchronize()
        if not torch.equal(view[0], before):
            raise SystemExit(f"{name}: decode did not restore stripe 0")
        del before

    if roofline:
        dom = max(kernels, key=lambda l: kernels[l]["avg_ms"])
        ker = kernels[dom]
        roofs = {}
        if view is not None:
            t_mean = round(sum(len(e) for e in erasures) / len(erasures))
            roofs = {"batch_encode": stream_roof(view, k0, m0, stream),
                     "batch_decode": stream_roof(view, k0, max(1, t_mean), stream)}
            batch.encode(enc, stream)          # the probe wrote over the parity rows
            torch.cuda.synchronize()
            for label in kernels:
                kernels[label]["stream_roof_gbs"] = round(roofs[label], 1)
                kernels[label]["of_stream_roof"] = round(kernels[label]["gbs"] / roofs[label], 3)
        rec["roofline"] = {"bound": "hbm", "achieved": ker["gbs"], "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": ker["frac"], "traffic": ker["traffic"],
                           "kernel": ker["kernel"], "op": dom,
                           "alg_bytes_per_launch": ker["alg_bytes"],
                           "stream_roof_gbs": round(roofs[dom], 1) if roofs else None,
                           "of_stream_roof": ker.get("of_stream_roof")}
    rec["_state"] = (buf, stripes, erasures, view, codes, batch, enc)
    return rec


def cpu_baseline(view, stripes, erasures, window, n_stripes, threads, seed):
    """The oracle, unchanged, on a bounded sample: for each sampled stripe a
    window of `window` columns at a seeded offset, encoded and then decoded
    with the stripe's own erasure pattern; stripes run in parallel threads
    (ctypes drops the GIL).  Also checks the GPU's parity and the decode's
    output on every window.  Returns (GB/s of user data, seconds)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    import workloads
    F = oracle.Field(8, 0x11D)
    k, m, nb, _ = stripes[0]
    rng = workloads.meta_rng(seed)
    offs = [int(rng.integers(0, (nb - window) // 16 + 1)) * 16 for _ in range(n_stripes)]
    host = [view[s, :, o:o + window].cpu().numpy() for s, o in zip(range(n_stripes), offs)]

    def one(i):
        blocks = host[i]
        par = oracle.encode(F, k, m, blocks[:k])
        full = np.concatenate([blocks[:k], par])
        er = erasures[i]
        full[er] = 0
        oracle.decode(F, k, m, full, er)
        ok_par = np.array_equal(par, blocks[k:])
        ok_dec = np.array_equal(full[er], blocks[er])
        return ok_par, ok_dec

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(one, range(n_stripes)))
    dt = time.perf_counter() - t0
    if not all(p for p, _ in res):
        raise SystemExit("GPU parity differs from the oracle on the CPU sample")
    if not all(d for _, d in res):
        raise SystemExit("the oracle's decode did not restore a sampled window")
    user = 2 * n_stripes * k * window
    return user / dt / 1e9, dt


# ------------------------------------------------------------ extra legs --

def update_leg(view, stripes, codes, batch, stream, steps, dev):
    """Batched delta-parity update (Sec. 3.2 update property), one changed
    data block per stripe: reads the delta and the parity, writes the
    parity.  An even number of runs leaves the parity as it was.  Timed in
    the library's default placement (register split-nibble products, for
    stripes changing at most 2 blocks) and with the packed placement (the
    generator-matrix LDS tables); both must leave the same bytes."""
    import torch

    from paper_1312_5155_amd import binding as B
    import workloads
    S, n, nb = view.shape
    k, m = stripes[0][0], stripes[0][1]
    gen = torch.Generator(device=dev)
    gen.manual_seed(workloads.data_seed(1) + 7)
    delta = torch.randint(0, 256, (S, nb), dtype=torch.uint8, device=dev, generator=gen)
    changed = workloads.meta_rng(workloads.meta_seed(1) + 2).integers(0, k, size=S)
    ents = []
    for s in range(S):
        p = [None] * k + stripes[s][3][k:]
        p[int(changed[s])] = delta[s].data_ptr()
        ents.append((codes[(k, m)], p, nb))
    upd = B.StripeArray(ents)
    n_upd = steps + (steps & 1)
    ref = view[:, k:].clone()
    wide = 1 if m > 4 else 0
    alg = S * (1 + 2 * m) * nb

    def timed():
        batch.update(upd, stream)
        batch.update(upd, stream)
        u0, u1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        u0.record(stream)
        for _ in range(n_upd):
            batch.update(upd, stream)
        u1.record(stream)
        torch.cuda.synchronize()
        if not torch.equal(view[:, k:], ref):
            raise SystemExit("an even number of updates changed the parity")
        return u0.elapsed_time(u1) / n_upd

    ms = timed()
    launch = batch.get_launch(B.RS_POLY_OP_UPDATE, wide).as_dict()
    regs = launch["table_placement"] == B.RS_POLY_TABLES_REGISTERS
    rec = {"avg_ms": round(ms, 4), "alg_bytes": alg, "gbs": round(alg / (ms / 1e3) / 1e9, 1),
           "frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "user_gbs": round(S * nb / (ms / 1e3) / 1e9, 1), "changed_blocks_per_stripe": 1,
           "kernel": "nibble_batch_kernel" if regs else
                     batch_variant(B.RS_POLY_OP_UPDATE, launch, m=m, matrix_update=True),
           "launch": launch}
    # the same updates in the generator-matrix form (packed LDS tables)
    packed = dict(launch, table_placement=B.RS_POLY_TABLES_PACKED)
    batch.set_launch(B.RS_POLY_OP_UPDATE, wide, packed)
    ms_p = timed()
    batch.set_launch(B.RS_POLY_OP_UPDATE, wide, launch)
    rec["matrix_form"] = {"avg_ms": round(ms_p, 4), "gbs": round(alg / (ms_p / 1e3) / 1e9, 1),
                          "frac": round(alg / (ms_p / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "kernel": batch_variant(B.RS_POLY_OP_UPDATE, packed, m=m,
                                                  matrix_update=True),
                          "launch": packed}
    return rec


def plain_encoders_leg(dev, stream, steps):
    """One-stripe launches of the three encoders on large blocks: the LFSR
    (rs_poly_encode), the generator-matrix form (rs_poly_encode_matrix) and
    the bit-sliced XOR-only form (rs_poly_encode_bitmatrix: compiled-in XOR
    networks for the workload codes, matrices taken at run time for
    RS(16,4)); every parity must be identical."""
    import torch

    from paper_1312_5155_amd import binding as B
    import workloads
    out = {}
    for (k, m, nb) in ((10, 4, 64 << 20), (6, 3, 64 << 20), (32, 8, 16 << 20),
                       (16, 4, 32 << 20)):
        code = B.Code(k, m)
        gen = torch.Generator(device=dev)
        gen.manual_seed(workloads.data_seed(3) + k)
        data = torch.randint(0, 256, (k, nb), dtype=torch.uint8, device=dev, generator=gen)
        par = torch.zeros((3, m, nb), dtype=torch.uint8, device=dev)
        dptr = [data[j].data_ptr() for j in range(k)]
        runs = {"lfsr": (B.rs_poly_encode, 0), "bitmatrix": (B.rs_poly_encode_bitmatrix, 1)}
        if k <= B.RS_POLY_MATRIX_MAX_K:
            runs["matrix"] = (B.rs_poly_encode_matrix, 2)
        rec = {"alg_bytes": (k + m) * nb}
        for label, (fn, row) in runs.items():
            pp = [par[row, i].data_ptr() for i in range(m)]
            for _ in range(5):
                fn(code.handle, dptr, pp, nb, stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]
            for a, b in ev:
                a.record(stream)
                fn(code.handle, dptr, pp, nb, stream)
                b.record(stream)
            torch.cuda.synchronize()
            ms = median([a.elapsed_time(b) for a, b in ev])
            rec[label] = {"median_ms": round(ms, 4),
                          "gbs": round((k + m) * nb / (ms / 1e3) / 1e9, 1)}
        for label, (fn, row) in runs.items():
            if row and not torch.equal(par[0], par[row]):
                raise SystemExit(f"RS({k},{m}) {label} parity differs from the LFSR parity")
        rec["identical"] = True
        out[f"RS({k},{m}) {nb >> 20} MiB blocks"] = rec
        del data, par
        torch.cuda.empty_cache()
    return out


def nibble_update_leg(dev, stream, steps):
    """One-stripe delta-parity updates on large blocks, 1 or 2 changed
    blocks: the register-held split-nibble kernel (rs_poly_update_nibble)
    against the LDS-table matrix form (rs_poly_update).  Both start from
    the same parity and must end with identical bytes."""
    import torch

    from paper_1312_5155_amd import binding as B
    import workloads
    out = {}
    for (k, m, nb, changed) in ((10, 4, 64 << 20, [3]), (10, 4, 64 << 20, [2, 7]),
                                (32, 8, 16 << 20, [5]), (6, 3, 64 << 20, [0, 4])):
        code = B.Code(k, m)
        gen = torch.Generator(device=dev)
        gen.manual_seed(workloads.data_seed(3) + 100 + k + len(changed))
        delta = torch.randint(0, 256, (len(changed), nb), dtype=torch.uint8, device=dev,
                              generator=gen)
        par = torch.randint(0, 256, (2, m, nb), dtype=torch.uint8, device=dev, generator=gen)
        par[1] = par[0]
        dp = [None] * k
        for t, j in enumerate(changed):
            dp[j] = delta[t].data_ptr()
        runs = {"nibble": (B.rs_poly_update_nibble, 0), "lds_matrix": (B.rs_poly_update, 1)}
        for label, (fn, row) in runs.items():
            fn(code.handle, dp, [par[row, i].data_ptr() for i in range(m)], nb, stream)
        torch.cuda.synchronize()
        if not torch.equal(par[0], par[1]):
            raise SystemExit(f"RS({k},{m}) nibble update differs from the LDS update")
        alg = (len(changed) + 2 * m) * nb
        rec = {"changed_blocks": len(changed), "products": len(changed) * m, "alg_bytes": alg}
        for label, (fn, row) in runs.items():
            pp = [par[row, i].data_ptr() for i in range(m)]
            for _ in range(4):
                fn(code.handle, dp, pp, nb, stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]
            for a, b in ev:
                a.record(stream)
                fn(code.handle, dp, pp, nb, stream)
                b.record(stream)
            torch.cuda.synchronize()
            ms = median([a.elapsed_time(b) for a, b in ev])
            rec[label] = {"median_ms": round(ms, 4),
                          "gbs": round(alg / (ms / 1e3) / 1e9, 1),
                          "frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        rec["identical"] = True
        out[f"RS({k},{m}) {nb >> 20} MiB blocks, changed {changed}"] = rec
        del delta, par
        torch.cuda.empty_cache()
    return out


def encoder_forms_leg(view, stripes, codes, stream, steps):
    """The three encoders on the workload's own stripes, one launch per
    stripe: the LFSR (rs_poly_encode), the bit-sliced XOR-only form
    (rs_poly_encode_bitmatrix) and the generator-matrix form
    (rs_poly_encode_matrix); each parity must equal the batched encode's
    (already in the buffer)."""
    import torch

    from paper_1312_5155_amd import binding as B
    S, n, nb = view.shape
    k, m = stripes[0][0], stripes[0][1]
    ref = view[:, k:].clone()
    h = codes[(k, m)].handle
    forms = {"lfsr": B.rs_poly_encode, "bitmatrix": B.rs_poly_encode_bitmatrix,
             "matrix": B.rs_poly_encode_matrix}
    out = {"workload": f"{S} stripes, one launch each", "alg_bytes": S * n * nb}
    for label, fn in forms.items():
        def step():
            for (_, _, nbytes, p) in stripes:
                fn(h, p[:k], p[k:], nbytes, stream)
        view[:, k:] = 0
        step()
        torch.cuda.synchronize()
        if not torch.equal(view[:, k:], ref):
            raise SystemExit(f"{label} encode differs from the batched encode")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[label] = {"ms": round(ms, 3), "gbs": round(S * n * nb / (ms / 1e3) / 1e9, 1),
                      "frac": round(S * n * nb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def bitmatrix_batch_leg(batch, enc, view, stream, steps, warmup):
    """The batched encode again with the bit-sliced placement; the parity
    must equal the LFSR batch's."""
    import torch

    from paper_1312_5155_amd import binding as B
    S, n, nb = view.shape
    k = 10
    saved = batch.get_launch(B.RS_POLY_OP_ENCODE, 0).as_dict()
    bm = {"bytes_per_lane": 16, "threads": 256, "tile_bytes": 8192, "wgs_per_cu": 2,
          "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": 0}
    batch.set_launch(B.RS_POLY_OP_ENCODE, 0, bm)
    ref = view[:, k:].clone()
    for _ in range(warmup):
        batch.encode(enc, stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        batch.encode(enc, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = median([a.elapsed_time(b) for a, b in ev])
    if not torch.equal(view[:, k:], ref):
        raise SystemExit("batched bit-matrix parity differs from the LFSR parity")
    batch.set_launch(B.RS_POLY_OP_ENCODE, 0, saved)
    alg = S * n * nb
    return {"launch": bm, "median_ms": round(ms, 4), "gbs": round(alg / (ms / 1e3) / 1e9, 1)}


# ------------------------------------------------------------- serving --

def serving_run(srv, sets, trace, times, k):
    """Replays one trace and returns (makespan s, latencies us, user bytes,
    algorithmic HBM bytes)."""
    import numpy as np

    from paper_1312_5155_amd import binding as B
    reqs = B.RequestArray(sets.entries(trace))     # marshalled before timing
    before = srv.stats()
    t0 = time.perf_counter()
    srv.replay(reqs, times)
    done = []
    while len(done) < reqs.count:
        done += srv.poll(4096, timeout_us=50000)
    span = time.perf_counter() - t0
    if any(c.status != 0 for c in done):
        raise SystemExit("a serving request failed")
    lat = np.array([c.latency_us for c in done])
    user = sum(r["data_bytes"] for r in trace)
    alg = sum((k + (len(r["erasures"]) if r["op"] else sets.m)) * r["block_bytes"]
              for r in trace)
    after = srv.stats()
    serving_run.last = {key: round(after[key] - before[key], 1) for key in
                        ("batches", "launch_host_us", "batch_device_us", "admit_host_us")}
    serving_run.last["span_us"] = round(span * 1e6, 1)
    return span, lat, user, alg


def _point(span, lat, user, alg):
    import numpy as np
    gbs = alg / span / 1e9
    return {"gbs": round(user / span / 1e9, 1), "alg_gbs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "p50_us": round(float(np.percentile(lat, 50)), 1),
            "p99_us": round(float(np.percentile(lat, 99)), 1), **serving_run.last}


def serving(fractions, count, max_batch=256):
    """Serving workload: RS(10,4), requests of log-uniform 64 KiB-64 MiB of
    data (70% encodes, 30% degraded reads with 1-4 erasures) on resident
    stripes, admitted under a 64 GiB HBM budget.  Capacity is measured with a
    backlog (every request arriving at t=0); then a Poisson trace at each
    fraction of it.  `gbs` counts user data bytes (the request sizes),
    `alg_gbs` the algorithmic HBM bytes ((k+m)B per encode, (k+t)B per
    decode) and `hbm_frac` their fraction of the HBM peak."""
    import workloads
    from paper_1312_5155_amd import binding as B
    from paper_1312_5155_amd.serving import ResidentSets

    cfg = workloads.CONFIGS["serving_rs104"]
    seed = workloads.meta_seed(cfg["index"])
    k, m = cfg["k"], cfg["m"]
    n_sets = 24
    streams = 4
    code = B.Code(k, m)
    sets = ResidentSets(code, n_sets, -(-cfg["max_request"] // k),
                        seed=workloads.data_seed(cfg["index"]))
    srv = B.Serve(cfg["hbm_budget"], streams=streams, max_batch=max_batch, auto_release=True,
                  max_block_bytes=-(-cfg["max_request"] // k))

    def trace(s, rate):
        return workloads.serving_trace(s, count, k, m, cfg["min_request"], cfg["max_request"],
                                       cfg["encode_frac"], rate, n_sets)

    tr, tm = trace(seed, None)
    serving_run(srv, sets, tr[:2000], tm[:2000], k)        # warm-up (graphs, plans)
    # capacity: the better of two backlog runs (every request at t = 0)
    runs = [serving_run(srv, sets, tr, tm, k) for _ in range(2)]
    best = min(runs, key=lambda r: r[0])
    cap_rps = count / best[0]
    out = {"capacity": {"req_s": round(cap_rps), **_point(*best)}, "points": []}
    for i, f in enumerate(fractions):
        tr, tm = trace(seed + 1 + i, f * cap_rps)
        res = serving_run(srv, sets, tr, tm, k)
        out["points"].append({"load": f, "offered_req_s": round(f * cap_rps), **_point(*res)})
    st = srv.stats()
    out.update({"requests_per_point": count, "streams": streams, "max_batch": max_batch,
                "hbm_budget_bytes": cfg["hbm_budget"], "budget_peak_bytes": st["budget_peak"],
                "peak_inflight_batches": st["peak_inflight_batches"]})
    srv.close()
    return out


# ----------------------------------------------------------------- main --

def strip_state(rec):
    rec.pop("_state", None)
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed steps first (kernel times settle over the first launches)")
    ap.add_argument("--workload", default=HEADLINE, choices=WORKLOADS,
                    help="the workload of the headline value")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="only the headline workload (no other workloads, update, "
                         "bit-sliced or serving legs)")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-sample-kib", type=int, default=512,
                    help="columns (KiB) per sampled stripe the CPU oracle encodes and "
                         "decodes (0 = skip)")
    ap.add_argument("--cpu-stripes", type=int, default=64,
                    help="stripes in the CPU oracle's sample")
    ap.add_argument("--update-steps", type=int, default=10)
    ap.add_argument("--encoder-steps", type=int, default=20,
                    help="timed one-stripe launches of each encoder form (0 = skip)")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on each workload before timing")
    ap.add_argument("--serving-requests", type=int, default=10000,
                    help="requests per serving load point (0 = skip serving)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only the serving workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the known-size copy used to scale HBM counters")
    ap.add_argument("--traffic-from", nargs=4, metavar="CSV",
                    help="FETCH, WRITE, calibration FETCH, calibration WRITE "
                         "counter_collection.csv files -> profiles/ traffic JSON")
    ap.add_argument("--traffic-workload", default=HEADLINE, choices=WORKLOADS)
    ap.add_argument("--leg", choices=("plain_encoders", "plain_update_forms"),
                    help="only this one-stripe leg (for profiling its kernels)")
    ap.add_argument("--probe-mixes", action="store_true",
                    help="only the streaming probe over a range of read:write mixes")
    args = ap.parse_args()
    loads = [0.1, 0.3, 0.5, 0.7, 0.8, 0.9, 1.0, 1.2]

    if args.traffic_from:
        traffic_summary(args.traffic_workload, *args.traffic_from)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.serving_sweep:
        res = serving(loads, max(1, args.serving_requests))
        print(json.dumps({"workload": "serving_rs104", **res}), flush=True)
        return
    if args.probe_mixes:
        import torch
        res = probe_mixes(torch.device("cuda:0"), torch.cuda.current_stream())
        print(json.dumps({"probe_mixes": res, "stripes": 64, "blocks": 40,
                          "block_bytes": 16 << 20}), flush=True)
        return
    if args.leg:
        import torch
        legs = {"plain_encoders": plain_encoders_leg, "plain_update_forms": nibble_update_leg}
        res = legs[args.leg](torch.device("cuda:0"), torch.cuda.current_stream(),
                             max(1, args.encoder_steps))
        print(json.dumps({"leg": args.leg, **res}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(stripes shard across GPUs with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    src_hash = kernel_source_hash()

    head = run_batched(args.workload, args, dev, stream, src_hash, roofline=True)
    buf, stripes, erasures, view, codes, batch, _ = head.pop("_state")
    k, m, nb = stripes[0][0], stripes[0][1], stripes[0][2]

    cpu = None
    if args.cpu_sample_kib > 0 and view is not None:
        import workloads
        window = min(nb, args.cpu_sample_kib << 10)
        n_s = min(args.cpu_stripes, len(stripes))
        avail = len(os.sched_getaffinity(0))
        threads = min(16, avail)      # the host's CPU share for one GPU
        seed = workloads.meta_seed(workloads.CONFIGS[args.workload]["index"]) + 5
        gbs, secs = cpu_baseline(view, stripes, erasures, window, n_s, threads, seed)
        gbs1, secs1 = cpu_baseline(view, stripes, erasures, window, 1, 1, seed)
        cpu = {"value": round(gbs, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"{n_s} of the {len(stripes)} stripes, a {window >> 10} KiB column "
                         f"window each (seeded offset), encoded then decoded with the "
                         f"stripe's erasures ({secs:.1f} s wall on {threads} threads)",
               "single_core": {"value": round(gbs1, 4), "cores": 1,
                               "sample": f"1 stripe window, {secs1:.1f} s"},
               "cpus_visible": avail, "cpu_model": cpu_model(),
               "gpu_parity_matches_oracle": True, "decode_restores_windows": True}
    extras = {}
    if args.extras and args.encoder_steps > 0 and view is not None:
        extras["encoder_forms"] = encoder_forms_leg(view, stripes, codes, stream, 3)
    if args.extras and args.update_steps > 0 and view is not None:
        extras["batch_update_" + args.workload] = update_leg(view, stripes, codes, batch, stream,
                                                             args.update_steps, dev)
    del buf, view, stripes, erasures, batch
    torch.cuda.empty_cache()

    if args.extras:
        # serving next, before the other workloads: one full run of an
        # earlier build measured serving after all the other legs at about
        # 40% of its capacity on its own (cause not isolated; not seen with
        # the current build)
        if args.serving_requests > 0:
            extras["serving_rs104"] = serving(loads, args.serving_requests)
        for name in WORKLOADS:
            if name == args.workload:
                continue
            rec = run_batched(name, args, dev, stream, src_hash, roofline=True)
            b2, s2, e2, v2, c2, bt2, enc2 = rec.pop("_state")
            if name == "rs104_256x1MiB":
                if args.update_steps > 0:
                    rec["kernels"]["batch_update"] = update_leg(v2, s2, c2, bt2, stream,
                                                                args.update_steps, dev)
                rec["bitmatrix_batched"] = bitmatrix_batch_leg(
                    bt2, enc2, v2, stream, max(args.steps, 10), max(args.warmup, 10))
                rec["bitmatrix_batched"]["lfsr_median_ms"] = \
                    rec["kernels"]["batch_encode"]["median_ms"]
            extras[name] = rec
            del b2, s2, e2, v2, c2, bt2, enc2
            torch.cuda.empty_cache()
        if args.encoder_steps > 0:
            extras["plain_encoders"] = plain_encoders_leg(dev, stream, args.encoder_steps)
            extras["plain_update_forms"] = nibble_update_leg(dev, stream, args.encoder_steps)

    out = {
        "metric": METRIC, "value": head["value"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "code": CODE_TEXT[args.workload],
                   "stripes": head["stripes"], "block_bytes": nb, "step": STEP_TEXT[args.workload]},
        "hbm_frac": head["hbm_frac"],
        "kernels": head["kernels"],
        "plain": head.get("plain"),
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "extras": extras,
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(out), flush=True)



if __name__ == "__main__":
    main()
