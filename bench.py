#!/usr/bin/env python3
"""Throughput of batched polynomial RS encode + erasure decode on one MI355X.

Workload (the headline configuration): RS(10,4) over GF(2^8) (field
polynomial 0x11D, roots alpha^0..alpha^3), 256 stripes x 10 data blocks x
1 MiB of uniform random bytes (2.5 GiB of data) resident in HBM.  One step =
one batched encode of all 256 stripes + one batched decode of all 256
stripes, each with 1-4 uniformly random erased blocks (one persistent,
graph-replayed launch each).  `value` is user data per second: k * B bytes
per stripe, counted once for the encode and once for the decode.

Also reported: the plain one-launch-per-stripe path on the same buffers, the
dominant kernel against the HBM roofline (algorithmic bytes per launch /
launch time from HIP events on the launch stream), and the CPU oracle timed
on a bounded sample of the same stripes on this host.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
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
K, M, STRIPES, BLOCK = 10, 4, 256, 1 << 20


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("codec.hip", "rs_internal.h"):
        with open(os.path.join(ROOT, "paper_1312_5155_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, src_hash, variant):
    """HBM bytes per launch from the committed counter summary, or None if
    it is missing, was taken on other kernel sources, or on another kernel
    variant than the one this run launched."""
    path = os.path.join(ROOT, "profiles", "traffic_rs104_256x1MiB.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != src_hash:
        return None
    entry = rec.get("kernels", {}).get(kernel, {})
    if entry.get("kernel") != variant:
        return None
    return entry.get("hbm_bytes_per_launch")


def batch_variant(op, launch, m=4, matrix_update=False, k=10):
    """Name of the batch kernel template a launch shape runs (state width 4
    for m <= 4), as the profiler prints it.  An update of at most 8 changed
    blocks per stripe runs the generator-matrix form (mode 3), which has no
    table-placement variants; an encode with the bit-sliced placement runs
    bitmatrix_batch_kernel<k, m> (the workloads that time it use one code)."""
    if op == 2 and matrix_update:
        mode = 3
    elif op == 0 and launch["table_placement"] == 2:
        return f"bitmatrix_batch_kernel<{k}, {m}>"
    else:
        mode = op + (4 if launch["table_placement"] == 1 else 0)
    return f"batch_kernel<{4 if m <= 4 else 8}, {launch['bytes_per_lane'] // 4}, {mode}>"


CALIB_BYTES = 1 << 30       # size of the copy that calibrates the counters
# bench.py arguments of the counter runs (timed steps only, no serving)
PMC_BENCH_ARGS = ("--steps 3 --warmup 1 --plain-steps 0 --cpu-sample 0 --serving-requests 0 "
                  "--bitmatrix-steps 0")


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
    """Mean counter value per kernel name (first 60 chars) from a rocprofv3
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


def traffic_summary(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, out_path):
    """Writes the per-launch HBM bytes of the batch kernels: the FETCH_SIZE
    and WRITE_SIZE means (KiB per dispatch), each scaled so that the
    calibration copy reads and writes exactly CALIB_BYTES."""
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
    variants = [(label, f"batch_kernel<4, {w}, {op + tp}>")
                for label, op in (("batch_encode", 0), ("batch_decode", 1), ("batch_update", 2),
                                  ("batch_update", 3))
                for w in (4, 2, 1) for tp in ((0, 4) if op < 3 else (0,))]
    for label, key in variants:
        fv = [v for n, (v, c) in fetch.items() if key in n]
        wv = [v for n, (v, c) in write.items() if key in n]
        if not fv or not wv:
            continue
        fb, wb = fv[0] * 1024.0 * f_scale, wv[0] * 1024.0 * w_scale
        kernels[label] = {"kernel": key, "fetch_kib_raw": fv[0], "write_kib_raw": wv[0],
                          "fetch_bytes": round(fb), "write_bytes": round(wb),
                          "hbm_bytes_per_launch": round(fb + wb)}
    cmd = "rocprofv3 --pmc {c} -d <out> -o run --output-format csv -- python3 bench.py {a}"
    rec = {"workload": "rs104_256x1MiB", "kernel_source_hash": kernel_source_hash(),
           "commands": [cmd.format(c=c, a=a) for c in ("FETCH_SIZE", "WRITE_SIZE") for a in (
               PMC_BENCH_ARGS, "--calibrate-copy")] +
           ["python3 bench.py --traffic-from <FETCH csv> <WRITE csv> <calibration FETCH csv> "
            "<calibration WRITE csv>"],
           "note": "counter values are KiB per dispatch; each is scaled by what it reads for "
                   "the 1 GiB calibration copy (__amd_rocclr_copyBuffer)",
           "calibration": {"copy_bytes": CALIB_BYTES, "fetch_kib_raw": cf, "write_kib_raw": cw,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec), flush=True)


def serving_run(srv, sets, trace, times):
    """Replays one trace and returns (makespan s, latencies us, user bytes)."""
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
    after = srv.stats()
    serving_run.last = {k: round(after[k] - before[k], 1) for k in
                        ("batches", "launch_host_us", "batch_device_us", "admit_host_us")}
    serving_run.last["span_us"] = round(span * 1e6, 1)
    return span, lat, user


def serving(fractions, count):
    """Serving workload: RS(10,4), requests of log-uniform 64 KiB-64 MiB of
    data (70% encodes, 30% degraded reads with 1-4 erasures) on resident
    stripes, admitted under a 64 GiB HBM budget.  Capacity is measured with a
    backlog (every request arriving at t=0); then a Poisson trace at each
    fraction of it.  GB/s counts user data bytes (the request sizes)."""
    import numpy as np

    import workloads
    from paper_1312_5155_amd import binding as B
    from paper_1312_5155_amd.serving import ResidentSets

    cfg = workloads.CONFIGS["serving_rs104"]
    seed = workloads.meta_seed(cfg["index"])
    k, m = cfg["k"], cfg["m"]
    n_sets = 24
    code = B.Code(k, m)
    sets = ResidentSets(code, n_sets, -(-cfg["max_request"] // k),
                        seed=workloads.data_seed(cfg["index"]))
    srv = B.Serve(cfg["hbm_budget"], streams=4, max_batch=64, auto_release=True,
                  max_block_bytes=-(-cfg["max_request"] // k))

    def trace(s, rate):
        return workloads.serving_trace(s, count, k, m, cfg["min_request"], cfg["max_request"],
                                       cfg["encode_frac"], rate, n_sets)

    tr, tm = trace(seed, None)
    serving_run(srv, sets, tr[:2000], tm[:2000])        # warm-up (graphs, plans)
    # capacity: the better of two backlog runs (every request at t = 0)
    runs = [serving_run(srv, sets, tr, tm) for _ in range(2)]
    span, lat, user = min(runs, key=lambda r: r[0])
    cap_rps = count / span
    out = {"capacity": {"req_s": round(cap_rps), "gbs": round(user / span / 1e9, 1),
                        "p50_us": round(float(np.percentile(lat, 50)), 1),
                        "p99_us": round(float(np.percentile(lat, 99)), 1),
                        **serving_run.last},
           "points": []}
    for i, f in enumerate(fractions):
        tr, tm = trace(seed + 1 + i, f * cap_rps)
        span, lat, user = serving_run(srv, sets, tr, tm)
        out["points"].append({"load": f, "offered_req_s": round(f * cap_rps),
                              "gbs": round(user / span / 1e9, 1),
                              "p50_us": round(float(np.percentile(lat, 50)), 1),
                              "p99_us": round(float(np.percentile(lat, 99)), 1),
                              **serving_run.last})
    st = srv.stats()
    out.update({"requests_per_point": count, "streams": 4, "max_batch": 64,
                "hbm_budget_bytes": cfg["hbm_budget"], "budget_peak_bytes": st["budget_peak"],
                "peak_inflight_batches": st["peak_inflight_batches"]})
    srv.close()
    return out


def cpu_baseline(host_stripes, erasures, threads):
    """The oracle, unchanged, on a bounded sample: encode then decode of each
    sampled stripe; stripes run in parallel threads (ctypes drops the GIL).
    Returns (GB/s of user data, seconds, the oracle's parity per stripe)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    F = oracle.Field(8, 0x11D)

    def one(i):
        data = host_stripes[i]
        par = oracle.encode(F, K, M, data)
        full = np.concatenate([data, par])
        full[erasures[i]] = 0
        oracle.decode(F, K, M, full, erasures[i])
        return par

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parity = list(ex.map(one, range(len(host_stripes))))
    dt = time.perf_counter() - t0
    user = 2 * len(host_stripes) * K * BLOCK
    return user / dt / 1e9, dt, parity


def bitmatrix_compare(dev, stream, steps):
    """Plain (one launch) encode of one RS(10,4) stripe of 64 MiB blocks:
    the LFSR kernel against the bit-sliced XOR-only kernel, same buffers;
    the two parities must be identical."""
    import torch

    import workloads
    from paper_1312_5155_amd import binding as B
    nb = 64 << 20
    code = B.Code(K, M)
    gen = torch.Generator(device=dev)
    gen.manual_seed(workloads.data_seed(3))
    data = torch.randint(0, 256, (K, nb), dtype=torch.uint8, device=dev, generator=gen)
    par = torch.zeros((2, M, nb), dtype=torch.uint8, device=dev)
    dptr = [data[j].data_ptr() for j in range(K)]
    runs = {"lfsr": lambda: B.rs_poly_encode(code.handle, dptr,
                                             [par[0, i].data_ptr() for i in range(M)], nb, stream),
            "bitmatrix": lambda: B.rs_poly_encode_bitmatrix(
                code.handle, dptr, [par[1, i].data_ptr() for i in range(M)], nb, stream)}
    out = {"workload": "RS(10,4) one stripe, 64 MiB blocks, plain launch",
           "alg_bytes": (K + M) * nb}
    for name, fn in runs.items():
        for _ in range(5):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        ms = median([a.elapsed_time(b) for a, b in ev])
        out[name] = {"median_ms": round(ms, 4), "gbs": round((K + M) * nb / (ms / 1e3) / 1e9, 1)}
    if not torch.equal(par[0], par[1]):
        raise SystemExit("bit-matrix parity differs from the LFSR parity")
    out["identical"] = True
    del data, par
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def copy_roof(dev):
    """GB/s of a plain device copy of 1 GiB (torch copy_, the runtime's
    copy kernel): the streaming rate this part reaches without any coding
    work, a practical roof beside the 8 TB/s peak."""
    import torch
    src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device=dev)
    src.fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del src, dst
    torch.cuda.empty_cache()
    return 2 * CALIB_BYTES / (ms / 1e3) / 1e9


def build_workload(name, dev):
    """Device arena, per-stripe (k, m, B, block pointers) and decode erasure
    lists of a parity workload: the mixed uneven batch or RS(32,8)."""
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
    return buf, stripes, erasures


def other_workload(name, args):
    """Batched (and plain) encode + decode of another workload; one JSON line
    with each kernel's time, algorithmic HBM bytes and fraction of peak."""
    import torch

    from paper_1312_5155_amd import binding as B
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    buf, stripes, erasures = build_workload(name, dev)
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
    for _ in range(args.warmup):
        batch.encode(enc, stream)
        batch.decode(dec, stream)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        batch.encode(enc, stream)
        ev[i][1].record(stream)
        batch.decode(dec, stream)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    enc_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
    dec_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps
    user = sum(k * nb for (k, m, nb, _) in stripes)
    enc_alg = sum((k + m) * nb for (k, m, nb, _) in stripes)
    dec_alg = sum((k + len(e)) * nb for (k, m, nb, _), e in zip(stripes, erasures))

    plain = None
    if args.plain_steps > 0:
        def plain_step():
            for (k, m, nb, p) in stripes:
                B.rs_poly_encode(codes[(k, m)].handle, p[:k], p[k:], nb, stream)
            for (k, m, nb, p), e in zip(stripes, erasures):
                B.rs_poly_decode(codes[(k, m)].handle, p, nb, e, 0, stream)
        plain_step()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - p0) * 1e3 / args.plain_steps
        plain = {"ms_per_step": round(plain_ms, 3),
                 "value": round(2 * user / (plain_ms / 1e3) / 1e9, 1),
                 "launches_per_step": 2 * len(stripes)}

    def kern(ms, alg):
        gbs = alg / (ms / 1e3) / 1e9
        return {"avg_ms": round(ms, 4), "alg_bytes": alg, "gbs": round(gbs, 1),
                "frac": round(gbs / HBM_PEAK_GBS, 4), "user_gbs": round(user / (ms / 1e3) / 1e9, 1)}

    out = {"workload": name, "stripes": len(stripes), "user_bytes": user,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "value": round(2 * user / (ms_per_step / 1e3) / 1e9, 1), "unit": "GB/s",
           "kernels": {"batch_encode": kern(enc_ms, enc_alg), "batch_decode": kern(dec_ms, dec_alg)},
           "launch": {"encode": [batch.get_launch(B.RS_POLY_OP_ENCODE, w).as_dict() for w in (0, 1)],
                      "decode": [batch.get_launch(B.RS_POLY_OP_DECODE, w).as_dict() for w in (0, 1)]},
           "plain": plain}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30,
                    help="untimed steps first (the clocks settle over the first tens)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--bitmatrix-steps", type=int, default=20,
                    help="timed launches of the plain LFSR and bit-matrix encodes of one "
                         "RS(10,4) stripe of 64 MiB blocks (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=48,
                    help="stripes the CPU oracle encodes+decodes (0 = skip)")
    ap.add_argument("--update-steps", type=int, default=10,
                    help="timed batched delta-parity updates (one changed block per "
                         "stripe; rounded up to even so the parity ends unchanged)")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on this workload before timing")
    ap.add_argument("--serving-requests", type=int, default=10000,
                    help="requests per serving load point (0 = skip serving)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only the serving workload, at 0.1..1.2 of capacity")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the known-size copy used to scale HBM counters")
    ap.add_argument("--traffic-from", nargs=4, metavar="CSV",
                    help="FETCH, WRITE, calibration FETCH, calibration WRITE "
                         "counter_collection.csv files -> profiles/ traffic JSON")
    ap.add_argument("--workload", default="rs104_256x1MiB",
                    choices=["rs104_256x1MiB", "mixed_4096_uneven", "rs328_64x16MiB"],
                    help="the headline workload, or another one measured on its own "
                         "(encode + decode kernels, no CPU or serving legs)")
    args = ap.parse_args()

    if args.traffic_from:
        traffic_summary(*args.traffic_from,
                        os.path.join(ROOT, "profiles", "traffic_rs104_256x1MiB.json"))
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.serving_sweep:
        res = serving([0.1, 0.3, 0.5, 0.7, 0.8, 0.9, 1.0, 1.2], max(1, args.serving_requests))
        print(json.dumps({"workload": "serving_rs104", **res}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(stripes shard across GPUs with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "rs104_256x1MiB":
        other_workload(args.workload, args)
        return

    import torch

    import workloads
    from paper_1312_5155_amd import binding as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # Stripes resident in HBM: (stripe, block, byte).
    buf = torch.empty((STRIPES, K + M, BLOCK), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(workloads.data_seed(1))
    for s in range(STRIPES):
        buf[s, :K] = torch.randint(0, 256, (K, BLOCK), dtype=torch.uint8, device=dev,
                                   generator=gen)
    rng = workloads.meta_rng(workloads.meta_seed(1))
    erasures = []
    for s in range(STRIPES):
        t = int(rng.integers(1, M + 1))
        erasures.append(workloads.random_erasures(rng, K + M, t))

    code = B.Code(K, M)
    ptrs = [[buf[s, b].data_ptr() for b in range(K + M)] for s in range(STRIPES)]
    enc = B.StripeArray([(code, ptrs[s], BLOCK) for s in range(STRIPES)])
    dec = B.StripeArray([(code, ptrs[s], BLOCK, erasures[s], 0) for s in range(STRIPES)])
    batch = B.Batch()
    if args.tune:
        batch.tune(B.RS_POLY_OP_ENCODE, enc, stream)
        batch.tune(B.RS_POLY_OP_DECODE, dec, stream)

    def step():
        batch.encode(enc, stream)
        batch.decode(dec, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        batch.encode(enc, stream)
        ev[i][1].record(stream)
        batch.decode(dec, stream)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_all = sorted(e[0].elapsed_time(e[1]) for e in ev)
    dec_all = sorted(e[1].elapsed_time(e[2]) for e in ev)
    enc_ms = sum(enc_all) / args.steps
    dec_ms = sum(dec_all) / args.steps
    ms_per_step = wall * 1e3 / args.steps

    user_per_op = STRIPES * K * BLOCK
    enc_alg = STRIPES * (K + M) * BLOCK                          # read k, write m
    dec_alg = sum((K + len(e)) * BLOCK for e in erasures)         # read k, write t
    value = 2 * user_per_op / (ms_per_step / 1e3) / 1e9

    # Plain: one launch per stripe, same buffers and patterns.
    def plain_step():
        for s in range(STRIPES):
            B.rs_poly_encode(code.handle, ptrs[s][:K], ptrs[s][K:], BLOCK, stream)
        for s in range(STRIPES):
            B.rs_poly_decode(code.handle, ptrs[s], BLOCK, erasures[s], 0, stream)

    plain = None
    if args.plain_steps > 0:
        plain_step()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - p0) * 1e3 / args.plain_steps
        plain = {"ms_per_step": round(plain_ms, 4),
                 "value": round(2 * user_per_op / (plain_ms / 1e3) / 1e9, 1),
                 "launches_per_step": 2 * STRIPES}

    # Delta-parity update (Sec. 3.2 update property), a small write: one
    # changed data block per stripe; reads the delta and the parity, writes
    # the parity.  An even number of runs leaves the parity as it was.
    update = None
    n_upd = args.update_steps + (args.update_steps & 1)
    if n_upd > 0:
        delta = torch.randint(0, 256, (STRIPES, BLOCK), dtype=torch.uint8, device=dev,
                              generator=gen)
        changed = workloads.meta_rng(workloads.meta_seed(1) + 2).integers(0, K, size=STRIPES)
        upd_ents = []
        for s in range(STRIPES):
            p = [None] * K + ptrs[s][K:]
            p[int(changed[s])] = delta[s].data_ptr()
            upd_ents.append((code, p, BLOCK))
        upd = B.StripeArray(upd_ents)
        batch.update(upd, stream)
        batch.update(upd, stream)
        u0 = torch.cuda.Event(enable_timing=True)
        u1 = torch.cuda.Event(enable_timing=True)
        u0.record(stream)
        for _ in range(n_upd):
            batch.update(upd, stream)
        u1.record(stream)
        torch.cuda.synchronize()
        upd_ms = u0.elapsed_time(u1) / n_upd
        upd_alg = STRIPES * (1 + 2 * M) * BLOCK
        update = {"avg_ms": round(upd_ms, 4), "alg_bytes": upd_alg,
                  "gbs": round(upd_alg / (upd_ms / 1e3) / 1e9, 1),
                  "user_gbs": round(STRIPES * BLOCK / (upd_ms / 1e3) / 1e9, 1),
                  "changed_blocks_per_stripe": 1}
        del delta

    bitmatrix = None
    if args.bitmatrix_steps > 0:
        bitmatrix = bitmatrix_compare(dev, stream, args.bitmatrix_steps)
        # the batched encode above, again with the bit-sliced kernel
        saved = batch.get_launch(B.RS_POLY_OP_ENCODE, 0).as_dict()
        bm_launch = {"bytes_per_lane": 16, "threads": 256, "tile_bytes": 8192, "wgs_per_cu": 2,
                     "table_placement": B.RS_POLY_TABLES_BITMATRIX, "tile_order": 0}
        batch.set_launch(B.RS_POLY_OP_ENCODE, 0, bm_launch)
        ref = buf[:, K:].clone()
        for _ in range(args.warmup):
            batch.encode(enc, stream)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for a, b in ev:
            a.record(stream)
            batch.encode(enc, stream)
            b.record(stream)
        torch.cuda.synchronize()
        bm_ms = median([a.elapsed_time(b) for a, b in ev])
        if not torch.equal(buf[:, K:], ref):
            raise SystemExit("batched bit-matrix parity differs from the LFSR parity")
        del ref
        batch.set_launch(B.RS_POLY_OP_ENCODE, 0, saved)
        bitmatrix["batched"] = {"workload": "rs104_256x1MiB encode", "launch": bm_launch,
                                "median_ms": round(bm_ms, 4),
                                "gbs": round(enc_alg / (bm_ms / 1e3) / 1e9, 1),
                                "lfsr_median_ms": round(median(enc_all), 4)}

    # Self-consistency of the timed buffers (GPU path only): wiping stripe
    # 0's erased blocks and decoding again restores them.
    before = buf[0].clone()
    buf[0, erasures[0]] = 0
    B.rs_poly_decode(code.handle, ptrs[0], BLOCK, erasures[0], 0, stream)
    torch.cuda.synchronize()
    assert torch.equal(buf[0], before), "decode did not restore stripe 0"
    del before

    src_hash = kernel_source_hash()
    kernels = {
        "batch_encode": {"avg_ms": round(enc_ms, 4), "median_ms": round(median(enc_all), 4),
                         "alg_bytes": enc_alg, "gbs": round(enc_alg / (enc_ms / 1e3) / 1e9, 1)},
        "batch_decode": {"avg_ms": round(dec_ms, 4), "median_ms": round(median(dec_all), 4),
                         "alg_bytes": dec_alg, "gbs": round(dec_alg / (dec_ms / 1e3) / 1e9, 1)},
    }
    if update:
        kernels["batch_update"] = update
    ops = {"batch_encode": B.RS_POLY_OP_ENCODE, "batch_decode": B.RS_POLY_OP_DECODE,
           "batch_update": B.RS_POLY_OP_UPDATE}
    for label in kernels:
        variant = batch_variant(ops[label], batch.get_launch(ops[label], 0).as_dict(),
                                matrix_update=True)   # one changed block per stripe
        kernels[label]["kernel"] = variant
        kernels[label]["traffic"] = measured_traffic(label, src_hash, variant)
    dom = "batch_encode" if enc_ms >= dec_ms else "batch_decode"
    achieved = kernels[dom]["gbs"]
    traffic = kernels[dom]["traffic"]
    roof = copy_roof(dev)
    for label in kernels:
        kernels[label]["of_copy_roof"] = round(kernels[label]["gbs"] / roof, 3)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernels[dom]["kernel"], "op": dom,
                "alg_bytes_per_launch": kernels[dom]["alg_bytes"],
                "copy_roof_gbs": round(roof, 1)}

    cpu = None
    if args.cpu_sample > 0:
        n = min(args.cpu_sample, STRIPES)
        host = [buf[s, :K].cpu().numpy() for s in range(n)]
        threads = min(16, os.cpu_count() or 1)
        gbs, secs, want = cpu_baseline(host, erasures[:n], threads)
        # one core, on the first few of the same stripes
        n1 = min(3, n)
        gbs1, secs1, _ = cpu_baseline(host[:n1], erasures[:n1], 1)
        # the GPU's parity of the sampled stripes against the oracle's
        exact = all((buf[s, K:].cpu().numpy() == want[s]).all() for s in range(n))
        cpu = {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": f"{n} of the {STRIPES} stripes, encode + decode each "
                         f"({secs:.1f} s wall on {threads} threads)",
               "single_core": {"value": round(gbs1, 3), "sample": f"{n1} stripes, "
                               f"{secs1:.1f} s"},
               "cpu_model": cpu_model(),
               "gpu_parity_matches_oracle": bool(exact)}
        if not exact:
            raise SystemExit("GPU parity differs from the oracle on the CPU sample")

    serve = None
    if args.serving_requests > 0:
        del buf
        torch.cuda.empty_cache()
        serve = serving([0.8], args.serving_requests)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "rs104_256x1MiB",
                   "code": "RS(10,4) GF(2^8) poly 0x11D roots alpha^0..alpha^3",
                   "stripes": STRIPES, "block_bytes": BLOCK,
                   "step": "batched encode + batched decode, 1-4 random erasures per stripe"},
        "hbm_frac": round((enc_alg + dec_alg) / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kernels,
        "launch": {"encode": batch.get_launch(B.RS_POLY_OP_ENCODE, 0).as_dict(),
                   "decode": batch.get_launch(B.RS_POLY_OP_DECODE, 0).as_dict(),
                   "update": batch.get_launch(B.RS_POLY_OP_UPDATE, 0).as_dict()},
        "plain": plain,
        "bitmatrix": bitmatrix,
        "serving": serve,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
