"""GPU tests of the continuous-batching serving engine: results are the same
alone and in a concurrent mix (0-byte tolerance), match the oracle, admission
never exceeds the HBM budget, and every request of a Poisson trace
completes."""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads
from paper_1312_5155_amd import binding as B
from paper_1312_5155_amd.serving import ResidentSets

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K, M = 10, 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_trace(seed, count, rate=None, max_request=4 << 20):
    return workloads.serving_trace(seed, count, K, M, 64 << 10, max_request, 0.7, rate, 6)


def drain(srv, count, timeout_s=60):
    done = []
    t0 = time.time()
    while len(done) < count:
        done += srv.poll(256, timeout_us=20000)
        assert time.time() - t0 < timeout_s, f"only {len(done)} of {count} completed"
    return done


def outputs_of(c, nbytes):
    return [torch.tensor([], dtype=torch.uint8) if not c.out[r] else
            _dev_bytes(c.out[r], nbytes) for r in range(c.n_out)]


def _hip():
    import ctypes
    lib = ctypes.CDLL("libamdhip64.so.7")
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return lib


def _dev_tensor(ptr, nbytes):
    # a device copy of nbytes at ptr (device to device), as a torch tensor
    out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    assert _hip().hipMemcpy(out.data_ptr(), ptr, nbytes, 3) == 0
    return out


def _dev_bytes(ptr, nbytes):
    # copy nbytes of device memory at ptr to a host numpy array; opening the
    # runtime by its soname reuses the copy already loaded in the process
    import ctypes
    host = np.empty(nbytes, dtype=np.uint8)
    lib = ctypes.CDLL("libamdhip64.so.7")
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert lib.hipMemcpy(host.ctypes.data, ptr, nbytes, 2) == 0   # device to host
    return host


def test_results_identical_alone_and_in_the_mix():
    say("serve: alone vs mix")
    code = B.Code(K, M)
    trace, _ = small_trace(31, 60)
    sets = ResidentSets(code, 6, max(r["block_bytes"] for r in trace), seed=77)
    entries = sets.entries(trace)

    alone = {}
    srv = B.Serve(8 << 30, streams=1, max_batch=1, auto_release=False)
    for i, e in enumerate(entries):
        srv.submit(e)
        c = drain(srv, 1)[0]
        assert c.status == 0 and c.user_tag == i
        alone[i] = [o.copy() for o in outputs_of(c, e["block_bytes"])]
        srv.release(c.ticket)
    srv.close()

    srv = B.Serve(8 << 30, streams=4, max_batch=16, auto_release=False)
    times = np.linspace(0, 300, len(entries))      # all within 0.3 ms: they overlap
    srv.replay(entries, times)
    done = drain(srv, len(entries))
    st = srv.stats()
    assert st["batches"] < len(entries)             # requests really were batched
    assert st["peak_inflight_batches"] >= 2         # and batches ran at the same time
    for c in done:
        i = c.user_tag
        assert c.status == 0
        got = outputs_of(c, entries[i]["block_bytes"])
        assert len(got) == len(alone[i])
        for a, b in zip(got, alone[i]):
            assert np.array_equal(a, b), (i, trace[i])
        srv.release(c.ticket)
    srv.close()

    # and what they are: the oracle's parity / the lost blocks themselves
    F = oracle.Field(8, 0x11D)
    for i in range(0, len(trace), 7):
        r = trace[i]
        nb = r["block_bytes"]
        stripe = sets.buf[r["set"], :, :nb].cpu().numpy()
        if r["op"] == B.RS_POLY_OP_ENCODE:
            want = oracle.encode(F, K, M, stripe[:K])
            for p in range(M):
                assert np.array_equal(alone[i][p], want[p])
        else:
            for j, b in enumerate(sorted(r["erasures"])):
                assert np.array_equal(alone[i][j], stripe[b])


def test_admission_respects_the_budget():
    say("serve: budget")
    code = B.Code(K, M)
    trace, _ = small_trace(32, 80, max_request=4 << 20)
    sets = ResidentSets(code, 6, max(r["block_bytes"] for r in trace), seed=78)
    budget = 24 << 20          # a few requests at a time
    charges = [(K + (M if r["op"] == 0 else len(r["erasures"]))) * r["block_bytes"]
               for r in trace]
    keep = [i for i, c in enumerate(charges) if c <= budget]
    entries = [sets.entries(trace)[i] for i in keep]
    srv = B.Serve(budget, streams=4, max_batch=8, auto_release=True)
    srv.replay(entries, np.zeros(len(entries)))
    done = drain(srv, len(entries))
    st = srv.stats()
    assert all(c.status == 0 for c in done)
    assert st["completed"] == len(entries)
    assert 0 < st["budget_peak"] <= budget
    assert st["budget_in_use"] == 0
    srv.close()


def test_poisson_trace_completes_with_latencies():
    say("serve: poisson trace")
    code = B.Code(K, M)
    trace, times = small_trace(33, 3000, rate=20000.0, max_request=1 << 20)
    sets = ResidentSets(code, 6, max(r["block_bytes"] for r in trace), seed=79)
    srv = B.Serve(4 << 30, streams=4, max_batch=64, auto_release=True)
    srv.replay(sets.entries(trace), times)
    done = drain(srv, len(trace))
    lat = np.array([c.latency_us for c in done])
    q = np.array([c.queue_us for c in done])
    assert (lat > 0).all() and (q >= 0).all() and (q <= lat).all()
    assert sorted(c.user_tag for c in done) == list(range(len(trace)))
    st = srv.stats()
    assert st["peak_inflight_batches"] >= 1 and st["completed"] == len(trace)
    say(f"p50 {np.percentile(lat, 50):.0f} us p99 {np.percentile(lat, 99):.0f} us "
        f"batches {st['batches']}")
    srv.close()


def test_bad_requests_are_rejected():
    code = B.Code(K, M)
    sets = ResidentSets(code, 1, 4096, seed=80)
    srv = B.Serve(1 << 20, streams=1, max_batch=4)
    good = {"op": 0, "code": code, "blocks": sets.ptrs(0), "block_bytes": 4096}
    srv.submit(good)
    for bad, err in (({**good, "op": 5}, B.RS_EINVAL),
                     ({**good, "block_bytes": 0}, B.RS_EINVAL),
                     ({**good, "block_bytes": 1 << 20}, B.RS_EINVAL),   # over budget
                     ({**good, "op": 1, "erasures": []}, B.RS_EINVAL),
                     ({**good, "op": 1, "erasures": [0, 0]}, B.RS_ERANGE),
                     ({**good, "op": 1, "erasures": [0, 1, 2, 3, 4]}, B.RS_ETOOMANY)):
        with pytest.raises(B.RsPolyError) as ei:
            srv.submit(bad)
        assert ei.value.code == err
    assert len(drain(srv, 1)) == 1
    srv.close()


def test_serving_config_at_full_size():
    # The serving workload as the benchmark runs it: RS(10,4), requests of
    # log-uniform 64 KiB - 64 MiB of data, 70% encodes / 30% degraded reads
    # with 1-4 erasures on 24 resident sets, a 64 GiB budget, 4 streams,
    # batches of up to 64.  Every completion is checked before it is
    # released: a decode's outputs are the lost blocks themselves, an
    # encode's outputs equal the resident parity and match the oracle on a
    # seeded window of up to 64 KiB.
    say("serve: full-size serving config")
    cfg = workloads.CONFIGS["serving_rs104"]
    k, m = cfg["k"], cfg["m"]
    code = B.Code(k, m)
    max_block = -(-cfg["max_request"] // k)
    n_sets = 24
    sets = ResidentSets(code, n_sets, max_block, seed=workloads.data_seed(cfg["index"]))
    seed = workloads.meta_seed(cfg["index"]) + 50
    trace, _ = workloads.serving_trace(seed, 400, k, m, cfg["min_request"],
                                       cfg["max_request"], cfg["encode_frac"], None, n_sets)
    assert max(r["block_bytes"] for r in trace) > (32 << 20) // k    # large requests too
    srv = B.Serve(cfg["hbm_budget"], streams=4, max_batch=64, auto_release=False,
                  max_block_bytes=max_block)
    srv.replay(sets.entries(trace), np.zeros(len(trace)))
    F = oracle.Field(8, 0x11D)
    rng = workloads.meta_rng(seed + 1)
    seen = set()
    t0 = time.time()
    while len(seen) < len(trace):
        for c in srv.poll(64, timeout_us=20000):
            i = c.user_tag
            r = trace[i]
            nb = r["block_bytes"]
            assert c.status == 0 and i not in seen
            seen.add(i)
            res = sets.buf[r["set"]]
            if r["op"] == B.RS_POLY_OP_ENCODE:
                assert c.n_out == m
                outs = [_dev_tensor(c.out[p], nb) for p in range(m)]
                for p in range(m):
                    assert c.out_index[p] == k + p
                    assert torch.equal(outs[p], res[k + p, :nb]), (i, p)
                w = min(nb, 64 << 10)
                c0 = int(rng.integers(0, nb - w + 1))
                want = oracle.encode(F, k, m, res[:k, c0:c0 + w].cpu().numpy())
                got = np.stack([o[c0:c0 + w].cpu().numpy() for o in outs])
                assert np.array_equal(got, want), i
            else:
                lost = sorted(r["erasures"])
                assert c.n_out == len(lost)
                for j, b in enumerate(lost):
                    assert c.out_index[j] == b
                    assert torch.equal(_dev_tensor(c.out[j], nb), res[b, :nb]), (i, b)
            srv.release(c.ticket)
        assert time.time() - t0 < 240, f"only {len(seen)} of {len(trace)} completed"
    st = srv.stats()
    assert st["completed"] == len(trace) and st["budget_in_use"] == 0
    assert 0 < st["budget_peak"] <= cfg["hbm_budget"]
    srv.close()
