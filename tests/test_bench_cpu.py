"""CPU checks of bench.py's bookkeeping: the kernel names it derives from a
launch shape are kernels the library instantiates, and the committed HBM
traffic summaries were taken with the current library sources and cover the
kernels of each workload's default launches (otherwise the bench would report
`traffic` as null)."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1312_5155_amd", "librs_poly.so")

PACKED, NIBBLE, BITMATRIX = 0, 1, 2


def launch(bpl=16, placement=PACKED):
    return {"bytes_per_lane": bpl, "threads": 1024, "tile_bytes": 65536, "wgs_per_cu": 2,
            "table_placement": placement, "tile_order": 1}


@pytest.mark.parametrize("op,lc,m,matrix,name", [
    (0, launch(), 8, False, "batch_kernel<8, 4, 16>"),          # interleaved encode
    (1, launch(), 8, False, "batch_kernel<8, 4, 17>"),          # interleaved decode
    (2, launch(), 8, False, "batch_kernel<8, 4, 18>"),          # interleaved LFSR update
    (2, launch(), 8, True, "batch_kernel<8, 4, 3>"),            # matrix-form update
    (1, launch(placement=NIBBLE), 8, False, "batch_kernel<8, 4, 5>"),
    (1, launch(bpl=8), 8, False, "batch_kernel<8, 2, 1>"),
    (0, launch(), 4, False, "batch_kernel<4, 4, 0>"),
    (1, launch(bpl=4), 3, False, "batch_kernel<4, 1, 1>"),
    (0, launch(placement=BITMATRIX), 4, False, "bitmatrix_batch_kernel<10, 4>"),
])
def test_batch_variant_names(op, lc, m, matrix, name):
    assert bench.batch_variant(op, lc, m=m, matrix_update=matrix) == name


def mangled(name):
    """Itanium-mangled template arguments of a batch_kernel<a, b, c> name."""
    args = name[name.index("<") + 1:-1].split(", ")
    return "batch_kernelI" + "".join(f"Li{a}E" for a in args) + "E"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("name", ["batch_kernel<8, 4, 16>", "batch_kernel<8, 4, 17>",
                                  "batch_kernel<8, 4, 18>", "batch_kernel<8, 4, 3>",
                                  "batch_kernel<4, 4, 0>", "batch_kernel<4, 4, 1>"])
def test_named_kernels_are_in_the_library(name):
    with open(LIB, "rb") as fh:
        blob = fh.read()
    assert mangled(name).encode() in blob, name


@pytest.mark.parametrize("workload,m", [("rs328_64x16MiB", 8), ("rs104_256x1MiB", 4)])
def test_traffic_summaries_are_current(workload, m):
    with open(bench.traffic_file(workload)) as fh:
        rec = json.load(fh)
    assert rec["kernel_source_hash"] == bench.kernel_source_hash(), \
        "counter summary taken with other library sources: re-take FETCH_SIZE/WRITE_SIZE"
    # the kernels of the default encode and decode launches of this workload
    for op in (0, 1):
        wide = m > 4
        lc = launch() if wide else {"bytes_per_lane": 16, "threads": 512,
                                    "tile_bytes": 8192, "wgs_per_cu": 2,
                                    "table_placement": PACKED, "tile_order": 0}
        name = bench.batch_variant(op, lc, m=m)
        assert name in rec["kernels"], (workload, name)
        assert rec["kernels"][name]["hbm_bytes_per_launch"] > 0
