"""The host-side launch helpers over every grid lz_init accepts (no GPU).

`lz_launch_plan` runs the helpers lz_init uses to size its launches (the
density band groups, the projector-dot chunks, the update blocks, the choice
of plane kernels) on the host alone.  Every cubic grid that lz_init accepts,
in every precision, with band, k-point, plane-wave and projector counts from
one of each up to the large cell's, must give positive sizes that cover the
work exactly, and arguments lz_init refuses must be refused here too.  No
device is touched: the test runs where there is none.
"""
import ctypes
import math

import numpy as np
import pytest

import paper_2111_06623_amd as lz

CT_SIZES = {24, 32, 40, 48, 64, 72, 96}
REGISTER_FP32 = {24, 32, 48, 64, 72, 96}   # register lines (24-48) and lane pairs (64-96)


def _smooth(n):
    for r in (2, 3, 5):
        while n % r == 0:
            n //= r
    return n == 1


GRIDS = [n for n in range(2, 129) if _smooth(n) and n * n <= 9216]

# (nbnd, nks, npwx, nproj): single band and plane wave, the 24^3 and 48^3
# cells, the largest batched member, the 96^3 cell, and awkward counts
SIZES = [(1, 1, 1, 0), (1, 1, 7, 0), (4, 1, 739, 0), (16, 8, 6500, 32), (48, 16, 21823, 96),
         (128, 4, 51443, 256), (7, 3, 100, 5), (300, 2, 3000, 0)]
SLOTS = [0, 1, 256, 768, 4096]


def _round_rule(n3, nb, slots):
    """The documented round rule: fewest rounds x bands per block plus 0.05
    of a band per group partial, ties to the larger group."""
    best, best_t = 1, math.inf
    for g in range(1, min(nb, 16) + 1):
        ng = -(-nb // g)
        t = -(-(n3 * ng) // slots) * g + 0.05 * ng
        if t <= best_t + 1e-9:
            best, best_t = g, t
    return best


@pytest.mark.parametrize("prec", ["fp64", "fp32", "splitbf16"])
def test_every_grid_gives_covering_launch_sizes(prec):
    lz.load()
    for n in GRIDS:
        for nbnd, nks, npwx, nproj in SIZES:
            nb = nbnd * nks
            for slots in SLOTS:
                p = lz.lz_launch_plan(n, prec, nbnd, nks, npwx, nproj, slots)
                case = (n, prec, nbnd, nks, npwx, nproj, slots, p)
                assert p["ct_size"] == (n if n in CT_SIZES else 0), case
                reg = n if (prec != "fp64" and n in REGISTER_FP32) else 0
                assert p["reg_plane"] == reg, case
                for key in ("group_reg", "group_lds"):
                    assert p[key] >= 1, case
                if slots:
                    assert 1 <= p["group_round"] <= min(nb, 16), case
                    assert p["group_round"] == _round_rule(n, nb, slots), case
                    assert p["group_lds"] == p["group_round"], case
                else:
                    assert p["group_round"] == 0, case
                if reg == 0:
                    assert p["group_reg"] == p["group_lds"], case
                assert 1 <= p["gsize"] <= nb and p["gsize"] == min(p["group_reg"], nb), case
                assert p["ngroups"] == -(-nb // p["gsize"]), case
                for path in ("valu", "mfma"):
                    c, m = p[f"{path}_chunk"], p[f"{path}_nchunk"]
                    assert c >= 1 and m == -(-npwx // c), case
                    assert p[f"{path}_upd_blocks"] >= 1 and p[f"{path}_upd_blocks_proj"] >= 1, case
                assert p["valu_chunk"] == 64, case


def test_the_benchmark_cells_plans():
    # 48^3 in FP64: LDS passes, groups of 8 bands (one round of 768 blocks at
    # three blocks per compute unit); in FP32 register lines, groups of 4
    p = lz.lz_launch_plan(48, "fp64", 16, 8, 6500, 32, 3 * 256)
    assert (p["reg_plane"], p["gsize"], p["ngroups"]) == (0, 8, 16)
    p = lz.lz_launch_plan(48, "fp32", 16, 8, 6500, 32, 0)
    assert (p["reg_plane"], p["gsize"], p["ngroups"]) == (48, 4, 32)
    # 96^3 in FP64, one block per compute unit: groups of 16
    p = lz.lz_launch_plan(96, "fp64", 128, 4, 51443, 256, 256)
    assert (p["gsize"], p["ngroups"]) == (16, 32)


@pytest.mark.parametrize("args", [
    (1, 0, 4, 1, 100, 0, 0), (7, 0, 4, 1, 100, 0, 0), (97, 0, 4, 1, 100, 0, 0),
    (130, 0, 4, 1, 100, 0, 0), (0, 0, 4, 1, 100, 0, 0), (-8, 0, 4, 1, 100, 0, 0),
    (48, 3, 4, 1, 100, 0, 0), (48, -1, 4, 1, 100, 0, 0), (48, 0, 0, 1, 100, 0, 0),
    (48, 0, 4, 0, 100, 0, 0), (48, 0, 4, 1, 0, 0, 0), (48, 0, 4, 1, 100, -1, 0),
    (48, 0, 4, 1, 100, 0, -1), (48, 0, 1 << 20, 1 << 10, 100, 0, 0)])
def test_refused_arguments(args):
    lib = lz.load()
    out = np.full(lz.LZ_PLAN_LEN, -7, dtype=np.int32)
    st = lib.lz_launch_plan(*args, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert st == lz.LZ_ERR_ARG and lz.lz_last_error()
    assert lib.lz_launch_plan(48, 0, 4, 1, 100, 0, 0, None) == lz.LZ_ERR_ARG
