"""Host-side planning (no GPU): the mixed path's int32 slice sums stay exact
under every plan the autotuner can pick.

The mixed precision multiplies balanced base-256 digits (|d| <= 128) on the
INT8 matrix cores and sums each slice level in int32.  A level holds at most 4
digit pairs of |d_i d_j| <= 2^14 per inner index, so a sum over n indices is
exact while 4 n 2^14 < 2^31, i.e. n <= 32767.  jk_plan_describe reports the
deepest such sum of a plan (the half-transform's padded nao, or one exchange
split of a chunk's slab-rank index) and the cap; the planner must split the
exchange so that every plan stays within it.
"""
import itertools

import pytest

from paper_2608_06536_amd import _lib, jk

CHUNKS_MB = (64, 128, 256, 512, 1024, 2048, 4096)
CAP = 32767


def _mixed(nao, naux, nd, r):
    return jk.make_problem(nao, naux, nd, r, "mixed")


def test_cap_value():
    info = jk.plan_describe(_mixed(48, 192, 1, 8), 4, 1024)
    assert info["int_depth_cap"] == CAP
    assert 4 * CAP * 2 ** 14 < 2 ** 31 <= 4 * (CAP + 1) * 2 ** 14


def test_deep_single_density_splits():
    # nao = 2000, one density of rank 200, 4 GiB chunks: 670 slabs of rank 200
    # is 134,000 inner indices per chunk, more than one int32 sum may take
    p = _mixed(2000, 8000, 1, 200)
    info = jk.plan_describe(p, 4, 4096)
    assert info["chunk_slabs"] * 200 > CAP           # the chunk alone would overflow
    assert info["nsplit"] >= 5 and info["nsplit_sym"] >= 5
    assert info["int_depth"] <= CAP


@pytest.mark.parametrize("nao", [48, 130, 300, 500, 1000, 2000, 4096, 16384])
def test_every_plan_within_cap(nao):
    for nd, r in itertools.product((1, 2, 8, 16), (1, 8, 40, 200, 1024)):
        if r > nao or 2 * nd * r > (1 << 20):
            continue
        naux = 4 * nao
        p = _mixed(nao, naux, nd, r)
        for mb in CHUNKS_MB:
            info = jk.plan_describe(p, 4, mb)
            assert info["int_depth_cap"] == CAP
            assert 0 < info["int_depth"] <= CAP, (nao, nd, r, mb, info)


def test_fp64_plans_report_no_int_sums():
    info = jk.plan_describe(jk.make_problem(500, 2000, 8, 40, "fp64"), 4, 1024)
    assert info["int_depth"] == 0 and info["int_depth_cap"] == 0
    assert info["chunk_slabs"] > 0 and info["nsplit"] >= 1


def test_describe_rejects_bad_plans():
    p = _mixed(48, 192, 1, 8)
    for tile, mb in ((5, 1024), (4, 32), (4, 8192), (-1, 1024)):
        with pytest.raises(_lib.JKError):
            jk.plan_describe(p, tile, mb)
