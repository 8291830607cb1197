"""sdd_solve_noalloc (every device buffer in the library's static scratch,
no allocation during the call) against sdd_solve on the same requests,
called twice in a row, the second time with a smaller request: bitwise the
same results (the same kernels run in the same order), the counters of the
first call not leaking into the second; a request beyond the scratch is
rejected with SDD_E_NOMEM."""
import numpy as np
import pytest

from paper_1603_09311_amd import sdd
from paper_1603_09311_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "var_re", "var_im", "cov", "se", "paths_done", "steps", "unfinished", "mean_exit_time")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = sdd.Context(0, workspace_bytes=4 << 30)
    yield c
    c.close()


def assert_same(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
    assert a["records"].tobytes() == b["records"].tobytes()


def test_noalloc_equals_solve_on_two_calls_in_a_row(ctx):
    big = W.quarter_space(paths=512, precision=W.FP32_MIXED, M=2048).subset(np.arange(0, 512, 2))
    small = W.unit_square(paths=300, precision=W.FP64, seed=5)
    for p in (big, small):
        print(f"noalloc: {p.name} {p.n_nodes} nodes x {int(p.path_count[0])} paths", flush=True)
        a = ctx.solve_noalloc(p, records=True)
        b = ctx.solve(p, records=True)
        assert_same(a, b)
        assert np.all(a["unfinished"] == 0)


def test_noalloc_generic_model_with_sigma_grid(ctx):
    regions = [W.Region(W.HALF_Z_LT, (0.0,), 0.0), W.Region(W.BOX, (-2.0, 0.0, 0.5, 1.5), 1.0),
               W.Region(W.BOX, (0.5, 2.0, 1.0, 2.5), 0.3), W.Region(W.TRIANGLE, (-4.0, 2.0, -3.0, 4.0, -1.0, 3.0), 0.5)]
    p = W.quarter_space(paths=256, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 16))
    p = p.replace(regions=regions, sigma_background=0.01,
                  g=W.column_tables(regions, 0.01, W.QS_WALLS, 1.0, W.DELTA1, 0.0, 1024))
    assert_same(ctx.solve_noalloc(p, records=True), ctx.solve(p, records=True))


def test_noalloc_rejects_requests_beyond_the_scratch(ctx):
    p = W.unit_square(paths=1 << 18, precision=W.FP32_MIXED)   # 2^21 paths: 64 MiB of records alone
    with pytest.raises(sdd.SddError) as e:
        ctx.solve_noalloc(p)
    assert e.value.status == sdd.SDD_E_NOMEM
    assert "static scratch" in str(e.value)
    # still usable afterwards
    q = W.unit_square(paths=64, precision=W.FP32_MIXED, seed=2)
    assert np.array_equal(ctx.solve_noalloc(q)["mean"], ctx.solve(q)["mean"])
