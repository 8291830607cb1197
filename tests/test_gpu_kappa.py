"""Parity of the HIP discontinuous-kappa walk (sdd_solve_kappa, through the C
ABI) with the FP64 CPU oracle (Secs. 2.2 and 3.1).

Bar (FP64 on both sides, same random streams): identical per-path decisions
(steps, exit wall), values and exit times equal to ~1e-11, per-node
statistics equal to 1e-9; results independent of the launch shape.
"""
import sys

import numpy as np
import pytest

from paper_1603_09311_amd import sdd
from paper_1603_09311_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9
SQ = (-1.0, 1.0, -1.0, 1.0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = sdd.Context(0, workspace_bytes=8 << 30)
    yield c
    c.close()


def assert_records_match(grec, orec):
    assert grec.shape == orec.shape
    assert np.array_equal(grec["steps"], orec["steps"])
    assert np.array_equal(grec["wall"], orec["wall"])
    for f in ("w_re", "w_im", "tau"):
        assert np.allclose(grec[f], orec[f], rtol=1e-11, atol=1e-13), f


def assert_fp64_parity(g, o, tol=TOL_FP64):
    e_o = o["mean_re"] + 1j * o["mean_im"]
    scale = np.fmax(np.abs(e_o), np.nan_to_num(o["se"]))
    d = np.abs(g["mean"] - e_o)
    assert np.all(d <= tol * np.fmax(scale, 1e-300)), (d / scale).max()
    assert np.array_equal(g["paths_done"], o["paths_done"])
    assert np.array_equal(g["steps"], o["steps"])
    assert np.array_equal(g["unfinished"], o["unfinished"])
    for k in ("var_re", "var_im", "cov", "se"):
        ok = np.isfinite(o[k])
        assert np.allclose(g[k][ok], o[k][ok], rtol=1e-9, atol=1e-300), k
    assert np.allclose(g["mean_exit_time"], o["mean_exit_time"], rtol=1e-12)


def two_media(paths=300, dt=1e-3, kappa=(1.0, 10.0), lam=(5j, 1 + 2j), seed=0x5EED1234ABCD, stream=5):
    """Both rates and both diffusivities differ; nodes on the interface,
    next to it on both sides, next to walls and corners."""
    g = W.tables_from_function(lambda y, z: np.exp(1j * y) * (1.0 + 0.5 * z) + 0.2 * z * z, SQ, 96)
    nodes = np.array([[0.0, 0.0], [-0.01, 0.3], [0.012, -0.4], [0.6, 0.6], [-0.97, 0.2], [0.98, -0.98],
                      [-0.3, -0.95], [0.25, 0.5]])
    n = nodes.shape[0]
    return W.KappaProblem(*SQ, y_if=0.0, kappa=kappa, lam=lam, g=g, nodes=nodes,
                          path_begin=np.arange(n, dtype=np.uint32) * 1000, path_count=np.full(n, paths, np.uint32),
                          dt=dt, seed=seed, stream=stream)


def test_kappa_records_match_oracle_path_by_path(ctx, orc):
    for kappa in ((1.0, 10.0), (10.0, 1.0), (3.0, 3.0)):
        p = two_media(kappa=kappa)
        log(f"kappa records: kappa={kappa} nodes={p.n_nodes} paths={p.total_paths}")
        g = ctx.solve_kappa(p, records=True)
        o, orec = orc.ksolve(p, records=True)
        assert_records_match(g["records"], orec)
        assert_fp64_parity(g, o)


def test_kappa_interface_off_centre_and_tm_like_rates(ctx, orc):
    """Interface at y = 0.37 of a wider rectangle; kappa = 2 / sigma with
    sigma 0.1 | 1 and lambda = i (the TM form of Eq. 9)."""
    walls = (-1.5, 2.0, -1.0, 1.2)
    g = W.tables_from_function(lambda y, z: 1.0 + 0.3 * y - 0.2j * z, walls, 128)
    nodes = np.array([[0.37, 0.1], [0.3, -0.2], [0.45, 0.9], [-1.0, 0.0], [1.7, 0.5]])
    n = nodes.shape[0]
    p = W.KappaProblem(*walls, y_if=0.37, kappa=(20.0, 2.0), lam=(1j, 1j), g=g, nodes=nodes,
                       path_begin=np.zeros(n, np.uint32), path_count=np.full(n, 500, np.uint32), dt=2e-4,
                       seed=99, stream=0)
    log("kappa off-centre interface")
    g_ = ctx.solve_kappa(p, records=True)
    o, orec = orc.ksolve(p, records=True)
    assert_records_match(g_["records"], orec)
    assert_fp64_parity(g_, o)


def test_kappa_launch_shape_does_not_change_a_bit(ctx):
    p = two_media(paths=777)
    ref = ctx.solve_kappa(p, records=True)
    try:
        for tile in (64, 100, 4096):
            ctx.set_tuning(tile_paths=tile)
            g = ctx.solve_kappa(p, records=True)
            assert g["records"].tobytes() == ref["records"].tobytes(), tile
            assert np.array_equal(g["mean"], ref["mean"])
    finally:
        ctx.set_tuning()


def test_kappa_edge_cases(ctx, orc):
    # one path per node (SE undefined), and a step cap that leaves paths unfinished
    p = two_media(paths=1)
    g = ctx.solve_kappa(p, records=True)
    o, orec = orc.ksolve(p, records=True)
    assert_records_match(g["records"], orec)
    for cap in (1, 2, 3, 40):
        q = two_media(paths=200).replace(max_steps=cap)
        g = ctx.solve_kappa(q, records=True)
        o, orec = orc.ksolve(q, records=True)
        assert_records_match(g["records"], orec)
        assert np.array_equal(g["unfinished"], o["unfinished"])
        assert np.all(g["records"]["steps"] <= cap)
    # no nodes
    e = ctx.solve_kappa(two_media().replace(nodes=np.zeros((0, 2)), path_begin=np.zeros(0, np.uint32),
                                            path_count=np.zeros(0, np.uint32)))
    assert e["mean"].size == 0
    # a ragged mix of path counts across nodes and tiles
    q = two_media().replace(path_count=np.array([1, 63, 64, 65, 511, 513, 2, 1000], np.uint32))
    g = ctx.solve_kappa(q, records=True)
    o, orec = orc.ksolve(q, records=True)
    assert_records_match(g["records"], orec)
    assert_fp64_parity(g, o)


def test_kappa_invalid_requests_rejected(ctx):
    p = two_media(paths=10)
    bad = [p.replace(kappa=(0.0, 1.0)), p.replace(kappa=(1.0, float("nan"))), p.replace(y_if=-1.0),
           p.replace(lam=(-0.5, 1j)), p.replace(dt=0.05), p.replace(nodes=p.nodes + 5.0),
           p.replace(path_count=np.zeros(p.n_nodes, np.uint32)), p.replace(stream=1 << 30),
           p.replace(path_begin=np.full(p.n_nodes, 0xFFFFFFF8, np.uint32))]
    for b in bad:
        with pytest.raises(sdd.SddError) as ei:
            ctx.solve_kappa(b)
        assert ei.value.status == -1


def test_kappa_analytic_grid_sampled_at_full_size(ctx, orc):
    """Sec. 4.1 at all 49 x 49 interior points of the 51 x 51 mesh with
    10000 paths each (the paper's configuration, as timed): sampled nodes
    against the oracle on the same streams, and every node against the exact
    solution within the Monte-Carlo error plus the interface bias."""
    p = W.kappa_analytic_grid()
    log(f"kappa grid: nodes={p.n_nodes} paths={p.total_paths}")
    g = ctx.solve_kappa(p)
    log(f"kappa grid: walk {ctx.stats()['last_walk_ms']:.1f} ms")
    # sampled nodes, walked by the oracle with their own node indices
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([[0, 24, 1200, 1176, p.n_nodes - 1], rng.choice(p.n_nodes, 3, False)]))
    for j, rec in zip(idx, orc.kwalk_nodes(p, idx)):
        done = rec["wall"] >= 0
        w = rec["w_re"][done] + 1j * rec["w_im"][done]
        m = w.mean()
        assert abs(g["mean"][j] - m) <= TOL_FP64 * max(abs(m), 1e-300), j
        assert g["steps"][j] == rec["steps"].sum() and g["paths_done"][j] == done.sum()
        se = np.sqrt((w.real.var(ddof=1) + w.imag.var(ddof=1)) / done.sum())
        assert abs(g["se"][j] - se) <= 1e-9 * se
    exact = W.kappa_model_field(p.nodes[:, 0], p.nodes[:, 1])
    err = np.abs(g["mean"] - exact)
    assert np.all(g["unfinished"] == 0)
    # interface bias at dt = 1e-4 measured on the oracle at a few hundredths at most
    assert np.all(err <= 5.0 * g["se"] + 0.03), (err - 5 * g["se"]).max()
    assert np.median(err / g["se"]) < 1.5


# ---------------------------------------------------------------------------
# FP32-mixed kappa walk: same random numbers, FP32 rounding.
# ---------------------------------------------------------------------------
FP32 = sdd.SDD_FP32_MIXED


def assert_within_3se(g, o):
    e_o = o["mean_re"] + 1j * o["mean_im"]
    d = g["mean"] - e_o
    z = np.concatenate([np.abs(d.real) / o["se_re"], np.abs(d.imag) / o["se_im"]])
    z = z[np.isfinite(z)]
    assert z.max() <= 3.0, z.max()
    from scipy import stats
    assert np.sum(z ** 2) <= stats.chi2.ppf(0.999, z.size)


def test_kappa_fp32_within_3se_and_paired_with_fp64(ctx, orc):
    for kappa in ((1.0, 10.0), (10.0, 1.0), (3.0, 3.0)):
        p = two_media(paths=4000, kappa=kappa)
        log(f"kappa fp32: kappa={kappa} nodes={p.n_nodes} paths={p.total_paths}")
        g32 = ctx.solve_kappa(p, precision=FP32)
        g64 = ctx.solve_kappa(p)
        o, _ = orc.ksolve(p)
        assert_within_3se(g32, o)
        assert_fp64_parity(g64, o)
        # the same paths up to rounding: far inside the Monte-Carlo error
        se = np.hypot(g64["se_re"], g64["se_im"])
        assert np.all(np.abs(g32["mean"] - g64["mean"]) <= 0.5 * se)
        assert np.all(g32["unfinished"] == 0)


def test_kappa_fp32_launch_shape_and_caps(ctx):
    p = two_media(paths=777)
    ref = ctx.solve_kappa(p, records=True, precision=FP32)
    try:
        for tile in (64, 4096):
            ctx.set_tuning(tile_paths=tile)
            g = ctx.solve_kappa(p, records=True, precision=FP32)
            assert g["records"].tobytes() == ref["records"].tobytes(), tile
    finally:
        ctx.set_tuning()
    for cap in (1, 2, 3, 40):
        g = ctx.solve_kappa(two_media(paths=200).replace(max_steps=cap), records=True, precision=FP32)
        rec = g["records"]
        assert np.all(rec["steps"] <= cap)
        assert np.all((rec["wall"] >= 0) | (rec["steps"] == cap))
    with pytest.raises(sdd.SddError):
        ctx.solve_kappa(p, precision=2)


def test_kappa_fp32_analytic_grid_full_size(ctx):
    """Sec. 4.1 on the full 51 x 51 mesh (10000 paths per node): FP32-mixed
    against the FP64 walk on the same streams, and against the exact
    solution as for FP64."""
    p = W.kappa_analytic_grid()
    g32 = ctx.solve_kappa(p, precision=FP32)
    ms32 = ctx.stats()["last_walk_ms"]
    g64 = ctx.solve_kappa(p)
    log(f"kappa grid fp32 walk {ms32:.1f} ms, fp64 {ctx.stats()['last_walk_ms']:.1f} ms")
    z = np.concatenate([np.abs((g32["mean"] - g64["mean"]).real) / g64["se_re"],
                        np.abs((g32["mean"] - g64["mean"]).imag) / g64["se_im"]])
    assert np.nanmax(z) <= 3.0, np.nanmax(z)
    exact = W.kappa_model_field(p.nodes[:, 0], p.nodes[:, 1])
    err = np.abs(g32["mean"] - exact)
    assert np.all(g32["unfinished"] == 0)
    assert np.all(err <= 5.0 * g32["se"] + 0.03)


def test_kappa_both_precisions_match_the_exact_scheme_on_a_strip(ctx):
    """The HIP kappa walks, FP64 and FP32-mixed (each with its own code for
    the interface time split), against the exact expectation of the discrete
    scheme on a strip (kappa_chain: the walk's one-dimensional Markov chain
    evaluated without sampling): kappa (1, 4), lambda (20, 0), dt = 1e-2,
    |y| < 1.5 with the z-walls out of reach, 8e6 paths per node; within 4 SE
    plus the chain's quadrature error.  Splits of an interface step's time
    that converge to the same continuum limit differ from it by 0.015 or more
    at y = -0.05 (about 100 SE here)."""
    from kappa_chain import StripChain
    a, kappa, lam, dt = 1.5, (1.0, 4.0), (20.0, 0.0), 1e-2
    chain = StripChain(a, kappa, lam, 1.0, 1.0, dt, n_side=300).solve()
    ys = np.array([-0.3, -0.05, 0.05, 0.3])
    exact = np.array([chain.value(y) for y in ys])
    walls = (-a, a, -40.0, 40.0)
    g = W.tables_from_function(lambda y, z: np.ones_like(y, dtype=np.complex128), walls, 4096)
    nodes = np.stack([ys, np.zeros_like(ys)], axis=1)
    n = nodes.shape[0]
    p = W.KappaProblem(*walls, y_if=0.0, kappa=kappa, lam=lam, g=g, nodes=nodes,
                       path_begin=np.zeros(n, np.uint32), path_count=np.full(n, 8_000_000, np.uint32), dt=dt,
                       seed=12, stream=1)
    for prec in (0, FP32):
        r = ctx.solve_kappa(p, precision=prec)
        d = (r["mean"] - exact).real
        log(f"kappa strip precision {prec}: mean {r['mean'].real} exact {exact.real} diff/se {d / r['se_re']}")
        assert np.all(np.abs(r["mean"].imag) == 0.0)
        assert np.all(np.abs(d) <= 4.0 * r["se_re"] + 1e-4), (d, r["se_re"])
        assert np.all(r["unfinished"] == 0)
