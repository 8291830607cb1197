"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars:
  * FP64 walk: identical per-path decisions (steps, exit wall) and weights
    equal to ~1e-12; per node |E_gpu - E_oracle| <= 1e-9 max(|E_oracle|, SE).
  * FP32-mixed walk: per node within 3 SE of the oracle per component plus
    a chi-square gate over all components; paired with the FP64 walk on the
    same streams, the difference is far below SE.
  * Scheduling never changes a bit: plain == persistent, alone == in a batch,
    any tile/block shape, served == blocking.
"""
import math
import os
import sys
import time

import numpy as np
import pytest
from scipy import stats

from paper_1603_09311_amd import sdd
from paper_1603_09311_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = sdd.Context(0, workspace_bytes=24 << 30)
    yield c
    c.close()


def oracle_solve(orc, p, records=False):
    res, recs = orc.solve(p, records=records)
    return res, recs


def assert_fp64_parity(g, o, tol=TOL_FP64):
    e_o = o["mean_re"] + 1j * o["mean_im"]
    scale = np.fmax(np.abs(e_o), o["se"])      # SE is NaN for a one-path node
    d = np.abs(g["mean"] - e_o)
    assert np.all(d <= tol * scale), (d / scale).max()
    assert np.array_equal(g["paths_done"], o["paths_done"])
    assert np.array_equal(g["steps"], o["steps"])
    assert np.array_equal(g["unfinished"], o["unfinished"])
    for k in ("var_re", "var_im", "cov", "se"):
        ok = np.isfinite(o[k])
        assert np.allclose(g[k][ok], o[k][ok], rtol=1e-9, atol=1e-300), k
    assert np.allclose(g["mean_exit_time"], o["mean_exit_time"], rtol=1e-12)


def assert_within_se(g, o, zmax=3.0):
    e_o = o["mean_re"] + 1j * o["mean_im"]
    d = g["mean"] - e_o
    z = np.concatenate([np.abs(d.real) / o["se_re"], np.abs(d.imag) / o["se_im"]])
    assert z.max() <= zmax, z.max()
    assert np.sum(z ** 2) <= stats.chi2.ppf(0.999, z.size)


def assert_records_match(grec, orec):
    assert grec.shape == orec.shape
    assert np.array_equal(grec["steps"], orec["steps"])
    assert np.array_equal(grec["wall"], orec["wall"])
    for f in ("w_re", "w_im", "tau"):
        assert np.allclose(grec[f], orec[f], rtol=1e-11, atol=1e-13), f


def small_mixed_model():
    regions = [W.Region(W.HALF_Z_LT, (0.3,), 0.0), W.Region(W.BOX, (0.5, 0.8, 0.4, 0.7), 5.0),
               W.Region(W.TRIANGLE, (0.1, 0.5, 0.1, 0.95, 0.45, 0.95), 2.0)]
    p = W.unit_square(alpha=30.0, g_fn=lambda y, z: np.exp(1j * y) * (1 + z), M=64, dt=1e-3,
                      nodes=np.array([[0.5, 0.5], [0.02, 0.5], [0.97, 0.03], [0.3, 0.8], [0.6, 0.45],
                                      [0.2, 0.6], [0.7, 0.35], [0.45, 0.9]]),
                      paths=200, seed=0x123456789, stream=3)
    return p.replace(regions=regions, sigma_background=1.0)


# ---------------------------------------------------------------------------

def test_records_fp64_match_oracle_path_by_path(ctx, orc):
    p = small_mixed_model()
    log(f"records fp64: nodes={p.n_nodes} paths={p.total_paths}")
    g = ctx.solve(p, precision=sdd.SDD_FP64, records=True)
    o, orec = oracle_solve(orc, p, records=True)
    assert_records_match(g["records"], orec)
    assert_fp64_parity(g, o)


def test_plain_equals_persistent_fp64_bitwise(ctx):
    p = small_mixed_model().with_paths(333)
    a = ctx.solve(p, precision=sdd.SDD_FP64, records=True)
    b = ctx.solve_plain(p, records=True)
    assert a["records"].tobytes() == b["records"].tobytes()
    assert np.array_equal(a["mean"], b["mean"])


def test_unit_square_fp64_parity(ctx, orc):
    """The homogeneous toy at full size: 8 nodes x 4096 paths, dt = 1e-4."""
    p = W.unit_square(paths=4096, precision=W.FP64)
    log("unit square fp64 full size")
    g = ctx.solve(p)
    o, _ = oracle_solve(orc, p)
    assert_fp64_parity(g, o)
    exact = -0.0021278355286973 - 0.2057296574127508j
    z = np.abs(g["mean"] - exact) / g["se"]
    assert z.max() < 4.5


def test_unit_square_fp32_within_se(ctx, orc):
    p = W.unit_square(paths=4096, precision=W.FP32_MIXED)
    g = ctx.solve(p)
    o, _ = oracle_solve(orc, p)
    assert_within_se(g, o)
    # paired with the FP64 walk on the same streams
    g64 = ctx.solve(p, precision=sdd.SDD_FP64)
    assert np.all(np.abs(g["mean"] - g64["mean"]) < 0.2 * g64["se"])


def test_g_one_alpha_zero_exact_both_precisions(ctx):
    p = W.unit_square(alpha=0.0, g_fn=lambda y, z: np.ones_like(y) + 0j, paths=1000, dt=4e-4)
    for prec in (sdd.SDD_FP64, sdd.SDD_FP32_MIXED):
        g = ctx.solve(p, precision=prec)
        assert np.all(g["mean"] == 1.0) and np.all(g["var_re"] == 0.0)


def test_quarter_space_subset_fp64_parity(ctx, orc):
    """Quarter-space geometry (lengths in skin depths, air, two half-spaces),
    a node subset with fewer paths so the oracle finishes in seconds."""
    p = W.quarter_space(paths=96, precision=W.FP64, M=4096).subset([0, 37, 128, 255, 256, 300, 383, 511])
    p = p.replace(path_count=np.array([96, 17, 64, 65, 96, 1, 130, 33], np.uint32))
    log(f"quarter space subset fp64: {p.total_paths} paths")
    g = ctx.solve(p, records=True)
    o, orec = oracle_solve(orc, p, records=True)
    assert_records_match(g["records"], orec)
    assert_fp64_parity(g, o)


def test_quarter_space_subset_fp32_within_se(ctx, orc):
    p = W.quarter_space(paths=2048, precision=W.FP32_MIXED, M=4096).subset([10, 100, 200, 260, 400, 500])
    log(f"quarter space subset fp32: {p.total_paths} paths")
    g = ctx.solve(p)
    o, _ = oracle_solve(orc, p)
    assert_within_se(g, o)


def test_block_and_triangle_fp64_parity(ctx, orc):
    blk = W.block_in_half_space(10.0, paths=64, precision=W.FP64, M=2048).subset([0, 130, 260, 400, 600, 1000])
    tri = W.triangle_request(5, precision=W.FP64, M=2048)
    tri = tri.subset(np.arange(0, tri.n_nodes, max(1, tri.n_nodes // 6))[:6]).with_paths(48)
    for p in (blk, tri):
        g = ctx.solve(p, records=True)
        o, orec = oracle_solve(orc, p, records=True)
        assert_records_match(g["records"], orec)
        assert_fp64_parity(g, o)


def _sample_paths(p, per, seed=3):
    """(node, path) pairs: three random paths at every 8th node."""
    rng = np.random.default_rng(seed)
    return [(int(j), int(k)) for j in range(0, p.n_nodes, 8) for k in rng.choice(per, 3, replace=False)]


def test_quarter_space_full_size_sampled_paths(ctx, orc):
    """The timed workload at full size and in the timed launch form (512
    nodes x 65536 paths, FP32-mixed, one prepared batch replayed as a HIP
    graph): every path finished; 192 paths (3 at every 8th node) walked one
    by one by the FP64 oracle with their own node and path indices take the
    same number of steps to the same wall (all but at most two: a proposal
    that FP32 rounding moves across a wall or a bridge threshold) and agree in
    value.  The FP32 walk counts full steps per region exactly and forms the
    phase in FP64, so a path's value differs from the oracle's only by FP32
    rounding of its positions (about 1e-5 of a skin depth at the exit,
    times |dg/dt| <= |k E0| = 0.16 on the walls) unless FP32 rounding moves a
    proposal across the contact or the surface: then one full step's phase
    goes to the other region, |delta S| <= max alpha dt / 2 = 4e-3.  Bound:
    max alpha dt / 2 |g|max + 1e-4.  The per-node reduction equals the mean
    of the records."""
    p = W.quarter_space()
    log(f"quarter space full size fp32: {p.n_nodes} nodes x {int(p.path_count[0])} paths")
    b = ctx.batch([p], records=True)
    try:
        r = b.run()[0]
    finally:
        b.close()
    rec = r["records"]
    per = int(p.path_count[0])
    assert rec.shape[0] == p.n_nodes * per
    assert np.all(r["unfinished"] == 0) and np.all(rec["wall"] >= 0)
    same, n, dev = 0, 0, []
    for j, k in _sample_paths(p, per):
        o = orc.walk_path(p, j, k)
        g = rec[j * per + k]
        n += 1
        if g["steps"] == o["steps"] and g["wall"] == o["wall"]:
            same += 1
            dev.append(abs(complex(g["w_re"], g["w_im"]) - complex(o["w_re"], o["w_im"])))
    dev = np.array(dev)
    bound = p.alphas().max() * p.dt / 2.0 * p.g_norm + 1e-4
    log(f"fp32 sampled paths: {same}/{n} same steps and wall, value deviation median {np.median(dev):.2e} "
        f"max {dev.max():.2e} (bound {bound:.2e})")
    assert same >= n - 2, (same, n)
    assert np.median(dev) <= 1e-6 and dev.max() <= bound, (np.median(dev), dev.max(), bound)
    m = (rec["w_re"] + 1j * rec["w_im"]).reshape(p.n_nodes, per).mean(axis=1)
    assert np.allclose(m, r["mean"], rtol=1e-12, atol=1e-15)
    d = r["diag"]
    assert d["rho_dt"] == pytest.approx(p.alphas().max() * p.dt / 2.0, rel=1e-12) and not d["dt_unresolved"]


def test_quarter_space_fp64_full_size_and_fp32_per_node(ctx, orc):
    """The timed workload at full size with the FP64 persistent walker (the
    parity form, 512 nodes x 65536 paths, 1.9e12 steps, prepared batch
    replayed as a HIP graph): 192 sampled paths walked one by one by the
    oracle under their own indices take the same steps to the same wall with
    weights equal to 1e-11.  Then the headline FP32-mixed result at full size
    against this FP64 result, node by node: every component within 3 FP64
    standard errors and the sum of squared z-scores inside the 99.9%
    chi-square quantile (the two walks share their random numbers, so the
    z-scores are far below 1)."""
    p64 = W.quarter_space(precision=W.FP64)
    per = int(p64.path_count[0])
    log(f"quarter space full size fp64: {p64.n_nodes} nodes x {per} paths")
    b = ctx.batch([p64], records=True)
    try:
        r64 = b.run()[0]
    finally:
        b.close()
    rec = r64["records"]
    assert np.all(r64["unfinished"] == 0) and np.all(rec["wall"] >= 0)
    idx = _sample_paths(p64, per)
    got = np.array([rec[j * per + k] for j, k in idx], dtype=rec.dtype)
    want = np.zeros(len(idx), dtype=got.dtype)
    for i, (j, k) in enumerate(idx):
        o = orc.walk_path(p64, j, k)
        want[i] = (o["w_re"], o["w_im"], o["tau"], o["steps"], o["wall"])
    assert_records_match(got, want)
    m = (rec["w_re"] + 1j * rec["w_im"]).reshape(p64.n_nodes, per).mean(axis=1)
    assert np.allclose(m, r64["mean"], rtol=1e-12, atol=1e-15)
    del rec, r64["records"]
    log("quarter space full size fp32 for the per-node comparison")
    r32 = ctx.solve(W.quarter_space())
    d = r32["mean"] - r64["mean"]
    z = np.concatenate([np.abs(d.real) / r64["se_re"], np.abs(d.imag) / r64["se_im"]])
    log(f"fp32 vs fp64 at full size: max |z| {z.max():.4f}, sum z^2 {np.sum(z ** 2):.3f} over {z.size}")
    assert z.max() <= 3.0
    assert np.sum(z ** 2) <= stats.chi2.ppf(0.999, z.size)
    assert np.array_equal(r32["paths_done"], r64["paths_done"])


def test_block_four_frequencies_one_launch_fp32_within_3se(ctx, orc):
    """The block-in-half-space batch: the four frequencies 0.1, 1, 10 and
    100 Hz as four FP32-mixed requests in one persistent launch, each within
    3 SE of the FP64 oracle on the same streams (nodes on the block edges and
    the surface)."""
    sel = [5, 200, 300, 700]
    ps = [W.block_in_half_space(f, paths=1024, precision=W.FP32_MIXED, M=2048).subset(sel)
          for f in (0.1, 1.0, 10.0, 100.0)]
    log(f"block batch: {len(ps)} requests x {ps[0].n_nodes} nodes x 1024 paths")
    got = ctx.solve_batch(ps)
    for p, g in zip(ps, got):
        o, _ = oracle_solve(orc, p)
        assert_within_se(g, o)
        assert np.all(g["unfinished"] == 0)


def test_triangle_uneven_graph_batch_fp32_within_3se(ctx, orc):
    """The triangle family as an uneven batch (different models, frequencies,
    node counts and path counts) prepared once and replayed as a HIP graph:
    every replay bitwise equal, each request within 3 SE of the FP64 oracle."""
    ps = []
    for m, (k, paths) in enumerate([(2, 256), (3, 512), (5, 1024), (7, 384)]):
        t = W.triangle_request(11 + m, precision=W.FP32_MIXED, M=2048)
        idx = np.linspace(0, t.n_nodes - 1, k).astype(int)
        ps.append(t.subset(idx).with_paths(paths))
    log(f"triangle batch: nodes {[p.n_nodes for p in ps]}")
    b = ctx.batch(ps)
    try:
        first = b.run()
        again = b.run()
    finally:
        b.close()
    for p, g, h in zip(ps, first, again):
        assert np.array_equal(g["mean"], h["mean"]) and np.array_equal(g["se"], h["se"])
        o, _ = oracle_solve(orc, p)
        assert_within_se(g, o)


def multi_body_model(seed, paths=128):
    """A seeded model with 4-11 bodies (boxes, triangles, a half-space) under
    air on the quarter-space domain, nodes on edges, at corners and at random
    points (the walker's generic signature)."""
    rng = np.random.default_rng(seed)
    regions = [W.Region(W.HALF_Z_LT, (0.0,), 0.0)]
    nodes = []
    for _ in range(int(rng.integers(4, 12))):
        kind = rng.choice([W.BOX, W.BOX, W.TRIANGLE, W.HALF_Y_LT], p=[0.45, 0.1, 0.35, 0.1])
        sig = float(10.0 ** rng.uniform(-2, 0.5))
        if kind == W.BOX:
            y0, z0 = rng.uniform(-6, 5), rng.uniform(0.1, 6)
            y1, z1 = y0 + rng.uniform(0.3, 3), z0 + rng.uniform(0.3, 2)
            regions.append(W.Region(W.BOX, (y0, y1, z0, z1), sig))
            nodes += [(y0, z0), (y1, (z0 + z1) / 2), ((y0 + y1) / 2, z1)]
        elif kind == W.TRIANGLE:
            v = [(rng.uniform(-6, 6), rng.uniform(0.1, 7)) for _ in range(3)]
            regions.append(W.Region(W.TRIANGLE, tuple(x for pt in v for x in pt), sig))
            nodes += [v[0], ((v[1][0] + v[2][0]) / 2, (v[1][1] + v[2][1]) / 2)]
        else:
            regions.append(W.Region(W.HALF_Y_LT, (rng.uniform(-7, 7),), sig))
    nodes += [tuple(x) for x in rng.uniform((-7.5, -5.5), (7.5, 7.5), (8, 2))]
    nodes = np.array([(y, z) for y, z in nodes if -8 < y < 8 and -6 < z < 8])
    p = W.unit_square(paths=paths, precision=W.FP32_MIXED, dt=4e-4, M=1024, nodes=nodes, seed=seed)
    g = W.column_tables(regions, 0.01, W.QS_WALLS, 1.0, W.DELTA1, 0.0, 1024)
    return p.replace(y_lo=W.QS_WALLS[0], y_hi=W.QS_WALLS[1], z_lo=W.QS_WALLS[2], z_hi=W.QS_WALLS[3],
                     regions=regions, sigma_background=0.01, length_unit_m=W.DELTA1, freq_hz=1.0,
                     alpha_direct=0.0, g=g)


def test_sigma_grid_equals_primitive_loop_bitwise(ctx, orc):
    """FP32-mixed walks on multi-body models: the sigma grid staged in LDS
    (the default for a launch of one grid), the grid read from global memory
    and the loop over the primitives give every path the same record, bit for
    bit; a batch of two models with different grids (one launch that cannot
    stage either in LDS) gives each the same records again; and the results
    are within 3 SE of the FP64 oracle."""
    for seed in range(6):
        p = multi_body_model(seed)
        log(f"sigma grid: seed {seed}, {len(p.regions)} primitives, {p.n_nodes} nodes")
        a = ctx.solve(p, records=True)
        b = ctx.solve(p, records=True, flags=sdd.SDD_FLAG_NO_SIGMA_GRID)
        c = ctx.solve(p, records=True, flags=sdd.SDD_FLAG_NO_LDS_GRID)
        assert a["records"].tobytes() == b["records"].tobytes(), seed
        assert a["records"].tobytes() == c["records"].tobytes(), seed
        assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["mean"], c["mean"])
        if seed < 2:
            o, _ = oracle_solve(orc, p.with_paths(2048))
            assert_within_se(ctx.solve(p.with_paths(2048)), o)
    p0, p1 = multi_body_model(0), multi_body_model(1)
    both = ctx.solve_batch([p0, p1], records=True)
    for p, got in zip((p0, p1), both):
        assert got["records"].tobytes() == ctx.solve(p, records=True)["records"].tobytes()
    # the seeded multi-body workload of the benchmark: 6 bodies, 128 surface nodes
    q = W.multi_body(seed=0, paths=256, M=1024)
    a = ctx.solve(q, records=True)
    for fl in (sdd.SDD_FLAG_NO_SIGMA_GRID, sdd.SDD_FLAG_NO_LDS_GRID):
        assert ctx.solve(q, records=True, flags=fl)["records"].tobytes() == a["records"].tobytes()


def _reversed_triangle(p, k):
    """p with primitive k (a triangle) entered in the other vertex order."""
    r = p.regions[k]
    v = np.asarray(r.params, dtype=np.float64).reshape(3, 2)[::-1].reshape(-1)
    regions = list(p.regions)
    regions[k] = W.Region(W.TRIANGLE, tuple(float(x) for x in v), r.sigma)
    return p.replace(regions=regions)


def test_triangle_either_vertex_order(ctx, orc):
    """A triangle entered clockwise and counter-clockwise is one region: the
    FP32 walkers (the specialised air + triangle signature, and the generic
    signature's sigma grid in LDS, in global memory and by the loop) give the
    two orders the same estimates to far below the Monte-Carlo error (the
    host orients the edges; the two orders' edge coefficients differ by
    rounding only), and both orders stay within 3 SE of the FP64 oracle."""
    tri = W.triangle_request(5, precision=W.FP32_MIXED, M=1024)
    tri = tri.subset(np.arange(0, tri.n_nodes, max(1, tri.n_nodes // 8))[:8]).with_paths(2048)
    rev = _reversed_triangle(tri, 1)
    a, b = ctx.solve(tri), ctx.solve(rev)
    se = np.hypot(a["se_re"], a["se_im"])
    assert np.all(np.abs(a["mean"] - b["mean"]) <= 0.05 * se), (np.abs(a["mean"] - b["mean"]) / se).max()
    o, _ = oracle_solve(orc, tri)
    assert_within_se(b, o)
    gen = W.multi_body(seed=1, paths=512, M=1024)
    k = next(i for i, r in enumerate(gen.regions) if r.kind == W.TRIANGLE)
    grev = _reversed_triangle(gen, k)
    for fl in (0, sdd.SDD_FLAG_NO_LDS_GRID, sdd.SDD_FLAG_NO_SIGMA_GRID):
        log(f"triangle vertex order, generic signature, flags {fl}")
        x, y = ctx.solve(gen, flags=fl), ctx.solve(grev, flags=fl)
        se = np.hypot(x["se_re"], x["se_im"])
        assert np.all(np.abs(x["mean"] - y["mean"]) <= 0.05 * se), fl


def test_batch_equals_alone_bitwise(ctx):
    """Uneven node counts, path counts, frequencies, models and precisions in
    one persistent launch: each result is bitwise the one it gets alone."""
    a = small_mixed_model()
    b = W.quarter_space(paths=40, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 37))
    c = W.block_in_half_space(1.0, paths=24, precision=W.FP64, M=1024).subset(np.arange(0, 1024, 101))
    d = W.unit_square(paths=777, precision=W.FP32_MIXED, seed=9)
    batch = ctx.solve_batch([a, b, c, d], records=True)
    for p, got in zip([a, b, c, d], batch):
        alone = ctx.solve(p, records=True)
        assert got["records"].tobytes() == alone["records"].tobytes()
        assert np.array_equal(got["mean"], alone["mean"]) and np.array_equal(got["se"], alone["se"])


def test_launch_shape_does_not_change_a_bit(ctx):
    p = W.unit_square(paths=1500, precision=W.FP32_MIXED, seed=4)
    ref = ctx.solve(p, records=True)
    try:
        for bt, bpc, tile, rf in [(64, 1, 1, 1), (128, 2, 64, 2), (192, 1, 4096, 8), (256, 3, 100, 64)]:
            ctx.set_tuning(block_threads=bt, blocks_per_cu=bpc, tile_paths=tile, refill_every=rf)
            got = ctx.solve(p, records=True)
            assert got["records"].tobytes() == ref["records"].tobytes(), (bt, bpc, tile, rf)
            assert np.array_equal(got["mean"], ref["mean"])
        for bad in ({"block_threads": 512}, {"refill_every": 3}, {"refill_every": 128}):
            with pytest.raises(sdd.SddError) as e:
                ctx.set_tuning(**bad)
            assert e.value.status == sdd.SDD_E_INVALID
    finally:
        ctx.set_tuning()


def test_edge_cases(ctx, orc):
    # no nodes
    p0 = W.unit_square(paths=4).subset([])
    g = ctx.solve(p0)
    assert g["mean"].size == 0
    # one path: variance undefined (NaN), mean is the path's weight
    p1 = W.unit_square(paths=1, precision=W.FP64, nodes=np.array([[0.5, 0.5]]))
    g = ctx.solve(p1, records=True)
    assert g["paths_done"][0] == 1 and np.isnan(g["var_re"][0])
    assert g["mean"][0] == complex(g["records"]["w_re"][0], g["records"]["w_im"][0])
    # ragged path counts and begins (not multiples of 64 or of the tile)
    pr = W.unit_square(paths=1, precision=W.FP64).replace(
        path_begin=np.array([0, 5, 1000, 7, 0, 3, 64, 1], np.uint32),
        path_count=np.array([1, 63, 65, 127, 129, 513, 2, 1000], np.uint32))
    g = ctx.solve(pr, records=True)
    o, orec = oracle_solve(orc, pr, records=True)
    assert_records_match(g["records"], orec)
    assert_fp64_parity(g, o)
    # the top of the 32-bit path range: path indices up to 2^32 - 1
    top = np.array([0xFFFFFFFF - 299, 0xFFFFFFFF - 64, 0xFFFFFFFF, 0xFFFFFF00, 0, 1, 2, 0xFFFFFFFF - 1], np.uint32)
    cnt = np.array([300, 65, 1, 256, 3, 3, 3, 2], np.uint32)
    pt = W.unit_square(paths=1, precision=W.FP64, dt=4e-4).replace(path_begin=top, path_count=cnt)
    g = ctx.solve(pt, records=True)
    o, orec = oracle_solve(orc, pt, records=True)
    assert_records_match(g["records"], orec)
    assert_fp64_parity(g, o)
    g32 = ctx.solve(pt, precision=sdd.SDD_FP32_MIXED, records=True)
    assert np.array_equal(g32["paths_done"], cnt.astype(np.uint64))
    assert np.mean(g32["records"]["steps"] == g["records"]["steps"]) > 0.98   # paired walks
    # a tiny step cap: unfinished paths counted and left out of the estimate
    pc = W.unit_square(paths=300, precision=W.FP64, dt=4e-4).replace(max_steps=25)
    g = ctx.solve(pc, records=True)
    o, orec = oracle_solve(orc, pc, records=True)
    assert g["unfinished"].sum() > 0 and np.array_equal(g["unfinished"], o["unfinished"])
    assert_records_match(g["records"], orec)
    for prec in (sdd.SDD_FP32_MIXED,):
        g32 = ctx.solve(pc, precision=prec)
        assert np.all(g32["paths_done"] + g32["unfinished"] == 300)


def test_naive_exit_ablation(ctx, orc):
    """SDD_FLAG_EXIT_NAIVE (exits on crossings only): FP64 records path by
    path as the oracle's naive walk, FP32 within 3 SE of it; both exit later
    than the bridge walk on the same streams."""
    p = small_mixed_model().with_paths(150).replace(naive_exit=True)
    g = ctx.solve(p, precision=sdd.SDD_FP64, records=True)
    o, orec = oracle_solve(orc, p, records=True)
    assert_records_match(g["records"], orec)
    assert_fp64_parity(g, o)
    q = W.unit_square(paths=4096, precision=W.FP32_MIXED, dt=4e-4)
    g32 = ctx.solve(q.replace(naive_exit=True))
    o32, _ = oracle_solve(orc, q.replace(naive_exit=True))
    assert_within_se(g32, o32)
    bridge = ctx.solve(q)
    assert np.all(g32["mean_exit_time"] > bridge["mean_exit_time"])
    assert np.all(g32["steps"] >= bridge["steps"])


def test_invalid_requests_rejected(ctx):
    p = W.unit_square(paths=8)
    bad = [p.replace(dt=0.0), p.replace(dt=0.02), p.replace(nodes=np.array([[0.0, 0.5]] * 8)),
           p.replace(nodes=np.array([[0.5, 1.0]] * 8)), p.replace(path_count=np.zeros(8, np.uint32)),
           p.replace(stream=2 ** 31)]
    for b in bad:
        with pytest.raises(sdd.SddError) as e:
            ctx.solve(b)
        assert e.value.status == sdd.SDD_E_INVALID
    with pytest.raises(sdd.SddError) as e:
        ctx.solve(p, precision=7)
    assert e.value.status == sdd.SDD_E_INVALID


def test_workspace_exhaustion_is_reported():
    import torch
    c = sdd.Context(0, workspace_bytes=1 << 20)
    try:
        p = W.unit_square(paths=100000)
        with pytest.raises(sdd.SddError) as e:
            c.solve(p)
        assert e.value.status == sdd.SDD_E_NOMEM
        g = c.solve(W.unit_square(paths=64))   # still usable
        assert g["paths_done"].sum() == 8 * 64
    finally:
        c.close()
    torch.cuda.synchronize()


def test_target_rel_se_pilot_and_extension(ctx, orc):
    """Pilot of 4096 paths, then N = ceil((s / (target |g|inf))^2) on the same
    streams; the oracle decides N from its own pilot."""
    p = W.unit_square(paths=1, precision=W.FP64, dt=4e-4, n_nodes=4)
    target = 4e-3
    g = ctx.solve(p, target_rel_se=target)
    pil = p.with_paths(4096)
    o1, _ = oracle_solve(orc, pil)
    gnorm = p.g_norm
    want = np.ceil((o1["var_re"] + o1["var_im"]) / (target * gnorm) ** 2)
    want = np.clip(want, 4096, 1 << 20).astype(np.uint32)
    assert np.array_equal(g["paths_done"], want)
    full = p.replace(path_begin=np.zeros(4, np.uint32), path_count=want)
    o2, _ = oracle_solve(orc, full)
    assert_fp64_parity(g, o2)
    assert np.all(g["se"] <= target * gnorm * 1.25)


def test_served_results_equal_blocking(ctx):
    ps = [small_mixed_model(), W.unit_square(paths=500, precision=W.FP32_MIXED, seed=3),
          W.quarter_space(paths=16, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 64)),
          W.unit_square(paths=300, precision=W.FP64, seed=8)]
    tickets = [ctx.submit(p, records=True) for p in ps]
    got = [ctx.wait(t, timeout_s=120) for t in tickets]
    for p, r in zip(ps, got):
        alone = ctx.solve(p, records=True)
        assert r["records"].tobytes() == alone["records"].tobytes()
        assert np.array_equal(r["mean"], alone["mean"])
    # cancel: either it is cancelled (wait reports it) or it had finished
    t = ctx.submit(W.unit_square(paths=64))
    st = ctx.cancel(t)
    if st == sdd.SDD_OK:
        with pytest.raises(sdd.SddError) as e:
            ctx.wait(t, timeout_s=60)
        assert e.value.status == sdd.SDD_E_CANCELLED
    else:
        assert st == sdd.SDD_E_BUSY
        assert ctx.wait(t, timeout_s=60)["paths_done"].sum() == 8 * 64
    with pytest.raises(sdd.SddError) as e:
        ctx.poll(987654321)
    assert e.value.status == sdd.SDD_E_NOTFOUND


def test_served_fp32_at_1e3_rel_se_within_3se_of_oracle(ctx, orc):
    """The served target: FP32-mixed requests of two families submitted
    together, each asking for a relative standard error of 1e-3 of |g|inf
    (pilot of 4096 paths, then the extension the pilot variance asks for),
    each node within 3 SE of the FP64 oracle on the same paths, and every SE
    at the target (25% slack for the pilot's variance estimate)."""
    ps = [W.unit_square(paths=1, precision=W.FP32_MIXED, dt=4e-4, n_nodes=4),
          W.layered_check(n_nodes=4, paths=1, dt=1e-3, precision=W.FP32_MIXED)]
    tickets = [ctx.submit(p, target_rel_se=1e-3) for p in ps]
    got = [ctx.wait(t, timeout_s=120) for t in tickets]
    for p, g in zip(ps, got):
        n = g["paths_done"].astype(np.uint32)
        log(f"{p.name}: paths {n.tolist()}, max SE / |g|inf {(g['se'] / p.g_norm).max():.3e}")
        assert np.all(n > 4096)
        assert np.all(g["se"] <= 1e-3 * p.g_norm * 1.25)
        o, _ = oracle_solve(orc, p.replace(path_begin=np.zeros(p.n_nodes, np.uint32), path_count=n))
        assert_within_se(g, o)


def test_served_time_slices_are_exact(ctx):
    """Tiny slices: walkers are suspended and resumed thousands of times;
    every result is still bitwise the blocking one (alone vs in the mix)."""
    ps = [small_mixed_model().with_paths(150), W.unit_square(paths=400, precision=W.FP32_MIXED, seed=3),
          W.quarter_space(paths=24, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 40)),
          W.block_in_half_space(10.0, paths=20, precision=W.FP64, M=1024).subset(np.arange(0, 1024, 90)),
          W.unit_square(paths=1, precision=W.FP32_MIXED, n_nodes=3, dt=4e-4)]
    try:
        ctx.set_tuning(slice_iters=8, tile_paths=37)
        tickets = [ctx.submit(p, records=True) for p in ps[:4]]
        tickets.append(ctx.submit(ps[4], target_rel_se=2e-2))
        got = [ctx.wait(t, timeout_s=100) for t in tickets]
        # generic-signature walkers (64-bit phase sums) suspended and resumed
        # in slices of the LDS-grid walker (the flight's launches hold one grid)
        gen = W.multi_body(seed=3, paths=64, M=1024).subset(np.arange(0, 128, 8))
        g_served = ctx.wait(ctx.submit(gen, records=True), timeout_s=100)
    finally:
        ctx.set_tuning()
    assert g_served["records"].tobytes() == ctx.solve(gen, records=True)["records"].tobytes()
    for p, r in zip(ps[:4], got[:4]):
        alone = ctx.solve(p, records=True)
        assert r["records"].tobytes() == alone["records"].tobytes()
        assert np.array_equal(r["mean"], alone["mean"]) and np.array_equal(r["se"], alone["se"])
    alone = ctx.solve(ps[4], target_rel_se=2e-2)
    assert np.array_equal(got[4]["mean"], alone["mean"]) and np.array_equal(got[4]["paths_done"], alone["paths_done"])


def test_served_slices_at_the_top_of_the_path_range(ctx):
    """Tiles that end at path 2^32, suspended and resumed in tiny slices:
    every path is walked once, bitwise as in a blocking solve."""
    top = np.array([0xFFFFFFFF - 299, 0xFFFFFFFF - 64, 0xFFFFFFFF, 0xFFFFFF00], np.uint32)
    cnt = np.array([300, 65, 1, 256], np.uint32)
    p = W.unit_square(paths=1, precision=W.FP32_MIXED, dt=4e-4, n_nodes=4).replace(path_begin=top,
                                                                                  path_count=cnt)
    try:
        ctx.set_tuning(slice_iters=8, tile_paths=37)
        r = ctx.wait(ctx.submit(p, records=True), timeout_s=100)
    finally:
        ctx.set_tuning()
    alone = ctx.solve(p, records=True)
    assert np.array_equal(r["paths_done"], cnt.astype(np.uint64))
    assert r["records"].tobytes() == alone["records"].tobytes()


def test_concurrent_callers_share_one_context(ctx):
    """Six host threads drive one context at once, mixing blocking solves,
    served requests and a prepared batch; every result is bitwise the one a
    single caller gets (one launch sequence at a time on the context's
    stream, the served worker yielding to waiting callers)."""
    import threading
    ps = [W.unit_square(paths=300, precision=W.FP32_MIXED, seed=s) for s in range(3)] + \
         [small_mixed_model().with_paths(100), W.unit_square(paths=200, precision=W.FP64, seed=9)]
    ref = [ctx.solve(p, records=True)["records"].tobytes() for p in ps]
    ok, errs = {}, []

    def worker(i):
        try:
            p, want = ps[i % len(ps)], ref[i % len(ps)]
            for r in range(3):
                kind = (i + r) % 3
                if kind == 0:
                    g = ctx.solve(p, records=True)
                elif kind == 1:
                    g = ctx.wait(ctx.submit(p, records=True), timeout_s=100)
                else:
                    b = ctx.batch([p], records=True)
                    try:
                        g = b.run()[0]
                    finally:
                        b.close()
                ok[(i, r)] = g["records"].tobytes() == want
        except Exception as e:   # reported below
            errs.append(repr(e))

    threads = [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(6)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=150)
    assert not any(t.is_alive() for t in threads), "a caller did not finish"
    assert not errs, errs
    assert len(ok) == 18 and all(ok.values()), ok


def test_served_requests_join_while_others_run(ctx):
    """Continuous batching: a small request submitted while a long one is on
    the GPU finishes first, and its result equals the blocking one."""
    big = W.quarter_space(paths=4096, precision=W.FP32_MIXED, M=2048)
    small = W.unit_square(paths=256, precision=W.FP32_MIXED, seed=21)
    t_big = ctx.submit(big)
    time.sleep(0.05)
    t_small = ctx.submit(small, records=True)
    r_small = ctx.wait(t_small, timeout_s=100)
    big_done_early = ctx.poll(t_big)
    r_big = big_done_early if big_done_early is not None else ctx.wait(t_big, timeout_s=100)
    assert big_done_early is None, "the long request should still be running"
    assert r_small["records"].tobytes() == ctx.solve(small, records=True)["records"].tobytes()
    assert r_big["paths_done"].sum() == big.total_paths


def test_served_slices_survive_a_narrower_launch(ctx):
    """Walkers suspended by a wide launch can outnumber the lanes of the next,
    narrower one (another tuning, or another walker build with less
    occupancy): the ones no wave resumes carry over to later slices and the
    result is still bitwise the blocking one."""
    p = W.quarter_space(paths=256, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 4))
    try:
        ctx.set_tuning(slice_iters=64)
        t = ctx.submit(p, records=True)
        time.sleep(0.02)
        ctx.set_tuning(slice_iters=64, blocks_per_cu=1, block_threads=64)
        r = ctx.wait(t, timeout_s=100)
    finally:
        ctx.set_tuning()
    alone = ctx.solve(p, records=True)
    assert r["records"].tobytes() == alone["records"].tobytes()
    assert np.array_equal(r["mean"], alone["mean"])


def test_batch_graph_replays_bitwise(ctx):
    """A prepared batch replayed as a HIP graph several times, with eager
    work and synchronisations in between: every replay equals the eager
    batch solve bitwise."""
    import torch
    ps = [small_mixed_model().with_paths(90), W.unit_square(paths=300, precision=W.FP32_MIXED, seed=12),
          W.quarter_space(paths=16, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 50))]
    eager = ctx.solve_batch(ps, records=True)
    b = ctx.batch(ps, records=True)
    try:
        times = []
        for rep in range(3):
            got = b.run()
            times.append(ctx.stats()["last_walk_ms"])
            for e, g in zip(eager, got):
                assert g["records"].tobytes() == e["records"].tobytes(), rep
                assert np.array_equal(g["mean"], e["mean"]) and np.array_equal(g["var_re"], e["var_re"])
            ctx.solve(W.unit_square(paths=64, seed=rep))   # eager work between replays
            torch.cuda.synchronize()
        # every replay times its own walk (the eager solves in between record
        # other timings)
        assert all(t > 0 for t in times)
        assert ctx.stats()["last_walk_ms"] not in times
    finally:
        b.close()


def test_autotune_changes_speed_not_results(ctx):
    """The autotuner's trials cover its candidate sweep, it leaves the chosen
    tuning on the context, and solves under that tuning are bitwise the
    solves under the default."""
    p = W.quarter_space(paths=64, precision=W.FP32_MIXED, M=1024).subset(np.arange(0, 512, 8))
    ref = ctx.solve(p, records=True)
    try:
        chosen, trials = ctx.autotune(p, sample_paths=64)
        assert len(trials) >= 8
        assert all(t["walk_ms"] > 0 and t["walk_steps_per_s"] > 0 for t in trials)
        assert ctx.get_tuning() == chosen
        assert chosen["block_threads"] in (64, 128, 256) and chosen["refill_every"] in (1, 2, 4, 8)
        fastest = min(t["walk_ms"] for t in trials[1:])
        assert any(t["walk_ms"] == fastest and all(t[k] == chosen[k] for k in chosen) for t in trials[1:])
        got = ctx.solve(p, records=True)
        assert got["records"].tobytes() == ref["records"].tobytes()
    finally:
        ctx.set_tuning()


def test_multi_frequency_one_walk(ctx, orc):
    """One walk weighted for four frequencies: each frequency's result
    matches the oracle solved at that frequency with the same streams (FP64
    bar); at the walk's own frequency it is bitwise the ordinary solve."""
    freqs = [0.1, 1.0, 10.0, 100.0]
    sel = [0, 130, 260, 400, 600, 1000]
    probs = [W.block_in_half_space(f, paths=48, precision=W.FP64, M=1024).subset(sel) for f in freqs]
    base = probs[1]
    got = ctx.solve_multi_freq(base, freqs, [q.g for q in probs])
    assert len(got) == 4
    for f, q, g in zip(freqs, probs, got):
        o, orec = oracle_solve(orc, q, records=True)
        log(f"multi-frequency fp64 f={f}")
        # The oracle sums the phase at frequency f; the one walk sums it at the
        # walk's frequency and scales.  The two sums of n terms differ by at
        # most n 2^-52 |S| (relative rounding per term), which moves a weight
        # by at most |g|max times that: per node, the mean of this bound.
        gmax = np.abs(q.g).max()
        bound = ((orec["steps"].astype(float) + 2) * 2.0 ** -52 * np.abs(orec["S"]) * gmax)
        bound = bound.reshape(q.n_nodes, -1).mean(axis=1)
        e_o = o["mean_re"] + 1j * o["mean_im"]
        d = np.abs(g["mean"] - e_o)
        assert np.all(d <= TOL_FP64 * np.fmax(np.abs(e_o), o["se"]) + bound), (f, d, bound)
        assert np.array_equal(g["steps"], o["steps"]) and np.array_equal(g["paths_done"], o["paths_done"])
        assert np.allclose(g["mean_exit_time"], o["mean_exit_time"], rtol=1e-12)
        assert np.allclose(g["se"], o["se"], rtol=1e-6)
    alone = ctx.solve(base)
    assert np.array_equal(got[1]["mean"], alone["mean"]) and np.array_equal(got[1]["se"], alone["se"])
    # FP32-mixed walk: within SE of the oracle at every frequency
    probs32 = [W.block_in_half_space(f, paths=2048, precision=W.FP32_MIXED, M=1024).subset(sel[:4])
               for f in freqs[:3]]
    got32 = ctx.solve_multi_freq(probs32[1], freqs[:3], [q.g for q in probs32])
    for q, g in zip(probs32, got32):
        o, _ = oracle_solve(orc, q)
        assert_within_se(g, o)
    with pytest.raises(sdd.SddError):
        ctx.solve_multi_freq(base, [1.0, -2.0], [probs[0].g, probs[1].g])


def test_mt_response_fp64_matches_oracle(ctx, orc):
    """Pointwise TE responses on the COMMEMI 2D-1 geometry: the fields at the
    three points of each site match the oracle (FP64 bar), and so do the
    apparent resistivity and phase computed from them."""
    ps = W.commemi_te_points(paths=48, sites=(0.0, 1.0), precision=W.FP64, M=2048)
    got = ctx.solve_batch(ps)
    exp = []
    for p, g in zip(ps, got):
        o, _ = oracle_solve(orc, p)
        assert_fp64_parity(g, o)
        exp.append(o["mean_re"] + 1j * o["mean_im"])
    rho, phi = sdd.mt_te_response(*[g["mean"] for g in got], 0.01, 1000.0, 10.0)
    rho_o, phi_o = sdd.mt_te_response(*exp, 0.01, 1000.0, 10.0)
    assert np.allclose(rho, rho_o, rtol=1e-5) and np.allclose(phi, phi_o, atol=1e-4)


def test_mt_response_half_space_physics(ctx):
    """TE apparent resistivity and phase of a uniform 100 ohm m half-space at
    10 Hz from the FP32 walk: rho_a within 12% of 100 (4 standard deviations
    of 2^18-path estimates, measured over seeds) and phase within 2.5 degrees
    of 45 (first-order differencing across the surface adds about 1%)."""
    ps = W.commemi_te_points(paths=1 << 18, sites=(0.0, 2.0, 4.0), block=False, dt=4e-4, h=0.05, M=8192)
    got = ctx.solve_batch(ps)
    rho, phi = sdd.mt_te_response(*[g["mean"] for g in got], 0.05, 1000.0, 10.0)
    log(f"half-space rho_a {rho} phase {phi}")
    assert np.all(np.abs(rho - 100.0) < 12.0) and np.all(np.abs(phi - 45.0) < 2.5)


def _surface_jump_bias(h_km):
    """|rho_a / 100 - 1| of the jump-corrected difference on the exact
    half-space (0.01 S/m under air, 10 Hz) at spacing h: its own bias."""
    al = W._alpha_of(np.array([0.0, 0.01]), 10.0, 1000.0, 0.0)
    e = W.layered_1d(np.array([W.COMMEMI_WALLS[2], 0.0]), al, np.array([-h_km, 0.0, h_km]))
    rho, _ = sdd.mt_te_response(*[np.atleast_1d(x) for x in e], h_km, 1000.0, 10.0, sigma_jump=0.01)
    return abs(rho[0] / 100.0 - 1.0)


def test_mt_response_commemi_within_table2(ctx):
    """TE apparent resistivity of COMMEMI 2D-1 at 10 Hz at the five sites of
    Sec. 4.3 (Table 2) from the FP32 walk: 16 independent seeds of 2^19 paths
    per point, the points h = 100 m above and below the surface at the two
    sites over the block (its top is 250 m down), 200 m at 1 km and 400 m at
    2 and 4 km, and the surface jump's first-order term removed from the
    difference (sdd_mt_te_response_jump).  The 16-seed mean lies inside the
    COMMEMI spread widened by its Monte-Carlo error (99% two-sided Student t,
    15 degrees of freedom, times the seed spread over 4) and by the
    difference's own bias on the exact half-space at the same h (at most
    0.13%).  At 2 and 4 km the Monte-Carlo part alone is narrower than the
    COMMEMI spread."""
    tab = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "commemi_te_table2.txt"))
    assert np.allclose(tab[:, 0], 1000.0 * np.asarray(W.COMMEMI_SITES_KM))
    H = np.asarray(W.COMMEMI_H_KM)
    n_seeds = 16
    rhos = []
    for seed in range(n_seeds):
        em, e0, ep = [g["mean"] for g in ctx.solve_batch(W.commemi_te_points(paths=1 << 19, seed=seed, dt=4e-4,
                                                                                h=H))]
        rhos.append([sdd.mt_te_response(em[j:j + 1], e0[j:j + 1], ep[j:j + 1], H[j], 1000.0, 10.0,
                                        sigma_jump=0.01)[0][0] for j in range(H.size)])
    rhos = np.array(rhos)
    mean, sd = rhos.mean(0), rhos.std(0, ddof=1)
    mc = stats.t.ppf(0.995, n_seeds - 1) * sd / math.sqrt(n_seeds)
    bias = np.array([_surface_jump_bias(h) for h in H]) * tab[:, 1]
    allow = tab[:, 2] + mc + bias
    log(f"COMMEMI rho_a {mean.round(2)} sd {sd.round(2)} MC allowance {mc.round(2)} bias {bias.round(3)}; "
        f"Table 2 {tab[:, 1]} +- {tab[:, 2]}")
    assert np.all(mc[3:] <= tab[3:, 2]), mc
    assert np.all(np.abs(mean - tab[:, 1]) <= allow), (mean - tab[:, 1]) / allow


def test_domain_decomposition_layered_model(ctx):
    """Stochastic domain decomposition end to end: FP32 walks at the 138
    interface nodes of air over a uniform half-space cut into three
    sub-domains, then RBF-FD in each; the field everywhere matches the exact
    1-D solution within the discretisation error (1.7e-4 at this grid) plus
    five standard errors of the interface walks."""
    from paper_1603_09311_amd import decompose as D
    walls = (-2.0, 2.0, -1.0, 3.0)
    h = 0.05
    y = np.arange(walls[0], walls[1] + 1e-9, h)
    z = np.arange(walls[2], walls[3] + 1e-9, h)
    iz0, iy0 = int(np.argmin(abs(z))), int(np.argmin(abs(y)))
    subs = [D.SubDomain(0, y.size - 1, 0, iz0, 0.0), D.SubDomain(0, iy0, iz0, z.size - 1, 2.0),
            D.SubDomain(iy0, y.size - 1, iz0, z.size - 1, 2.0)]
    p = W.layered_check(alpha_ground=2.0, walls=walls, paths=16384, precision=W.FP32_MIXED)
    regions = [W.Region(W.HALF_Z_LT, (0.0,), 0.0)]
    ex = W.column_field(regions, 1.0, y, z, walls[2], 0.0, 1.0, alpha_direct=2.0)
    outer = W.column_field(regions, 1.0, y, z, walls[2], 0.0, 1.0, alpha_direct=2.0, boundary_only=True)
    F, r = D.decompose(ctx, p, y, z, subs, outer, 1.0)
    assert r["mean"].size == 138
    err = np.abs(F - ex).max()
    log(f"decomposition: max error {err:.3e}, max interface SE {r['se'].max():.3e}")
    assert err <= 1.7e-4 + 5.0 * r["se"].max()


def test_both_precisions_match_the_exact_scheme_on_a_strip(ctx):
    """The walkers as discrete schemes, at a finite dt with no bias
    allowance: on the strip -1 < z < 1 (air over ground of rate 20, the side
    walls out of reach) the scheme's exact expectation (te_chain, its Markov
    chain evaluated with no sampling) against the FP64 and the FP32-mixed
    persistent walkers at dt = 1e-2 and 10^7 paths per node: within 4 SE per
    component plus 3e-5 (the chain's quadrature error is about 1e-5)."""
    import te_chain as TC
    zs = (-0.5, -0.05, 0.05, 0.5)
    chain = TC.z_strip_chain(20.0, 1e-2)
    exact = np.array([chain.value(z) for z in zs])
    for prec in (W.FP64, W.FP32_MIXED):
        r = ctx.solve(TC.z_strip_problem(20.0, 1e-2, zs, 10_000_000, precision=prec))
        d = r["mean"] - exact
        log(f"z strip precision {prec}: diff/se re {d.real / r['se_re']} im {d.imag / r['se_im']}")
        assert np.all(np.abs(d.real) <= 4.0 * r["se_re"] + 3e-5), (d, r["se_re"])
        assert np.all(np.abs(d.imag) <= 4.0 * r["se_im"] + 3e-5), (d, r["se_im"])
        assert np.all(r["unfinished"] == 0)


def test_generic_signature_matches_the_exact_scheme_on_a_strip(ctx):
    """The generic signature's walkers as discrete schemes: air over two
    full-width layers (sigma 3 on 0 <= z < 0.3, 0.5 on 0.3 <= z < 0.6) over
    the background, three primitives, so the FP32-mixed walk looks regions up
    in the sigma grid (in LDS, in global memory, or by the primitive loop) and
    sums fixed-point phases; the FP64 walk loops over the primitives.  Each
    against the scheme's exact expectation (te_chain) at dt = 1e-2 and 10^7
    paths per node, within 4 SE per component plus 3e-5; the three FP32
    lookups give the same records bit for bit."""
    import te_chain as TC
    layers = ((0.0, 0.3, 3.0), (0.3, 0.6, 0.5))
    zs = (-0.5, -0.05, 0.05, 0.32, 0.7)
    chain = TC.z_strip_chain(20.0, 1e-2, layers=layers)
    exact = np.array([chain.value(z) for z in zs])
    p64 = TC.z_strip_problem(20.0, 1e-2, zs, 10_000_000, precision=W.FP64, layers=layers)
    p32 = TC.z_strip_problem(20.0, 1e-2, zs, 10_000_000, precision=W.FP32_MIXED, layers=layers)
    runs = [("fp64", ctx.solve(p64)), ("fp32 lds grid", ctx.solve(p32)),
            ("fp32 global grid", ctx.solve(p32, flags=sdd.SDD_FLAG_NO_LDS_GRID)),
            ("fp32 primitive loop", ctx.solve(p32, flags=sdd.SDD_FLAG_NO_SIGMA_GRID))]
    for name, r in runs:
        d = r["mean"] - exact
        log(f"layered strip {name}: diff/se re {d.real / r['se_re']} im {d.imag / r['se_im']}")
        assert np.all(np.abs(d.real) <= 4.0 * r["se_re"] + 3e-5), (name, d, r["se_re"])
        assert np.all(np.abs(d.imag) <= 4.0 * r["se_im"] + 3e-5), (name, d, r["se_im"])
        assert np.all(r["unfinished"] == 0)
    for name, r in runs[2:]:
        assert np.array_equal(r["mean"], runs[1][1]["mean"]) and np.array_equal(r["steps"], runs[1][1]["steps"]), name


def test_multi_frequency_one_walk_matches_the_exact_scheme_on_a_strip(ctx):
    """The multi-frequency fan-out as a discrete scheme: one FP32-mixed walk
    on the strip (air over ground) weighted for rates 5, 20 and 80 (the
    walk's own rate 20 sets the phase scale), each against the exact
    expectation of the scheme at that rate (te_chain), dt = 1e-2 and 10^7
    paths per node: within 4 SE per component plus 3e-5."""
    import te_chain as TC
    zs = (-0.5, -0.05, 0.05, 0.5)
    rates = (5.0, 20.0, 80.0)
    p = TC.z_strip_problem(20.0, 1e-2, zs, 10_000_000, precision=W.FP32_MIXED)
    got = ctx.solve_multi_freq(p, list(rates), [p.g] * len(rates))
    for alpha, r in zip(rates, got):
        chain = TC.z_strip_chain(alpha, 1e-2)
        exact = np.array([chain.value(z) for z in zs])
        d = r["mean"] - exact
        log(f"strip fan-out rate {alpha}: diff/se re {d.real / r['se_re']} im {d.imag / r['se_im']}")
        assert np.all(np.abs(d.real) <= 4.0 * r["se_re"] + 3e-5), (alpha, d, r["se_re"])
        assert np.all(np.abs(d.imag) <= 4.0 * r["se_im"] + 3e-5), (alpha, d, r["se_im"])
