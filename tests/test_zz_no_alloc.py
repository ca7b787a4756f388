"""The allocation-free walk launch (wos_build_measure_noalloc) against wos_build_measure.

Its scratch lives in a static device array shared by every call on the GPU, so the test makes two
calls in a row, the second with a smaller input of another kind (polygon records staged, FP64
point mode with one work cursor per point), and compares counts, statistics and per-walk traces
with those of the allocating entry point bit for bit; a descriptor too large for the array is
refused on the host.
"""
import numpy as np
import pytest

import wos_inputs as wi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def wos():
    from paper_2409_03686_amd import wos as w
    w.lib()
    return w


@pytest.fixture(scope="module")
def ctx(wos):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = wos.wos_create(0)
    yield c
    wos.wos_destroy(c)


def _run(wos, ctx, inst, noalloc, precision, trace):
    M = wos.wos_element_count(inst.geom)
    n = inst.x_obs.shape[0]
    x = wos.device_inputs(inst)
    counts = torch.zeros((n, M), dtype=torch.int32, device="cuda")
    stats = torch.zeros(wos.WOS_STATS_WORDS, dtype=torch.int64, device="cuda")
    tr = torch.zeros((n, inst.n_walks, 2), dtype=torch.int32, device="cuda") if trace else None
    w = wos.walk_params_of(inst, precision=precision)
    f = wos.wos_build_measure_noalloc if noalloc else wos.wos_build_measure
    f(ctx, inst.geom, w, x, n, counts, stats, tr)
    torch.cuda.synchronize()
    return (counts.cpu().numpy(), stats.cpu().numpy(), None if tr is None else tr.cpu().numpy())


def _lshape(n_obs, n_walks):
    rng = np.random.default_rng(11)
    g = wi.Geometry(2, wi.POLYGON, (), (120,), verts=wi.L_SHAPE)
    g.gamma1_mask = (np.arange(120) % 2).astype(np.uint8)
    x = wi.sample_points(g, n_obs, rng, margin=0.02)
    return wi.Instance(g, np.array([[1.0, 0.5], [0.5, 2.0]]), x, n_walks, eps=1e-4, seed=3,
                       precision=wi.FP64, radius_mode=wi.RADIUS_MAPPED_EXACT, name="lshape")


def test_noalloc_matches_allocating_launch_twice(wos, ctx):
    first = wi.cfg2_annulus(n_walks=4000, n_obs=512, precision=wi.FP32_GEOM_FP64_EXIT)
    second = _lshape(48, 1500)
    for inst, prec, trace in ((first, wi.FP32_GEOM_FP64_EXIT, False), (second, wi.FP64, True)):
        ref = _run(wos, ctx, inst, False, prec, trace)
        got = _run(wos, ctx, inst, True, prec, trace)
        assert np.array_equal(got[0], ref[0]), inst.name
        assert np.all(got[0].view(np.uint32).sum(1) == inst.n_walks)
        assert np.array_equal(got[1], ref[1]), inst.name
        if trace:
            assert np.array_equal(got[2], ref[2])
        print(f"noalloc {inst.name}: {inst.x_obs.shape[0]} x {inst.n_walks} walks, counts and statistics equal")


def test_noalloc_refuses_oversized_descriptor(wos, ctx):
    # 2048 Bauer nodes on a ball: 2048 staged node records (96 B each) exceed the 64 KiB descriptor
    g = wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (2048, 0))
    g.gamma1_mask = np.ones(2048, np.uint8)
    x = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    counts = torch.zeros((4, 2048), dtype=torch.int32, device="cuda")
    w = wos.walk_params(np.eye(3), 1e-4, 0, 10)
    with pytest.raises(wos.WosError):
        wos.wos_build_measure_noalloc(ctx, g, w, x, 4, counts)
    torch.cuda.synchronize()
    assert int(counts.sum()) == 0


def test_noalloc_small_mesh_matches_allocating_launch(wos, ctx):
    """A small triangle mesh (the L-prism of 44 triangles) with the mapped-exact radius in FP32: both
    hierarchies (about 24 KB of records) fit the descriptor, and the allocation-free launch equals the
    allocating one bit for bit, counts, statistics and traces."""
    rng = np.random.default_rng(12)
    g = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.l_prism_mesh(2))
    x = wi.sample_points(g, 24, rng)
    K = np.array([[1.0, 0.3, 0.1], [0.3, 0.6, -0.2], [0.1, -0.2, 0.4]])
    inst = wi.Instance(g, K, x, 800, eps=1e-4, seed=4, precision=wi.FP32_GEOM_FP64_EXIT,
                       radius_mode=wi.RADIUS_MAPPED_EXACT, name="lprism")
    ref = _run(wos, ctx, inst, False, wi.FP32_GEOM_FP64_EXIT, True)
    got = _run(wos, ctx, inst, True, wi.FP32_GEOM_FP64_EXIT, True)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    assert np.all(got[0].sum(1) == 800)
