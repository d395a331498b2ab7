"""Per-face density weights on the GPU (dm_topology_set_weights): cell
clusters rendered as the paper's multimaterial meshes (walls as double
membranes, Sec. 3.3) and as piecewise-constant densities, against the
FP64 oracle's weighted transforms."""
import sys

import numpy as np
import pytest

from helpers import f32, f32_grid, rel_l2
from workloads import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_10440_amd as m
    return m


@pytest.fixture(scope="module")
def handle(dm):
    return dm.Handle(0)


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda:0")


def _small(mode, seed=0):
    return configs.foam_case(mode, seed=seed, cells=(2, 2, 2), sub=2, n=(32, 32, 32), spacing=(1.0, 1.0, 1.0),
                             block=16.0, sigma=(1.0, 2.0))


@pytest.mark.parametrize("mode", [configs.VOLUME, configs.SURFACE])
def test_weighted_cluster_image_and_gradients(dm, handle, ref, mode):
    c = _small(mode)
    g = f32_grid(c.grid)
    w = c.extra["tri_w"]
    say("weighted cluster", mode, c.F.shape[0], "faces")
    topo = handle.topology(c.F, n_verts=len(c.V))
    topo.set_weights(w)
    assert topo.closed == (mode == configs.VOLUME)
    V64, S64, w64 = c.V.astype(np.float64), tuple(float(f32(x)) for x in c.sigma), w.astype(np.float64)
    img = dm.render(handle, dev(c.V), topo, c.sigma, g).cpu().numpy()
    want = ref.render(V64, c.F, g, S64, tri_w=w64)
    e_img = rel_l2(img, want)
    G = np.random.default_rng(3).standard_normal(g.n).astype(np.float32)
    dv, ds, _ = dm.render_vjp(handle, dev(c.V), topo, c.sigma, g, dev(G))
    dvw, dsw = ref.render_vjp(V64, c.F, g, S64, G.astype(np.float64), tri_w=w64)
    e_dv, e_ds = rel_l2(dv.cpu().numpy(), dvw), rel_l2(ds.cpu().numpy(), dsw)
    say("  image", e_img, "dV", e_dv, "dSigma", e_ds)
    assert e_img < 1e-5 and e_dv < 1e-4 and e_ds < 1e-4


def test_unit_weights_are_bitwise_the_unweighted_render_and_can_be_removed(dm, handle):
    import torch
    c = _small(configs.SURFACE)
    g = f32_grid(c.grid)
    topo = handle.topology(c.F, n_verts=len(c.V))
    G = dev(np.random.default_rng(4).standard_normal(g.n))
    a = dm.render_vjp(handle, dev(c.V), topo, c.sigma, g, G, want_image=True)
    topo.set_weights(np.ones(c.F.shape[0]))
    b = dm.render_vjp(handle, dev(c.V), topo, c.sigma, g, G, want_image=True)
    topo.set_weights(c.extra["tri_w"])
    d = dm.render(handle, dev(c.V), topo, c.sigma, g)
    topo.set_weights(None)
    e = dm.render_vjp(handle, dev(c.V), topo, c.sigma, g, G, want_image=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    for x, y in zip(a, e):
        assert torch.equal(x, y)
    assert not torch.equal(d, a[2])


def test_volume_needs_weights_that_close_and_finite_weights(dm, handle):
    c = _small(configs.VOLUME)
    g = f32_grid(c.grid)
    topo = handle.topology(c.F, n_verts=len(c.V))
    assert not topo.closed                    # the cluster itself is not a closed manifold
    with pytest.raises(Exception):
        dm.render(handle, dev(c.V), topo, c.sigma, g)
    w = c.extra["tri_w"].copy()
    w[0] += 0.25                              # one face off: the density is no longer consistent
    topo.set_weights(w)
    assert not topo.closed
    with pytest.raises(Exception):
        dm.render(handle, dev(c.V), topo, c.sigma, g)
    topo.set_weights(c.extra["tri_w"])
    assert topo.closed
    dm.render(handle, dev(c.V), topo, c.sigma, g)
    bad = c.extra["tri_w"].copy()
    bad[3] = np.nan
    with pytest.raises(Exception):
        topo.set_weights(bad)


def test_weighted_cluster_in_a_batch_equals_the_single_call(dm, handle):
    import torch
    c = configs.foam_case(configs.SURFACE, cells=(2, 2, 2), sub=4, n=(64, 64, 64), spacing=(1.0, 1.0, 1.0),
                          block=32.0, sigma=(1.0, 2.0))
    topo = handle.topology(c.F, n_verts=len(c.V))
    topo.set_weights(c.extra["tri_w"])
    G = dev(np.random.default_rng(5).standard_normal(c.grid.n))
    single = dm.render_vjp(handle, dev(c.V), topo, c.sigma, c.grid, G, want_image=True)
    batch = dm.batch_run(handle, [(dev(c.V), topo, c.sigma, c.grid, G)])[0]
    torch.cuda.synchronize()
    e = rel_l2(batch[0].cpu().numpy(), single[2].cpu().numpy())
    ev = rel_l2(batch[1].cpu().numpy(), single[0].cpu().numpy())
    say("batch vs single: image", e, "dV", ev)
    assert e < 1e-5 and ev < 1e-4
