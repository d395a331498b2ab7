"""Smoothed vertex update (I + lambda L)^{-2} g on the GPU (dm_laplace_smooth)
against the FP64 oracle and closed forms.

Meshes of at most 3072 vertices (degrees <= 8) are solved by conjugate
gradients in one workgroup, larger ones (and higher degrees) by Chebyshev
iteration whose step count bounds the residual.  Tolerance: a solve stopped at
relative residual tol leaves a relative error of at most cond(I + lambda L) *
tol; with vertex degree <= 6 (icospheres) or <= 7 and lambda = 50 the
condition number is below 1 + 50 * 2 * 7 = 701, so tol = 1e-7 bounds the
error by 7e-5, inside the 1e-4 gradient tolerance."""
import sys

import numpy as np
import pytest

from oracle import smoothing as S
from workloads import configs, meshes

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _meshes():
    c1, c3 = configs.cfg1(), configs.cfg3()
    Vg, Fg = meshes.geodesic_sphere(45)
    return [("cfg1 sphere", c1.F, len(c1.V)), ("cfg3 cell", c3.F, len(c3.V)), ("geodesic-45", Fg, len(Vg))]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_smooth_matches_oracle(dm, handle, idx):
    name, F, nv = _meshes()[idx]
    say("laplace smooth vs oracle:", name, nv, "vertices")
    rng = np.random.default_rng(idx)
    g = rng.standard_normal((nv, 3)).astype(np.float32)
    topo = handle.topology(F, n_verts=nv)
    out, info = dm.laplace_smooth(handle, topo, dev(g), lam=50.0, max_iter=5000, tol=1e-7, with_info=True)
    want = S.laplace_smooth(F, nv, g.astype(np.float64), 50.0)
    err = rel(out.cpu().numpy().astype(np.float64), want)
    say("  rel L2", err, "info", info)
    assert err < 1e-4
    assert info["iters"][0] < 5000 and info["iters"][1] < 5000
    assert info["residual"][0] < 1e-6 and info["residual"][1] < 1e-6


def test_closed_forms_identity_alias_and_isolated_vertex(dm, handle):
    import torch
    F = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]])
    opp = np.array([1, 0, 3, 2, 5, 4])
    rng = np.random.default_rng(7)
    g = rng.standard_normal((6, 3)).astype(np.float32)
    lam = 3.0
    gd = g.astype(np.float64)
    mean = gd.mean(0, keepdims=True)
    want = mean + 0.5 * (gd - gd[opp]) / (1 + 4 * lam) ** 2 + (0.5 * (gd + gd[opp]) - mean) / (1 + 6 * lam) ** 2
    topo = handle.topology(F, n_verts=6)
    got = dm.laplace_smooth(handle, topo, dev(g), lam=lam, tol=1e-7).cpu().numpy()
    say("octahedron closed form rel", rel(got, want))
    assert rel(got, want) < 1e-6
    # lambda = 0: one iteration, alpha = 1 exactly, so the identity is exact
    x = dev(g)
    assert torch.equal(dm.laplace_smooth(handle, topo, x, lam=0.0), x)
    # out may be the input array; two calls are bitwise identical
    V, Fi = meshes.icosphere(2)
    nv = len(V) + 1                    # the last vertex is on no edge
    topo2 = handle.topology(Fi, n_verts=nv)
    g2 = rng.standard_normal((nv, 3)).astype(np.float32)
    a = dm.laplace_smooth(handle, topo2, dev(g2), lam=50.0, tol=1e-7)
    b = dm.laplace_smooth(handle, topo2, dev(g2), lam=50.0, tol=1e-7)
    y = dev(g2)
    dm.laplace_smooth(handle, topo2, y, lam=50.0, tol=1e-7, out=y)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, y)
    # the isolated vertex's row is the identity: the solves return its value to their tolerance
    assert np.allclose(a.cpu().numpy()[-1], g2[-1], rtol=1e-5, atol=1e-6 * float(np.abs(g2).max()))
    want2 = S.laplace_smooth(Fi, nv, g2.astype(np.float64), 50.0)
    say("isolated-vertex mesh rel", rel(a.cpu().numpy(), want2))
    assert rel(a.cpu().numpy(), want2) < 1e-4


def test_open_mesh_and_errors(dm, handle):
    V, F = meshes.icosphere(3)
    cz = V[F].mean(1)[:, 2]
    Fh = F[cz > 0.0]
    used = np.unique(Fh)
    remap = -np.ones(len(V), int)
    remap[used] = np.arange(len(used))
    Fh = remap[Fh]
    nv = len(used)
    rng = np.random.default_rng(9)
    g = rng.standard_normal((nv, 3)).astype(np.float32)
    topo = handle.topology(Fh, n_verts=nv)
    assert not topo.closed
    got = dm.laplace_smooth(handle, topo, dev(g), lam=50.0, tol=1e-7).cpu().numpy()
    err = rel(got, S.laplace_smooth(Fh, nv, g.astype(np.float64), 50.0))
    say("open hemisphere rel", err)
    assert err < 1e-4
    for kw in ({"lam": -1.0}, {"lam": float("nan")}, {"tol": 0.0}, {"max_iter": 0}):
        with pytest.raises(Exception):
            dm.laplace_smooth(handle, topo, dev(g), **kw)


def test_high_degree_vertices_use_the_list_path(dm, handle):
    """A 12-sided bipyramid: its apexes have degree 12, above the width of
    the neighbour table, so the adjacency lists are used."""
    n = 12
    ang = 2 * np.pi * np.arange(n) / n
    V = np.concatenate([np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], 1), [[0, 0, 1.0], [0, 0, -1.0]]])
    top, bot = n, n + 1
    F = np.array([[i, (i + 1) % n, top] for i in range(n)] + [[(i + 1) % n, i, bot] for i in range(n)])
    assert meshes.check_closed_oriented(F)
    rng = np.random.default_rng(11)
    g = rng.standard_normal((n + 2, 3)).astype(np.float32)
    topo = handle.topology(F, n_verts=n + 2)
    got = dm.laplace_smooth(handle, topo, dev(g), lam=50.0, tol=1e-7).cpu().numpy()
    err = rel(got, S.laplace_smooth(F, n + 2, g.astype(np.float64), 50.0))
    say("bipyramid (degree 12) rel", err)
    assert err < 1e-4
