"""GPU parity: the HIP path against the FP64 oracle, element by element.

Tolerances (float32 kernels vs float64 oracle): images and spectra within
1e-5 relative L2, gradients within 1e-4 relative L2; band membership and
frequency lists bit-exact."""
import dataclasses
import sys

import numpy as np
import pytest

from helpers import expected_band, f32_grid, f32_sigma, rel_l2, sort_entries
from workloads import configs, meshes

pytestmark = pytest.mark.gpu

VOLUME, SURFACE = configs.VOLUME, configs.SURFACE
IMG_TOL, GRAD_TOL = 1e-5, 1e-4


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
    return torch.tensor(np.ascontiguousarray(x), device="cuda:0")


def prepared(case, mode=None):
    g = f32_grid(case.grid if mode is None else case.grid.with_mode(mode))
    S = f32_sigma(case.sigma)
    return case.V, case.F, g, S


# ------------------------------------------------------------------ band
@pytest.mark.parametrize("name", ["cfg1", "cfg3", "odd_general", "tau0", "tau_big"])
def test_band_bit_exact(dm, handle, ref, name):
    say("band", name)
    if name == "cfg1":
        c = configs.cfg1()
        g, S = f32_grid(c.grid), f32_sigma(c.sigma)
    elif name == "cfg3":
        c = configs.cfg3()
        g, S = f32_grid(c.grid), f32_sigma(c.sigma)
    elif name == "odd_general":
        g = f32_grid(configs.Grid((15, 18, 11), (0.9, 1.1, 1.7), (0.3, -0.2, 0.5), 2e-2, VOLUME))
        S = f32_sigma((1.3, 0.9, 2.2, 0.35, -0.2, 0.15))
    elif name == "tau0":
        g = f32_grid(configs.Grid((12, 10, 8), (1.0, 1.0, 1.0), (0, 0, 0), 0.0, VOLUME))
        S = f32_sigma((1.0, 1.0, 4.0, 0.0, 0.0, 0.0))
    else:
        g = f32_grid(configs.Grid((12, 10, 8), (1.0, 1.0, 1.0), (0, 0, 0), 1.5, VOLUME))
        S = f32_sigma((1.0, 1.0, 4.0, 0.0, 0.0, 0.0))
    got = dm.band_export(handle, g, S)
    pos, k, w = expected_band(ref, g, S)
    assert len(got["pos"]) == len(pos)
    if name == "tau0":
        n0, n1, n2 = g.n
        assert len(pos) >= n0 * n1 * (n2 // 2 + 1)
    if name == "tau_big":
        assert len(pos) == 0
        return
    a = sort_entries(got["pos"], got["k"])
    b = sort_entries(pos, k)
    assert np.array_equal(got["pos"][a], pos[b])
    assert np.array_equal(got["k"][a], k[b])
    assert np.array_equal(got["weight"][a].astype(np.float64), w[b])


# ------------------------------------------------------- mesh transform
def _k_samples(g, rng, n=300):
    K = np.stack([rng.integers(-g.n[j] // 2, (g.n[j] + 1) // 2, size=n) for j in range(3)], 1)
    special = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [-g.n[0] // 2, 0, 0], [0, g.n[1] // 2, 3],
                        [2, -3, -(g.n[2] // 2)], [0, 0, 5], [4, 0, 0]])
    return np.concatenate([special, K]).astype(np.int32)


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
@pytest.mark.parametrize("shape", ["sphere", "box", "cfg3"])
def test_mesh_transform_pointwise(dm, handle, ref, mode, shape):
    say("mesh_transform", shape, mode)
    if shape == "sphere":
        c = configs.cfg1(mode)
    elif shape == "box":
        c = configs.box_case(mode=mode)
    else:
        c = configs.cfg3(mode)
    V, F, g, S = prepared(c, mode)
    rng = np.random.default_rng(5)
    K = _k_samples(g, rng)
    topo = handle.topology(F, n_verts=len(V))
    got = dm.mesh_transform(handle, dev(V), topo, g, dev(K)).cpu().numpy().astype(np.complex128)
    want = ref.mesh_transform(V.astype(np.float64), F, ref.xi_of_k(K, g), g, mode)
    scale = np.abs(want).max()
    err = np.abs(got - want)
    say("  max err / scale", err.max() / scale, "rel l2", rel_l2(got, want))
    assert err.max() < 2e-6 * scale, (err.max() / scale)
    assert rel_l2(got, want) < IMG_TOL


# ------------------------------------------------------------ rendering
def _render_case(name, mode):
    if name == "cfg1":
        return configs.cfg1(mode)
    if name == "box":
        return configs.box_case(mode=mode)
    if name == "odd_general":
        U, F = meshes.icosphere(2)
        g = configs.Grid((15, 18, 11), (0.9, 1.1, 1.7), (0.3, -0.2, 0.5), 2e-2, mode)
        V = meshes.sh_deform(U, 3.5, np.random.default_rng(3)) + g.centre
        return configs.Case("odd_general", V.astype(np.float32), F.astype(np.int32), g,
                            (1.3, 0.9, 2.2, 0.35, -0.2, 0.15))
    if name == "tau0":
        c = configs.sphere_case(1, 4.0, (16, 12, 10), (1, 1, 1), 1.0, 1.5, 0.0, mode)
        return c
    raise KeyError(name)


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
@pytest.mark.parametrize("name", ["cfg1", "box", "odd_general", "tau0"])
def test_render_image_and_spectrum(dm, handle, ref, name, mode):
    say("render", name, mode)
    c = _render_case(name, mode)
    V, F, g, S = prepared(c, mode)
    topo = handle.topology(F, n_verts=len(V))
    img, spec = dm.render(handle, dev(V), topo, S, g, spectrum=True)
    img = img.cpu().numpy().astype(np.float64)
    want = ref.render(V.astype(np.float64), F, g, S)
    say("  rel err image", rel_l2(img, want))
    assert rel_l2(img, want) < IMG_TOL, rel_l2(img, want)
    band = dm.band_export(handle, g, S)
    u_want = ref.mesh_transform(V.astype(np.float64), F, ref.xi_of_k(band["k"], g), g, mode)
    u_got = spec.cpu().numpy().astype(np.float64)
    u_got = u_got[:, 0] + 1j * u_got[:, 1]
    assert rel_l2(u_got, u_want) < IMG_TOL
    # image integral = transform at zero frequency (volume, or one for the surface density)
    total = img.sum() * np.prod(g.spacing)
    dc = np.prod(g.spacing) * want.sum()
    assert abs(total - dc) < 1e-5 * abs(dc)


def _surface_only_case(name):
    """Meshes only the surface density accepts: an open hemisphere (boundary
    edges, unused vertices), a box with a fin (an edge shared by three faces)
    and a sphere with two zero-area triangles (which add nothing)."""
    if name == "hemisphere":
        c = configs.cfg1(SURFACE)
        U, F = meshes.icosphere(2)
        F = F[U[F].mean(axis=1)[:, 2] > 0.1]
        return configs.Case("hemisphere", c.V, F.astype(np.int32), c.grid, c.sigma)
    if name == "degenerate":
        # zero-area triangles: a repeated vertex, and three points on one
        # axis-aligned line (collinear exactly, in float32 and in float64)
        c = configs.cfg1(SURFACE)
        n = len(c.V)
        line = [[10.0, 12.5, 14.0], [11.5, 12.5, 14.0], [13.25, 12.5, 14.0]]
        V = np.concatenate([c.V, line]).astype(np.float32)
        F = np.concatenate([c.F, [[0, 0, 1], [n, n + 1, n + 2]]]).astype(np.int32)
        return configs.Case("degenerate", V, F, c.grid, c.sigma)
    box = configs.box_case(mode=SURFACE)
    V = np.concatenate([box.V, [[15.0, 25.0, 16.0]]]).astype(np.float32)
    F = np.concatenate([box.F, [[box.F[0][0], box.F[0][1], len(box.V)]]]).astype(np.int32)
    return configs.Case("fin", V, F, box.grid, box.sigma)


@pytest.mark.parametrize("name", ["hemisphere", "fin", "degenerate"])
def test_surface_open_and_nonmanifold_meshes(dm, handle, ref, name):
    say("surface", name)
    c = _surface_only_case(name)
    V, F, g, S = prepared(c, SURFACE)
    topo = handle.topology(F, n_verts=len(V))
    img = dm.render(handle, dev(V), topo, S, g).cpu().numpy().astype(np.float64)
    want = ref.render(V.astype(np.float64), F, g, S)
    say("  rel err image", rel_l2(img, want))
    assert rel_l2(img, want) < IMG_TOL
    G = np.random.default_rng(12).standard_normal(g.n).astype(np.float32)
    dv, ds, _ = dm.render_vjp(handle, dev(V), topo, S, g, dev(G))
    dvw, dsw = ref.render_vjp(V.astype(np.float64), F, g, S, G.astype(np.float64))
    say("  rel err dV", rel_l2(dv.cpu().numpy(), dvw), "dSigma", rel_l2(ds.cpu().numpy(), dsw))
    assert rel_l2(dv.cpu().numpy(), dvw) < GRAD_TOL
    assert rel_l2(ds.cpu().numpy(), dsw) < GRAD_TOL


def test_render_empty_band_gives_zero_image(dm, handle, ref):
    say("render empty band")
    c = configs.cfg1()
    V, F, g, S = prepared(c)
    g = dataclasses.replace(g, tau=1.0)
    topo = handle.topology(F, n_verts=len(V))
    img = dm.render(handle, dev(V), topo, S, g)
    assert float(img.abs().max()) == 0.0


def test_mesh_without_triangles(dm, handle, ref):
    """A mesh with vertices but no triangles: the surface density renders a
    zero image and zero gradients (vertex and PSF), alone and inside a batch
    next to a non-empty request, and the mesh transform is zero; the
    indicator density refuses it (no enclosed region: not a closed
    surface)."""
    import torch
    say("mesh without triangles")
    c = configs.cfg1(SURFACE)
    V, F, g, S = prepared(c, SURFACE)
    V0 = V[:5].copy()
    F0 = np.zeros((0, 3), np.int32)
    topo0 = handle.topology(F0, n_verts=len(V0))
    G = np.random.default_rng(3).standard_normal(g.n).astype(np.float32)
    dv, ds, img = dm.render_vjp(handle, dev(V0), topo0, S, g, dev(G), want_image=True)
    assert tuple(dv.shape) == (5, 3)
    assert float(img.abs().max()) == 0.0 and float(dv.abs().max()) == 0.0 and float(ds.abs().max()) == 0.0
    K = _k_samples(g, np.random.default_rng(4), n=20)
    u = dm.mesh_transform(handle, dev(V0), topo0, g, dev(K))
    assert float(u.abs().max()) == 0.0
    topo = handle.topology(F, n_verts=len(V))
    out = dm.batch_run(handle, [(dev(V0), topo0, S, g, dev(G)), (dev(V), topo, S, g, dev(G))])
    alone = dm.batch_run(handle, [(dev(V), topo, S, g, dev(G))])
    torch.cuda.synchronize()
    assert all(float(x.abs().max()) == 0.0 for x in out[0])
    assert all(torch.equal(a, b) for a, b in zip(out[1], alone[0]))
    with pytest.raises(dm.DeltamicError):
        dm.render(handle, dev(V0), topo0, S, g.with_mode(VOLUME))


# ------------------------------------------------------------- gradients
@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
@pytest.mark.parametrize("name", ["cfg1", "box", "odd_general", "tau0"])
def test_vjp_random_cotangent(dm, handle, ref, name, mode):
    say("vjp", name, mode)
    c = _render_case(name, mode)
    V, F, g, S = prepared(c, mode)
    rng = np.random.default_rng(11)
    G = rng.standard_normal(g.n).astype(np.float32)
    topo = handle.topology(F, n_verts=len(V))
    dv, ds, img = dm.render_vjp(handle, dev(V), topo, S, g, dev(G), want_image=True)
    dvw, dsw = ref.render_vjp(V.astype(np.float64), F, g, S, G.astype(np.float64))
    say("  rel err dV", rel_l2(dv.cpu().numpy(), dvw), "dSigma", rel_l2(ds.cpu().numpy(), dsw))
    assert rel_l2(dv.cpu().numpy(), dvw) < GRAD_TOL, rel_l2(dv.cpu().numpy(), dvw)
    assert rel_l2(ds.cpu().numpy(), dsw) < GRAD_TOL, (ds.cpu().numpy(), dsw)
    want = ref.render(V.astype(np.float64), F, g, S)
    assert rel_l2(img.cpu().numpy(), want) < IMG_TOL


def test_largest_serving_shape_at_sampled_outputs(dm, handle, ref):
    """The largest request of the serving workload: a deformed geodesic
    sphere of 40,500 triangles in the 256x256x128 grid (unit voxels,
    sigma_xy = 1, band about 1.5M entries, |k| up to 128, so vertex phases
    reach about 40 revolutions), in the launch configuration of a single call.
    Checked on what the oracle can evaluate at this size: the band spectrum
    of dm_render at 600 sampled band entries (the extreme frequencies
    included), the mesh transform at 300 sampled frequencies, the image's
    integral (the k = 0 term, the enclosed volume) and the gradients of 4
    sampled vertices (from the triangles around them)."""
    import torch
    say("largest serving shape")
    c = configs.random_cell(np.random.default_rng(11), 40000, 40000, ((256, 256, 128),), "largest", VOLUME)
    V, F, g, S = prepared(c, VOLUME)
    say("  triangles", len(F), "band", dm.band_size(handle, g, S))
    topo = handle.topology(F, n_verts=len(V))
    _, spec = dm.render(handle, dev(V), topo, S, g, spectrum=True)
    kb = dm.band_export(handle, g, S)["k"]
    ext = [int(np.argmax(kb[:, j])) for j in range(3)] + [int(np.argmin(kb[:, j])) for j in range(3)]
    ext.append(int(np.argmax(np.abs(kb).sum(axis=1))))
    pick = np.concatenate([ext, np.random.default_rng(15).choice(len(kb), 600, replace=False)])
    sp = spec.cpu().numpy().astype(np.float64)[pick]
    got = sp[:, 0] + 1j * sp[:, 1]
    want = ref.mesh_transform(V.astype(np.float64), F, ref.xi_of_k(kb[pick], g), g, VOLUME)
    err = np.abs(got - want).max() / np.abs(want).max()
    say("  band spectrum: max err / scale", err, "rel l2", rel_l2(got, want))
    assert err < 2e-6 and rel_l2(got, want) < IMG_TOL
    del spec
    K = _k_samples(g, np.random.default_rng(12))
    got = dm.mesh_transform(handle, dev(V), topo, g, dev(K)).cpu().numpy().astype(np.complex128)
    want = ref.mesh_transform(V.astype(np.float64), F, ref.xi_of_k(K, g), g, VOLUME)
    err = np.abs(got - want).max() / np.abs(want).max()
    say("  transform: max err / scale", err, "rel l2", rel_l2(got, want))
    assert err < 2e-6 and rel_l2(got, want) < IMG_TOL
    G = np.random.default_rng(13).standard_normal(g.n).astype(np.float32)
    dv, _, img = dm.render_vjp(handle, dev(V), topo, S, g, dev(G), want_sigma=False, want_image=True)
    vol = float(np.real(ref.mesh_transform(V.astype(np.float64), F, np.zeros((1, 3)), g, VOLUME)[0]))
    dvol = float(np.prod(g.spacing))
    integral = float(img.double().sum()) * dvol
    say("  image integral", integral, "volume", vol)
    assert abs(integral - vol) < IMG_TOL * abs(vol)
    vs = np.random.default_rng(14).choice(len(V), 4, replace=False)
    tris = np.nonzero(np.isin(F, vs).any(axis=1))[0]
    dvw, _ = ref.render_vjp(V.astype(np.float64), F[tris], g, S, G.astype(np.float64))
    gerr = rel_l2(dv.cpu().numpy()[vs], dvw[vs])
    say("  gradient rel err at sampled vertices", gerr)
    assert gerr < GRAD_TOL, gerr
    del img, dv
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_cfg2_mse_gradient_vs_oracle_and_fd(dm, handle, ref, mode):
    """cfg2: jittered sphere, MSE against a noisy render of the unjittered
    sphere; gradient to vertices and (sigma_xy, sigma_z)."""
    say("cfg2", mode)
    c = configs.cfg2(mode)
    V, F, g, S = prepared(c, mode)
    Vt = c.extra["V_target"].astype(np.float64)
    target = ref.render(Vt, F, g, S)
    target = target + c.extra["noise_frac"] * np.abs(target).max() * c.extra["unit_noise"]
    img_o = ref.render(V.astype(np.float64), F, g, S)
    G = (2.0 * (img_o - target) / img_o.size).astype(np.float32)
    topo = handle.topology(F, n_verts=len(V))
    dv, ds, _ = dm.render_vjp(handle, dev(V), topo, S, g, dev(G))
    dvw, dsw = ref.render_vjp(V.astype(np.float64), F, g, S, G.astype(np.float64))
    assert rel_l2(dv.cpu().numpy(), dvw) < GRAD_TOL
    assert rel_l2(ds.cpu().numpy(), dsw) < GRAD_TOL
    # (sigma_xy, sigma_z) chain rule and central differences of the oracle loss (h = 1e-3)
    sxy, sz = np.sqrt(S[0]), np.sqrt(S[2])
    ds = ds.cpu().numpy().astype(np.float64)
    d_sxy = 2 * sxy * (ds[0] + ds[1])
    d_sz = 2 * sz * ds[2]

    def loss(Vx, a, b):   # band held fixed at the unperturbed covariance
        I = ref.render(Vx, F, g, (a * a, a * a, b * b, 0, 0, 0), band_sigma6=S)
        return float(np.sum((I - target) ** 2) / I.size)

    h = 1e-3
    fd_xy = (loss(V.astype(np.float64), sxy + h, sz) - loss(V.astype(np.float64), sxy - h, sz)) / (2 * h)
    fd_z = (loss(V.astype(np.float64), sxy, sz + h) - loss(V.astype(np.float64), sxy, sz - h)) / (2 * h)
    assert abs(d_sxy - fd_xy) < 1e-3 * abs(fd_xy) + 1e-12
    assert abs(d_sz - fd_z) < 1e-3 * abs(fd_z) + 1e-12
    dvn = dv.cpu().numpy().astype(np.float64)
    for vi, j in [(0, 0), (17, 1), (90, 2)]:
        Vp, Vm = V.astype(np.float64), V.astype(np.float64)
        Vp[vi, j] += h
        Vm[vi, j] -= h
        fd = (loss(Vp, sxy, sz) - loss(Vm, sxy, sz)) / (2 * h)
        assert abs(dvn[vi, j] - fd) < 1e-3 * np.abs(dvn).max(), (vi, j, dvn[vi, j], fd)


def test_autograd_function_matches_vjp(dm, handle, ref):
    import torch
    say("autograd")
    c = configs.cfg1()
    V, F, g, S = prepared(c)
    topo = handle.topology(F, n_verts=len(V))
    v = dev(V).requires_grad_(True)
    s = torch.tensor(S, dtype=torch.float32, device="cuda:0", requires_grad=True)
    img = dm.RenderFunction.apply(v, s, handle, topo, g)
    target = torch.zeros_like(img)
    loss = ((img - target) ** 2).mean()
    loss.backward()
    G = (2 * img.detach() / img.numel()).contiguous()
    # the backward reuses the forward's band spectrum: the same call with that
    # spectrum handed in gives the same bits
    _, spec = dm.render(handle, dev(V), topo, S, g, spectrum=True)
    dv, ds, _ = dm.render_vjp(handle, dev(V), topo, S, g, G, spectrum_in=spec)
    assert torch.equal(v.grad, dv) and torch.equal(s.grad, ds)
    # the one-call gradient (forward and gradient in one sweep) sums in
    # another order: float32 rounding apart
    dvf, dsf, _ = dm.render_vjp(handle, dev(V), topo, S, g, G)
    assert rel_l2(v.grad.cpu().numpy(), dvf.cpu().numpy()) < 1e-5
    assert rel_l2(s.grad.cpu().numpy(), dsf.cpu().numpy()) < 1e-5


# ------------------------------------------------------- determinism
def test_bitwise_deterministic(dm, handle):
    say("determinism")
    c = configs.cfg1(SURFACE)
    V, F, g, S = prepared(c, SURFACE)
    topo = handle.topology(F, n_verts=len(V))
    G = dev(np.random.default_rng(1).standard_normal(g.n).astype(np.float32))
    a = dm.render_vjp(handle, dev(V), topo, S, g, G, want_image=True)
    b = dm.render_vjp(handle, dev(V), topo, S, g, G, want_image=True)
    for x, y in zip(a, b):
        assert bool((x == y).all())


# ------------------------------------------------------------- errors
def test_error_paths(dm, handle):
    say("errors")
    c = configs.cfg1()
    V, F, g, S = prepared(c)
    bad = F.copy()
    bad[3, 1] = len(V)
    with pytest.raises(dm.DeltamicError) as e:
        handle.topology(bad, n_verts=len(V))
    assert e.value.status == -2
    openF = F[1:]
    topo_open = handle.topology(openF, n_verts=len(V))
    assert not topo_open.closed
    with pytest.raises(dm.DeltamicError) as e:
        dm.render(handle, dev(V), topo_open, S, g)
    assert e.value.status == -2
    img = dm.render(handle, dev(V), topo_open, S, g.with_mode(SURFACE))   # surfaces may be open
    assert np.isfinite(img.cpu().numpy()).all()
    topo = handle.topology(F, n_verts=len(V))
    with pytest.raises(dm.DeltamicError) as e:
        dm.render(handle, dev(V), topo, (1.0, 1.0, -1.0, 0, 0, 0), g)
    assert e.value.status == -3
    with pytest.raises(dm.DeltamicError) as e:
        dm.render(handle, dev(V[:-1]), topo, S, g)
    assert e.value.status == -1


def test_band_cache_stays_bounded_over_many_psfs(dm):
    """A handle that renders with a new covariance every call (a PSF fit, a
    server whose requests carry their own PSFs) keeps a bounded band cache:
    at most 32 bands (least recently used evicted), so its device memory stops
    growing; a band evicted and needed again is rebuilt identically."""
    import torch
    h = dm.Handle(0)
    c = configs.cfg1()
    g = f32_grid(c.grid)
    topo = h.topology(c.F, n_verts=len(c.V))
    V = dev(c.V)
    sig = lambda i: (1.0 + 0.01 * i, 1.0 + 0.01 * i, 2.5, 0.0, 0.0, 0.0)
    first = dm.render(h, V, topo, sig(0), g)
    mem, sizes = [], []
    for i in range(50):
        dm.render(h, V, topo, sig(i), g)
        torch.cuda.synchronize()
        mem.append(h.memory_in_use())
        sizes.append(dm.band_size(h, g, sig(i)))
    n_pos = g.n[0] * g.n[1] * (g.n[2] // 2 + 1)
    band_bytes = 24 * max(sizes) + 4 * n_pos + 4096
    say("band cache: memory after 1/32/50 PSFs", mem[0], mem[31], mem[49], "band <=", band_bytes)
    assert mem[49] <= mem[0] + 32 * band_bytes
    assert mem[49] <= mem[31] + 2 * band_bytes
    again = dm.render(h, V, topo, sig(0), g)   # its band was evicted and is rebuilt
    torch.cuda.synchronize()
    assert torch.equal(first, again)
