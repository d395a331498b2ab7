"""Batched persistent launch (dm_batch_run): same results as single calls and
as the oracle, and each request's result independent of the rest of the batch."""
import ctypes
import sys

import numpy as np
import pytest

from helpers import f32_grid, f32_sigma, rel_l2
from workloads import configs, meshes

pytestmark = pytest.mark.gpu
VOLUME, SURFACE = configs.VOLUME, configs.SURFACE


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


def _cases():
    out = [configs.cfg1(VOLUME), configs.cfg1(SURFACE), configs.box_case(mode=VOLUME)]
    U, F = meshes.icosphere(2)
    g = configs.Grid((15, 18, 11), (0.9, 1.1, 1.7), (0.3, -0.2, 0.5), 2e-2, SURFACE)
    V = meshes.sh_deform(U, 3.5, np.random.default_rng(3)) + g.centre
    out.append(configs.Case("odd", V.astype(np.float32), F.astype(np.int32), g, (1.3, 0.9, 2.2, 0.35, -0.2, 0.15)))
    rng = np.random.default_rng(4)
    out.append(configs.random_cell(rng, 1000, 3000, ((24, 28, 20),), "cell", VOLUME))
    return out


def _requests(dm, handle, cases, seed=0):
    rng = np.random.default_rng(seed)
    reqs = []
    for c in cases:
        g, S = f32_grid(c.grid), f32_sigma(c.sigma)
        topo = handle.topology(c.F, n_verts=len(c.V))
        G = rng.standard_normal(g.n).astype(np.float32)
        reqs.append((dev(c.V), topo, S, g, dev(G)))
    return reqs


def test_batch_matches_single_calls_and_oracle(dm, handle, ref):
    say("batch vs single")
    cases = _cases()
    reqs = _requests(dm, handle, cases)
    out = dm.batch_run(handle, reqs)
    for i, ((V, topo, S, g, G), (img, dv, ds)) in enumerate(zip(reqs, out)):
        dv1, ds1, img1 = dm.render_vjp(handle, V, topo, S, g, G, want_image=True)
        # the batch splits the sums into different chunks: agreement to rounding,
        # held to the same bar as parity with the oracle
        assert rel_l2(img.cpu().numpy(), img1.cpu().numpy()) < 1e-5, i
        assert rel_l2(dv.cpu().numpy(), dv1.cpu().numpy()) < 1e-4, i
        assert rel_l2(ds.cpu().numpy(), ds1.cpu().numpy()) < 1e-4, i
    for i in (0, 3):
        c = cases[i]
        V, topo, S, g, G = reqs[i]
        img, dv, ds = out[i]
        want = ref.render(c.V.astype(np.float64), c.F, g, S)
        dvw, dsw = ref.render_vjp(c.V.astype(np.float64), c.F, g, S, G.cpu().numpy().astype(np.float64))
        assert rel_l2(img.cpu().numpy(), want) < 1e-5
        assert rel_l2(dv.cpu().numpy(), dvw) < 1e-4
        assert rel_l2(ds.cpu().numpy(), dsw) < 1e-4


def test_batch_result_independent_of_the_mix(dm, handle):
    say("batch mix invariance")
    cases = _cases()
    reqs = _requests(dm, handle, cases)
    alone = dm.batch_run(handle, [reqs[3]])[0]
    mixed = dm.batch_run(handle, [reqs[4], reqs[0], reqs[3], reqs[1]])[2]
    for a, b in zip(alone, mixed):
        assert bool((a == b).all())


def test_batch_forward_only_request(dm, handle, ref):
    say("batch forward only")
    c = configs.cfg1(VOLUME)
    g, S = f32_grid(c.grid), f32_sigma(c.sigma)
    topo = handle.topology(c.F, n_verts=len(c.V))
    img, dv, ds = dm.batch_run(handle, [(dev(c.V), topo, S, g, None)])[0]
    assert dv is None and ds is None
    want = ref.render(c.V.astype(np.float64), c.F, g, S)
    assert rel_l2(img.cpu().numpy(), want) < 1e-5


def test_batch_rejects_whole_batch_and_writes_nothing(dm, handle):
    import torch
    say("batch validation")
    c = configs.cfg1(VOLUME)
    g, S = f32_grid(c.grid), f32_sigma(c.sigma)
    topo = handle.topology(c.F, n_verts=len(c.V))
    V = dev(c.V)
    G = dev(np.ones(g.n, np.float32))
    arr = (dm.CRequest * 2)()
    outs = []
    for i, sig in enumerate([S, (1.0, 1.0, -2.0, 0.0, 0.0, 0.0)]):
        img = torch.full(g.n, 7.0, device="cuda:0")
        dv = torch.full((len(c.V), 3), 7.0, device="cuda:0")
        r = arr[i]
        r.mesh = dm._mesh(V, topo)
        r.psf = dm._psf(sig)
        r.grid = dm._grid(g)
        r.dL_dimage_dev = G.data_ptr()
        r.image_dev = img.data_ptr()
        r.dL_dverts_dev = dv.data_ptr()
        r.dL_dsigma_dev = None
        outs.append((img, dv))
    st = dm.lib().dm_batch_run(handle.ptr, 2, ctypes.cast(arr, ctypes.c_void_p), dm._stream(0))
    torch.cuda.synchronize()
    assert st == -3
    for img, dv in outs:
        assert bool((img == 7.0).all()) and bool((dv == 7.0).all())


def test_large_request_in_the_shared_launch(dm, handle):
    """A request of 2.8e9 pairs (the single cell) in the shared persistent
    launch with a small one: its outputs agree with dm_render_vjp to float32
    rounding (the batch cuts it into larger tiles) and are bitwise those of a
    batch of itself alone; the small request's are bitwise those of a batch of
    itself alone."""
    import torch
    big = configs.cfg3()
    small = configs.cfg1()
    tb = handle.topology(big.F, n_verts=len(big.V))
    ts = handle.topology(small.F, n_verts=len(small.V))
    Gb = dev(np.random.default_rng(21).standard_normal(big.grid.n).astype(np.float32))
    Gs = dev(np.random.default_rng(22).standard_normal(small.grid.n).astype(np.float32))
    rb = (dev(big.V), tb, big.sigma, big.grid, Gb)
    rs = (dev(small.V), ts, small.sigma, small.grid, Gs)
    single = dm.render_vjp(handle, *rb, want_image=True)
    out = dm.batch_run(handle, [rs, rb])
    alone_s = dm.batch_run(handle, [rs])
    alone_b = dm.batch_run(handle, [rb])
    torch.cuda.synchronize()
    img, dv, ds = out[1]
    e_img = float((img - single[2]).norm() / single[2].norm())
    e_dv = float((dv - single[0]).norm() / single[0].norm())
    e_ds = float((ds - single[1]).norm() / single[1].norm())
    say("large request in batch vs single call: image", e_img, "dV", e_dv, "dSigma", e_ds)
    assert e_img < 1e-6 and e_dv < 1e-5 and e_ds < 1e-5
    for a, b in zip(out[1], alone_b[0]):
        assert torch.equal(a, b)
    for a, b in zip(out[0], alone_s[0]):
        assert torch.equal(a, b)


def test_several_large_requests_in_one_launch(dm, handle):
    """Three large requests (the single cell in both density modes, and the
    volume cell with another PSF) and two small ones in one batch, all in the
    shared persistent launches (one per density): every request's outputs are
    bitwise those of a batch of itself alone, and the large ones agree with
    dm_render_vjp to float32 rounding.  The batch is complete when the
    caller's stream is (read right after it, with no device-wide
    synchronisation)."""
    import torch
    big = configs.cfg3(VOLUME)
    bigs = configs.cfg3(SURFACE)
    small = configs.cfg1()
    tb = handle.topology(big.F, n_verts=len(big.V))
    tbs = handle.topology(bigs.F, n_verts=len(bigs.V))
    ts = handle.topology(small.F, n_verts=len(small.V))
    rng = np.random.default_rng(31)
    Gb = dev(rng.standard_normal(big.grid.n).astype(np.float32))
    Gbs = dev(rng.standard_normal(bigs.grid.n).astype(np.float32))
    Gs = dev(rng.standard_normal(small.grid.n).astype(np.float32))
    sig2 = configs.psf_diag(0.17, 0.5)
    reqs = [(dev(big.V), tb, big.sigma, big.grid, Gb),
            (dev(small.V), ts, small.sigma, small.grid, Gs),
            (dev(bigs.V), tbs, bigs.sigma, bigs.grid, Gbs),
            (dev(small.V) * 1.01, ts, small.sigma, small.grid, Gs),
            (dev(big.V), tb, sig2, big.grid, Gb)]
    large = {0, 2, 4}
    refs = [dm.batch_run(handle, [r])[0] for r in reqs]
    singles = {i: dm.render_vjp(handle, *reqs[i], want_image=True) for i in large}
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    out = dm.batch_run(handle, reqs)
    s.synchronize()
    for i, (o, ref) in enumerate(zip(out, refs)):
        eq = all(torch.equal(a, b) for a, b in zip(o, ref))
        say(f"request {i} ({'large' if i in large else 'small'}): outputs equal to the request alone: {eq}")
        assert eq
        if i in large:
            dv, ds, img = singles[i]
            assert float((o[0] - img).norm() / img.norm()) < 1e-6
            assert float((o[1] - dv).norm() / dv.norm()) < 1e-5


def test_cfg4_sized_request_in_the_shared_launch_vs_oracle(dm, handle, ref):
    """The largest cell of the 64-cell batched workload (by pairs), run in the
    shared persistent launch between two other cells of that workload: its
    vertex gradient at 12 sampled vertices against the FP64 oracle evaluated
    on the triangles around them (each triangle adds its own terms to its
    vertices' gradients, so those triangles fix them exactly), and its image
    against the single call to rounding."""
    import torch
    cases = configs.cfg4()
    sizes = [len(c.F) * dm.band_size(handle, f32_grid(c.grid), f32_sigma(c.sigma)) for c in cases]
    order = np.argsort(sizes)
    ib, i1, i2 = int(order[-1]), int(order[0]), int(order[len(order) // 2])
    say("cfg4 largest cell", cases[ib].name, "triangles", len(cases[ib].F), "pairs", sizes[ib])
    reqs = _requests(dm, handle, [cases[i1], cases[ib], cases[i2]], seed=7)
    out = dm.batch_run(handle, reqs)
    V, topo, S, g, G = reqs[1]
    dv1, ds1, img1 = dm.render_vjp(handle, V, topo, S, g, G, want_image=True)
    torch.cuda.synchronize()
    img, dv, ds = out[1]
    assert rel_l2(img.cpu().numpy(), img1.cpu().numpy()) < 1e-6
    c = cases[ib]
    Vd = c.V.astype(np.float64)
    bmask, xb, hb, Gb, W = ref.vjp_band(g, S, G.cpu().numpy().astype(np.float64))
    vs = np.random.default_rng(23).choice(len(Vd), 12, replace=False)
    tris = np.nonzero(np.isin(c.F, vs).any(axis=1))[0]
    Vr = Vd - np.asarray(g.origin, dtype=np.float64)
    want = ref.mesh_ft_vjp_raw(Vr, c.F[tris], xb, W, VOLUME)[vs]
    err = rel_l2(dv.cpu().numpy().astype(np.float64)[vs], want)
    say("cfg4 largest cell in the shared launch: dV rel l2 at 12 vertices", err)
    assert err < 1e-4


def test_batch_with_tabulated_otf_requests(dm, handle, ref):
    """Tabulated-OTF requests (aberrated tables: defocus phase, missing cone)
    in one batch with Gaussian ones: the OTF requests match the FP64 oracle
    (image, vertex gradient), agree with dm_render_otf_vjp to float32 rounding
    and are bitwise a batch of themselves alone; the Gaussian requests are
    bitwise unchanged by their company.  Each OTF request builds its band in
    its own workspace, so two different tables on one grid coexist."""
    import dataclasses

    import torch
    from workloads import psfs
    c_vol = configs.cfg1(VOLUME)
    c_surf = configs.cfg1(SURFACE)
    g_vol = f32_grid(c_vol.grid)
    g_surf = dataclasses.replace(f32_grid(c_surf.grid), n=(30, 31, 33), mode=SURFACE)
    otf_a = psfs.aberrated_otf(g_vol, 1.0, 2.0, defocus=0.9, cone=1.2)
    otf_b = psfs.aberrated_otf(g_vol, 1.2, 2.4, defocus=-0.6, cone=1.0)
    otf_c = psfs.aberrated_otf(g_surf, 1.0, 2.0, defocus=0.9, cone=1.2)
    rng = np.random.default_rng(41)
    t_vol = handle.topology(c_vol.F, n_verts=len(c_vol.V))
    t_surf = handle.topology(c_surf.F, n_verts=len(c_surf.V))
    gauss = _requests(dm, handle, [configs.box_case(mode=VOLUME), configs.cfg1(SURFACE)], seed=42)
    otf_dev = [dev(psfs.half_spectrum(o).astype(np.complex64)) for o in (otf_a, otf_b, otf_c)]
    otf_reqs = [
        (dev(c_vol.V), t_vol, None, g_vol, dev(rng.standard_normal(g_vol.n).astype(np.float32)), otf_dev[0]),
        (dev(c_vol.V * 1.02), t_vol, None, g_vol, dev(rng.standard_normal(g_vol.n).astype(np.float32)), otf_dev[1]),
        (dev(c_surf.V), t_surf, None, g_surf, dev(rng.standard_normal(g_surf.n).astype(np.float32)), otf_dev[2]),
    ]
    reqs = [otf_reqs[0], gauss[0], otf_reqs[1], gauss[1], otf_reqs[2]]
    out = dm.batch_run(handle, reqs)
    alone = [dm.batch_run(handle, [r])[0] for r in reqs]
    torch.cuda.synchronize()
    for i, (o, a) in enumerate(zip(out, alone)):
        eq = all((x is None and y is None) or torch.equal(x, y) for x, y in zip(o, a))
        say(f"request {i}: bitwise a batch of itself alone: {eq}")
        assert eq
    tables = [otf_a, otf_b, otf_c]
    for j, i in enumerate((0, 2, 4)):
        V, topo, _, g, G, otf = reqs[i]
        img, dv, ds = out[i]
        assert ds is None
        dv1, img1 = dm.render_otf_vjp(handle, V, topo, otf, g, G, want_image=True)
        torch.cuda.synchronize()
        # float32 summation orders of the batch tiles and the single call
        assert rel_l2(img.cpu().numpy(), img1.cpu().numpy()) < 1e-5
        assert rel_l2(dv.cpu().numpy(), dv1.cpu().numpy()) < 1e-5
        V64 = V.cpu().numpy().astype(np.float64)
        F = c_vol.F if g.mode == VOLUME else c_surf.F
        want = ref.render_otf(V64, F, g, tables[j].astype(np.complex128))
        dvw = ref.render_otf_vjp(V64, F, g, tables[j].astype(np.complex128), G.cpu().numpy().astype(np.float64))
        e_img, e_dv = rel_l2(img.cpu().numpy(), want), rel_l2(dv.cpu().numpy(), dvw)
        say(f"otf request {i}: image {e_img:.2e} dV {e_dv:.2e} against the oracle")
        assert e_img < 1e-5 and e_dv < 1e-4
