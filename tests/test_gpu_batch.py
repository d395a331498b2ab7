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


def test_large_request_in_a_batch_runs_its_own_sweeps(dm, handle):
    """A request of 2.8e9 pairs (the single cell) is large enough to run its
    own sweep launches inside a batch: its outputs are bitwise those of the
    single call, while a small request shares the persistent launch."""
    import torch
    big = configs.cfg3()
    small = configs.cfg1()
    tb = handle.topology(big.F, n_verts=len(big.V))
    ts = handle.topology(small.F, n_verts=len(small.V))
    Gb = dev(np.random.default_rng(21).standard_normal(big.grid.n).astype(np.float32))
    Gs = dev(np.random.default_rng(22).standard_normal(small.grid.n).astype(np.float32))
    single = dm.render_vjp(handle, dev(big.V), tb, big.sigma, big.grid, Gb, want_image=True)
    out = dm.batch_run(handle, [(dev(small.V), ts, small.sigma, small.grid, Gs),
                                (dev(big.V), tb, big.sigma, big.grid, Gb)])
    alone = dm.batch_run(handle, [(dev(small.V), ts, small.sigma, small.grid, Gs)])
    torch.cuda.synchronize()
    img, dv, ds = out[1]
    say("large request in batch: image equal", torch.equal(img, single[2]), "dV equal", torch.equal(dv, single[0]))
    assert torch.equal(img, single[2]) and torch.equal(dv, single[0]) and torch.equal(ds, single[1])
    for a, b in zip(out[0], alone[0]):
        assert torch.equal(a, b)


def test_several_large_requests_alternate_streams(dm, handle):
    """Three large requests (the single cell in both density modes, and the
    volume cell with another PSF) and two small ones in one batch: the large
    ones run their own sweeps, alternating between the caller's stream and
    the handle's second stream, and their outputs are bitwise the single
    call's; the small ones share the persistent launch and match a batch of
    themselves alone bitwise.  The batch is complete when the caller's stream
    is (read right after it, with no device-wide synchronisation)."""
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
    refs = []
    for i, r in enumerate(reqs):
        if i in large:
            dv, ds, img = dm.render_vjp(handle, *r, want_image=True)
            refs.append((img, dv, ds))
        else:
            refs.append(dm.batch_run(handle, [r])[0])
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    out = dm.batch_run(handle, reqs)
    s.synchronize()
    for i, (o, ref) in enumerate(zip(out, refs)):
        eq = all(torch.equal(a, b) for a, b in zip(o, ref))
        say(f"request {i} ({'own sweeps' if i in large else 'shared launch'}): outputs equal: {eq}")
        assert eq
