"""Continuous-batching server: every request's result equals the same request
run alone, batches form while earlier ones run, admission respects the HBM
budget, oversize requests are refused, state errors are reported."""
import sys
import threading
import time

import numpy as np
import pytest

from helpers import f32_grid, f32_sigma
from workloads import configs

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


def _cells(n, seed=0):
    rng = np.random.default_rng(seed)
    grids = ((24, 28, 20), (32, 32, 32), (40, 36, 24))
    out = []
    for i in range(n):
        c = configs.random_cell(rng, 300, 2500, grids, f"cell{i}", SURFACE if i % 3 == 2 else VOLUME)
        out.append(c)
    return out


def _buffers(c, seed):
    import torch
    g = f32_grid(c.grid)
    G = torch.tensor(np.random.default_rng(seed).standard_normal(g.n).astype(np.float32), device="cuda:0")
    img = torch.empty(g.n, device="cuda:0")
    dv = torch.empty((len(c.V), 3), device="cuda:0")
    ds = torch.empty(6, device="cuda:0")
    return g, G, img, dv, ds


def test_served_results_equal_alone(dm):
    import torch
    say("serve equal alone")
    cells = _cells(7)
    srv = dm.Server(0, max_batch=8, max_inflight=2)
    h = dm.Handle(0)
    try:
        ids = [srv.mesh_add(c.V, c.F) for c in cells]
        bufs = [_buffers(c, i) for i, c in enumerate(cells)]
        tickets = [srv.submit(mid, f32_sigma(c.sigma), b[0], b[1], b[2], b[3], b[4])
                   for mid, c, b in zip(ids, cells, bufs)]
        res = [srv.poll(t) for t in tickets]
        assert all(r["status"] == 0 for r in res)
        torch.cuda.synchronize()
        for c, b in zip(cells, bufs):
            g, G = b[0], b[1]
            topo = h.topology(c.F, n_verts=len(c.V))
            V = torch.tensor(c.V, device="cuda:0")
            img, dv, ds = dm.batch_run(h, [(V, topo, f32_sigma(c.sigma), g, G)])[0]
            assert bool((img == b[2]).all()) and bool((dv == b[3]).all()) and bool((ds == b[4]).all())
        st = srv.stats()
        assert st["completed"] == len(cells) and st["rejected"] == 0
    finally:
        srv.close()


def test_continuous_batching_under_staggered_arrivals(dm):
    import torch
    say("serve staggered")
    cells = _cells(24, seed=1)
    srv = dm.Server(0, max_batch=6, max_inflight=2)
    try:
        ids = [srv.mesh_add(c.V, c.F) for c in cells]
        bufs = [_buffers(c, i) for i, c in enumerate(cells)]
        tickets = []

        def client():
            rng = np.random.default_rng(7)
            for mid, c, b in zip(ids, cells, bufs):
                tickets.append(srv.submit(mid, f32_sigma(c.sigma), b[0], b[1], b[2], b[3], b[4]))
                time.sleep(float(rng.exponential(0.002)))

        th = threading.Thread(target=client)
        th.start()
        th.join()
        res = [srv.poll(t) for t in tickets]
        assert all(r["status"] == 0 for r in res)
        assert max(r["batch_size"] for r in res) > 1
        torch.cuda.synchronize()
        for b in bufs:
            assert bool(torch.isfinite(b[2]).all()) and bool(torch.isfinite(b[3]).all())
        st = srv.stats()
        assert st["completed"] == len(cells) and st["batches"] < len(cells)
    finally:
        srv.close()


def test_budget_admission_and_oversize_rejection(dm):
    say("serve budget")
    small = _cells(6, seed=2)
    big = configs.random_cell(np.random.default_rng(9), 3000, 3000, ((128, 128, 128),), "big", VOLUME)
    budget = 24 << 20
    srv = dm.Server(0, max_batch=8, max_inflight=2, hbm_budget_bytes=budget)
    try:
        ids = [srv.mesh_add(c.V, c.F) for c in small]
        bid = srv.mesh_add(big.V, big.F)
        bufs = [_buffers(c, i) for i, c in enumerate(small)]
        bb = _buffers(big, 99)
        tickets = [srv.submit(mid, f32_sigma(c.sigma), b[0], b[1], b[2], b[3], b[4])
                   for mid, c, b in zip(ids, small, bufs)]
        tb = srv.submit(bid, f32_sigma(big.sigma), bb[0], bb[1], bb[2], bb[3], bb[4])
        res = [srv.poll(t) for t in tickets]
        rb = srv.poll(tb)
        assert all(r["status"] == 0 for r in res)
        assert rb["status"] == -4          # its footprint alone exceeds the budget
        st = srv.stats()
        assert st["peak_inflight_bytes"] <= budget
        assert st["rejected"] == 1
        with pytest.raises(dm.DeltamicError):
            srv.poll(tb)                   # ticket consumed
    finally:
        srv.close()


def test_mesh_remove_with_pending_request_is_refused(dm):
    say("serve mesh remove")
    c = _cells(1, seed=3)[0]
    srv = dm.Server(0, max_batch=1, max_inflight=1)
    try:
        mid = srv.mesh_add(c.V, c.F)
        b = _buffers(c, 0)
        t = srv.submit(mid, f32_sigma(c.sigma), b[0], b[1], b[2], b[3], b[4])
        try:
            srv.mesh_remove(mid)
            removed = True
        except dm.DeltamicError as e:
            assert e.status == -8
            removed = False
        assert srv.poll(t)["status"] == 0 or removed
        if not removed:
            srv.mesh_remove(mid)
        with pytest.raises(dm.DeltamicError):
            srv.submit(mid, f32_sigma(c.sigma), b[0], b[1], b[2], b[3], b[4])
    finally:
        srv.close()


def test_served_large_requests_on_two_streams(dm):
    """Three requests large enough to run their own sweeps (the single cell,
    both density modes, and the volume cell with a wider PSF) submitted with
    small ones: in a batch the large ones alternate between the batch's
    stream and the slot's second stream, each handed out at its own
    completion.  Every result equals the same request run alone: the large
    ones bitwise dm_render_vjp (they run its sweep plan), the small ones
    bitwise a batch of themselves alone."""
    import torch
    say("serve large requests on two streams")
    big = configs.cfg3(VOLUME)
    bigs = configs.cfg3(SURFACE)
    small = _cells(2, seed=5)
    wide = configs.psf_diag(0.17, 0.5)
    jobs = [(big, big.sigma), (small[0], small[0].sigma), (bigs, bigs.sigma), (small[1], small[1].sigma),
            (big, wide)]
    srv = dm.Server(0, max_batch=8, max_inflight=2)
    h = dm.Handle(0)
    try:
        mids = {}
        for c, _ in jobs:
            if id(c) not in mids:
                mids[id(c)] = srv.mesh_add(c.V, c.F)
        bufs = [_buffers(c, 40 + i) for i, (c, _) in enumerate(jobs)]
        tickets = [srv.submit(mids[id(c)], f32_sigma(sig), b[0], b[1], b[2], b[3], b[4])
                   for (c, sig), b in zip(jobs, bufs)]
        res = [srv.poll(t) for t in tickets]
        say("statuses", [r["status"] for r in res])
        assert all(r["status"] == 0 for r in res)
        torch.cuda.synchronize()
        for i, ((c, sig), b) in enumerate(zip(jobs, bufs)):
            g, G = b[0], b[1]
            topo = h.topology(c.F, n_verts=len(c.V))
            V = torch.tensor(c.V, device="cuda:0")
            if c is big or c is bigs:
                dv, ds, img = dm.render_vjp(h, V, topo, f32_sigma(sig), g, G, want_image=True)
            else:
                img, dv, ds = dm.batch_run(h, [(V, topo, f32_sigma(sig), g, G)])[0]
            eq = bool((img == b[2]).all()) and bool((dv == b[3]).all()) and bool((ds == b[4]).all())
            say(f"request {i}: served equals alone: {eq}")
            assert eq
    finally:
        srv.close()


def test_served_tabulated_otf_requests(dm):
    """Requests with tabulated OTFs next to Gaussian ones in the server: each
    result is bitwise the same request run alone through dm_batch_run, and a
    request asking for the PSF gradient with a tabulated OTF is refused at
    submission."""
    import torch
    from workloads import psfs
    say("serve tabulated OTF requests")
    cells = _cells(3, seed=9)
    srv = dm.Server(0, max_batch=8, max_inflight=2)
    h = dm.Handle(0)
    try:
        mids = [srv.mesh_add(c.V, c.F) for c in cells]
        bufs = [_buffers(c, 60 + i) for i, c in enumerate(cells)]
        otfs = {}
        for i in (0, 2):
            g = bufs[i][0]
            otfs[i] = torch.tensor(psfs.half_spectrum(psfs.aberrated_otf(g, 1.1, 2.2, defocus=0.7, cone=1.1))
                                   .astype(np.complex64), device="cuda:0")
        tickets = []
        for i, c in enumerate(cells):
            g, G, img, dv, ds = bufs[i]
            if i in otfs:
                tickets.append(srv.submit(mids[i], None, g, G, img, dv, None, otf=otfs[i]))
            else:
                tickets.append(srv.submit(mids[i], f32_sigma(c.sigma), g, G, img, dv, ds))
        g0, G0, img0, dv0, _ = bufs[0]
        with pytest.raises(dm.DeltamicError):
            srv.submit(mids[0], None, g0, G0, torch.empty_like(img0), torch.empty_like(dv0),
                       torch.empty(6, device="cuda:0"), otf=otfs[0])
        res = [srv.poll(t) for t in tickets]
        assert all(r["status"] == 0 for r in res)
        torch.cuda.synchronize()
        for i, c in enumerate(cells):
            g, G, img, dv, ds = bufs[i]
            topo = h.topology(c.F, n_verts=len(c.V))
            V = torch.tensor(c.V, device="cuda:0")
            if i in otfs:
                a_img, a_dv, _ = dm.batch_run(h, [(V, topo, None, g, G, otfs[i])])[0]
                eq = torch.equal(a_img, img) and torch.equal(a_dv, dv)
            else:
                a_img, a_dv, a_ds = dm.batch_run(h, [(V, topo, f32_sigma(c.sigma), g, G)])[0]
                eq = torch.equal(a_img, img) and torch.equal(a_dv, dv) and torch.equal(a_ds, ds)
            say(f"request {i} ({'otf' if i in otfs else 'gaussian'}): served equals alone: {eq}")
            assert eq
    finally:
        srv.close()


def test_large_request_runs_alone_unless_a_backlog_builds(dm):
    """The scheduling rule for large requests (their own sweep launches, here
    the single cell, 2.8e9 pairs): with fewer than max_batch requests waiting,
    small requests submitted while it runs start only after it completes;
    once max_batch of them wait they start beside it.  Launch and completion
    times come from the server's per-request results (queue_ms, total_ms)
    and the submission times measured here."""
    import torch
    say("serve: large request alone unless backlog")
    big = configs.cfg3(VOLUME)
    small = _cells(3, seed=13)

    def run(max_batch):
        srv = dm.Server(0, max_batch=max_batch, max_inflight=2)
        try:
            mb = srv.mesh_add(big.V, big.F)
            ms = [srv.mesh_add(c.V, c.F) for c in small]
            bb = _buffers(big, 70)
            bs = [_buffers(c, 71 + i) for i, c in enumerate(small)]
            # warm-up: bands, FFT plans and workspace of every request
            ts = [srv.submit(mb, f32_sigma(big.sigma), *bb)]
            ts += [srv.submit(m, f32_sigma(c.sigma), *b) for m, c, b in zip(ms, small, bs)]
            assert all(srv.poll(t)["status"] == 0 for t in ts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tl = srv.submit(mb, f32_sigma(big.sigma), *bb)
            subs = []
            for m, c, b in zip(ms, small, bs):
                subs.append((time.perf_counter() - t0, srv.submit(m, f32_sigma(c.sigma), *b)))
            rl = srv.poll(tl)
            rs = [(dt, srv.poll(t)) for dt, t in subs]
            assert rl["status"] == 0 and all(r["status"] == 0 for _, r in rs)
            done_l = rl["total_ms"]   # from the large request's submission (t0)
            starts = [1e3 * dt + r["queue_ms"] for dt, r in rs]
            say(f"  max_batch {max_batch}: large done at {done_l:.2f} ms, small starts "
                + ", ".join(f"{x:.2f}" for x in starts))
            return done_l, starts
        finally:
            srv.close()

    done_l, starts = run(16)
    assert done_l > 1.0
    assert all(x >= done_l - 0.3 for x in starts)
    done_l, starts = run(2)
    assert min(starts) < done_l - 0.5
