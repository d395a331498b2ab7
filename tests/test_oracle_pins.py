"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each check compares the oracle with something other than its own formulas:
high-precision arithmetic (mpmath), the special cases printed in the paper
(Eq. 12a/12b), closed-form transforms of boxes and spheres, exact
invariances (translation, conjugate symmetry, subdivision, orientation,
scaling), quadrature and voxelisation brute force, and finite differences.
A dropped term, a wrong sign or a swapped index in the oracle breaks at least
one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from workloads import configs, meshes

VOLUME, SURFACE = configs.VOLUME, configs.SURFACE


# ------------------------------------------------------------------ helpers
def mp_dd_exp(nodes, dps=220, eps="1e-35"):
    """Divided difference of exp in high precision; repeated nodes are split
    by a tiny perturbation (error ~ eps) so the distinct-node formula applies."""
    with mp.workdps(dps):
        x = [mp.mpc(complex(z)) for z in nodes]
        e = mp.mpf(eps)
        seen = {}
        for i, z in enumerate(x):
            key = (float(z.real), float(z.imag))
            c = seen.get(key, 0)
            if c:
                x[i] = z + c * e
            seen[key] = c + 1
        s = mp.mpc(0)
        for i, xi in enumerate(x):
            d = mp.mpc(1)
            for j, xj in enumerate(x):
                if j != i:
                    d *= (xi - xj)
            s += mp.exp(xi) / d
        return complex(s)


def sinc(a):
    a = np.asarray(a, dtype=np.float64)
    out = np.ones_like(a)
    nz = a != 0
    out[nz] = np.sin(a[nz]) / a[nz]
    return out


def box_volume_ft(lo, hi, xi):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    L, c = hi - lo, (hi + lo) / 2
    s = sinc(xi * L / 2)
    return np.prod(L) * np.prod(s, axis=-1) * np.exp(-1j * xi @ c)


def box_surface_ft(lo, hi, xi):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    L, c = hi - lo, (hi + lo) / 2
    s = sinc(xi * L / 2)
    co = np.cos(xi * L / 2)
    t = (L[1] * L[2] * co[..., 0] * s[..., 1] * s[..., 2]
         + L[0] * L[2] * s[..., 0] * co[..., 1] * s[..., 2]
         + L[0] * L[1] * s[..., 0] * s[..., 1] * co[..., 2])
    return 2 * t * np.exp(-1j * xi @ c)


def xi_samples():
    rng = np.random.default_rng(7)
    xi = rng.uniform(-3, 3, size=(40, 3))
    special = np.array([[0, 0, 0], [0.7, 0, 0], [0, -1.3, 0], [0, 0, 2.1], [0.4, -0.9, 0],
                        [0, 1.7, 2.2], [1.1, 0, -0.6], [12.0, 0, 0], [0, 0, -9.5]], float)
    return np.concatenate([special, xi])


# ------------------------------------------------- divided differences of exp
@pytest.mark.parametrize("n", [3, 4, 5])
def test_dd_exp_matrix_matches_high_precision(ref, n):
    rng = np.random.default_rng(100 + n)
    worst = 0.0
    for trial in range(60):
        base = rng.uniform(-100, 100)
        gaps = 10.0 ** rng.uniform(-12, 0.5, size=n - 1)
        y = base + np.concatenate([[0.0], np.cumsum(gaps * rng.choice([-1, 1], n - 1))])
        if trial % 5 == 0:
            y[-1] = y[0]                      # exact repeat
        if trial % 7 == 0:
            y[:] = y[0]                       # all equal
        z = -1j * y
        got = ref.dd_exp(z)
        want = mp_dd_exp(z)
        worst = max(worst, abs(got - want) / abs(want))
    assert worst < 1e-13, worst


def test_dd_exp_real_nodes_textbook(ref):
    # DD[0,1] exp = e - 1 ; DD[0,0,0] exp = 1/2 ; DD[a]*4 = e^a/3!
    assert abs(ref.dd_exp([0, 1]) - (math.e - 1)) < 1e-14
    assert abs(ref.dd_exp([0, 0, 0]) - 0.5) < 1e-14
    assert abs(ref.dd_exp([0.3] * 4) - math.exp(0.3) / 6) < 1e-14


# ------------------------------------------------------- triangle transform
def test_tri_f_matches_high_precision_across_branch_switch(ref):
    rng = np.random.default_rng(3)
    worst = 0.0
    for gap in [1e-9, 1e-4, 9.9e-3, 1.01e-2, 0.05, 0.3, 2.0, 20.0]:
        for _ in range(6):
            y = rng.uniform(-80, 80) + np.array([0.0, gap, rng.uniform(-5, 5)])
            got = ref.tri_f(y)
            want = mp_dd_exp(-1j * y)
            worst = max(worst, abs(got - want) / abs(want))
    assert worst < 1e-10, worst


def test_tri_f_equals_paper_degenerate_forms(ref):
    """Eq. 12a g(t,t,u) and Eq. 12b g(u,u,u), with the exponent sign of Eq. 8."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        t, u = rng.uniform(-30, 30, size=2)
        eq12a = 1j * np.exp(-1j * t) / (t - u) + np.exp(-1j * t) / (t - u) ** 2 - np.exp(-1j * u) / (t - u) ** 2
        for y in ([t, t, u], [u, t, t], [t, u, t]):
            assert abs(ref.tri_f(y) - eq12a) < 1e-12 * max(1, abs(eq12a))
        assert abs(ref.tri_f([u, u, u]) - np.exp(-1j * u) / 2) < 1e-15


def test_tri_f_is_eq8_for_distinct_phases(ref):
    """Eq. 8 written from the paper's edge notation, for a triangle in space."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.normal(size=(3, 3)) * 2
        xi = rng.normal(size=3) * 2
        e = [v[(p + 2) % 3] - v[(p + 1) % 3] for p in range(3)]      # e_p = v_{p-} - v_{p+}
        f = sum(np.exp(-1j * v[p] @ xi) / ((e[(p + 2) % 3] @ xi) * (e[(p + 1) % 3] @ xi)) for p in range(3))
        assert abs(ref.tri_f(v @ xi) - f) < 1e-10 * abs(f)


def test_eq10_gradient_matches_finite_differences_and_high_precision(ref):
    rng = np.random.default_rng(6)
    for gap in [1e-7, 1e-3, 0.049, 0.051, 0.5, 3.0]:
        for _ in range(4):
            y = rng.uniform(-40, 40) + np.array([0.0, gap, rng.uniform(-4, 4)])
            B = ref.tri_dfdv(y)
            for p in range(3):
                z = list(-1j * y) + [-1j * y[p]]
                want = -1j * mp_dd_exp(z)
                assert abs(B[p] - want) < 1e-9 * abs(want), (gap, p)
            if gap >= 0.5:
                h = 1e-6
                for p in range(3):
                    yp, ym = y.copy(), y.copy()
                    yp[p] += h
                    ym[p] -= h
                    fd = (ref.tri_f(yp) - ref.tri_f(ym)) / (2 * h)
                    assert abs(B[p] - fd) < 1e-6 * abs(B[p])


def test_surface_quadrature_single_triangle(ref):
    """2 A_T f_T equals the surface integral of exp(-i x.xi) (Richardson-
    extrapolated centroid rule on n^2 sub-triangles)."""
    rng = np.random.default_rng(8)
    v = rng.normal(size=(3, 3)) * 1.5
    xi = np.array([1.3, -2.1, 0.7])

    def centroid_rule(n):
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        m = i + j < n
        up = np.stack([(i[m] + 1 / 3) / n, (j[m] + 1 / 3) / n], 1)
        m2 = i + j < n - 1
        dn = np.stack([(i[m2] + 2 / 3) / n, (j[m2] + 2 / 3) / n], 1)
        st = np.concatenate([up, dn])
        x = v[0] + st[:, :1] * (v[1] - v[0]) + st[:, 1:] * (v[2] - v[0])
        area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        return np.exp(-1j * x @ xi).sum() * area / n ** 2

    q = (4 * centroid_rule(512) - centroid_rule(256)) / 3
    twoA = np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    got = twoA * ref.tri_f(v @ xi)
    assert abs(got - q) < 1e-8 * abs(q)


# --------------------------------------------------------------- mesh level
@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_box_closed_form(ref, mode):
    lo, hi = (0.3, -1.2, 0.9), (2.8, 1.7, 4.15)
    V, F = meshes.box_mesh(lo, hi)
    xi = xi_samples()
    got = ref.mesh_ft_raw(V, F, xi, mode)
    want = box_volume_ft(lo, hi, xi) if mode == VOLUME else box_surface_ft(lo, hi, xi)
    scale = np.abs(want).max()
    assert np.max(np.abs(got - want)) < 1e-12 * scale


def test_zero_frequency_is_volume_and_area(ref):
    V, F = meshes.tetrahedron()
    assert abs(ref.mesh_ft_raw(V, F, np.zeros((1, 3)), VOLUME)[0] - 1 / 6) < 1e-15
    assert abs(ref.mesh_ft_raw(V, F, np.zeros((1, 3)), SURFACE)[0] - (1.5 + math.sqrt(3) / 2)) < 1e-14
    V, F = meshes.box_mesh((1, 2, 3), (2.5, 2.75, 5))
    assert abs(ref.mesh_ft_raw(V, F, np.zeros((1, 3)), VOLUME)[0] - 1.5 * 0.75 * 2) < 1e-13


def _deformed(sub=2, seed=0, R=5.0):
    U, F = meshes.icosphere(sub)
    V = meshes.sh_deform(U, R, np.random.default_rng(seed)) + np.array([1.0, -2.0, 0.5])
    return V, F


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_translation_is_phase_and_conjugate_symmetry(ref, mode):
    V, F = _deformed(1)
    xi = xi_samples()[:30] * 0.7
    t = np.array([0.37, -1.1, 2.3])
    u0 = ref.mesh_ft_raw(V, F, xi, mode)
    u1 = ref.mesh_ft_raw(V + t, F, xi, mode)
    assert np.max(np.abs(u1 - np.exp(-1j * xi @ t) * u0)) < 1e-11 * np.abs(u0).max()
    um = ref.mesh_ft_raw(V, F, -xi, mode)
    assert np.max(np.abs(um - np.conj(u0))) < 1e-12 * np.abs(u0).max()


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_subdivision_orientation_scaling(ref, mode):
    V, F = _deformed(1)
    xi = xi_samples()[:30] * 0.6
    u = ref.mesh_ft_raw(V, F, xi, mode)
    V2, F2 = meshes.subdivide_midpoint(V, F)
    assert np.max(np.abs(ref.mesh_ft_raw(V2, F2, xi, mode) - u)) < 1e-11 * np.abs(u).max()
    uf = ref.mesh_ft_raw(V, meshes.flip_faces(F), xi, mode)
    sign = -1 if mode == VOLUME else 1
    assert np.max(np.abs(uf - sign * u)) < 1e-12 * np.abs(u).max()
    s = 1.7
    us = ref.mesh_ft_raw(s * V, F, xi / s, mode)
    p = 3 if mode == VOLUME else 2
    assert np.max(np.abs(us - s ** p * u)) < 1e-11 * np.abs(us).max()


def test_volume_cone_decomposition_agrees(ref):
    V, F = _deformed(2, seed=3)
    xi = xi_samples() * 0.8
    a = ref.mesh_ft_raw(V, F, xi, VOLUME)
    b = ref.cone_volume_ft(V, F, xi, c=V.mean(0) + np.array([0.2, -0.1, 0.3]))
    assert np.max(np.abs(a - b)) < 1e-11 * np.abs(a).max()


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_sphere_limit(ref, mode):
    """Icospheres approach the transforms of the ball / sphere as they refine;
    the error falls by ~4x per subdivision (second order in the edge length)."""
    R = 3.0
    q = np.array([0.3, 0.9, 1.7, 2.6])
    xi = np.stack([q * 0.6, q * -0.48, q * 0.64], 1)     # |xi| = q
    if mode == VOLUME:
        exact = 4 * np.pi * (np.sin(q * R) - q * R * np.cos(q * R)) / q ** 3
    else:
        exact = 4 * np.pi * R ** 2 * np.sin(q * R) / (q * R)
    errs = []
    for sub in (3, 4):
        U, F = meshes.icosphere(sub)
        errs.append(np.max(np.abs(ref.mesh_ft_raw(U * R, F, xi, mode) - exact)))
    scale = np.abs(exact).max()
    assert errs[1] < 3e-3 * scale
    assert errs[1] < 0.35 * errs[0]


def _column_voxelise(V, F, xs, ys):
    """Inside intervals along z for every (x, y) column: crossings of the
    vertical line with the triangles (barycentric test in the xy projection)."""
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], 1)
    crossings = [[] for _ in range(len(P))]
    for a, b, c in F:
        A, B, C = V[a], V[b], V[c]
        d = (B[0] - A[0]) * (C[1] - A[1]) - (C[0] - A[0]) * (B[1] - A[1])
        if d == 0:
            continue
        l1 = ((P[:, 0] - A[0]) * (C[1] - A[1]) - (C[0] - A[0]) * (P[:, 1] - A[1])) / d
        l2 = ((B[0] - A[0]) * (P[:, 1] - A[1]) - (P[:, 0] - A[0]) * (B[1] - A[1])) / d
        inside = (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
        z = A[2] + l1 * (B[2] - A[2]) + l2 * (C[2] - A[2])
        for i in np.nonzero(inside)[0]:
            crossings[i].append(z[i])
    return P, crossings


def test_volume_supersampled_voxelisation(ref):
    """Indicator transform against brute force: the solid is voxelised on a
    supersampled grid (column crossings decide inside), every sub-voxel is a
    small box with its own sinc transform, and the sum is taken directly.  The
    error is first order in the sub-voxel size and must shrink when it halves."""
    U, F = meshes.icosphere(1)
    V = meshes.sh_deform(U, 3.0, np.random.default_rng(1)) + 8.0     # inside a 16^3 grid
    L = 16.0
    k = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 1], [2, -1, 0], [1, 1, -2], [0, 0, 3]], float)
    xi = 2 * np.pi * k / L
    exact = ref.mesh_ft_raw(V, F, xi, VOLUME)
    errs = []
    for s in (4, 8):
        h = 1.0 / s
        cs = (np.arange(int(L * s)) + 0.5) * h
        P, cr = _column_voxelise(V, F, cs, cs)
        zc = cs
        tot = np.zeros(len(xi), complex)
        for (x, y), zs in zip(P, cr):
            if not zs:
                continue
            zs = np.sort(zs)
            inside = np.zeros(len(zc), bool)
            for z0, z1 in zip(zs[0::2], zs[1::2]):
                inside |= (zc > z0) & (zc < z1)
            if not inside.any():
                continue
            zin = zc[inside]
            ph = np.exp(-1j * (xi[:, 0:1] * x + xi[:, 1:2] * y + xi[:, 2:3] * zin[None, :]))
            tot += ph.sum(1)
        sub = h ** 3 * np.prod(sinc(xi * h / 2), axis=1)
        approx = tot * sub
        errs.append(np.max(np.abs(approx - exact)) / abs(exact[0]))
    assert errs[1] < 2e-2, errs
    assert errs[1] < 0.75 * errs[0], errs


# ----------------------------------------------------------------- gradients
@pytest.mark.parametrize("mode", [VOLUME, SURFACE, 2])
def test_vertex_gradient_matches_finite_differences(ref, mode):
    """Mode 2 is the unnormalised surface transform sum_T 2 A_T f_T."""
    V, F = _deformed(1, seed=2, R=2.0)
    rng = np.random.default_rng(11)
    xi = rng.normal(size=(12, 3)) * 1.2
    xi[0] = 0.0
    W = rng.normal(size=12) + 1j * rng.normal(size=12)

    def loss(Vx):
        u = ref.mesh_ft_raw(Vx, F, xi, VOLUME if mode == VOLUME else SURFACE)
        if mode == SURFACE:
            u = u / ref.surface_area(Vx, F)
        return float(np.real(np.sum(W * u)))

    g = ref.mesh_ft_vjp_raw(V, F, xi, W, mode)
    h = 1e-5
    for vi in [0, 5, 17, 33]:
        for j in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[vi, j] += h
            Vm[vi, j] -= h
            fd = (loss(Vp) - loss(Vm)) / (2 * h)
            assert abs(g[vi, j] - fd) < 1e-6 * (np.abs(g).max()), (vi, j, g[vi, j], fd)


def test_surface_area_gradient_matches_finite_differences(ref):
    """d|Lambda|/dV (with and without density weights, and with a zero-area
    triangle, which adds nothing) against central differences of the area."""
    V, F = _deformed(1, seed=4)
    n = len(V)
    V = np.concatenate([V, V[F[0, 0]][None], V[F[0, 0]][None] + [0.3, 0.0, 0.0]])
    F = np.concatenate([F, [[F[0, 0], n, n + 1]]])   # collinear: zero area
    wts = np.random.default_rng(3).uniform(0.5, 1.5, len(F))
    for tw in (None, wts):
        g = ref.surface_area_grad(V, F, tw)
        h = 1e-6
        for vi in [0, 3, 11, 29, n]:
            for j in range(3):
                Vp, Vm = V.copy(), V.copy()
                Vp[vi, j] += h
                Vm[vi, j] -= h
                fd = (ref.surface_area(Vp, F[:-1], None if tw is None else tw[:-1])
                      - ref.surface_area(Vm, F[:-1], None if tw is None else tw[:-1])) / (2 * h)
                assert abs(g[vi, j] - fd) < 1e-7 * np.abs(g).max(), (vi, j, g[vi, j], fd)
    # the mesh is closed: moving it rigidly keeps the area, so the gradient sums to zero
    assert np.abs(ref.surface_area_grad(V[:n], F[:-1]).sum(axis=0)).max() < 1e-12 * ref.surface_area(V[:n], F[:-1])


def test_surface_gradient_assembles_from_triangle_terms(ref):
    """Eq. 6 split into its two parts: on every vertex, the normalised
    surface gradient equals (raw triangle terms of the triangles around the
    vertex - s d|Lambda|/dv) / |Lambda| with the global scalar
    s = sum_k Re[W_k u_k] of the normalised transform u.  This is how a
    large mesh's gradient is checked at a few vertices."""
    V, F = _deformed(1, seed=7, R=2.5)
    rng = np.random.default_rng(17)
    xi = rng.normal(size=(20, 3)) * 1.1
    W = rng.normal(size=20) + 1j * rng.normal(size=20)
    full = ref.mesh_ft_vjp_raw(V, F, xi, W, SURFACE)
    area = ref.surface_area(V, F)
    u = ref.mesh_ft_raw(V, F, xi, SURFACE) / area
    s = float(np.real(np.sum(W * u)))
    dA = ref.surface_area_grad(V, F)
    for v in [0, 9, 23]:
        tris = np.nonzero((F == v).any(axis=1))[0]
        local = ref.mesh_ft_vjp_raw(V, F[tris], xi, W, 2)[v]
        got = (local - s * dA[v]) / area
        assert np.abs(got - full[v]).max() < 1e-12 * np.abs(full).max(), (v, got, full[v])


def test_volume_gradient_at_zero_frequency_is_normal_sum(ref):
    """d(volume)/dv = sum over incident faces of (v2-v1)x(v3-v1)/6."""
    V, F = _deformed(1, seed=5)
    g = ref.mesh_ft_vjp_raw(V, F, np.zeros((1, 3)), np.ones(1), VOLUME)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    want = np.zeros_like(V)
    for p in range(3):
        np.add.at(want, F[:, p], n / 6)
    assert np.max(np.abs(g - want)) < 1e-12 * np.abs(want).max()


def test_surface_gradient_at_zero_frequency_vanishes(ref):
    """The normalised surface density integrates to one for every shape."""
    V, F = _deformed(1, seed=6)
    g = ref.mesh_ft_vjp_raw(V, F, np.zeros((1, 3)), np.ones(1), SURFACE)
    assert np.max(np.abs(g)) < 1e-14


# ------------------------------------------------------------ whole pipeline
def _small_case(mode, tau=1e-3):
    U, F = meshes.icosphere(1)
    g = configs.Grid((16, 14, 12), (1.0, 1.25, 1.5), (0.5, -0.25, 1.0), tau, mode)
    V = meshes.sh_deform(U, 3.0, np.random.default_rng(2)) + g.centre
    return V.astype(np.float32).astype(np.float64), F, g, configs.psf_diag(1.1, 2.0)


def test_gaussian_otf_is_transform_of_eq2_kernel(ref):
    """exp(-xi^T Sigma xi / 2) is the transform of the normalised Gaussian of
    Eq. 2 with covariance Sigma (checked by a fine Riemann sum)."""
    S = np.array([[1.2, 0.3, 0.1], [0.3, 0.8, -0.2], [0.1, -0.2, 2.0]])
    Si = np.linalg.inv(S)
    h = 0.1
    ax = np.arange(-9, 9 + h / 2, h)
    X = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    kern = np.exp(-0.5 * np.einsum("ni,ij,nj->n", X, Si, X)) / np.sqrt((2 * np.pi) ** 3 * np.linalg.det(S))
    for xi in [np.array([0.5, -0.3, 0.2]), np.array([1.0, 0.4, -0.7])]:
        num = np.sum(kern * np.exp(-1j * X @ xi)) * h ** 3
        q = ref.quad_form(xi[None], (1.2, 0.8, 2.0, 0.3, 0.1, -0.2))[0]
        assert abs(num - np.exp(-0.5 * q)) < 1e-6


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_image_integrates_to_volume_or_one(ref, mode):
    V, F, g, S = _small_case(mode)
    img = ref.render(V, F, g, S)
    dvol = np.prod(g.spacing)
    total = img.sum() * dvol
    want = ref.mesh_ft_raw(V - np.array(g.origin), F, np.zeros((1, 3)), VOLUME)[0].real if mode == VOLUME else 1.0
    assert abs(total - want) < 1e-11 * abs(want)


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_integer_voxel_shift_rolls_the_image(ref, mode):
    V, F, g, S = _small_case(mode)
    img = ref.render(V, F, g, S)
    m = np.array([3, -2, 1])
    img2 = ref.render(V + m * np.array(g.spacing), F, g, S)
    assert np.max(np.abs(img2 - np.roll(img, tuple(m), axis=(0, 1, 2)))) < 1e-12 * np.abs(img).max()


def test_band_threshold_and_full_spectrum(ref):
    V, F, g, S = _small_case(VOLUME, tau=0.0)
    _, h, band = ref.otf_and_band(g, S)
    assert band.all()
    _, h, band = ref.otf_and_band(g.with_tau(1.0), S)
    assert not band.any()
    img = ref.render(V, F, g.with_tau(1.0), S)
    assert np.all(img == 0)
    _, h, band = ref.otf_and_band(g.with_tau(0.05), S)
    assert np.all(h[band] > 0.05 * (1 - 1e-12)) and np.all(h[~band] <= 0.05 * (1 + 1e-12))


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_render_vjp_matches_finite_differences(ref, mode):
    V, F, g, S = _small_case(mode)
    rng = np.random.default_rng(9)
    target = rng.normal(size=g.n) * 1e-3

    def loss(Vx, Sx, band_S=None):
        return float(np.mean((ref.render(Vx, F, g, Sx, band_sigma6=band_S) - target) ** 2))

    img = ref.render(V, F, g, S)
    dLdI = 2 * (img - target) / img.size
    dV, dS = ref.render_vjp(V, F, g, S, dLdI)
    h = 1e-5
    for vi, j in [(0, 0), (7, 1), (20, 2), (41, 0)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[vi, j] += h
        Vm[vi, j] -= h
        fd = (loss(Vp, S) - loss(Vm, S)) / (2 * h)
        assert abs(dV[vi, j] - fd) < 1e-5 * np.abs(dV).max(), (vi, j)
    Sarr = np.array(S, float)
    Sarr[3] = 0.05   # perturb around a non-diagonal covariance too
    dV, dS = ref.render_vjp(V, F, g, tuple(Sarr), 2 * (ref.render(V, F, g, tuple(Sarr)) - target) / img.size)
    for i in range(6):
        Sp, Sm = Sarr.copy(), Sarr.copy()
        Sp[i] += h
        Sm[i] -= h
        fd = (loss(V, tuple(Sp), tuple(Sarr)) - loss(V, tuple(Sm), tuple(Sarr))) / (2 * h)
        assert abs(dS[i] - fd) < 1e-6 * np.abs(dS).max() + 1e-14, (i, dS[i], fd)


@pytest.mark.parametrize("mode", [VOLUME, SURFACE])
def test_adjoint_dot_product(ref, mode):
    """<G, J d> = <J^T G, d> for the linear map J: (dV, dSigma) -> dI, with
    J d taken by central differences of the image along one random
    direction of all vertices and all six covariance entries at once, and
    J^T G the gradient render_vjp returns for dL/dI = G (band fixed)."""
    V, F, g, S = _small_case(mode)
    rng = np.random.default_rng(13)
    G = rng.normal(size=g.n)
    dVd = rng.normal(size=V.shape)
    dSd = rng.normal(size=6) * 0.05
    S0 = np.array(S, float)
    h = 1e-4
    Ip = ref.render(V + h * dVd, F, g, tuple(S0 + h * dSd), band_sigma6=tuple(S0))
    Im = ref.render(V - h * dVd, F, g, tuple(S0 - h * dSd), band_sigma6=tuple(S0))
    lhs = float((G * (Ip - Im)).sum() / (2 * h))
    gV, gS = ref.render_vjp(V, F, g, tuple(S0), G)
    rhs = float((gV * dVd).sum() + (gS * dSd).sum())
    assert abs(lhs - rhs) < 1e-6 * max(abs(lhs), abs(rhs)), (lhs, rhs)
