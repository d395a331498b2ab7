"""Input generators and host-side marshalling (no GPU)."""
import ctypes

import numpy as np
import pytest

from workloads import configs, meshes


def _outward(V, F):
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    c = V.mean(0)
    return bool((np.einsum("ij,ij->i", n, V[F].mean(1) - c) > 0).all())


@pytest.mark.parametrize("sub,nv,nf", [(0, 12, 20), (1, 42, 80), (2, 162, 320), (4, 2562, 5120)])
def test_icosphere_counts_closed_outward(sub, nv, nf):
    V, F = meshes.icosphere(sub)
    assert V.shape == (nv, 3) and F.shape == (nf, 3)
    assert meshes.check_closed_oriented(F) and _outward(V, F)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)


@pytest.mark.parametrize("freq", [1, 3, 5, 16, 45])
def test_geodesic_counts_closed_outward(freq):
    V, F = meshes.geodesic_sphere(freq)
    assert V.shape == (10 * freq * freq + 2, 3) and F.shape == (20 * freq * freq, 3)
    assert meshes.check_closed_oriented(F) and _outward(V, F)


def test_box_and_tetrahedron_closed_outward():
    for V, F in (meshes.box_mesh((0, 0, 0), (1, 2, 3)), meshes.tetrahedron()):
        assert meshes.check_closed_oriented(F) and _outward(V, F)
    V, F = meshes.box_mesh((0, 0, 0), (1, 1, 1))
    assert not meshes.check_closed_oriented(F[1:])
    assert not meshes.check_closed_oriented(meshes.flip_faces(F)[:, [0, 0, 2]])


def test_configs_are_seeded_and_fit_their_grids():
    for mode in (configs.VOLUME, configs.SURFACE):
        a, b = configs.cfg3(mode), configs.cfg3(mode)
        assert np.array_equal(a.V, b.V) and np.array_equal(a.F, b.F)
    for c in (configs.cfg1(), configs.cfg2(), configs.cfg3(), configs.box_case()):
        L = np.array(c.grid.n) * np.array(c.grid.spacing)
        assert (c.V.min(0) > c.grid.origin).all() and (c.V.max(0) < np.array(c.grid.origin) + L).all()
        assert c.V.dtype == np.float32 and c.F.dtype == np.int32
        assert meshes.check_closed_oriented(c.F)
    cells = configs.cfg4(count=6)
    assert all(1000 * 0.8 <= c.F.shape[0] <= 20000 * 1.2 for c in cells)
    pool, t, idx, widx = configs.cfg5_pooled(count=50, pool=8)
    assert len(pool) == 8 and len(t) == 50 and np.all(np.diff(t) > 0) and idx.max() < 8


def test_binding_marshalling_without_gpu():
    dm = pytest.importorskip("paper_2303_10440_amd")
    g = configs.cfg3().grid
    cg = dm._grid(g)
    assert list(cg.n) == [128, 128, 64] and abs(cg.spacing[2] - 0.5) < 1e-7 and cg.mode == 0
    assert abs(cg.band_tau - np.float32(1e-3)) == 0
    p = dm._psf((1, 2, 3, 4, 5, 6))
    assert list(p.sigma) == [1, 2, 3, 4, 5, 6]
    with pytest.raises(ValueError):
        dm._psf((1, 2, 3))
    assert "dm_batch_run" in dm.header_symbols() and "dm_submit" in dm.header_symbols()


def test_ctypes_structs_match_the_c_header(tmp_path):
    """Field offsets and sizes of the binding's ctypes mirrors equal those the
    C compiler derives from include/deltamic.h."""
    import subprocess
    dm = pytest.importorskip("paper_2303_10440_amd")
    pairs = {"dm_grid": dm.CGrid, "dm_psf": dm.CPsf, "dm_mesh": dm.CMesh, "dm_request": dm.CRequest,
             "dm_kernel_time": dm.CKernelTime, "dm_server_config": dm.CServerConfig,
             "dm_serve_request": dm.CServeRequest, "dm_serve_result": dm.CServeResult,
             "dm_server_stats": dm.CServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{dm.HEADER}"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
