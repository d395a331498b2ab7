"""Strip order of the topologies (host logic, no GPU): every input face
appears once, consecutive triangles of a strip share the edge of the last two
vertices, and the orientation flag says whether the written vertex order is an
odd permutation of the input face."""
import numpy as np
import pytest

from workloads import configs, meshes


def _cases():
    out = {"ico2": meshes.icosphere(2)[1], "ico4": meshes.icosphere(4)[1], "geo5": meshes.geodesic_sphere(5)[1],
           "box": meshes.box_mesh((0, 0, 0), (1, 2, 3))[1], "tet": meshes.tetrahedron()[1]}
    V, F = meshes.icosphere(2)
    out["hemisphere"] = F[V[F].mean(axis=1)[:, 2] > 0.0]                 # open: boundary edges
    Vb, Fb = meshes.box_mesh((0, 0, 0), (1, 1, 1))
    out["fin"] = np.concatenate([Fb, [[0, 1, 8]]])                         # an edge shared by three faces
    out["one"] = np.array([[0, 1, 2]])
    return out


def _is_rotation(a, b):
    return any(tuple(a) == (b[r], b[(r + 1) % 3], b[(r + 2) % 3]) for r in range(3))


@pytest.mark.parametrize("name", list(_cases()))
def test_strip_order_is_a_valid_strip_cover(name):
    dm = pytest.importorskip("paper_2303_10440_amd")
    F = np.asarray(_cases()[name], dtype=np.int32)
    Fs, flags, n_strips = dm.topology_strips(F)
    assert Fs.shape == F.shape and flags.shape == (len(F),)
    # every input face exactly once (as a vertex set)
    key = lambda f: tuple(sorted(int(x) for x in f))
    assert sorted(map(key, F)) == sorted(map(key, Fs))
    # orientation flag
    by_key = {key(f): f for f in F}
    for f, fl in zip(Fs, flags):
        assert bool(fl & 2) == (not _is_rotation(f, by_key[key(f)]))
    # strips: starts counted, neighbours share the edge of the last two vertices
    assert flags[0] & 1 and int((flags & 1).sum()) == n_strips
    for i in range(1, len(Fs)):
        if not flags[i] & 1:
            assert (Fs[i][0], Fs[i][1]) == (Fs[i - 1][1], Fs[i - 1][2]), (name, i)
            assert Fs[i][2] not in (Fs[i][0], Fs[i][1])


def test_strips_are_long_on_the_benchmark_cells():
    dm = pytest.importorskip("paper_2303_10440_amd")
    F = configs.cfg3().F
    _, flags, n_strips = dm.topology_strips(F)
    assert len(F) / n_strips >= 20          # measured: 29.8 triangles per strip
    F5 = meshes.geodesic_sphere(16)[1]
    _, _, n5 = dm.topology_strips(F5)
    assert len(F5) / n5 >= 40                # measured: 64


def test_strips_argument_errors():
    dm = pytest.importorskip("paper_2303_10440_amd")
    Fs, flags, n = dm.topology_strips(np.zeros((0, 3), np.int32))
    assert Fs.shape == (0, 3) and n == 0
    with pytest.raises(dm.DeltamicError):
        dm._check(dm.lib().dm_topology_strips(None, -1, None, None, None), "dm_topology_strips")
