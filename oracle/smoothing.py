"""FP64 reference of the smoothed vertex update of the shape step.

TEST INFRASTRUCTURE ONLY.  The tests and the benchmark use it to check the
GPU library; the library never imports or calls anything here, and nothing
here imports the library.

Paper Sec. 5.2 moves the vertices along the loss gradient filtered by
(I + lambda L)^{-2}, L a Laplacian of the mesh.  Reading taken (listed in the
design notes): L = D - A, the combinatorial Laplacian of the graph of mesh
edges (A[i, j] = 1 when i and j share an edge, D the diagonal of vertex
degrees); a vertex on no edge has a zero row.  The filtered gradient is
obtained by two direct sparse solves in float64 (scipy's spsolve), one
column of the gradient at a time.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def edge_adjacency(F, n_verts: int) -> sp.csr_matrix:
    """Symmetric 0/1 adjacency of the vertices joined by a face edge."""
    F = np.asarray(F, dtype=np.int64).reshape(-1, 3)
    a = np.concatenate([F[:, 0], F[:, 1], F[:, 2]])
    b = np.concatenate([F[:, 1], F[:, 2], F[:, 0]])
    keep = a != b
    a, b = a[keep], b[keep]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    A = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n_verts, n_verts)).tocsr()
    A.data[:] = 1.0   # duplicates (an edge shared by two faces) count once
    return A


def graph_laplacian(F, n_verts: int) -> sp.csr_matrix:
    A = edge_adjacency(F, n_verts)
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(deg) - A).tocsr()


def laplace_smooth(F, n_verts: int, grad, lam: float) -> np.ndarray:
    """(I + lam L)^{-2} grad for grad of shape [n_verts, 3] (float64)."""
    g = np.asarray(grad, dtype=np.float64).reshape(n_verts, -1)
    M = (sp.identity(n_verts, format="csc") + lam * graph_laplacian(F, n_verts).tocsc()).tocsc()
    out = np.empty_like(g)
    for c in range(g.shape[1]):
        y = spla.spsolve(M, g[:, c])
        out[:, c] = spla.spsolve(M, y)
    return out
