// Host-side checks and mesh tables of the renderer: argument validation,
// face validation, closure and orientation, triangle strips, vertex incidence
// and adjacency, and the closure test of density weights.  Plain C++ with no
// HIP dependency, so the same code also builds and runs alone under the host
// sanitizers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/deltamic.h"

namespace dm {

// Per-triangle flags of the strip order.
constexpr int TRI_STRIP_START = 1;   // first triangle of a strip
constexpr int TRI_REVERSED = 2;      // strip order is an odd permutation of the input face

// Width of the fixed neighbour table of the Laplacian filter (-1 padded).
constexpr int LAP_TABLE_W = 8;

// Outcome of a check: st == DM_OK, or the status and a message.
struct Check {
  dm_status st = DM_OK;
  std::string msg;
};

// Grid: positive finite spacing, finite origin, n >= 1, a non-negative
// threshold, a known density mode, at most 2^29 half-spectrum positions.
Check validate_grid(const dm_grid* g);
// PSF: finite covariance entries, symmetric positive definite (Cholesky in
// double).
Check validate_psf(const dm_psf* p);

// Greedy triangle strips.  From each unused seed triangle (in input order)
// the strip is grown across the edge formed by its last two vertices while
// the triangle across it is unused; of the seed's three rotations the longest
// strip is kept.  Output: faces in strip order (s_i, s_i+1, s_i+2), per
// triangle TRI_STRIP_START / TRI_REVERSED flags and, if src is given, the
// input face of each strip-order triangle.  Returns the number of strips.
int build_strips(const std::vector<int32_t>& F, std::vector<int32_t>& Fs, std::vector<int32_t>& flags,
                 std::vector<int32_t>* src = nullptr);

// Host tables of a mesh connectivity.
struct TopoTables {
  std::vector<int32_t> faces;     // [nt][3] in strip order
  std::vector<int32_t> flags;     // [nt] TRI_STRIP_START | TRI_REVERSED
  std::vector<int32_t> src;       // [nt] input face of each strip-order triangle
  std::vector<int32_t> csr_off;   // [nv + 1] vertex incidence ...
  std::vector<int32_t> csr_ent;   // [3 nt] ... entries 3 t + p (strip-order t, slot p)
  std::vector<int32_t> adj_off;   // [nv + 1] vertex adjacency (mesh edges, both directions) ...
  std::vector<int32_t> adj_nbr;   // ... neighbours
  std::vector<int32_t> adj_tab;   // [nv][LAP_TABLE_W] neighbours, -1 padded; empty if a degree exceeds the width
  int n_strips = 0;
  int lap_mu = 0;                 // max over mesh edges of d_i + d_j (bounds the largest eigenvalue of D - A)
  bool closed = false;            // every directed edge exactly once, its reverse present
};

// Validates the faces F [nt][3] (indices in [0, n_verts): DM_ERR_MESH
// otherwise) and builds the tables.
Check build_topology(const std::vector<int32_t>& F, int n_verts, TopoTables* out);

// Density weights of the faces (input order, [nt]): DM_ERR_ARG if one is not
// finite; *closed tells whether they cancel across every edge (the sum of the
// weights of the faces on the edge, signed by the direction each face runs
// along it, within 1e-6 of the sum of their magnitudes).
Check weights_close(const std::vector<int32_t>& faces_in, const float* weights, int nt, bool* closed);

}  // namespace dm
