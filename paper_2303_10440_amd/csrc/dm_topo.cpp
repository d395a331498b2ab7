// Host-side checks and mesh tables (see dm_topo.h).  No HIP: the library
// links it, and the host sanitizer build of the tests compiles it alone.
#include "dm_topo.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <utility>

namespace dm {

namespace {

Check bad(dm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  Check c;
  c.st = st;
  c.msg = buf;
  return c;
}

}  // namespace

Check validate_grid(const dm_grid* g) {
  if (!g) return bad(DM_ERR_ARG, "grid is NULL");
  for (int j = 0; j < 3; ++j) {
    if (g->n[j] < 1) return bad(DM_ERR_ARG, "grid n[%d] = %d must be >= 1", j, g->n[j]);
    // keeps every vertex phase the sweeps pass to the hardware sine and
    // cosine inside their domain of [-256, 256] revolutions
    if (g->n[j] > DM_MAX_AXIS) return bad(DM_ERR_ARG, "grid n[%d] = %d exceeds %d", j, g->n[j], DM_MAX_AXIS);
    if (!(g->spacing[j] > 0.0f) || !std::isfinite(g->spacing[j]))
      return bad(DM_ERR_ARG, "grid spacing[%d] must be finite and > 0", j);
    if (!std::isfinite(g->origin[j])) return bad(DM_ERR_ARG, "grid origin[%d] must be finite", j);
  }
  // in double: the int32 sizes may multiply past 2^63
  const double npos = (double)g->n[0] * (double)g->n[1] * (double)(g->n[2] / 2 + 1);
  if (npos > (double)((int64_t)1 << 29)) return bad(DM_ERR_ARG, "grid too large (%.4g half-spectrum positions)", npos);
  if (!(g->band_tau >= 0.0f) || std::isnan(g->band_tau)) return bad(DM_ERR_ARG, "band_tau must be >= 0");
  if (g->mode != DM_VOLUME && g->mode != DM_SURFACE) return bad(DM_ERR_ARG, "unknown mode %d", g->mode);
  return Check{};
}

Check validate_psf(const dm_psf* p) {
  if (!p) return bad(DM_ERR_ARG, "psf is NULL");
  for (int j = 0; j < 6; ++j)
    if (!std::isfinite(p->sigma[j])) return bad(DM_ERR_PSF, "sigma[%d] is not finite", j);
  // Cholesky of [[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]] in double.
  const double a = p->sigma[0], b = p->sigma[3], c = p->sigma[4], d = p->sigma[1], e = p->sigma[5], f = p->sigma[2];
  if (!(a > 0)) return bad(DM_ERR_PSF, "covariance not positive definite (xx <= 0)");
  const double l21 = b / std::sqrt(a), l31 = c / std::sqrt(a);
  const double d2 = d - l21 * l21;
  if (!(d2 > 0)) return bad(DM_ERR_PSF, "covariance not positive definite");
  const double l32 = (e - l31 * l21) / std::sqrt(d2);
  const double d3 = f - l31 * l31 - l32 * l32;
  if (!(d3 > 0)) return bad(DM_ERR_PSF, "covariance not positive definite");
  return Check{};
}

int build_strips(const std::vector<int32_t>& F, std::vector<int32_t>& Fs, std::vector<int32_t>& flags,
                 std::vector<int32_t>* src) {
  const int nt = (int)(F.size() / 3);
  std::vector<std::pair<uint64_t, int>> edges;
  edges.reserve(F.size());
  for (int t = 0; t < nt; ++t)
    for (int p = 0; p < 3; ++p) {
      const uint32_t a = (uint32_t)F[3 * t + p], b = (uint32_t)F[3 * t + (p + 1) % 3];
      edges.push_back({((uint64_t)std::min(a, b) << 32) | std::max(a, b), t});
    }
  std::sort(edges.begin(), edges.end());
  std::vector<char> used((size_t)nt, 0), trial((size_t)nt, 0);
  // the unused triangle other than `from` across edge {x, y}, or -1
  auto across = [&](int32_t x, int32_t y, const std::vector<char>& taken) {
    const uint64_t key = ((uint64_t)std::min((uint32_t)x, (uint32_t)y) << 32) | std::max((uint32_t)x, (uint32_t)y);
    auto it = std::lower_bound(edges.begin(), edges.end(), std::make_pair(key, -1));
    for (; it != edges.end() && it->first == key; ++it)
      if (!used[(size_t)it->second] && !taken[(size_t)it->second]) return it->second;
    return -1;
  };
  // the vertex of triangle u left after removing one occurrence each of x and
  // y (its edge {x, y}), so that (x, y, third) is a permutation of the face
  // also when the face repeats a vertex
  auto third = [&](int u, int32_t x, int32_t y) {
    bool taken[3] = {false, false, false};
    for (const int32_t w : {x, y})
      for (int p = 0; p < 3; ++p)
        if (!taken[p] && F[3 * (size_t)u + p] == w) {
          taken[p] = true;
          break;
        }
    for (int p = 0; p < 3; ++p)
      if (!taken[p]) return F[3 * (size_t)u + p];
    return F[3 * (size_t)u];
  };
  Fs.clear();
  flags.clear();
  Fs.reserve(F.size());
  flags.reserve((size_t)nt);
  if (src) {
    src->clear();
    src->reserve((size_t)nt);
  }
  int n_strips = 0;
  std::vector<int> tris, best_tris;
  std::vector<int32_t> seq, best_seq;
  for (int s = 0; s < nt; ++s) {
    if (used[(size_t)s]) continue;
    best_tris.clear();
    for (int r = 0; r < 3; ++r) {
      seq = {F[3 * s + r], F[3 * s + (r + 1) % 3], F[3 * s + (r + 2) % 3]};
      tris = {s};
      trial[(size_t)s] = 1;
      for (;;) {
        const int32_t x = seq[seq.size() - 2], y = seq.back();
        const int u = across(x, y, trial);
        if (u < 0) break;
        trial[(size_t)u] = 1;
        tris.push_back(u);
        seq.push_back(third(u, x, y));
      }
      for (int u : tris) trial[(size_t)u] = 0;
      if (tris.size() > best_tris.size()) {
        best_tris = tris;
        best_seq = seq;
      }
    }
    for (size_t i = 0; i < best_tris.size(); ++i) {
      const int u = best_tris[i];
      used[(size_t)u] = 1;
      const int32_t a = best_seq[i], b = best_seq[i + 1], c = best_seq[i + 2];
      Fs.push_back(a);
      Fs.push_back(b);
      Fs.push_back(c);
      // (a, b, c) is a rotation of the input face (same orientation) or not
      bool same = false;
      for (int r = 0; r < 3; ++r)
        same = same || (F[3 * u + r] == a && F[3 * u + (r + 1) % 3] == b && F[3 * u + (r + 2) % 3] == c);
      flags.push_back((i == 0 ? TRI_STRIP_START : 0) | (same ? 0 : TRI_REVERSED));
      if (src) src->push_back(u);
    }
    ++n_strips;
  }
  return n_strips;
}

Check build_topology(const std::vector<int32_t>& F, int n_verts, TopoTables* out) {
  const size_t nt = F.size() / 3;
  for (size_t i = 0; i < F.size(); ++i)
    if (F[i] < 0 || F[i] >= n_verts)
      return bad(DM_ERR_MESH, "face %zu references vertex %d outside [0, %d)", i / 3, F[i], n_verts);
  // closed and consistently oriented: each directed edge once, with its reverse present
  std::vector<uint64_t> e;
  e.reserve(F.size());
  for (size_t t = 0; t < nt; ++t)
    for (int p = 0; p < 3; ++p) {
      const uint32_t a = (uint32_t)F[3 * t + p], b = (uint32_t)F[3 * t + (p + 1) % 3];
      e.push_back(((uint64_t)a << 32) | b);
    }
  std::sort(e.begin(), e.end());
  bool closed = nt > 0 && std::adjacent_find(e.begin(), e.end()) == e.end();
  if (closed)
    for (uint64_t x : e) {
      const uint64_t r = (x << 32) | (x >> 32);
      if (!std::binary_search(e.begin(), e.end(), r)) {
        closed = false;
        break;
      }
    }
  TopoTables& T = *out;
  T = TopoTables{};
  T.closed = closed;
  T.n_strips = build_strips(F, T.faces, T.flags, &T.src);
  const std::vector<int32_t>& Fs = T.faces;
  // vertex incidence (CSR)
  T.csr_off.assign((size_t)n_verts + 1, 0);
  T.csr_ent.assign(Fs.size(), 0);
  for (size_t i = 0; i < Fs.size(); ++i) T.csr_off[(size_t)Fs[i] + 1]++;
  for (int v = 0; v < n_verts; ++v) T.csr_off[(size_t)v + 1] += T.csr_off[(size_t)v];
  std::vector<int32_t> fill(T.csr_off.begin(), T.csr_off.end() - 1);
  for (size_t i = 0; i < Fs.size(); ++i) T.csr_ent[(size_t)fill[(size_t)Fs[i]]++] = (int32_t)i;   // i = 3 t + p
  // vertex adjacency: both directions of every undirected mesh edge, unique
  std::vector<uint64_t> und;
  und.reserve(2 * e.size());
  for (uint64_t x : e) {
    const uint64_t a = x >> 32, b = x & 0xffffffffu;
    if (a == b) continue;
    und.push_back((a << 32) | b);
    und.push_back((b << 32) | a);
  }
  std::sort(und.begin(), und.end());
  und.erase(std::unique(und.begin(), und.end()), und.end());
  T.adj_off.assign((size_t)n_verts + 1, 0);
  T.adj_nbr.assign(und.size(), 0);
  for (size_t i = 0; i < und.size(); ++i) {
    T.adj_off[(size_t)(und[i] >> 32) + 1]++;
    T.adj_nbr[i] = (int32_t)(und[i] & 0xffffffffu);
  }
  for (int v = 0; v < n_verts; ++v) T.adj_off[(size_t)v + 1] += T.adj_off[(size_t)v];
  int max_deg = 0;
  for (int v = 0; v < n_verts; ++v) max_deg = std::max(max_deg, T.adj_off[(size_t)v + 1] - T.adj_off[(size_t)v]);
  for (int v = 0; v < n_verts; ++v)
    for (int o = T.adj_off[(size_t)v]; o < T.adj_off[(size_t)v + 1]; ++o) {
      const int u = T.adj_nbr[(size_t)o];
      T.lap_mu = std::max(T.lap_mu, (T.adj_off[(size_t)v + 1] - T.adj_off[(size_t)v]) +
                                        (T.adj_off[(size_t)u + 1] - T.adj_off[(size_t)u]));
    }
  if (max_deg <= LAP_TABLE_W) {
    T.adj_tab.assign((size_t)n_verts * LAP_TABLE_W, -1);
    for (int v = 0; v < n_verts; ++v)
      for (int o = T.adj_off[(size_t)v]; o < T.adj_off[(size_t)v + 1]; ++o)
        T.adj_tab[(size_t)v * LAP_TABLE_W + (size_t)(o - T.adj_off[(size_t)v])] = T.adj_nbr[(size_t)o];
  }
  return Check{};
}

Check weights_close(const std::vector<int32_t>& faces_in, const float* weights, int nt, bool* closed) {
  for (int i = 0; i < nt; ++i)
    if (!std::isfinite(weights[i])) return bad(DM_ERR_ARG, "weight of face %d is not finite", i);
  // across every edge the weights of the incident faces, signed by the
  // direction in which each face runs along the edge, cancel
  std::vector<std::pair<uint64_t, std::pair<double, double>>> e;   // edge -> (signed weight, |weight|)
  e.reserve((size_t)nt * 3);
  for (int f = 0; f < nt; ++f)
    for (int p = 0; p < 3; ++p) {
      const uint32_t a = (uint32_t)faces_in[(size_t)3 * f + p], b = (uint32_t)faces_in[(size_t)3 * f + (p + 1) % 3];
      const double w = weights[f];
      const uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
      e.push_back({key, {a < b ? w : -w, std::fabs(w)}});
    }
  std::sort(e.begin(), e.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  bool ok = nt > 0;
  for (size_t i = 0; i < e.size() && ok;) {
    size_t j = i;
    double sum = 0.0, mag = 0.0;
    for (; j < e.size() && e[j].first == e[i].first; ++j) {
      sum += e[j].second.first;
      mag += e[j].second.second;
    }
    if (std::fabs(sum) > 1e-6 * mag) ok = false;
    i = j;
  }
  *closed = ok;
  return Check{};
}

}  // namespace dm
