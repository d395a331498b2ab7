// Host sanitizer harness of the renderer's host-side checks and mesh tables
// (paper_2303_10440_amd/csrc/dm_topo.cpp) and of its sweep launch planning
// (dm_plan.h), built alone with -fsanitize=address,undefined by
// tests/test_sanitize_cpu.py.  Exercises closed, open, non-manifold,
// degenerate, random and out-of-range face sets, empty meshes, density
// weights, bad grids and covariances, and the sweep plans over a range of band
// and mesh sizes, and checks the invariants of every table and plan.  Exit
// status 0 iff every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <map>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "dm_plan.h"
#include "dm_topo.h"

using dm::Check;
using dm::TopoTables;

static int g_fail = 0;
#define EXPECT(c)                                                    \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                      \
    }                                                                \
  } while (0)

// icosahedron refined by midpoint subdivision (vertex positions are not
// needed: only the connectivity), counter-clockwise seen from outside
static std::vector<int32_t> icosphere_faces(int sub, int* nv) {
  std::vector<int32_t> F = {0, 11, 5, 0, 5, 1, 0, 1, 7, 0, 7, 10, 0, 10, 11, 1, 5, 9, 5, 11, 4, 11, 10, 2, 10, 7, 6,
                            7, 1, 8, 3, 9, 4, 3, 4, 2, 3, 2, 6, 3, 6, 8, 3, 8, 9, 4, 9, 5, 2, 4, 11, 6, 2, 10, 8, 6, 7,
                            9, 8, 1};
  int n = 12;
  for (int s = 0; s < sub; ++s) {
    std::map<std::pair<int, int>, int> mid;
    auto m = [&](int a, int b) {
      const auto key = std::make_pair(std::min(a, b), std::max(a, b));
      auto it = mid.find(key);
      if (it != mid.end()) return it->second;
      mid[key] = n;
      return n++;
    };
    std::vector<int32_t> G;
    for (size_t t = 0; t < F.size() / 3; ++t) {
      const int a = F[3 * t], b = F[3 * t + 1], c = F[3 * t + 2];
      const int ab = m(a, b), bc = m(b, c), ca = m(c, a);
      const int tri[4][3] = {{a, ab, ca}, {b, bc, ab}, {c, ca, bc}, {ab, bc, ca}};
      for (auto& q : tri)
        for (int p = 0; p < 3; ++p) G.push_back(q[p]);
    }
    F.swap(G);
  }
  *nv = n;
  return F;
}

static std::vector<int32_t> box_faces() {
  // unit cube, 8 corners (x + 2y + 4z), outward orientation
  return {0, 2, 3, 0, 3, 1, 4, 5, 7, 4, 7, 6, 0, 1, 5, 0, 5, 4, 2, 6, 7, 2, 7, 3, 0, 4, 6, 0, 6, 2, 1, 3, 7, 1, 7, 5};
}

static bool is_rotation(const int32_t* f, int a, int b, int c) {
  for (int r = 0; r < 3; ++r)
    if (f[r] == a && f[(r + 1) % 3] == b && f[(r + 2) % 3] == c) return true;
  return false;
}

// invariants of the tables of a valid face set
static void check_tables(const std::vector<int32_t>& F, int nv, const TopoTables& T) {
  const size_t nt = F.size() / 3;
  EXPECT(T.faces.size() == F.size());
  EXPECT(T.flags.size() == nt && T.src.size() == nt);
  // strip order is a permutation of the input faces, each a rotation or a reversal
  std::vector<int> seen(nt, 0);
  int starts = 0;
  for (size_t t = 0; t < nt; ++t) {
    const int s = T.src[t];
    EXPECT(s >= 0 && (size_t)s < nt);
    if (s < 0 || (size_t)s >= nt) continue;
    seen[(size_t)s]++;
    const int a = T.faces[3 * t], b = T.faces[3 * t + 1], c = T.faces[3 * t + 2];
    const bool same = is_rotation(&F[3 * (size_t)s], a, b, c);
    const bool rev = is_rotation(&F[3 * (size_t)s], a, c, b);
    EXPECT(same || rev);
    EXPECT(((T.flags[t] & dm::TRI_REVERSED) != 0) == !same);
    if (T.flags[t] & dm::TRI_STRIP_START) {
      ++starts;
    } else {
      // (s_i, s_i+1, s_i+2) then (s_i+1, s_i+2, s_i+3)
      EXPECT(t > 0);
      if (t > 0) EXPECT(T.faces[3 * t] == T.faces[3 * (t - 1) + 1] && T.faces[3 * t + 1] == T.faces[3 * (t - 1) + 2]);
    }
  }
  for (size_t s = 0; s < nt; ++s) EXPECT(seen[s] == 1);
  EXPECT(starts == T.n_strips);
  EXPECT(nt == 0 || (T.flags[0] & dm::TRI_STRIP_START));
  // vertex incidence
  EXPECT(T.csr_off.size() == (size_t)nv + 1 && T.csr_ent.size() == 3 * nt);
  EXPECT(T.csr_off[0] == 0 && (size_t)T.csr_off[(size_t)nv] == 3 * nt);
  std::vector<int> used(3 * nt, 0);
  for (int v = 0; v < nv; ++v) {
    EXPECT(T.csr_off[(size_t)v] <= T.csr_off[(size_t)v + 1]);
    for (int o = T.csr_off[(size_t)v]; o < T.csr_off[(size_t)v + 1]; ++o) {
      const int i = T.csr_ent[(size_t)o];
      EXPECT(i >= 0 && (size_t)i < 3 * nt);
      if (i < 0 || (size_t)i >= 3 * nt) continue;
      used[(size_t)i]++;
      EXPECT(T.faces[(size_t)i] == v);
    }
  }
  for (size_t i = 0; i < 3 * nt; ++i) EXPECT(used[i] == 1);
  // adjacency: symmetric, no self loops, exactly the mesh edges
  std::set<std::pair<int, int>> edges;
  for (size_t t = 0; t < nt; ++t)
    for (int p = 0; p < 3; ++p) {
      const int a = F[3 * t + p], b = F[3 * t + (p + 1) % 3];
      if (a != b) {
        edges.insert({a, b});
        edges.insert({b, a});
      }
    }
  EXPECT(T.adj_off.size() == (size_t)nv + 1 && T.adj_nbr.size() == edges.size());
  std::set<std::pair<int, int>> got;
  int max_deg = 0;
  for (int v = 0; v < nv; ++v) {
    max_deg = std::max(max_deg, T.adj_off[(size_t)v + 1] - T.adj_off[(size_t)v]);
    for (int o = T.adj_off[(size_t)v]; o < T.adj_off[(size_t)v + 1]; ++o) got.insert({v, T.adj_nbr[(size_t)o]});
  }
  EXPECT(got == edges);
  // the Laplacian's eigenvalue bound: the largest d_i + d_j over the edges
  {
    std::map<int, int> deg;
    for (const auto& e : edges) deg[e.first]++;
    int mu = 0;
    for (const auto& e : edges) mu = std::max(mu, deg[e.first] + deg[e.second]);
    EXPECT(T.lap_mu == mu);
  }
  if (max_deg <= dm::LAP_TABLE_W) {
    EXPECT(T.adj_tab.size() == (size_t)nv * dm::LAP_TABLE_W);
    for (int v = 0; v < nv && T.adj_tab.size() == (size_t)nv * dm::LAP_TABLE_W; ++v) {
      const int d = T.adj_off[(size_t)v + 1] - T.adj_off[(size_t)v];
      for (int k = 0; k < dm::LAP_TABLE_W; ++k) {
        const int32_t x = T.adj_tab[(size_t)v * dm::LAP_TABLE_W + (size_t)k];
        EXPECT(k < d ? x == T.adj_nbr[(size_t)(T.adj_off[(size_t)v] + k)] : x == -1);
      }
    }
  } else {
    EXPECT(T.adj_tab.empty());
  }
}

static TopoTables build_ok(const std::vector<int32_t>& F, int nv) {
  TopoTables T;
  const Check c = dm::build_topology(F, nv, &T);
  EXPECT(c.st == DM_OK);
  if (c.st == DM_OK) check_tables(F, nv, T);
  return T;
}

static void test_meshes() {
  for (int sub = 0; sub <= 3; ++sub) {
    int nv = 0;
    const std::vector<int32_t> F = icosphere_faces(sub, &nv);
    const TopoTables T = build_ok(F, nv);
    EXPECT(T.closed);
    // strips exist and are long on a subdivided sphere
    EXPECT(T.n_strips >= 1 && (size_t)T.n_strips < F.size() / 3 + 1);
    // a reversed face breaks the orientation; removing faces opens the mesh
    std::vector<int32_t> G = F;
    std::swap(G[1], G[2]);
    EXPECT(!build_ok(G, nv).closed);
    std::vector<int32_t> H(F.begin(), F.end() - 6);
    EXPECT(!build_ok(H, nv).closed);
    // the same faces in another order: closed, same count
    std::vector<int32_t> P = F;
    std::mt19937 rng(7u + (unsigned)sub);
    for (size_t t = P.size() / 3; t > 1; --t) {
      const size_t u = rng() % t;
      for (int p = 0; p < 3; ++p) std::swap(P[3 * (t - 1) + p], P[3 * u + p]);
    }
    EXPECT(build_ok(P, nv).closed);
  }
  // box, with a fin (an edge shared by three faces) and with an isolated vertex
  std::vector<int32_t> B = box_faces();
  EXPECT(build_ok(B, 8).closed);
  std::vector<int32_t> fin = B;
  fin.insert(fin.end(), {0, 2, 8});
  EXPECT(!build_ok(fin, 9).closed);
  EXPECT(build_ok(B, 10).closed);   // vertices 8, 9 on no face
  // degenerate faces: a repeated vertex, and a face given twice
  std::vector<int32_t> D = B;
  D.insert(D.end(), {1, 1, 3});
  EXPECT(!build_ok(D, 8).closed);
  std::vector<int32_t> twice = B;
  twice.insert(twice.end(), B.begin(), B.begin() + 3);
  EXPECT(!build_ok(twice, 8).closed);
  // empty meshes
  EXPECT(!build_ok({}, 0).closed);
  EXPECT(!build_ok({}, 5).closed);
  // out-of-range indices are refused
  for (int32_t badv : {-1, 8, 1 << 30, std::numeric_limits<int32_t>::min()}) {
    std::vector<int32_t> X = B;
    X[7] = badv;
    TopoTables T;
    EXPECT(dm::build_topology(X, 8, &T).st == DM_ERR_MESH);
  }
  // random face soups: any valid index set builds consistent tables
  std::mt19937 rng(1234u);
  for (int rep = 0; rep < 200; ++rep) {
    const int nv = 1 + (int)(rng() % 40);
    const int nt = (int)(rng() % 120);
    std::vector<int32_t> S((size_t)nt * 3);
    for (auto& x : S) x = (int32_t)(rng() % (unsigned)nv);
    build_ok(S, nv);
  }
  // a high-degree vertex (a fan of 12 triangles around vertex 0): no neighbour table
  std::vector<int32_t> fan;
  for (int k = 0; k < 12; ++k) fan.insert(fan.end(), {0, 1 + k, 1 + (k + 1) % 12});
  EXPECT(build_ok(fan, 13).adj_tab.empty());
}

static void test_weights() {
  const std::vector<int32_t> B = box_faces();
  const int nt = (int)B.size() / 3;
  std::vector<float> w((size_t)nt, 1.0f);
  bool closed = false;
  EXPECT(dm::weights_close(B, w.data(), nt, &closed).st == DM_OK && closed);
  w[3] = 2.0f;
  EXPECT(dm::weights_close(B, w.data(), nt, &closed).st == DM_OK && !closed);
  w[3] = std::numeric_limits<float>::quiet_NaN();
  EXPECT(dm::weights_close(B, w.data(), nt, &closed).st == DM_ERR_ARG);
  w[3] = std::numeric_limits<float>::infinity();
  EXPECT(dm::weights_close(B, w.data(), nt, &closed).st == DM_ERR_ARG);
  // two cells sharing the wall x = 1 (cell A = [0,1]^3 of density 1, cell B =
  // [1,2]x[0,1]^2 of density 2): A's faces, the wall once as A's +x face with
  // the density jump across it (behind minus in front, 1 - 2), B's faces but
  // its own copy of the wall; the weights then cancel across every edge
  {
    auto gid = [](int c, bool b) {   // corner c = x + 2y + 4z of cell A or B
      const int x = c & 1, y = (c >> 1) & 1, z = (c >> 2) & 1;
      if (!b) return c;
      return x == 0 ? 1 + 2 * y + 4 * z : 8 + y + 2 * z;
    };
    std::vector<int32_t> C;
    std::vector<float> cw;
    for (int cell = 0; cell < 2; ++cell)
      for (int t = 0; t < nt; ++t) {
        const int32_t* f = &B[3 * (size_t)t];
        const bool xface0 = (f[0] & 1) == 0 && (f[1] & 1) == 0 && (f[2] & 1) == 0;
        const bool xface1 = (f[0] & 1) && (f[1] & 1) && (f[2] & 1);
        if (cell == 1 && xface0) continue;   // B's copy of the wall
        for (int p = 0; p < 3; ++p) C.push_back(gid(f[p], cell == 1));
        cw.push_back(cell == 0 ? (xface1 ? 1.0f - 2.0f : 1.0f) : 2.0f);
      }
    const int nc = (int)cw.size();
    EXPECT(nc == 22);
    EXPECT(dm::weights_close(C, cw.data(), nc, &closed).st == DM_OK && closed);
    cw[0] += 0.5f;
    EXPECT(dm::weights_close(C, cw.data(), nc, &closed).st == DM_OK && !closed);
    EXPECT(!build_ok(C, 12).closed);   // unweighted, the cluster is not a closed surface
  }
  EXPECT(dm::weights_close({}, nullptr, 0, &closed).st == DM_OK && !closed);
  std::mt19937 rng(99u);
  for (int rep = 0; rep < 100; ++rep) {
    const int nv = 1 + (int)(rng() % 20), n = (int)(rng() % 60);
    std::vector<int32_t> S((size_t)n * 3);
    for (auto& x : S) x = (int32_t)(rng() % (unsigned)nv);
    std::vector<float> ww((size_t)n);
    for (auto& x : ww) x = (float)((int)(rng() % 7) - 3);
    EXPECT(dm::weights_close(S, ww.data(), n, &closed).st == DM_OK);
  }
}

static dm_grid good_grid() {
  dm_grid g{};
  g.n[0] = 32;
  g.n[1] = 16;
  g.n[2] = 8;
  for (int j = 0; j < 3; ++j) {
    g.spacing[j] = 0.5f;
    g.origin[j] = -1.0f;
  }
  g.band_tau = 1e-3f;
  g.mode = DM_VOLUME;
  return g;
}

static void test_grid_and_psf() {
  const float nan = std::numeric_limits<float>::quiet_NaN(), inf = std::numeric_limits<float>::infinity();
  dm_grid g = good_grid();
  EXPECT(dm::validate_grid(&g).st == DM_OK);
  EXPECT(dm::validate_grid(nullptr).st == DM_ERR_ARG);
  for (int j = 0; j < 3; ++j) {
    for (int32_t n : {0, -1, std::numeric_limits<int32_t>::min()}) {
      dm_grid b = good_grid();
      b.n[j] = n;
      EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
    }
    for (float s : {0.0f, -1.0f, nan, inf, -inf}) {
      dm_grid b = good_grid();
      b.spacing[j] = s;
      EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
    }
    for (float o : {nan, inf, -inf}) {
      dm_grid b = good_grid();
      b.origin[j] = o;
      EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
    }
  }
  for (float t : {-1e-3f, nan, -inf}) {
    dm_grid b = good_grid();
    b.band_tau = t;
    EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
  }
  {
    dm_grid b = good_grid();
    b.band_tau = inf;   // an empty band is not an error
    EXPECT(dm::validate_grid(&b).st == DM_OK);
    b.mode = 7;
    EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
    b = good_grid();
    b.n[0] = b.n[1] = b.n[2] = 1 << 30;   // far beyond the position limit (no overflow)
    EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
    for (int j = 0; j < 3; ++j) {   // the per-axis limit, on grids of few positions
      b = good_grid();
      b.n[0] = b.n[1] = b.n[2] = 1;
      b.n[j] = DM_MAX_AXIS;
      EXPECT(dm::validate_grid(&b).st == DM_OK);
      b.n[j] = DM_MAX_AXIS + 1;
      EXPECT(dm::validate_grid(&b).st == DM_ERR_ARG);
    }
  }
  dm_psf p{};
  EXPECT(dm::validate_psf(nullptr).st == DM_ERR_ARG);
  const float good[6] = {1.0f, 1.5f, 6.25f, 0.2f, -0.1f, 0.3f};
  for (int j = 0; j < 6; ++j) p.sigma[j] = good[j];
  EXPECT(dm::validate_psf(&p).st == DM_OK);
  for (int j = 0; j < 6; ++j)
    for (float v : {nan, inf, -inf}) {
      dm_psf b = p;
      b.sigma[j] = v;
      EXPECT(dm::validate_psf(&b).st == DM_ERR_PSF);
    }
  const float notspd[][6] = {{0, 1, 1, 0, 0, 0}, {1, -1, 1, 0, 0, 0}, {1, 1, 0, 0, 0, 0}, {1, 1, 1, 1, 0, 0},
                             {1, 1, 1, 0, 1, 0},  {1, 1, 1, 0, 0, 1}, {1, 1, 1, 0.8f, 0.8f, -0.8f}};
  for (const auto& s : notspd) {
    dm_psf b;
    for (int j = 0; j < 6; ++j) b.sigma[j] = s[j];
    EXPECT(dm::validate_psf(&b).st == DM_ERR_PSF);
  }
  std::mt19937 rng(5u);
  std::uniform_real_distribution<float> U(-2.0f, 2.0f);
  for (int rep = 0; rep < 1000; ++rep) {
    dm_psf b;
    for (int j = 0; j < 6; ++j) b.sigma[j] = U(rng);
    const dm_status st = dm::validate_psf(&b).st;
    EXPECT(st == DM_OK || st == DM_ERR_PSF);
  }
}

// Sweep plans: every entry and triangle covered, no empty range, the bounds
// the kernels and partial buffers assume, and the shared launch's fused plan
// against the single call's (same entry chunks, never more triangle ranges, so
// never larger forward partials; tiles of at most max(single tile, 4M pairs);
// at least min(single-call tiles, half the tile floor) tiles).
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static void test_plans() {
  const int64_t nEs[] = {0, 1, 767, 768, 769, 1023, 1024, 1025, 45000, 140000, 549888, 1100000, 8585088};
  const int nts[] = {0, 1, 31, 32, 33, 500, 1000, 2880, 5120, 20480, 40500};
  for (int mode = 0; mode < 2; ++mode)
    for (int64_t nE : nEs)
      for (int nt : nts) {
        const int64_t n = std::max(nt, 1);
        const dm::SweepPlan f = dm::plan_fwd(nE, nt);
        EXPECT(f.n_chunks >= 1 && f.per_chunk >= 1);
        EXPECT((int64_t)f.n_chunks * f.per_chunk >= nt && (int64_t)(f.n_chunks - 1) * f.per_chunk < n);
        EXPECT(nt < 32 || f.per_chunk >= 32);
        const dm::SweepPlan v = dm::plan_vjp(nE, nt, mode);
        EXPECT(v.n_chunks >= 1 && v.n_chunks <= 256 && v.sub >= 1);
        EXPECT(v.per_chunk == v.sub * dm::vjp_chunk(mode));
        EXPECT((int64_t)v.n_chunks * v.per_chunk >= nE);
        EXPECT(v.tpb >= 1 && v.tpb <= dm::VJP_TPB_MAX);
        const dm::SweepPlan s1 = dm::plan_fused(nE, nt, mode);
        EXPECT(s1.per_chunk == dm::fused_chunk(mode) && s1.n_chunks == std::max<int64_t>(1, cdiv(nE, s1.per_chunk)));
        EXPECT(s1.tpb >= 1 && (nt < 32 || s1.tpb >= 32));
        const dm::SweepPlan r1 = dm::fused_fwd_plan(s1, nt);
        EXPECT(r1.per_chunk == s1.tpb && (int64_t)r1.n_chunks * r1.per_chunk >= nt);
        EXPECT((int64_t)(r1.n_chunks - 1) * r1.per_chunk < n);
        const dm::SweepPlan sb = dm::plan_fused_batch(nE, nt, mode);
        const dm::SweepPlan rb = dm::fused_fwd_plan(sb, nt);
        EXPECT(sb.n_chunks == s1.n_chunks && sb.per_chunk == s1.per_chunk);
        EXPECT(sb.tpb >= s1.tpb && rb.n_chunks <= r1.n_chunks);
        EXPECT((int64_t)rb.n_chunks * rb.per_chunk >= nt && (int64_t)(rb.n_chunks - 1) * rb.per_chunk < n);
        const int64_t want = cdiv(dm::FUSED_BATCH_TILE_PAIRS, dm::fused_chunk(mode));
        EXPECT(sb.tpb <= std::max<int64_t>(s1.tpb, std::min(n, want)));
        const int64_t tiles_s = (int64_t)s1.n_chunks * r1.n_chunks, tiles_b = (int64_t)sb.n_chunks * rb.n_chunks;
        EXPECT(tiles_b >= std::min(tiles_s, dm::FUSED_BATCH_MIN_TILES / 2));
        const dm::SweepPlan fb = dm::plan_fwd_batch(nE, nt);
        EXPECT(fb.per_chunk >= 1 && fb.n_chunks <= 8 && (nt == 0 || fb.n_chunks >= 1));   // no sweep runs for nt = 0
        EXPECT((int64_t)fb.n_chunks * fb.per_chunk >= nt && (nt < 640 || fb.per_chunk >= 640));
        const dm::SweepPlan vb = dm::plan_vjp_batch(nE, nt, mode);
        EXPECT(vb.n_chunks == v.n_chunks && vb.per_chunk == v.per_chunk);
        EXPECT(vb.tpb >= 1 && vb.tpb <= dm::VJP_TPB_MAX && vb.tpb <= n);
      }
  // a small cell of the serving pool (64^3 band, 2880 triangles) alone in the
  // shared launch: the single call's tiling, thousands of tiles, not dozens
  const dm::SweepPlan s1 = dm::plan_fused(45000, 2880, 0), sb = dm::plan_fused_batch(45000, 2880, 0);
  EXPECT(sb.tpb == s1.tpb && (int64_t)sb.n_chunks * dm::fused_fwd_plan(sb, 2880).n_chunks >= 2048);
  // the single cell's band (549,888 entries, 5120 triangles): larger tiles than
  // the single call's, still at least the tile floor
  const dm::SweepPlan c1 = dm::plan_fused(549888, 5120, 0), cb = dm::plan_fused_batch(549888, 5120, 0);
  EXPECT(cb.tpb > c1.tpb && (int64_t)cb.n_chunks * dm::fused_fwd_plan(cb, 5120).n_chunks >= dm::FUSED_BATCH_MIN_TILES);
}

int main() {
  test_meshes();
  test_weights();
  test_grid_and_psf();
  test_plans();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("topo harness: all checks passed\n");
  return 0;
}
