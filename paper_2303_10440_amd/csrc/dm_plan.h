// Launch planning of the mesh-transform sweeps: how a request's band entries
// and triangles are cut into workgroup tiles.  Plain integer arithmetic with
// no device code, shared by the library and its host-side tests.
#pragma once

#include <algorithm>
#include <cstdint>

namespace dm {

// Lane-per-entry gradient sweep: vjp_j(mode) band entries per lane (entry
// chunks of 4 waves x 64 lanes x vjp_j(mode) entries), chosen with the
// occupancy: 5 per lane at 5 waves per SIMD (volume), 6 at 4 waves (surface,
// whose ten accumulators per triangle need the larger register budget).
constexpr int VJP_J_MAX = 8;
constexpr int vjp_j(int mode) { return mode == 0 ? 5 : 6; }
constexpr int vjp_chunk(int mode) { return 256 * vjp_j(mode); }
// Fused forward and gradient sweep (given cotangent): one entry per lane fewer
// than the gradient sweep, for the forward sums each entry carries; blocks of
// one chunk of fused_chunk(mode) entries.
constexpr int fused_j(int mode) { return mode == 0 ? 4 : 4; }
constexpr int fused_chunk(int mode) { return 256 * fused_j(mode); }
// Forward sweep: FWD_J band entries per lane, FWD_CHUNK entries per block.
constexpr int FWD_J = 3;
constexpr int FWD_CHUNK = 256 * FWD_J;
static_assert(FWD_J <= 8 && VJP_J_MAX <= 8, "queued pairs store the entry step in 3 bits");
// Most triangles per gradient-sweep block.
constexpr int VJP_TPB_MAX = 256;

// Launch geometry of the two sweeps.
struct SweepPlan {
  int n_chunks = 1, per_chunk = 1;
  int sub = 1, tpb = 1;   // lane-per-entry gradient sweep: entry chunks per block, triangles per block
};

// Both sweeps hold about 1280 blocks of 4 waves resident at once (5 waves
// per SIMD); a grid of several times that keeps the last, partly filled round
// short.
constexpr int64_t FWD_TARGET_BLOCKS = 20480, VJP_TARGET_BLOCKS = 20480;

// Forward sweep (band entries on lanes): blocks of FWD_CHUNK entries times
// triangle chunks of at least 32 triangles, FWD_TARGET_BLOCKS blocks in all.
inline SweepPlan plan_fwd(int64_t nE, int nt) {
  SweepPlan sp;
  const int64_t eblocks = std::max<int64_t>(1, (nE + FWD_CHUNK - 1) / FWD_CHUNK);
  const int64_t want = (FWD_TARGET_BLOCKS + eblocks - 1) / eblocks;
  const int64_t most = std::max<int64_t>(1, nt / 32);
  sp.n_chunks = (int)std::max<int64_t>(1, std::min(want, most));
  sp.per_chunk = std::max(1, (nt + sp.n_chunks - 1) / sp.n_chunks);
  sp.n_chunks = std::max(1, (nt + sp.per_chunk - 1) / sp.per_chunk);
  return sp;
}

// Gradient sweep (lane per band entry): n_chunks blocks along the band of
// sub x vjp_chunk(mode) entries each (one chunk per block up to 256 chunks,
// which bounds the partials to 4 B x channels x triangles x 256), times
// triangle chunks of tpb so the grid has about VJP_TARGET_BLOCKS blocks.
// Each block rereads its entries' records once per chunk of triangles, so
// long triangle ranges (few entries per block) keep that traffic low.
inline SweepPlan plan_vjp(int64_t nE, int nt, int mode) {
  SweepPlan sp;
  const int64_t chunk = vjp_chunk(mode);
  const int64_t units = std::max<int64_t>(1, (nE + chunk - 1) / chunk);
  sp.sub = (int)((units + 255) / 256);
  sp.n_chunks = (int)((units + sp.sub - 1) / sp.sub);
  sp.per_chunk = (int)(sp.sub * chunk);
  const int64_t want = (VJP_TARGET_BLOCKS + sp.n_chunks - 1) / sp.n_chunks;
  const int64_t most = std::max<int64_t>(1, (nt + 7) / 8);
  const int64_t tchunks = std::max<int64_t>((nt + VJP_TPB_MAX - 1) / VJP_TPB_MAX, std::min(want, most));
  sp.tpb = (int)std::max<int64_t>(1, (nt + tchunks - 1) / tchunks);
  return sp;
}

// Fused sweep (forward and gradient in one pass): one entry chunk of
// fused_chunk(mode) entries per block times triangle ranges of tpb, about
// FUSED_TARGET_BLOCKS blocks in all (ranges of at least 32 triangles).  The
// forward partials take 8 B x entries per triangle range and the gradient
// partials 4 B x channels x triangles per entry chunk.  In the returned plan
// n_chunks/per_chunk/tpb describe the entry chunks (gradient partials); the
// triangle ranges are fused_fwd_plan's.
constexpr int64_t FUSED_TARGET_BLOCKS = 20480;

inline SweepPlan plan_fused(int64_t nE, int nt, int mode) {
  SweepPlan sp;
  const int64_t chunk = fused_chunk(mode);
  const int64_t units = std::max<int64_t>(1, (nE + chunk - 1) / chunk);
  sp.sub = 1;
  sp.n_chunks = (int)units;
  sp.per_chunk = (int)chunk;
  const int64_t want = (FUSED_TARGET_BLOCKS + units - 1) / units;
  const int64_t most = std::max<int64_t>(1, nt / 32);
  const int64_t tchunks = std::max<int64_t>(1, std::min(want, most));
  sp.tpb = (int)std::max<int64_t>(1, (nt + tchunks - 1) / tchunks);
  return sp;
}

// The fused plan of a request inside a batch's shared launch: the same entry
// chunks, triangle ranges of at least FUSED_BATCH_TILE_PAIRS / fused_chunk
// triangles (the whole mesh when it is smaller), so that many small requests
// do not turn into many small tiles; the shared queue fills the GPU.  But a
// request is cut into at least FUSED_BATCH_MIN_TILES tiles (four rounds of
// resident workgroups) where ranges of the single-call plan's size allow it:
// a small request that runs alone (a server at low load) still spreads over
// the GPU instead of a few dozen workgroups, and the shared queue's tail is
// shorter.  The plan depends on the request alone.
constexpr int64_t FUSED_BATCH_TILE_PAIRS = (int64_t)1 << 22;
constexpr int64_t FUSED_BATCH_MIN_TILES = 4096;

inline SweepPlan plan_fused_batch(int64_t nE, int nt, int mode) {
  SweepPlan sp = plan_fused(nE, nt, mode);
  const int64_t n = std::max(nt, 1);
  const int64_t want = (FUSED_BATCH_TILE_PAIRS + fused_chunk(mode) - 1) / fused_chunk(mode);
  const int64_t ranges = std::max<int64_t>(1, (FUSED_BATCH_MIN_TILES + sp.n_chunks - 1) / sp.n_chunks);
  const int64_t cap = (n + ranges - 1) / ranges;   // triangles per range for that many ranges
  sp.tpb = (int)std::max<int64_t>(sp.tpb, std::min(n, std::min(want, cap)));
  return sp;
}

// Triangle ranges of a fused plan as a forward plan (the forward partials).
inline SweepPlan fused_fwd_plan(const SweepPlan& v, int nt) {
  SweepPlan sp;
  sp.per_chunk = v.tpb;
  sp.n_chunks = std::max(1, (nt + v.tpb - 1) / v.tpb);
  return sp;
}

// Batch chunking depends on the request alone, so a request's result is the
// same whichever other requests share its batch.  A request that wants the
// image (or dL/dSigma) and the vertex gradient runs plan_fused_batch's tiles.
// Forward-only and gradient-only requests: at least 640 triangles per forward
// tile so small requests still give long sweeps, at most 8 forward chunks so
// the partials of large requests stay bounded (8 B x entries x 8); gradient
// items cover sub x vjp_chunk(mode) entries (at most 256 chunks, as in
// plan_vjp) and up to VJP_TPB_MAX triangles.
// The server runs a request of at least this many (entry, triangle) pairs with
// its own sweep launches (it fills the GPU alone), after the shared launch of
// the batch's smaller requests, so that those complete first; dm_batch_run
// puts every request in the shared launch.  The choice depends on the request
// alone, so its result is still the same in any batch.
constexpr double BATCH_DIRECT_PAIRS = 5e8;

inline SweepPlan plan_fwd_batch(int64_t nE, int nt) {
  SweepPlan sp;
  (void)nE;
  sp.per_chunk = std::max(1, std::min(nt, std::max(640, (nt + 7) / 8)));
  sp.n_chunks = (nt + sp.per_chunk - 1) / sp.per_chunk;
  return sp;
}

inline SweepPlan plan_vjp_batch(int64_t nE, int nt, int mode) {
  SweepPlan sp = plan_vjp(nE, nt, mode);
  int tpb = 32;   // about 2^20 pairs per gradient item
  while (tpb < VJP_TPB_MAX && (int64_t)2 * tpb * sp.per_chunk <= ((int64_t)1 << 20)) tpb *= 2;
  sp.tpb = std::max(1, std::min(nt, tpb));
  return sp;
}

}  // namespace dm
