// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dm_plan.h"   // sweep sizes (entries per lane and per block), launch planning
#include "dm_topo.h"   // strip flags, neighbour-table width

namespace dm {

// Per-call mesh quantities computed on the device by the mesh-prep kernels.
struct MeshInfo {
  float c[3];        // reference point for phases: vertex centroid
  float pad0;
  double cu[3];      // (c - origin) / L, revolutions per unit integer frequency
  double area;       // |Lambda| = sum_T A_T
  double volume;     // enclosed volume (signed cones from c)
};

// Grid constants passed by value to kernels.
struct GridC {
  int n0, n1, n2, n2h;     // voxel counts, n2h = n2/2 + 1
  double L[3];             // box lengths n_j * spacing_j
  double origin[3];
  float Linv[3];           // 1 / L_j (float)
  float two_pi_over_L[3];  // 2 pi / L_j (float)
  float inv_LV;            // 1 / (Lx Ly Lz)
};

// Band description on the device (see band.hip).
struct BandDev {
  int64_t n_entries;
  int64_t n_pos;           // n0 * n1 * n2h
  float4* kf;              // [n_entries] {kx, ky, kz, h_hat}
  float* wgt;              // [n_entries] alias weight (1 or 1/2)
  int32_t* pos;            // [n_entries] half-spectrum position
  int32_t* map;            // [n_pos] first entry | (count-1) << 30, or -1
  // Tabulated OTF per half-spectrum position [n_pos] (complex), or nullptr:
  // then the Gaussian value kf.w of each entry is the OTF.
  const float2* otf;
};

// Triangle record for the sweeps: 16 floats (one 64-byte scalar load), for
// the triangle (v1, v2, v3) in strip order (v3 is the vertex it adds).
//  [0..2] u3_hi, [3..5] u3_lo : (v3 - c)/L split into a 12-bit grid part and rest
//  [6..8] e2 = 2 pi (v2 - v1)/L,  [9..11] e3 = 2 pi (v3 - v1)/L  (k.e: relative phases in radians)
//  [12..14] VOLUME: n_T / L, n_T the outward (v2-v1)x(v3-v1);  SURFACE: [12] = 2 A_T
//  [15] 1 for the first triangle of a strip, else 0
constexpr int TRI_REC = 16;
constexpr float PHASE_GRID = 4096.0f;   // 2^12

// Band-entry record of the VJP sweeps: ERC float4 per entry,
//  {kx, ky, kz, Wr}, {Wi, xi_x, xi_y, xi_z}, {|W|, arg(W) / (2 pi), 0, 0}
constexpr int ERC = 3;

// Work item of the persistent batched sweeps: one tile of one request's
// forward sweep (kind 0: FWD_CHUNK band entries from x0, triangle chunk c) or
// gradient sweep (kind 1: entry chunk c of epc entries, triangles x0.. x0+vtpb).
// The fused sweep's tiles need no items (see launch_batch_sweep).
struct SweepItem {
  int kind, req, x0, c;
};

// Per-request pointers and chunking for the batched sweep.  Fused requests:
// tile0 is the request's first tile in its launch and ntr its triangle ranges
// of vtpb triangles per entry chunk of fused_chunk(mode) entries.
struct SweepReq {
  int mode, nE, nt, tpc, epc, vsub, vtpb, tile0;
  float tpx, tpy, tpz;   // 2 pi / L (SURFACE gradient)
  int ntr;
  const float4* kf;
  const float* rec;
  float2* fpart;       // [fwd chunks][nE]
  const float4* erec;  // [nE][ERC]
  float* vpart;        // [vjp chunks][NC][nt]
};

constexpr int SWEEP_THREADS = 256;

// ---- launchers (defined in dm_kernels.hip); all enqueue on `s` ----
// The persistent launches of a batch.  Groups 0-3 (2 kind + mode: forward
// volume, forward surface, gradient volume, gradient surface) run the sorted
// items, group g being items [group_end[g-1], group_end[g]).  Groups 4 and 5
// run the fused tiles of each density: fused_reqs[m] lists n_fused_reqs[m]
// requests, request r owning tiles [tile0_r, tile0_{r+1}) of the
// n_fused_tiles[m] (entry chunk major, ntr triangle ranges per chunk), handed
// out in increasing order.  counters[0..BATCH_GROUPS) are zeroed first.
constexpr int BATCH_GROUPS = 6;
hipError_t launch_batch_sweep(const SweepItem* items, const int* group_end, const SweepReq* reqs,
                              const SweepReq* const* fused_reqs, const int* n_fused_reqs, const int* n_fused_tiles,
                              int* counters, hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t launch_band_count(const GridC& g, const double* sigma6, double qmax, int32_t* cnt, int64_t n_slots,
                             hipStream_t s);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* block_tmp, int64_t* total,
                       hipStream_t s);
int64_t scan_tmp_elems(int64_t n);
// Band of a tabulated OTF: positions with Re^2 + Im^2 > tau2 (float64), all
// their aliases; entries get kf.w = 1.
hipError_t launch_band_count_otf(const GridC& g, const float2* otf, double tau2, int32_t* cnt, int64_t n_slots,
                                 hipStream_t s);
hipError_t launch_band_fill_otf(const GridC& g, const float2* otf, double tau2, const int32_t* cnt,
                                const int32_t* off, int64_t n_slots, BandDev b, hipStream_t s);
hipError_t launch_band_fill(const GridC& g, const double* sigma6, double qmax, const int32_t* cnt,
                            const int32_t* off, int64_t n_slots, BandDev b, hipStream_t s);

// tri_w: per-triangle density weights in strip order, or nullptr (all 1).
hipError_t launch_mesh_prep(int mode, const GridC& g, const float* verts, int nv, const int32_t* faces,
                            const int32_t* flags, const float* tri_w, int nt,
                            float* tri_rec, MeshInfo* info, double* block_tmp, int tmp_blocks, hipStream_t s);
int mesh_prep_blocks(int nt);

// Forward sweep with band entries on lanes: ceil(nE / FWD_CHUNK) x n_chunks
// blocks, triangle chunks of tris_per_chunk strip-ordered triangles; writes
// part[chunk][nE].
hipError_t launch_fwd_lanes(int mode, const float4* kf, int64_t nE, const float* tri_rec, int nt, int tris_per_chunk,
                            int n_chunks, float2* part, hipStream_t s);

hipError_t launch_fwd_finalize(int mode, const GridC& g, BandDev b, const float2* part, int n_chunks,
                               const MeshInfo* info, float2* spec_out, float2* xhalf, hipStream_t s);
hipError_t launch_spec_scatter(const GridC& g, BandDev b, const float2* spec, float2* xhalf, hipStream_t s);

hipError_t launch_adjoint(int mode, const GridC& g, BandDev b, const float2* ghat, const MeshInfo* info, float4* erec,
                          hipStream_t s);
hipError_t launch_dsig(const GridC& g, BandDev b, const float2* ghat, const float2* spec, double* dsig_part,
                       int dsig_blocks, hipStream_t s);
int adjoint_blocks(const GridC& g);
hipError_t launch_dsig_final(const double* dsig_part, int nblk, float* out6, hipStream_t s);

// Lane-per-entry gradient sweep: n_chunks blocks along the band, each covering
// chunks_per_block x vjp_chunk(mode) entries, times triangle chunks of tris_per_block
// (at most VJP_TPB_MAX); same partial layout [chunk][NC][nt].
hipError_t launch_vjp_lanes(int mode, const GridC& g, const float* tri_rec, int nt, int tris_per_block,
                            int chunks_per_block, int n_chunks, const float4* erec, int64_t nE, float* part,
                            hipStream_t s);
// Fused sweep: ceil(nE / fused_chunk(mode)) x ceil(nt / tris_per_block) blocks;
// gradient partials part[entry block][NC][nt] (as launch_vjp_lanes with one
// chunk per block) and forward partials fpart[triangle block][nE] (as
// launch_fwd_lanes).  The volume density needs the record's normal (as both
// sweeps do).
hipError_t launch_fused_lanes(int mode, const GridC& g, const float* tri_rec, int nt, int tris_per_block,
                              const float4* erec, int64_t nE, float* part, float2* fpart, hipStream_t s);
int vjp_reduce_groups(int n_chunks);
hipError_t launch_vjp_reduce(int mode, const float* part, int n_chunks, int nt, float* tmp, float* red,
                             hipStream_t s);
hipError_t launch_surface_scalar(const float* red, const float* tri_rec, int nt, const MeshInfo* info,
                                 double* out_R, hipStream_t s);
hipError_t launch_vertex_gather(int mode, const float* verts, int nv, const int32_t* faces, const int32_t* flags,
                                const float* tri_w, int nt,
                                const int32_t* csr_off, const int32_t* csr_ent, const float* red,
                                const double* R, float* dV, hipStream_t s);

hipError_t launch_points_prepare(const GridC& g, const int32_t* k, int64_t n, float4* kf, hipStream_t s);
hipError_t launch_points_finalize(int mode, const GridC& g, const float4* kf, int64_t n, const float2* part,
                                  int n_chunks, const MeshInfo* info, float2* out, hipStream_t s);

inline int nchannels(int mode) { return mode == 0 ? 3 : 10; }

// Smoothed gradient (I + lam L)^{-2} g of the shape step (dm_precond.hip).
// Meshes of at most 3072 vertices whose degrees fit the neighbour table
// (adj_tab [nv][LAP_TABLE_W], -1 padded; nullptr when a degree exceeds it):
// one workgroup runs Jacobi-preconditioned CG with the vectors resident on
// the chip.  Larger meshes: Chebyshev iteration, one launch per step, over
// the table or the CSR lists (adj_off, adj_nbr), mu >= the largest eigenvalue
// of L (the largest d_i + d_j over the edges).  ws holds
// laplace_smooth_workspace(nv) bytes; info (device, optional) receives
// {iterations, relative residual} of each of the two solves.
size_t laplace_smooth_workspace(int nv);
// Chebyshev steps that bound each column's relative residual by tol (at most max_iter; 0: the identity).
int chebyshev_steps(float lam, int mu, float tol, int max_iter);
hipError_t launch_laplace_smooth(int nv, const int32_t* adj_off, const int32_t* adj_nbr, const int32_t* adj_tab,
                                 int mu, float lam, const float* g, float* out, float* ws, int max_iter, float tol,
                                 float* info, hipStream_t s);

// Fixed scratch of the allocation-free entry point (dm_scratch.hip):
// scratch_init resolves its device address for `device`, which must be the
// current device (once per device; later calls return at once);
// scratch_ptr returns that address, or nullptr before scratch_init.
hipError_t scratch_init(int device);
void* scratch_ptr(int device);

}  // namespace dm
