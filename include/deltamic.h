/*
 * deltamic.h -- C ABI of the MI355X (gfx950) mesh-transform microscope renderer.
 *
 * The library renders a synthetic 3D fluorescence image from a closed
 * triangle mesh and a Gaussian point-spread function, and returns the
 * gradient of a scalar loss with respect to the vertex positions and the PSF
 * covariance.  It follows the image-formation model of the paper (Sec. 3):
 * the image is the convolution of a fluorophore density with the PSF
 * (Eq. 1), computed as a product in Fourier space; the density's transform is
 * the closed-form transform of the triangle mesh (Sec. 4, Eq. 5-12); the
 * PSF is the Gaussian of Eq. 2 with covariance Sigma; the mesh transform is
 * evaluated only on the narrow band of frequencies where the PSF transform
 * exceeds a threshold (Sec. 5.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Units     vertex positions, grid spacing, grid origin and the PSF
 *            covariance use one length unit (Sigma in length^2).
 *  Grid      n[0] x n[1] x n[2] voxels (x, y, z), voxel (i,j,k) centred at
 *            origin + (i, j, k) * spacing; images are float32 arrays laid out
 *            [n0][n1][n2], z fastest.  The image is periodic over the box
 *            L = n * spacing (it is produced by an inverse DFT).
 *  Spectrum  frequencies xi = 2 pi k / L with k the integer DFT frequencies
 *            (fftfreq order); the image is Re(ifftn(h_hat * u_hat * band)) /
 *            (spacing_x spacing_y spacing_z).  On even axes the Nyquist
 *            coefficient of that real part is the average of the two aliases
 *            +-N/2; the library evaluates both.
 *  Band      a frequency is evaluated iff xi^T Sigma xi < -2 ln(band_tau)
 *            (equivalently h_hat(xi) > band_tau), decided in float64 with the
 *            order ((((Sxx x x + Syy y y) + Szz z z) + 2 Sxy x y) + 2 Sxz x z)
 *            + 2 Syz y z and xi_j = (2 pi k_j) / (n_j spacing_j).
 *            band_tau = 0 evaluates the full spectrum; band_tau >= 1 gives an
 *            empty band and a zero image.
 *  Density   DM_VOLUME:  indicator function of the region the closed mesh
 *            encloses (the paper's suggested volumetric extension, Sec. 3.3
 *            and Sec. 7); its transform at xi = 0 is the enclosed volume.
 *            DM_SURFACE: fluorophores on the surface, normalised by the total
 *            area so that the image integrates to one (Eq. 3-5).
 *  Memory    pointers named *_dev are device (HBM) pointers on the handle's
 *            device, owned by the caller and never freed by the library.
 *            Host structs are read during the call only.
 *  Streams   `stream` is a hipStream_t (NULL = default stream).  Calls
 *            enqueue their work on it and return; outputs are valid once the
 *            stream has been synchronised.  A handle is not thread-safe:
 *            serialise calls on one handle.
 *  Errors    every entry point returns a dm_status and dm_last_error()
 *            describes a failure.  Input checks happen on the host before
 *            any work is enqueued, so a call refused for its arguments, its
 *            mesh, its PSF or the budget has written nothing.  A device or
 *            FFT failure after work was enqueued (DM_ERR_DEVICE, DM_ERR_FFT)
 *            may leave outputs partly written; the handle stays usable and
 *            its next call is still ordered after the enqueued work.
 *  Results   deterministic: the same inputs give bitwise identical outputs
 *            (all reductions run in a fixed order; no floating-point
 *            atomics).
 */
#ifndef DELTAMIC_H
#define DELTAMIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DM_OK = 0,
  DM_ERR_ARG = -1,      /* null pointer, bad size or option */
  DM_ERR_MESH = -2,     /* face index out of range, open mesh in VOLUME mode */
  DM_ERR_PSF = -3,      /* covariance not symmetric positive definite */
  DM_ERR_BUDGET = -4,   /* the call's device memory would exceed the handle budget */
  DM_ERR_DEVICE = -5,   /* a HIP runtime call failed */
  DM_ERR_FFT = -6,      /* a rocFFT call failed */
  DM_ERR_BUSY = -7,     /* serving queue full */
  DM_ERR_STATE = -8     /* object used in the wrong state (e.g. unknown ticket) */
} dm_status;

typedef enum {
  DM_VOLUME = 0,        /* indicator density of the enclosed region */
  DM_SURFACE = 1        /* area-normalised surface density (Eq. 3-5) */
} dm_mode;

typedef struct dm_handle dm_handle;
typedef struct dm_topology dm_topology;

/* Most voxels along one grid axis: the sweeps pass vertex phases of less
 * than (sum of |k_j|) / 8192 + 3/2 revolutions in magnitude (k the integer
 * frequency, at most n_j / 2 per axis) to the hardware sine and cosine, whose
 * domain is [-256, 256] revolutions. */
#define DM_MAX_AXIS (1 << 20)

typedef struct {
  int32_t n[3];         /* voxels along x, y, z (each in [1, DM_MAX_AXIS]) */
  float spacing[3];     /* voxel size along x, y, z (> 0) */
  float origin[3];      /* position of voxel (0,0,0) */
  float band_tau;       /* band threshold on the PSF transform, in [0, inf) */
  int32_t mode;         /* dm_mode */
} dm_grid;

typedef struct {
  float sigma[6];       /* covariance xx, yy, zz, xy, xz, yz (length^2) */
} dm_psf;

typedef struct {
  const float* verts_dev;     /* [n_verts][3] positions */
  int32_t n_verts;
  const dm_topology* topo;    /* faces, validated at dm_topology_create */
} dm_mesh;

/* ---------------------------------------------------------------- handle */

/* Create a handle bound to HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the handle's workspaces and caches may hold (0 = no cap).
 * Returns DM_ERR_DEVICE if the device is absent or not gfx950. */
dm_status dm_create(dm_handle** out, int device, size_t hbm_budget_bytes);

/* Free the handle, its caches, FFT plans and workspaces.  Synchronises the
 * device first.  NULL is accepted. */
dm_status dm_destroy(dm_handle* h);

/* Bytes of device memory the handle currently holds. */
dm_status dm_memory_in_use(const dm_handle* h, size_t* bytes);

/* ------------------------------------------------------------- topology */

/* Validate the faces of a triangle mesh and build its vertex-incidence
 * table (the one-ring of each vertex, the triangles "v star" of Eq. 6).
 * faces: [n_faces][3] int32 vertex indices, counter-clockwise seen from
 * outside; a host pointer if faces_on_device == 0, else a device pointer.
 * Fails with DM_ERR_MESH if an index is outside [0, n_verts).  Records
 * whether the mesh is closed and consistently oriented (every directed edge
 * matched by its reverse exactly once), which DM_VOLUME requires.  The
 * topology keeps its own device copy of the faces.  Synchronous. */
dm_status dm_topology_create(dm_handle* h, const int32_t* faces, int32_t n_faces, int32_t n_verts,
                             int faces_on_device, dm_topology** out);
dm_status dm_topology_destroy(dm_topology* t);
/* closed = 1 if closed and consistently oriented. */
dm_status dm_topology_info(const dm_topology* t, int32_t* n_faces, int32_t* n_verts, int32_t* closed);

/* Density weights of the faces (paper Sec. 3.3: several surfaces or
 * materials rendered as a weighted sum of densities; cell-cell interfaces
 * modelled as double membranes).  weights: host [n_faces] float32 in the
 * order of the faces given to dm_topology_create; NULL removes them (every
 * face weighs 1).  Each face's term of the mesh transform is multiplied by its
 * weight:
 *   DM_SURFACE: u = sum_T w_T 2 A_T f_T / sum_T w_T A_T (w_T = 2 for a wall
 *     shared by two cells of a non-manifold cluster mesh, 1 elsewhere);
 *   DM_VOLUME: w_T is the density jump across face T (density behind minus
 *     density in front of its counter-clockwise normal), so that the weighted
 *     divergence sum is the transform of a piecewise-constant density.  Such
 *     weights cancel across every edge (sum of the weights of the faces on
 *     the edge, signed by the direction each face runs along it); the
 *     topology is then reported closed and accepted by DM_VOLUME, otherwise
 *     DM_VOLUME renders fail with DM_ERR_MESH.
 * The vertex gradients and the PSF gradient follow.  Synchronises the device
 * (the weights are copied to it).  Errors: DM_ERR_ARG for a NULL topology or
 * a weight that is not finite. */
dm_status dm_topology_set_weights(dm_topology* t, const float* weights);

/* Smoothed update direction of the shape step (paper Sec. 5.2): the vertex
 * gradient filtered twice by the inverse of I + lambda L,
 *     out = (I + lambda L)^{-2} grad,
 * with L = D - A the combinatorial Laplacian of the mesh graph (D the vertex
 * degrees, A the adjacency of the mesh edges; a vertex on no edge has a row
 * of the identity).  The paper uses lambda = 50.
 * grad, out: device [n_verts][3] float32 (row-major, the layout of
 * dm_render_vjp's dL_dverts); out may be the same array as grad.  Each solve
 * runs conjugate gradients (Jacobi preconditioner, float64 dot products) on
 * the three columns together until every column's residual is at most tol
 * times its right-hand side, or for max_iter iterations.  info (device, 4
 * floats, optional) receives {iterations, relative residual} of the first and
 * of the second solve; reaching max_iter is not an error, the residuals tell.
 * The topology owns the workspace (13 n_verts floats, allocated on the first
 * call and counted against the budget), so calls with one topology must be
 * ordered on one stream.  Asynchronous on stream.  Errors: DM_ERR_ARG for
 * NULL pointers, a topology of another handle, lambda negative or not
 * finite, max_iter < 1 or tol <= 0; DM_ERR_BUDGET for the workspace. */
dm_status dm_laplace_smooth(dm_handle* h, dm_topology* topo, float lambda, const float* grad, float* out,
                            int32_t max_iter, float tol, float* info, void* stream);

/* The triangle order a topology uses internally, computed on the host (no
 * device needed): greedy triangle strips, in which every triangle after the
 * first of a strip shares the edge formed by the previous triangle's last two
 * vertices and so adds one vertex.  The mesh transform is a sum over
 * triangles (Eq. 5, and the volume form of the indicator), so the order only
 * changes rounding; the sweeps use it to share vertex phase factors.
 * faces: [n_faces][3] host array (indices are not checked here).
 * faces_out: [n_faces][3] host array, the faces in strip order, each written
 * as (s_i, s_i+1, s_i+2).  flags_out: [n_faces] host array, bit 0 = first
 * triangle of a strip, bit 1 = the written vertex order is an odd
 * permutation of the input face (opposite orientation).  n_strips may be NULL.
 * DM_ERR_ARG for a negative count or NULL arrays with n_faces > 0. */
dm_status dm_topology_strips(const int32_t* faces, int32_t n_faces, int32_t* faces_out, int32_t* flags_out,
                             int32_t* n_strips);

/* ------------------------------------------------------------------ band */

/* Number of frequency entries evaluated for (grid, psf): the in-band
 * positions of the half spectrum [n0][n1][n2/2+1], counting both aliases of
 * Nyquist positions.  Builds and caches the band on the device if needed
 * (synchronises `stream` on a cache miss). */
dm_status dm_band_size(dm_handle* h, const dm_grid* g, const dm_psf* psf, int64_t* n_entries, void* stream);

/* Copy the band to host memory, in the library's evaluation order:
 * k_out [n][3] integer frequencies, pos_out [n] linear half-spectrum
 * position (i0*n1 + i1)*(n2/2+1) + i2, weight_out [n] the alias weight
 * (1/2 for entries at Nyquist positions, else 1).  Any output may be NULL.
 * Synchronous. */
dm_status dm_band_export(dm_handle* h, const dm_grid* g, const dm_psf* psf, int32_t* k_out,
                         int64_t* pos_out, float* weight_out, void* stream);

/* ---------------------------------------------------------------- render */

/* Forward render (Sec. 3-4): image_dev [n0][n1][n2] float32 receives the
 * image.  If spectrum_dev is not NULL it receives the mesh transform u_hat
 * at every band entry (complex64 as float pairs, [n_entries][2], band order),
 * which dm_render_vjp can reuse.  DM_VOLUME requires a closed topology.
 * Either output may be NULL (both NULL is an argument error). */
dm_status dm_render(dm_handle* h, const dm_mesh* mesh, const dm_psf* psf, const dm_grid* g,
                    float* image_dev, float* spectrum_dev, void* stream);

/* Gradient of a scalar loss L(image) (the paper's backward pass, Eq. 6-10,
 * and the PSF gradient of Sec. 5.2) given dL_dimage_dev [n0][n1][n2]:
 *   dL_dverts_dev [n_verts][3]  (may be NULL)
 *   dL_dsigma_dev [6] with respect to (xx, yy, zz, xy, xz, yz); an
 *                 off-diagonal entry stands for both symmetric positions
 *                 of Sigma (may be NULL)
 *   image_dev     optional: the forward image, computed in the same call
 *                 (with dL_dverts_dev, by the fused sweep that evaluates the
 *                 forward and gradient sums together: dm_render's image up to
 *                 the order of float32 additions)
 * The band is held fixed (it depends on Sigma only through the threshold).
 * spectrum_in_dev, if not NULL, is the spectrum dm_render returned for the
 * same mesh, psf and grid, and saves the forward sweep when image_dev is
 * NULL.  Without it the forward sweep runs when image_dev or dL_dsigma_dev
 * is requested. */
dm_status dm_render_vjp(dm_handle* h, const dm_mesh* mesh, const dm_psf* psf, const dm_grid* g,
                        const float* dL_dimage_dev, float* dL_dverts_dev, float* dL_dsigma_dev,
                        float* image_dev, const float* spectrum_in_dev, void* stream);

/* Mesh transform at arbitrary integer frequencies: out_dev [n][2] receives
 * u_hat(2 pi k / L) for k_dev [n][3] (int32, device), with the grid's
 * origin as phase origin and the grid's mode (DM_SURFACE normalised by the
 * area).  No band, no PSF. */
dm_status dm_mesh_transform(dm_handle* h, const dm_mesh* mesh, const dm_grid* g, const int32_t* k_dev,
                            int64_t n, float* out_dev, void* stream);

/* Size of the fixed device scratch of dm_mesh_transform_noalloc, per GPU. */
#define DM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* dm_mesh_transform without any allocation, for callers that cannot allocate
 * device memory: work enqueued under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, same result up to the
 * order of float32 additions (bitwise the same whenever dm_mesh_transform's
 * triangle chunking fits the scratch).  The call allocates nothing: no
 * hipMalloc or hipFree, no library routine that allocates, no growth of the
 * handle's workspace; its intermediates (triangle records, mesh totals, the
 * frequency table and the per-chunk partial sums) live in a fixed array of
 * DM_NOALLOC_SCRATCH_BYTES bytes in the library's code object, one per GPU,
 * whose address dm_create resolves for its device.  With the triangles in c
 * chunks it needs 64 n_faces + 16 n + 8 n c bytes plus at most 20 KiB; when
 * dm_mesh_transform's chunking does not fit, fewer chunks are used (down to
 * one), and a request that does not fit with one chunk returns DM_ERR_BUDGET
 * before anything is enqueued.  Every call on a
 * GPU shares that GPU's scratch and leaves its contents behind (nothing in it
 * needs to start at zero): calls on one handle are ordered, but calls that
 * overlap on one GPU through different handles, or from several threads,
 * race on the scratch and give wrong results.  Kernel timing
 * (dm_timing_enable) does not cover this call. */
dm_status dm_mesh_transform_noalloc(dm_handle* h, const dm_mesh* mesh, const dm_grid* g, const int32_t* k_dev,
                                    int64_t n, float* out_dev, void* stream);

/* ----------------------------------------------------------------- batch */

/* One request of a batch: the forward render and/or gradient of one mesh on
 * its own grid with its own PSF (same meaning as dm_render_vjp's arguments).
 * dL_dimage_dev may be NULL for a forward-only request; any output may be
 * NULL, but each request must ask for at least one.  With otf_dev set, the
 * PSF is that tabulated OTF (as in dm_render_otf, band from grid.band_tau)
 * and psf is ignored; such a request has no PSF gradient (dL_dsigma_dev
 * must be NULL: DM_ERR_ARG). */
typedef struct {
  dm_mesh mesh;
  dm_psf psf;
  dm_grid grid;
  const float* dL_dimage_dev;   /* [n0][n1][n2] or NULL */
  float* image_dev;             /* [n0][n1][n2] or NULL */
  float* dL_dverts_dev;         /* [n_verts][3] or NULL (needs dL_dimage_dev) */
  float* dL_dsigma_dev;         /* [6] or NULL (needs dL_dimage_dev) */
  const void* otf_dev;          /* complex64 [n0][n1][n2/2+1] (dm_render_otf's table) or NULL */
} dm_request;

/* Rendering with a tabulated PSF (paper Sec. 3.2 and Sec. 7: measured or
 * physics-based PSFs beyond the Gaussian).  otf: device complex64
 * [n0][n1][n2/2+1], the PSF's transform at the half-spectrum DFT frequencies
 * (the layout of a real-to-complex FFT of the PSF; it must be Hermitian,
 * i.e. come from a real PSF, and is normalised like the Gaussian's, value 1 at
 * xi = 0 for a unit-mass PSF).  The band is the set of positions whose value
 * has |OTF|^2 > band_tau^2 (decided in float64); positions on the Nyquist
 * planes of even axes use the same value for both of their aliases.  Then
 * the image is I = Re(ifftn(OTF u 1_band)) / (Dx Dy Dz) with u the mesh
 * transform of the grid's density mode, as in dm_render.  The band is rebuilt
 * on every call (the table may change), which synchronises the stream once.
 * dm_render_otf_vjp returns dL/dverts (and optionally the image) for a given
 * dL/dimage, the band held fixed; there is no PSF gradient.  Batches and the
 * server take tabulated OTFs per request (dm_request.otf_dev,
 * dm_serve_request.otf_dev).  Errors as dm_render. */
dm_status dm_render_otf(dm_handle* h, const dm_mesh* mesh, const void* otf, const dm_grid* g, float* image_out,
                        void* stream);
dm_status dm_render_otf_vjp(dm_handle* h, const dm_mesh* mesh, const void* otf, const dm_grid* g,
                            const float* dL_dimage, float* dL_dverts, float* image_out, void* stream);

/* Runs n independent requests of uneven sizes and grids as one batch: the
 * mesh-transform sweeps of all of them (forward, Eq. 5/7-8, and gradient,
 * Eq. 6/9-10) execute in persistent launches (one per kind of sweep and
 * density present) whose workgroups draw work tiles of every request from a
 * shared queue, longest first; the small per-request steps (band, mesh prep,
 * FFTs, adjoint weights, reductions) run around them on the same stream.  A
 * request with dL_dimage and both an image (or dL_dsigma) and dL_dverts runs
 * dm_render_vjp's fused sweep in tiles of at least 4M (entry, triangle)
 * pairs, but in no fewer than 4096 tiles where triangle ranges of the single
 * call's size allow it (so a small request alone still spreads over the GPU);
 * forward-only and gradient-only requests have tiles of their own.
 * Results equal the single calls' up to float32 summation order.  Each
 * request's tiles and summation order depend on that request alone, so its
 * results are bitwise the same whatever else is in the batch.  A request with
 * a tabulated OTF counts its band while the batch is planned (one stream
 * synchronisation) and builds it in its own workspace.  All validation
 * happens before anything is enqueued; on error no output is written. */
dm_status dm_batch_run(dm_handle* h, int32_t n, const dm_request* reqs, void* stream);

/* --------------------------------------------------------------- serving */

/* A continuous-batching server for render + gradient requests on many
 * independent meshes.  A worker thread owns its own handle.  Meshes are made
 * resident once (dm_server_mesh_add); requests name a resident mesh and carry
 * their own PSF, grid and device buffers.  Whenever one of max_inflight stream
 * slots is free, the worker admits queued requests in arrival order, as many
 * as max_batch and the HBM budget allow (a request's footprint is its
 * workspace: band-sized partials, spectra, FFT buffers), and launches them
 * as one batch (the dm_batch_run machinery, workspace from the stream-ordered
 * allocator); requests that arrive meanwhile join the next batch, which runs
 * while the earlier ones are still on the GPU.  A request of at least 5e8
 * (band entry, triangle) pairs runs its own sweep launches after the batch's
 * shared launch; unless max_batch requests are waiting, it starts only when
 * nothing else is in flight and nothing starts beside it.  Results are bitwise
 * independent of which requests shared a batch.  Thread-safe: any thread may
 * submit and poll. */
typedef struct dm_server dm_server;

typedef struct {
  int32_t max_batch;          /* most requests launched together (>= 1) */
  int32_t max_inflight;       /* batches on the GPU at once, one stream each (1..8) */
  int32_t queue_capacity;     /* queued requests beyond this: DM_ERR_BUSY (>= 1) */
  size_t hbm_budget_bytes;    /* cap on the summed footprint of in-flight batches (0 = none) */
} dm_server_config;

typedef struct {
  int32_t mesh_id;            /* from dm_server_mesh_add */
  dm_psf psf;
  dm_grid grid;
  const float* dL_dimage_dev; /* [n0][n1][n2], or NULL for a forward-only request */
  float* image_dev;           /* outputs as in dm_request; device buffers owned by */
  float* dL_dverts_dev;       /* the caller and kept valid until dm_poll reports  */
  float* dL_dsigma_dev;       /* the request finished                            */
  const void* otf_dev;        /* tabulated OTF as in dm_request (psf ignored), or */
                              /* NULL; kept valid and unchanged until finished   */
} dm_serve_request;

typedef struct {
  dm_status status;           /* DM_OK, or why the request failed (DM_ERR_BUDGET: */
                              /* its footprint alone exceeds the budget)          */
  int32_t batch_size;         /* requests in the batch that carried it */
  double queue_ms;            /* submission to launch */
  double total_ms;            /* submission to completion seen by the server */
} dm_serve_result;

typedef struct {
  int64_t submitted, completed, rejected, batches;
  double mean_batch;
  size_t peak_inflight_bytes;
} dm_server_stats;

dm_status dm_server_create(int device, const dm_server_config* cfg, dm_server** out);
/* Finishes every queued and in-flight request, then frees everything. */
dm_status dm_server_destroy(dm_server* s);
/* Uploads a mesh (host arrays) and validates its faces; DM_ERR_MESH as for
 * dm_topology_create. */
dm_status dm_server_mesh_add(dm_server* s, const float* verts_host, int32_t n_verts, const int32_t* faces_host,
                             int32_t n_faces, int32_t* mesh_id);
/* DM_ERR_STATE while requests on the mesh are pending. */
dm_status dm_server_mesh_remove(dm_server* s, int32_t mesh_id);
/* Validates and queues a request; DM_ERR_BUSY if the queue is full. */
dm_status dm_submit(dm_server* s, const dm_serve_request* r, uint64_t* ticket);
/* DM_ERR_BUSY (non-blocking) while the request is not finished; once it has
 * finished, fills `out` and forgets the ticket (DM_ERR_STATE afterwards). */
dm_status dm_poll(dm_server* s, uint64_t ticket, int blocking, dm_serve_result* out);
dm_status dm_server_stats_read(dm_server* s, dm_server_stats* out);

/* ------------------------------------------------------------ diagnostics */

/* Kernel timing: while enabled, the handle records HIP events on the call's
 * stream around every launch of the mesh-transform sweeps (the forward sweep
 * of Eq. 5/7-8, the gradient sweep of Eq. 6/9-10, the fused sweep that
 * evaluates both in one pass when dL/dimage is given and the forward result
 * is wanted too, and the batched sweep of dm_batch_run).  dm_timing_read
 * waits for those events and returns, per sweep kind, the number of
 * launches, the summed duration in milliseconds and the summed
 * frequency-triangle pairs they evaluated (a fused pair counts once);
 * reset != 0 clears the counters.  Any output may be NULL. */
typedef struct {
  int64_t launches;
  double ms;
  double pairs;
} dm_kernel_time;

dm_status dm_timing_enable(dm_handle* h, int enable);
dm_status dm_timing_read(dm_handle* h, dm_kernel_time* fwd_sweep, dm_kernel_time* vjp_sweep,
                         dm_kernel_time* batch_sweep, dm_kernel_time* fused_sweep, int reset);

/* Thread-local description of the last error on this thread ("" if none). */
const char* dm_last_error(void);

/* Library version string. */
const char* dm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DELTAMIC_H */
