// Host side of the C ABI in include/deltamic.h: validation, handle state
// (workspace, band cache, FFT plans), and the launch sequences of the
// forward render and its vector-Jacobian product.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/deltamic.h"
#include "dm_internal.h"

using namespace dm;

namespace {

thread_local std::string g_err;

dm_status fail(dm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(DM_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define FFT_TRY(expr)                                                          \
  do {                                                                         \
    rocfft_status s_ = (expr);                                                 \
    if (s_ != rocfft_status_success) return fail(DM_ERR_FFT, "%s: rocfft status %d", #expr, (int)s_); \
  } while (0)

#define DM_TRY(expr)              \
  do {                            \
    dm_status s_ = (expr);        \
    if (s_ != DM_OK) return s_;   \
  } while (0)

std::once_flag g_fft_once;
rocfft_status g_fft_setup = rocfft_status_success;

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

struct BandKey {
  int n[3];
  uint32_t spacing[3];
  uint32_t sigma[6];
  uint32_t tau;
  bool operator<(const BandKey& o) const { return memcmp(this, &o, sizeof(BandKey)) < 0; }
  bool operator==(const BandKey& o) const { return memcmp(this, &o, sizeof(BandKey)) == 0; }
};

struct BandEntry {
  BandDev dev{};
  void* mem = nullptr;
  size_t bytes = 0;
};

struct FftPlans {
  rocfft_plan c2r = nullptr, r2c = nullptr;
  size_t work_c2r = 0, work_r2c = 0;
};

// Event pairs recorded around sweep launches while timing is enabled.
struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;   // 0 forward sweep, 1 gradient sweep
  double pairs = 0.0;
};

}  // namespace

struct dm_handle {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::map<BandKey, BandEntry> bands;
  std::list<BandKey> band_lru;   // front = most recent
  std::map<std::tuple<int, int, int>, FftPlans> ffts;
  rocfft_execution_info exec_info = nullptr;
  hipEvent_t last_ev = nullptr;
  bool have_last = false;
  int topo_count = 0;
  size_t topo_bytes = 0;
  bool timing = false;
  std::vector<TimedLaunch> pending;   // recorded, not yet read
  std::vector<hipEvent_t> event_pool;
  dm_kernel_time acc[2] = {{0, 0.0, 0.0}, {0, 0.0, 0.0}};
};

struct dm_topology {
  dm_handle* h = nullptr;
  int nt = 0, nv = 0, closed = 0;
  int32_t* faces = nullptr;     // device [nt][3]
  int32_t* csr_off = nullptr;   // device [nv+1]
  int32_t* csr_ent = nullptr;   // device [3 nt] = 3 t + p
  size_t bytes = 0;
};

namespace {

dm_status dev_alloc(dm_handle* h, void** p, size_t bytes, bool count = true) {
  if (count && h->budget && h->in_use + bytes > h->budget)
    return fail(DM_ERR_BUDGET, "allocation of %zu bytes exceeds the budget (%zu of %zu in use)", bytes, h->in_use,
                h->budget);
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(DM_ERR_DEVICE, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  if (count) h->in_use += bytes;
  return DM_OK;
}

void dev_free(dm_handle* h, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  h->in_use -= std::min(h->in_use, bytes);
}

void evict_one_band(dm_handle* h) {
  if (h->band_lru.empty()) return;
  BandKey k = h->band_lru.back();
  h->band_lru.pop_back();
  auto it = h->bands.find(k);
  if (it != h->bands.end()) {
    (void)hipDeviceSynchronize();
    dev_free(h, it->second.mem, it->second.bytes);
    h->bands.erase(it);
  }
}

// Workspace: one growable device buffer carved per call.
dm_status ensure_ws(dm_handle* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return DM_OK;
  while (h->budget && h->in_use - h->ws_bytes + bytes > h->budget && !h->band_lru.empty()) evict_one_band(h);
  if (h->ws) {
    HIP_TRY(hipDeviceSynchronize());
    dev_free(h, h->ws, h->ws_bytes);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (h->budget && h->in_use + want > h->budget) want = bytes;
  DM_TRY(dev_alloc(h, &h->ws, want));
  h->ws_bytes = want;
  return DM_OK;
}

struct Carver {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    size_t o = off;
    off += align_up(count * sizeof(T));
    return o;
  }
};

template <typename T>
T* at(dm_handle* h, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(h->ws) + off);
}

dm_status check_grid(const dm_grid* g) {
  if (!g) return fail(DM_ERR_ARG, "grid is NULL");
  for (int j = 0; j < 3; ++j) {
    if (g->n[j] < 1) return fail(DM_ERR_ARG, "grid n[%d] = %d must be >= 1", j, g->n[j]);
    if (!(g->spacing[j] > 0.0f) || !std::isfinite(g->spacing[j]))
      return fail(DM_ERR_ARG, "grid spacing[%d] must be finite and > 0", j);
    if (!std::isfinite(g->origin[j])) return fail(DM_ERR_ARG, "grid origin[%d] must be finite", j);
  }
  const int64_t npos = (int64_t)g->n[0] * g->n[1] * (g->n[2] / 2 + 1);
  if (npos > (int64_t)1 << 29) return fail(DM_ERR_ARG, "grid too large (%lld half-spectrum positions)", (long long)npos);
  if (!(g->band_tau >= 0.0f) || std::isnan(g->band_tau)) return fail(DM_ERR_ARG, "band_tau must be >= 0");
  if (g->mode != DM_VOLUME && g->mode != DM_SURFACE) return fail(DM_ERR_ARG, "unknown mode %d", g->mode);
  return DM_OK;
}

dm_status check_psf(const dm_psf* p) {
  if (!p) return fail(DM_ERR_ARG, "psf is NULL");
  for (int j = 0; j < 6; ++j)
    if (!std::isfinite(p->sigma[j])) return fail(DM_ERR_PSF, "sigma[%d] is not finite", j);
  // Cholesky of [[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]] in double.
  const double a = p->sigma[0], b = p->sigma[3], c = p->sigma[4], d = p->sigma[1], e = p->sigma[5], f = p->sigma[2];
  if (!(a > 0)) return fail(DM_ERR_PSF, "covariance not positive definite (xx <= 0)");
  const double l21 = b / std::sqrt(a), l31 = c / std::sqrt(a);
  const double d2 = d - l21 * l21;
  if (!(d2 > 0)) return fail(DM_ERR_PSF, "covariance not positive definite");
  const double l32 = (e - l31 * l21) / std::sqrt(d2);
  const double d3 = f - l31 * l31 - l32 * l32;
  if (!(d3 > 0)) return fail(DM_ERR_PSF, "covariance not positive definite");
  return DM_OK;
}

GridC make_gridc(const dm_grid* g) {
  GridC c{};
  c.n0 = g->n[0];
  c.n1 = g->n[1];
  c.n2 = g->n[2];
  c.n2h = g->n[2] / 2 + 1;
  double LV = 1.0;
  for (int j = 0; j < 3; ++j) {
    c.L[j] = (double)g->n[j] * (double)g->spacing[j];
    c.origin[j] = (double)g->origin[j];
    c.Linv[j] = (float)(1.0 / c.L[j]);
    c.two_pi_over_L[j] = (float)(6.283185307179586476925286766559 / c.L[j]);
    LV *= c.L[j];
  }
  c.inv_LV = (float)(1.0 / LV);
  return c;
}

BandKey make_key(const dm_grid* g, const dm_psf* p) {
  BandKey k;
  memset(&k, 0, sizeof(k));
  for (int j = 0; j < 3; ++j) {
    k.n[j] = g->n[j];
    memcpy(&k.spacing[j], &g->spacing[j], 4);
  }
  for (int j = 0; j < 6; ++j) memcpy(&k.sigma[j], &p->sigma[j], 4);
  memcpy(&k.tau, &g->band_tau, 4);
  return k;
}

double band_qmax(float tau) {
  if (!(tau > 0.0f)) return INFINITY;
  return -2.0 * std::log((double)tau);
}

// Builds (or fetches) the band for (grid, psf).  Synchronises `s` on a miss.
dm_status get_band(dm_handle* h, const dm_grid* g, const dm_psf* p, hipStream_t s, BandDev* out) {
  const BandKey key = make_key(g, p);
  auto it = h->bands.find(key);
  if (it != h->bands.end()) {
    h->band_lru.remove(key);
    h->band_lru.push_front(key);
    *out = it->second.dev;
    return DM_OK;
  }
  const GridC gc = make_gridc(g);
  const int64_t n_pos = (int64_t)gc.n0 * gc.n1 * gc.n2h;
  const int64_t n_slots = (int64_t)((gc.n0 + 3) / 4) * ((gc.n1 + 3) / 4) * ((gc.n2h + 3) / 4) * 64;
  const int64_t ntmp = scan_tmp_elems(n_slots);
  // temporary build buffers in the workspace
  Carver cv;
  const size_t o_cnt = cv.take<int32_t>(n_slots), o_off = cv.take<int32_t>(n_slots), o_tmp = cv.take<int32_t>(ntmp),
               o_tot = cv.take<int64_t>(1);
  DM_TRY(ensure_ws(h, cv.off));
  int32_t* cnt = at<int32_t>(h, o_cnt);
  int32_t* off = at<int32_t>(h, o_off);
  double sig[6];
  for (int j = 0; j < 6; ++j) sig[j] = (double)p->sigma[j];
  const double qmax = band_qmax(g->band_tau);
  HIP_TRY(launch_band_count(gc, sig, qmax, cnt, n_slots, s));
  HIP_TRY(launch_scan(cnt, off, n_slots, at<int32_t>(h, o_tmp), at<int64_t>(h, o_tot), s));
  int64_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, at<int64_t>(h, o_tot), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // allocate the band (evicting older bands if the budget requires)
  Carver bc;
  const int64_t ne = std::max<int64_t>(total, 1);
  const size_t o_kf = bc.take<float4>(ne), o_w = bc.take<float>(ne), o_pos = bc.take<int32_t>(ne),
               o_map = bc.take<int32_t>(n_pos);
  while (h->budget && h->in_use + bc.off > h->budget && !h->band_lru.empty()) evict_one_band(h);
  BandEntry be;
  DM_TRY(dev_alloc(h, &be.mem, bc.off));
  be.bytes = bc.off;
  char* base = static_cast<char*>(be.mem);
  be.dev.n_entries = total;
  be.dev.n_pos = n_pos;
  be.dev.kf = reinterpret_cast<float4*>(base + o_kf);
  be.dev.wgt = reinterpret_cast<float*>(base + o_w);
  be.dev.pos = reinterpret_cast<int32_t*>(base + o_pos);
  be.dev.map = reinterpret_cast<int32_t*>(base + o_map);
  hipError_t e = launch_band_fill(gc, sig, qmax, cnt, off, n_slots, be.dev, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dev_free(h, be.mem, be.bytes);
    return fail(DM_ERR_DEVICE, "band fill: %s", hipGetErrorString(e));
  }
  h->bands[key] = be;
  h->band_lru.push_front(key);
  *out = be.dev;
  return DM_OK;
}

dm_status get_fft(dm_handle* h, const dm_grid* g, FftPlans** out) {
  std::call_once(g_fft_once, [] { g_fft_setup = rocfft_setup(); });
  if (g_fft_setup != rocfft_status_success) return fail(DM_ERR_FFT, "rocfft_setup failed");
  auto key = std::make_tuple(g->n[0], g->n[1], g->n[2]);
  auto it = h->ffts.find(key);
  if (it != h->ffts.end()) {
    *out = &it->second;
    return DM_OK;
  }
  FftPlans fp;
  const size_t len[3] = {(size_t)g->n[2], (size_t)g->n[1], (size_t)g->n[0]};   // fastest first
  FFT_TRY(rocfft_plan_create(&fp.c2r, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                             rocfft_precision_single, 3, len, 1, nullptr));
  FFT_TRY(rocfft_plan_create(&fp.r2c, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                             rocfft_precision_single, 3, len, 1, nullptr));
  FFT_TRY(rocfft_plan_get_work_buffer_size(fp.c2r, &fp.work_c2r));
  FFT_TRY(rocfft_plan_get_work_buffer_size(fp.r2c, &fp.work_r2c));
  auto r = h->ffts.emplace(key, fp);
  *out = &r.first->second;
  return DM_OK;
}

dm_status run_fft(dm_handle* h, rocfft_plan plan, void* in, void* out, void* work, size_t work_bytes, hipStream_t s) {
  if (!h->exec_info) FFT_TRY(rocfft_execution_info_create(&h->exec_info));
  FFT_TRY(rocfft_execution_info_set_stream(h->exec_info, s));
  if (work_bytes) FFT_TRY(rocfft_execution_info_set_work_buffer(h->exec_info, work, work_bytes));
  void* ib[1] = {in};
  void* ob[1] = {out};
  FFT_TRY(rocfft_execute(plan, ib, ob, h->exec_info));
  return DM_OK;
}

dm_status check_mesh(const dm_mesh* m, int mode) {
  if (!m) return fail(DM_ERR_ARG, "mesh is NULL");
  if (!m->topo) return fail(DM_ERR_ARG, "mesh topology is NULL");
  if (m->n_verts != m->topo->nv)
    return fail(DM_ERR_ARG, "mesh has %d vertices but its topology was built for %d", m->n_verts, m->topo->nv);
  if (m->n_verts > 0 && !m->verts_dev) return fail(DM_ERR_ARG, "verts_dev is NULL");
  if (mode == DM_VOLUME && !m->topo->closed)
    return fail(DM_ERR_MESH, "DM_VOLUME needs a closed, consistently oriented mesh");
  return DM_OK;
}

// Launch geometry of the two sweeps.
struct SweepPlan {
  int n_chunks = 1, per_chunk = 1;
};

SweepPlan plan_fwd(int64_t nE, int nt) {
  SweepPlan sp;
  const int64_t tiles = (nE + 255) / 256;
  int64_t want = (16384 + tiles - 1) / std::max<int64_t>(tiles, 1);
  const int64_t maxc = std::max<int64_t>(1, nt / 32);
  sp.n_chunks = (int)std::max<int64_t>(1, std::min(want, maxc));
  sp.per_chunk = (int)((nt + sp.n_chunks - 1) / sp.n_chunks);
  if (sp.per_chunk < 1) sp.per_chunk = 1;
  sp.n_chunks = (int)((nt + sp.per_chunk - 1) / sp.per_chunk);
  if (sp.n_chunks < 1) sp.n_chunks = 1;
  return sp;
}

SweepPlan plan_vjp(int64_t nE, int nt) {
  SweepPlan sp;
  const int64_t tiles = (nt + 255) / 256;
  int64_t want = (16384 + tiles - 1) / std::max<int64_t>(tiles, 1);
  const int64_t maxc = std::max<int64_t>(1, nE / 64);
  sp.n_chunks = (int)std::max<int64_t>(1, std::min(want, maxc));
  sp.per_chunk = (int)((nE + sp.n_chunks - 1) / sp.n_chunks);
  if (sp.per_chunk < 1) sp.per_chunk = 1;
  sp.n_chunks = (int)((nE + sp.per_chunk - 1) / sp.per_chunk);
  if (sp.n_chunks < 1) sp.n_chunks = 1;
  return sp;
}

hipEvent_t pooled_event(dm_handle* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one sweep launch with events when timing is enabled.
struct SweepTimer {
  dm_handle* h;
  hipStream_t s;
  TimedLaunch t;
  SweepTimer(dm_handle* h_, hipStream_t s_, int kind, double pairs) : h(h_), s(s_) {
    if (!h->timing) return;
    t.kind = kind;
    t.pairs = pairs;
    t.a = pooled_event(h);
    t.b = pooled_event(h);
    if (t.a) (void)hipEventRecord(t.a, s);
  }
  void done() {
    if (!h->timing || !t.a || !t.b) return;
    (void)hipEventRecord(t.b, s);
    h->pending.push_back(t);
  }
};

// Orders a call after the previous call of the handle (the workspace is shared).
dm_status begin_call(dm_handle* h, hipStream_t s) {
  if (h->have_last) HIP_TRY(hipStreamWaitEvent(s, h->last_ev, 0));
  return DM_OK;
}

dm_status end_call(dm_handle* h, hipStream_t s) {
  HIP_TRY(hipEventRecord(h->last_ev, s));
  h->have_last = true;
  return DM_OK;
}

dm_status zero_fill(float* p, int64_t n, hipStream_t s) {
  if (!p || n <= 0) return DM_OK;
  HIP_TRY(launch_fill_zero(p, n, s));
  return DM_OK;
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char* dm_last_error(void) { return g_err.c_str(); }

const char* dm_version(void) { return "deltamic-mi355x 0.1 (gfx950)"; }

dm_status dm_create(dm_handle** out, int device, size_t hbm_budget_bytes) {
  g_err.clear();
  if (!out) return fail(DM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(DM_ERR_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(DM_ERR_DEVICE, "device %d out of range (%d devices)", device, ndev);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DM_ERR_DEVICE, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
  DeviceGuard dg(device);
  auto h = std::make_unique<dm_handle>();
  h->device = device;
  h->budget = hbm_budget_bytes;
  HIP_TRY(hipEventCreateWithFlags(&h->last_ev, hipEventDisableTiming));
  *out = h.release();
  return DM_OK;
}

dm_status dm_destroy(dm_handle* h) {
  g_err.clear();
  if (!h) return DM_OK;
  DeviceGuard dg(h->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : h->bands) (void)hipFree(kv.second.mem);
  for (auto& kv : h->ffts) {
    if (kv.second.c2r) rocfft_plan_destroy(kv.second.c2r);
    if (kv.second.r2c) rocfft_plan_destroy(kv.second.r2c);
  }
  if (h->exec_info) rocfft_execution_info_destroy(h->exec_info);
  for (auto& t : h->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
  if (h->ws) (void)hipFree(h->ws);
  if (h->last_ev) (void)hipEventDestroy(h->last_ev);
  delete h;
  return DM_OK;
}

dm_status dm_timing_enable(dm_handle* h, int enable) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  h->timing = enable != 0;
  return DM_OK;
}

dm_status dm_timing_read(dm_handle* h, dm_kernel_time* fwd_sweep, dm_kernel_time* vjp_sweep, int reset) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DeviceGuard dg(h->device);
  for (auto& t : h->pending) {
    HIP_TRY(hipEventSynchronize(t.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    h->acc[t.kind].launches += 1;
    h->acc[t.kind].ms += ms;
    h->acc[t.kind].pairs += t.pairs;
    h->event_pool.push_back(t.a);
    h->event_pool.push_back(t.b);
  }
  h->pending.clear();
  if (fwd_sweep) *fwd_sweep = h->acc[0];
  if (vjp_sweep) *vjp_sweep = h->acc[1];
  if (reset) h->acc[0] = h->acc[1] = dm_kernel_time{0, 0.0, 0.0};
  return DM_OK;
}

dm_status dm_memory_in_use(const dm_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(DM_ERR_ARG, "NULL argument");
  *bytes = h->in_use;
  return DM_OK;
}

dm_status dm_topology_create(dm_handle* h, const int32_t* faces, int32_t n_faces, int32_t n_verts,
                             int faces_on_device, dm_topology** out) {
  g_err.clear();
  if (!h || !out) return fail(DM_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (n_faces < 0 || n_verts < 0) return fail(DM_ERR_ARG, "negative size");
  if (n_faces > 0 && !faces) return fail(DM_ERR_ARG, "faces is NULL");
  if ((int64_t)n_faces * 3 >= ((int64_t)1 << 31)) return fail(DM_ERR_ARG, "too many faces");
  DeviceGuard dg(h->device);
  std::vector<int32_t> F((size_t)n_faces * 3);
  if (n_faces > 0) {
    if (faces_on_device)
      HIP_TRY(hipMemcpy(F.data(), faces, F.size() * 4, hipMemcpyDeviceToHost));
    else
      memcpy(F.data(), faces, F.size() * 4);
  }
  for (size_t i = 0; i < F.size(); ++i)
    if (F[i] < 0 || F[i] >= n_verts)
      return fail(DM_ERR_MESH, "face %zu references vertex %d outside [0, %d)", i / 3, F[i], n_verts);
  // closed and consistently oriented: each directed edge once, with its reverse present
  std::vector<uint64_t> e;
  e.reserve(F.size());
  for (int t = 0; t < n_faces; ++t)
    for (int p = 0; p < 3; ++p) {
      const uint32_t a = (uint32_t)F[3 * t + p], b = (uint32_t)F[3 * t + (p + 1) % 3];
      e.push_back(((uint64_t)a << 32) | b);
    }
  std::sort(e.begin(), e.end());
  bool closed = n_faces > 0 && std::adjacent_find(e.begin(), e.end()) == e.end();
  if (closed)
    for (uint64_t x : e) {
      const uint64_t r = (x << 32) | (x >> 32);
      if (!std::binary_search(e.begin(), e.end(), r)) {
        closed = false;
        break;
      }
    }
  // vertex incidence (CSR)
  std::vector<int32_t> off((size_t)n_verts + 1, 0), ent(F.size());
  for (size_t i = 0; i < F.size(); ++i) off[(size_t)F[i] + 1]++;
  for (int v = 0; v < n_verts; ++v) off[v + 1] += off[v];
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (size_t i = 0; i < F.size(); ++i) ent[fill[F[i]]++] = (int32_t)i;   // i = 3 t + p
  auto t = std::make_unique<dm_topology>();
  t->h = h;
  t->nt = n_faces;
  t->nv = n_verts;
  t->closed = closed ? 1 : 0;
  const size_t bf = align_up(F.size() * 4), bo = align_up(off.size() * 4), be = align_up(ent.size() * 4);
  void* mem = nullptr;
  DM_TRY(dev_alloc(h, &mem, bf + bo + be));
  t->bytes = bf + bo + be;
  t->faces = static_cast<int32_t*>(mem);
  t->csr_off = reinterpret_cast<int32_t*>(static_cast<char*>(mem) + bf);
  t->csr_ent = reinterpret_cast<int32_t*>(static_cast<char*>(mem) + bf + bo);
  hipError_t err = hipSuccess;
  if (!F.empty()) err = hipMemcpy(t->faces, F.data(), F.size() * 4, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(t->csr_off, off.data(), off.size() * 4, hipMemcpyHostToDevice);
  if (err == hipSuccess && !ent.empty()) err = hipMemcpy(t->csr_ent, ent.data(), ent.size() * 4, hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    dev_free(h, mem, t->bytes);
    return fail(DM_ERR_DEVICE, "topology upload: %s", hipGetErrorString(err));
  }
  h->topo_count++;
  *out = t.release();
  return DM_OK;
}

dm_status dm_topology_destroy(dm_topology* t) {
  g_err.clear();
  if (!t) return DM_OK;
  DeviceGuard dg(t->h->device);
  (void)hipDeviceSynchronize();
  dev_free(t->h, t->faces, t->bytes);
  t->h->topo_count--;
  delete t;
  return DM_OK;
}

dm_status dm_topology_info(const dm_topology* t, int32_t* n_faces, int32_t* n_verts, int32_t* closed) {
  if (!t) return fail(DM_ERR_ARG, "topology is NULL");
  if (n_faces) *n_faces = t->nt;
  if (n_verts) *n_verts = t->nv;
  if (closed) *closed = t->closed;
  return DM_OK;
}

dm_status dm_band_size(dm_handle* h, const dm_grid* g, const dm_psf* psf, int64_t* n_entries, void* stream) {
  g_err.clear();
  if (!h || !n_entries) return fail(DM_ERR_ARG, "NULL argument");
  DM_TRY(check_grid(g));
  DM_TRY(check_psf(psf));
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)stream;
  DM_TRY(begin_call(h, s));
  BandDev b;
  DM_TRY(get_band(h, g, psf, s, &b));
  DM_TRY(end_call(h, s));
  *n_entries = b.n_entries;
  return DM_OK;
}

dm_status dm_band_export(dm_handle* h, const dm_grid* g, const dm_psf* psf, int32_t* k_out, int64_t* pos_out,
                         float* weight_out, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_psf(psf));
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)stream;
  DM_TRY(begin_call(h, s));
  BandDev b;
  DM_TRY(get_band(h, g, psf, s, &b));
  const int64_t n = b.n_entries;
  if (n > 0) {
    std::vector<float4> kf((size_t)n);
    std::vector<int32_t> pos((size_t)n);
    std::vector<float> w((size_t)n);
    HIP_TRY(hipMemcpyAsync(kf.data(), b.kf, n * sizeof(float4), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(pos.data(), b.pos, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(w.data(), b.wgt, n * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
      if (k_out) {
        k_out[3 * i] = (int32_t)kf[i].x;
        k_out[3 * i + 1] = (int32_t)kf[i].y;
        k_out[3 * i + 2] = (int32_t)kf[i].z;
      }
      if (pos_out) pos_out[i] = pos[i];
      if (weight_out) weight_out[i] = w[i];
    }
  }
  DM_TRY(end_call(h, s));
  return DM_OK;
}

// The forward and backward passes share one implementation.
static dm_status render_impl(dm_handle* h, const dm_mesh* m, const dm_psf* psf, const dm_grid* g, float* image,
                             float* spec_out, const float* dLdI, float* dV, float* dS, const float* spec_in,
                             hipStream_t s) {
  const int mode = g->mode;
  const GridC gc = make_gridc(g);
  const int nt = m->topo->nt, nv = m->n_verts;
  const int64_t nvox = (int64_t)g->n[0] * g->n[1] * g->n[2];
  const bool want_vjp = dLdI && (dV || dS);
  DM_TRY(begin_call(h, s));
  BandDev b;
  DM_TRY(get_band(h, g, psf, s, &b));
  const int64_t nE = b.n_entries;
  FftPlans* fp = nullptr;
  if (image || want_vjp) DM_TRY(get_fft(h, g, &fp));

  // Empty band or empty mesh: zero outputs.
  if (nE == 0 || nt == 0) {
    DM_TRY(zero_fill(image, nvox, s));
    DM_TRY(zero_fill(spec_out, 2 * nE, s));
    DM_TRY(zero_fill(dV, 3 * (int64_t)nv, s));
    DM_TRY(zero_fill(dS, 6, s));
    return end_call(h, s);
  }

  const bool need_spec = (image && !spec_in) || (dS && !spec_in) || spec_out;
  const SweepPlan fsp = plan_fwd(nE, nt);
  const SweepPlan vsp = plan_vjp(nE, nt);
  const int nc = nchannels(mode);
  const int prep_blocks = mesh_prep_blocks(nt);
  const int adj_blocks = adjoint_blocks(gc);
  Carver cv;
  const size_t o_rec = cv.take<float>((size_t)nt * TRI_REC);
  const size_t o_info = cv.take<MeshInfo>(1);
  const size_t o_ptmp = cv.take<double>(2 * (size_t)prep_blocks);
  const size_t o_part = need_spec ? cv.take<float2>((size_t)fsp.n_chunks * nE) : 0;
  const size_t o_spec = (need_spec && !spec_out) ? cv.take<float2>(nE) : 0;
  const size_t o_x = image ? cv.take<float2>(b.n_pos) : 0;
  const size_t o_fftw = cv.take<char>(fp ? std::max(fp->work_c2r, fp->work_r2c) : 0);
  const size_t o_gin = want_vjp ? cv.take<float>(nvox) : 0;
  const size_t o_ghat = want_vjp ? cv.take<float2>(b.n_pos) : 0;
  const size_t o_erec = want_vjp ? cv.take<float4>(2 * (size_t)nE) : 0;
  const size_t o_dsp = (want_vjp && dS) ? cv.take<double>(6 * (size_t)adj_blocks) : 0;
  const size_t o_vpart = (want_vjp && dV) ? cv.take<float>((size_t)vsp.n_chunks * nc * nt) : 0;
  const size_t o_red = (want_vjp && dV) ? cv.take<float>((size_t)nc * nt) : 0;
  const size_t o_R = cv.take<double>(1);
  DM_TRY(ensure_ws(h, cv.off));

  float* rec = at<float>(h, o_rec);
  MeshInfo* info = at<MeshInfo>(h, o_info);
  HIP_TRY(launch_mesh_prep(mode, gc, m->verts_dev, nv, m->topo->faces, nt, rec, info, at<double>(h, o_ptmp),
                           prep_blocks, s));

  const float2* spec = reinterpret_cast<const float2*>(spec_in);
  if (need_spec) {
    float2* part = at<float2>(h, o_part);
    float2* sp = spec_out ? reinterpret_cast<float2*>(spec_out) : at<float2>(h, o_spec);
    SweepTimer tm(h, s, 0, (double)nE * nt);
    HIP_TRY(launch_fwd_sweep(mode, b.kf, nE, rec, nt, fsp.per_chunk, fsp.n_chunks, part, s));
    tm.done();
    float2* xh = image ? at<float2>(h, o_x) : nullptr;
    HIP_TRY(launch_fwd_finalize(mode, gc, b, part, fsp.n_chunks, info, sp, xh, s));
    spec = sp;
  } else if (image) {
    HIP_TRY(launch_spec_scatter(gc, b, spec, at<float2>(h, o_x), s));
  }
  if (image)
    DM_TRY(run_fft(h, fp->c2r, at<float2>(h, o_x), image, at<char>(h, o_fftw), fp->work_c2r, s));

  if (want_vjp) {
    float* gin = at<float>(h, o_gin);
    HIP_TRY(hipMemcpyAsync(gin, dLdI, (size_t)nvox * sizeof(float), hipMemcpyDeviceToDevice, s));
    float2* ghat = at<float2>(h, o_ghat);
    DM_TRY(run_fft(h, fp->r2c, gin, ghat, at<char>(h, o_fftw), fp->work_r2c, s));
    float4* erec = at<float4>(h, o_erec);
    double* dsp = dS ? at<double>(h, o_dsp) : nullptr;
    HIP_TRY(launch_adjoint(mode, gc, b, ghat, info, dS ? spec : nullptr, erec, dsp, adj_blocks, s));
    if (dS) HIP_TRY(launch_dsig_final(dsp, adj_blocks, dS, s));
    if (dV) {
      float* vpart = at<float>(h, o_vpart);
      float* red = at<float>(h, o_red);
      SweepTimer tm(h, s, 1, (double)nE * nt);
      HIP_TRY(launch_vjp_sweep(mode, rec, nt, erec, nE, vsp.per_chunk, vsp.n_chunks, vpart, s));
      tm.done();
      HIP_TRY(launch_vjp_reduce(mode, vpart, vsp.n_chunks, nt, red, s));
      double* R = at<double>(h, o_R);
      if (mode == DM_SURFACE) HIP_TRY(launch_surface_scalar(red, rec, nt, info, R, s));
      HIP_TRY(launch_vertex_gather(mode, m->verts_dev, nv, m->topo->faces, nt, m->topo->csr_off, m->topo->csr_ent, red,
                                   R, dV, s));
    }
  }
  return end_call(h, s);
}

dm_status dm_render(dm_handle* h, const dm_mesh* mesh, const dm_psf* psf, const dm_grid* g, float* image_dev,
                    float* spectrum_dev, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_psf(psf));
  DM_TRY(check_mesh(mesh, g->mode));
  if (!image_dev && !spectrum_dev) return fail(DM_ERR_ARG, "no output requested");
  DeviceGuard dg(h->device);
  return render_impl(h, mesh, psf, g, image_dev, spectrum_dev, nullptr, nullptr, nullptr, nullptr,
                     (hipStream_t)stream);
}

dm_status dm_render_vjp(dm_handle* h, const dm_mesh* mesh, const dm_psf* psf, const dm_grid* g,
                        const float* dL_dimage_dev, float* dL_dverts_dev, float* dL_dsigma_dev, float* image_dev,
                        const float* spectrum_in_dev, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_psf(psf));
  DM_TRY(check_mesh(mesh, g->mode));
  if (!dL_dimage_dev) return fail(DM_ERR_ARG, "dL_dimage is NULL");
  if (!dL_dverts_dev && !dL_dsigma_dev && !image_dev) return fail(DM_ERR_ARG, "no output requested");
  DeviceGuard dg(h->device);
  return render_impl(h, mesh, psf, g, image_dev, nullptr, dL_dimage_dev, dL_dverts_dev, dL_dsigma_dev,
                     spectrum_in_dev, (hipStream_t)stream);
}

dm_status dm_mesh_transform(dm_handle* h, const dm_mesh* mesh, const dm_grid* g, const int32_t* k_dev, int64_t n,
                            float* out_dev, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_mesh(mesh, g->mode));
  if (n < 0 || (n > 0 && (!k_dev || !out_dev))) return fail(DM_ERR_ARG, "bad frequency list");
  if (n >= ((int64_t)1 << 31)) return fail(DM_ERR_ARG, "too many frequencies");
  if (n == 0) return DM_OK;
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)stream;
  const int mode = g->mode;
  const GridC gc = make_gridc(g);
  const int nt = mesh->topo->nt;
  DM_TRY(begin_call(h, s));
  if (nt == 0) {
    DM_TRY(zero_fill(out_dev, 2 * n, s));
    return end_call(h, s);
  }
  const SweepPlan sp = plan_fwd(n, nt);
  const int prep_blocks = mesh_prep_blocks(nt);
  Carver cv;
  const size_t o_rec = cv.take<float>((size_t)nt * TRI_REC), o_info = cv.take<MeshInfo>(1),
               o_ptmp = cv.take<double>(2 * (size_t)prep_blocks), o_kf = cv.take<float4>(n),
               o_part = cv.take<float2>((size_t)sp.n_chunks * n);
  DM_TRY(ensure_ws(h, cv.off));
  float* rec = at<float>(h, o_rec);
  MeshInfo* info = at<MeshInfo>(h, o_info);
  HIP_TRY(launch_mesh_prep(mode, gc, mesh->verts_dev, mesh->n_verts, mesh->topo->faces, nt, rec, info,
                           at<double>(h, o_ptmp), prep_blocks, s));
  float4* kf = at<float4>(h, o_kf);
  HIP_TRY(launch_points_prepare(gc, k_dev, n, kf, s));
  float2* part = at<float2>(h, o_part);
  SweepTimer tm(h, s, 0, (double)n * nt);
  HIP_TRY(launch_fwd_sweep(mode, kf, n, rec, nt, sp.per_chunk, sp.n_chunks, part, s));
  tm.done();
  HIP_TRY(launch_points_finalize(mode, gc, kf, n, part, sp.n_chunks, info, reinterpret_cast<float2*>(out_dev), s));
  return end_call(h, s);
}

}  // extern "C"
