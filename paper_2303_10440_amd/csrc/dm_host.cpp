// Host side of the C ABI in include/deltamic.h: validation, handle state
// (workspace, band cache, FFT plans), and the launch sequences of the
// forward render and its vector-Jacobian product.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
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
#include "dm_topo.h"

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

// Limits of a handle's band cache (a band per grid, covariance and threshold:
// a fit that changes the PSF every step, or a server whose requests carry
// their own PSFs, would otherwise keep one band per covariance forever).
// Beyond either limit the least recently used band that no batch in
// preparation holds is freed.
constexpr size_t BAND_CACHE_MAX_COUNT = 32;
constexpr size_t BAND_CACHE_MAX_BYTES = (size_t)4 << 30;

// Second stream of a batch (created on first use, default priority) and the
// events that fork work onto it and join it back.  A handle has one for
// dm_batch_run; each serving slot has its own, so batches in flight on
// different slots do not queue behind each other's second stream.
// Streams beside a call's own stream (default priority, non-blocking): the
// small per-request steps of a batch are spread over them, and large requests
// alternate with the call's stream.  fork orders them after the call's stream,
// join[k] orders the call's stream after stream k.
constexpr int AUX_STREAMS = 3;
struct AuxStream {
  hipStream_t s[AUX_STREAMS] = {};
  hipEvent_t fork = nullptr, join[AUX_STREAMS] = {};
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
  int pins = 0;   // > 0 while a batch being enqueued uses this band
};

struct FftPlans {
  rocfft_plan c2r = nullptr, r2c = nullptr;
  size_t work_c2r = 0, work_r2c = 0;
};

// Event pairs recorded around sweep launches while timing is enabled.
struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;   // 0 forward sweep, 1 gradient sweep, 2 batched sweep, 3 fused sweep
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
  size_t band_bytes = 0;         // device memory of the cached bands
  BandEntry otf_band;            // band of the last tabulated-OTF call (rebuilt every call)
  std::map<std::tuple<int, int, int>, FftPlans> ffts;
  rocfft_execution_info exec_info = nullptr;
  hipEvent_t last_ev = nullptr;
  bool have_last = false;
  AuxStream aux;   // second stream of dm_batch_run
  int topo_count = 0;
  size_t topo_bytes = 0;
  bool timing = false;
  std::vector<TimedLaunch> pending;   // recorded, not yet read
  std::vector<hipEvent_t> event_pool;
  dm_kernel_time acc[4] = {{0, 0.0, 0.0}, {0, 0.0, 0.0}, {0, 0.0, 0.0}, {0, 0.0, 0.0}};
};

// Triangles are kept in strip order: consecutive triangles of a strip share
// an edge, triangle i of a strip is (s_i, s_i+1, s_i+2), so each one brings a
// single new vertex (the sweeps reuse the other two vertex phases).
struct dm_topology {
  dm_handle* h = nullptr;
  int nt = 0, nv = 0, closed = 0, n_strips = 0;
  int32_t* faces = nullptr;     // device [nt][3], strip order
  int32_t* csr_off = nullptr;   // device [nv+1]
  int32_t* csr_ent = nullptr;   // device [3 nt] = 3 t + p (strip-order t, p)
  int32_t* flags = nullptr;     // device [nt]: TRI_STRIP_START, TRI_REVERSED
  int32_t* adj_off = nullptr;   // device [nv+1]: vertex adjacency (mesh edges), CSR
  int32_t* adj_nbr = nullptr;   // device [2 n_edges]
  int32_t* adj_tab = nullptr;   // device [nv][LAP_TABLE_W], -1 padded; nullptr if a degree exceeds the width
  // density weights (dm_topology_set_weights): device [nt] in strip order, or nullptr (all 1)
  float* weights = nullptr;
  int closed_plain = 0;                    // closed and consistently oriented, ignoring weights
  int lap_mu = 0;                          // bound on the largest eigenvalue of the mesh Laplacian
  std::vector<int32_t> faces_in;           // host copy of the input faces
  std::vector<int32_t> src;                // input face of each strip-order triangle
  size_t bytes = 0;
  float* smooth_ws = nullptr;   // device workspace of dm_laplace_smooth (allocated on first use)
  size_t smooth_bytes = 0;
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

// Frees the least recently used band that no batch in preparation holds.
// Returns false if every cached band is pinned.
bool evict_one_band(dm_handle* h) {
  for (auto lit = h->band_lru.rbegin(); lit != h->band_lru.rend(); ++lit) {
    auto it = h->bands.find(*lit);
    if (it == h->bands.end() || it->second.pins > 0) continue;
    (void)hipDeviceSynchronize();
    dev_free(h, it->second.mem, it->second.bytes);
    h->band_bytes -= std::min(h->band_bytes, it->second.bytes);
    h->bands.erase(it);
    h->band_lru.erase(std::next(lit).base());
    return true;
  }
  return false;
}

// Workspace: one growable device buffer carved per call.
dm_status ensure_ws(dm_handle* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return DM_OK;
  while (h->budget && h->in_use - h->ws_bytes + bytes > h->budget && evict_one_band(h)) {
  }
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
  const Check c = validate_grid(g);
  return c.st == DM_OK ? DM_OK : fail(c.st, "%s", c.msg.c_str());
}

dm_status check_psf(const dm_psf* p) {
  const Check c = validate_psf(p);
  return c.st == DM_OK ? DM_OK : fail(c.st, "%s", c.msg.c_str());
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
dm_status get_band(dm_handle* h, const dm_grid* g, const dm_psf* p, hipStream_t s, BandDev* out, bool pin = false) {
  const BandKey key = make_key(g, p);
  auto it = h->bands.find(key);
  if (it != h->bands.end()) {
    h->band_lru.remove(key);
    h->band_lru.push_front(key);
    if (pin) it->second.pins++;
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
  // allocate the band (evicting the least recently used unpinned bands if the
  // budget or the cache's own limits require)
  Carver bc;
  const int64_t ne = std::max<int64_t>(total, 1);
  const size_t o_kf = bc.take<float4>(ne), o_w = bc.take<float>(ne), o_pos = bc.take<int32_t>(ne),
               o_map = bc.take<int32_t>(n_pos);
  while (((h->budget && h->in_use + bc.off > h->budget) || h->bands.size() >= BAND_CACHE_MAX_COUNT ||
          h->band_bytes + bc.off > BAND_CACHE_MAX_BYTES) &&
         evict_one_band(h)) {
  }
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
  be.pins = pin ? 1 : 0;
  h->bands[key] = be;
  h->band_bytes += be.bytes;
  h->band_lru.push_front(key);
  *out = be.dev;
  return DM_OK;
}

// Slots of the band build: 4x4x4 bricks of the half spectrum.
int64_t band_slots(const GridC& gc) {
  return (int64_t)((gc.n0 + 3) / 4) * ((gc.n1 + 3) / 4) * ((gc.n2h + 3) / 4) * 64;
}

double otf_tau2(const dm_grid* g) {
  const double tau = (double)(g->band_tau > 0.0f ? g->band_tau : 0.0f);
  return tau * tau;
}

// Layout of a tabulated-OTF band: entry arrays, then the position map.
struct OtfBandLayout {
  size_t o_kf = 0, o_w = 0, o_pos = 0, o_map = 0;
  void take(Carver& c, int64_t n_entries, int64_t n_pos) {
    const int64_t ne = std::max<int64_t>(n_entries, 1);
    o_kf = c.take<float4>(ne);
    o_w = c.take<float>(ne);
    o_pos = c.take<int32_t>(ne);
    o_map = c.take<int32_t>(n_pos);
  }
  void bind(char* base, BandDev& b) const {
    b.kf = reinterpret_cast<float4*>(base + o_kf);
    b.wgt = reinterpret_cast<float*>(base + o_w);
    b.pos = reinterpret_cast<int32_t*>(base + o_pos);
    b.map = reinterpret_cast<int32_t*>(base + o_map);
  }
};

// Counts the band of a tabulated OTF, with the per-slot counts and offsets in
// the workspace (cnt, off) for a fill that follows on the same stream.
// Synchronises s.
dm_status count_otf_band(dm_handle* h, const dm_grid* g, const float2* otf, hipStream_t s, int64_t* total,
                         int32_t** cnt, int32_t** off) {
  const GridC gc = make_gridc(g);
  const int64_t n_slots = band_slots(gc);
  Carver cv;
  const size_t o_cnt = cv.take<int32_t>(n_slots), o_off = cv.take<int32_t>(n_slots),
               o_tmp = cv.take<int32_t>(scan_tmp_elems(n_slots)), o_tot = cv.take<int64_t>(1);
  DM_TRY(ensure_ws(h, cv.off));
  *cnt = at<int32_t>(h, o_cnt);
  *off = at<int32_t>(h, o_off);
  HIP_TRY(launch_band_count_otf(gc, otf, otf_tau2(g), *cnt, n_slots, s));
  HIP_TRY(launch_scan(*cnt, *off, n_slots, at<int32_t>(h, o_tmp), at<int64_t>(h, o_tot), s));
  *total = 0;
  HIP_TRY(hipMemcpyAsync(total, at<int64_t>(h, o_tot), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DM_OK;
}

// Band of a tabulated OTF (half spectrum, device) for a single call: rebuilt
// on every call since the table may change between calls; its memory is the
// handle's and is reused.  Synchronises s.
dm_status get_otf_band(dm_handle* h, const dm_grid* g, const float2* otf, hipStream_t s, BandDev* out) {
  const GridC gc = make_gridc(g);
  const int64_t n_pos = (int64_t)gc.n0 * gc.n1 * gc.n2h;
  const int64_t n_slots = band_slots(gc);
  int64_t total = 0;
  int32_t *cnt = nullptr, *off = nullptr;
  DM_TRY(count_otf_band(h, g, otf, s, &total, &cnt, &off));
  Carver bc;
  OtfBandLayout bl;
  bl.take(bc, total, n_pos);
  BandEntry& be = h->otf_band;
  if (be.bytes < bc.off) {
    dev_free(h, be.mem, be.bytes);
    be.mem = nullptr;
    be.bytes = 0;
    DM_TRY(dev_alloc(h, &be.mem, bc.off));
    be.bytes = bc.off;
  }
  be.dev.n_entries = total;
  be.dev.n_pos = n_pos;
  bl.bind(static_cast<char*>(be.mem), be.dev);
  be.dev.otf = otf;
  HIP_TRY(launch_band_fill_otf(gc, otf, otf_tau2(g), cnt, off, n_slots, be.dev, s));
  *out = be.dev;
  return DM_OK;
}

void unpin_band(dm_handle* h, const dm_grid* g, const dm_psf* p) {
  auto it = h->bands.find(make_key(g, p));
  if (it != h->bands.end() && it->second.pins > 0) it->second.pins--;
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

dm_status ensure_aux(AuxStream* a) {
  if (!a->fork) HIP_TRY(hipEventCreateWithFlags(&a->fork, hipEventDisableTiming));
  for (int k = 0; k < AUX_STREAMS; ++k) {
    if (!a->s[k]) HIP_TRY(hipStreamCreateWithFlags(&a->s[k], hipStreamNonBlocking));
    if (!a->join[k]) HIP_TRY(hipEventCreateWithFlags(&a->join[k], hipEventDisableTiming));
  }
  return DM_OK;
}

// Orders the first n aux streams after everything enqueued so far on s.
dm_status aux_fork(AuxStream* a, int n, hipStream_t s) {
  if (n <= 0) return DM_OK;
  HIP_TRY(hipEventRecord(a->fork, s));
  for (int k = 0; k < n; ++k) HIP_TRY(hipStreamWaitEvent(a->s[k], a->fork, 0));
  return DM_OK;
}

// Orders s after everything enqueued so far on the first n aux streams.
dm_status aux_join(AuxStream* a, int n, hipStream_t s) {
  for (int k = 0; k < n; ++k) {
    HIP_TRY(hipEventRecord(a->join[k], a->s[k]));
    HIP_TRY(hipStreamWaitEvent(s, a->join[k], 0));
  }
  return DM_OK;
}

void destroy_aux(AuxStream* a) {
  if (a->fork) (void)hipEventDestroy(a->fork);
  for (int k = 0; k < AUX_STREAMS; ++k) {
    if (a->join[k]) (void)hipEventDestroy(a->join[k]);
    if (a->s[k]) (void)hipStreamDestroy(a->s[k]);
  }
  *a = AuxStream{};
}

dm_status end_call(dm_handle* h, hipStream_t s) {
  HIP_TRY(hipEventRecord(h->last_ev, s));
  h->have_last = true;
  return DM_OK;
}

// A call's ordering on the handle: begin() makes s wait for the handle's
// previous call, end() records the handle's last-call event on s.  If the
// call fails after begin() (work may already be enqueued on s), the
// destructor still records the event, so that the next call on any stream
// waits for what this one left running in the shared workspace.
struct CallScope {
  dm_handle* h;
  hipStream_t s;
  bool open = false;
  CallScope(dm_handle* h_, hipStream_t s_) : h(h_), s(s_) {}
  dm_status begin() {
    DM_TRY(begin_call(h, s));
    open = true;
    return DM_OK;
  }
  dm_status end() {
    open = false;
    return end_call(h, s);
  }
  ~CallScope() {
    if (open && hipEventRecord(h->last_ev, s) == hipSuccess) h->have_last = true;
  }
};

dm_status zero_fill(float* p, int64_t n, hipStream_t s) {
  if (!p || n <= 0) return DM_OK;
  HIP_TRY(launch_fill_zero(p, n, s));
  return DM_OK;
}

// ---------------------------------------------------------------------------
// One render / gradient request, split into stages so that a single call and
// a batch of many requests share everything except the sweep launch.
struct ReqPlan {
  const dm_mesh* m = nullptr;
  dm_grid g{};
  dm_psf psf{};
  const float* dLdI = nullptr;
  float* image = nullptr;
  float* dV = nullptr;
  float* dS = nullptr;
  const float* spec_in = nullptr;
  float* spec_out = nullptr;
  const float2* otf = nullptr;   // tabulated OTF (half spectrum) instead of the Gaussian PSF
  bool otf_ws = false;   // the OTF band lives in this request's workspace, built by stage_pre
  OtfBandLayout obl;
  size_t o_bcnt = 0, o_boff = 0, o_btmp = 0, o_btot = 0;
  int mode = 0, nt = 0, nv = 0, nc = 3, prep_blocks = 1, adj_blocks = 1;
  int64_t nvox = 0, nE = 0;
  bool want_vjp = false, need_spec = false, empty = false, pinned = false;
  bool fused = false;    // forward and gradient sweeps in one launch (k_fused_lanes)
  bool direct = false;   // in a batch: large enough to run its own sweep launches
  GridC gc{};
  BandDev b{};
  FftPlans* fp = nullptr;
  SweepPlan fsp, vsp;
  size_t o_rec = 0, o_info = 0, o_ptmp = 0, o_part = 0, o_spec = 0, o_x = 0, o_fftw = 0, o_gin = 0, o_ghat = 0,
         o_erec = 0, o_dsp = 0, o_vpart = 0, o_red = 0, o_rtmp = 0, o_R = 0, bytes = 0;
  char* base = nullptr;
  template <typename T>
  T* ptr(size_t off) const {
    return reinterpret_cast<T*>(base + off);
  }
};

// batch: the request is part of a batch; requests of at least direct_pairs
// (entry, triangle) pairs then run their own sweep launches instead of joining
// the shared persistent launch.
dm_status plan_request(dm_handle* h, ReqPlan& P, hipStream_t s, bool batch, double direct_pairs = INFINITY) {
  P.mode = P.g.mode;
  P.gc = make_gridc(&P.g);
  P.nt = P.m->topo->nt;
  P.nv = P.m->n_verts;
  P.nvox = (int64_t)P.g.n[0] * P.g.n[1] * P.g.n[2];
  P.want_vjp = P.dLdI && (P.dV || P.dS);
  if (P.otf && batch) {
    // a batch holds several tables at once: count now (for the plan), build
    // the band in the request's own workspace with its pre-steps
    int64_t total = 0;
    int32_t *cnt = nullptr, *off = nullptr;
    DM_TRY(count_otf_band(h, &P.g, P.otf, s, &total, &cnt, &off));
    P.b = BandDev{};
    P.b.n_entries = total;
    P.b.n_pos = (int64_t)P.gc.n0 * P.gc.n1 * P.gc.n2h;
    P.b.otf = P.otf;
    P.otf_ws = true;
    P.pinned = false;
  } else if (P.otf) {
    DM_TRY(get_otf_band(h, &P.g, P.otf, s, &P.b));
    P.pinned = false;
  } else {
    DM_TRY(get_band(h, &P.g, &P.psf, s, &P.b, batch));
    P.pinned = batch;
  }
  P.nE = P.b.n_entries;
  if (P.image || P.want_vjp) DM_TRY(get_fft(h, &P.g, &P.fp));
  P.empty = P.nE == 0 || P.nt == 0;
  P.need_spec = (P.image && !P.spec_in) || (P.dS && !P.spec_in) || P.spec_out;
  P.direct = batch && (double)P.nE * P.nt >= direct_pairs;
  const bool shared = batch && !P.direct;
  // the forward value comes with the gradient sweep when both are wanted (in a
  // batch too, in the shared launch's tiles of plan_fused_batch)
  P.fused = P.need_spec && P.want_vjp && P.dV;
  if (P.fused) {
    P.vsp = shared ? plan_fused_batch(P.nE, P.nt, P.g.mode) : plan_fused(P.nE, P.nt, P.g.mode);
    P.fsp = fused_fwd_plan(P.vsp, P.nt);
  } else {
    P.fsp = shared ? plan_fwd_batch(P.nE, P.nt) : plan_fwd(P.nE, P.nt);
    P.vsp = shared ? plan_vjp_batch(P.nE, P.nt, P.g.mode) : plan_vjp(P.nE, P.nt, P.g.mode);
  }
  P.nc = nchannels(P.mode);
  P.prep_blocks = mesh_prep_blocks(P.nt);
  P.adj_blocks = adjoint_blocks(P.gc);
  Carver cv;
  if (!P.empty) {
    const bool vjp_v = P.want_vjp && P.dV;
    P.o_rec = cv.take<float>((size_t)P.nt * TRI_REC);
    P.o_info = cv.take<MeshInfo>(1);
    P.o_ptmp = cv.take<double>(2 * (size_t)P.prep_blocks);
    P.o_part = P.need_spec ? cv.take<float2>((size_t)P.fsp.n_chunks * P.nE) : 0;
    P.o_spec = (P.need_spec && !P.spec_out) ? cv.take<float2>(P.nE) : 0;
    P.o_x = P.image ? cv.take<float2>(P.b.n_pos) : 0;
    P.o_fftw = cv.take<char>(P.fp ? std::max(P.fp->work_c2r, P.fp->work_r2c) : 0);
    P.o_gin = P.want_vjp ? cv.take<float>(P.nvox) : 0;
    P.o_ghat = P.want_vjp ? cv.take<float2>(P.b.n_pos) : 0;
    P.o_erec = vjp_v ? cv.take<float4>((size_t)ERC * P.nE) : 0;
    P.o_dsp = (P.want_vjp && P.dS) ? cv.take<double>(6 * (size_t)P.adj_blocks) : 0;
    P.o_vpart = vjp_v ? cv.take<float>((size_t)P.vsp.n_chunks * P.nc * P.nt) : 0;
    P.o_red = vjp_v ? cv.take<float>((size_t)P.nc * P.nt) : 0;
    P.o_rtmp = vjp_v ? cv.take<float>((size_t)vjp_reduce_groups(P.vsp.n_chunks) * P.nc * P.nt) : 0;
    P.o_R = cv.take<double>(1);
    if (P.otf_ws) {
      const int64_t n_slots = band_slots(P.gc);
      P.obl.take(cv, P.nE, P.b.n_pos);
      P.o_bcnt = cv.take<int32_t>(n_slots);
      P.o_boff = cv.take<int32_t>(n_slots);
      P.o_btmp = cv.take<int32_t>(scan_tmp_elems(n_slots));
      P.o_btot = cv.take<int64_t>(1);
    }
  }
  P.bytes = cv.off;
  return DM_OK;
}

// Drops the pin a batch request holds on its cached band (none for a
// tabulated OTF, whose band is the request's own).
void release_band(dm_handle* h, ReqPlan& P) {
  if (P.pinned) unpin_band(h, &P.g, &P.psf);
  P.pinned = false;
}

const float2* spectrum_of(const ReqPlan& P) {
  if (P.need_spec) return P.spec_out ? reinterpret_cast<const float2*>(P.spec_out) : P.ptr<float2>(P.o_spec);
  return reinterpret_cast<const float2*>(P.spec_in);
}

// Points the band of a request whose band lives in its workspace at that
// workspace (once P.base is set).
void bind_band(ReqPlan& P) {
  if (P.otf_ws && !P.empty) P.obl.bind(P.base, P.b);
}

// Mesh prep and, for the gradient, FFT of dL/dI and adjoint weights; the
// band first when it lives in the request's workspace.
dm_status stage_pre(dm_handle* h, ReqPlan& P, hipStream_t s) {
  if (P.empty) {
    DM_TRY(zero_fill(P.image, P.nvox, s));
    DM_TRY(zero_fill(P.spec_out, 2 * P.nE, s));
    DM_TRY(zero_fill(P.dV, 3 * (int64_t)P.nv, s));
    DM_TRY(zero_fill(P.dS, 6, s));
    return DM_OK;
  }
  if (P.otf_ws) {
    // the same count as at planning (the table is read again), then the fill
    const int64_t n_slots = band_slots(P.gc);
    int32_t* cnt = P.ptr<int32_t>(P.o_bcnt);
    int32_t* off = P.ptr<int32_t>(P.o_boff);
    HIP_TRY(launch_band_count_otf(P.gc, P.otf, otf_tau2(&P.g), cnt, n_slots, s));
    HIP_TRY(launch_scan(cnt, off, n_slots, P.ptr<int32_t>(P.o_btmp), P.ptr<int64_t>(P.o_btot), s));
    HIP_TRY(launch_band_fill_otf(P.gc, P.otf, otf_tau2(&P.g), cnt, off, n_slots, P.b, s));
  }
  HIP_TRY(launch_mesh_prep(P.mode, P.gc, P.m->verts_dev, P.nv, P.m->topo->faces, P.m->topo->flags, P.m->topo->weights,
                           P.nt, P.ptr<float>(P.o_rec),
                           P.ptr<MeshInfo>(P.o_info), P.ptr<double>(P.o_ptmp), P.prep_blocks, s));
  if (P.want_vjp) {
    HIP_TRY(hipMemcpyAsync(P.ptr<float>(P.o_gin), P.dLdI, (size_t)P.nvox * sizeof(float), hipMemcpyDeviceToDevice, s));
    DM_TRY(run_fft(h, P.fp->r2c, P.ptr<float>(P.o_gin), P.ptr<float2>(P.o_ghat), P.ptr<char>(P.o_fftw),
                   P.fp->work_r2c, s));
    if (P.dV)
      HIP_TRY(launch_adjoint(P.mode, P.gc, P.b, P.ptr<float2>(P.o_ghat), P.ptr<MeshInfo>(P.o_info),
                             P.ptr<float4>(P.o_erec), s));
  }
  return DM_OK;
}

// The two sweeps as separate launches, or the fused sweep (single-request path).
dm_status stage_sweeps(dm_handle* h, ReqPlan& P, hipStream_t s) {
  if (P.empty) return DM_OK;
  if (P.fused) {
    SweepTimer tm(h, s, 3, (double)P.nE * P.nt);
    HIP_TRY(launch_fused_lanes(P.mode, P.gc, P.ptr<float>(P.o_rec), P.nt, P.vsp.tpb, P.ptr<float4>(P.o_erec), P.nE,
                               P.ptr<float>(P.o_vpart), P.ptr<float2>(P.o_part), s));
    tm.done();
    return DM_OK;
  }
  if (P.need_spec) {
    SweepTimer tm(h, s, 0, (double)P.nE * P.nt);
    HIP_TRY(launch_fwd_lanes(P.mode, P.b.kf, P.nE, P.ptr<float>(P.o_rec), P.nt, P.fsp.per_chunk, P.fsp.n_chunks,
                             P.ptr<float2>(P.o_part), s));
    tm.done();
  }
  if (P.want_vjp && P.dV) {
    SweepTimer tm(h, s, 1, (double)P.nE * P.nt);
    HIP_TRY(launch_vjp_lanes(P.mode, P.gc, P.ptr<float>(P.o_rec), P.nt, P.vsp.tpb, P.vsp.sub, P.vsp.n_chunks,
                             P.ptr<float4>(P.o_erec), P.nE, P.ptr<float>(P.o_vpart), s));
    tm.done();
  }
  return DM_OK;
}

// Work items of this request for the persistent batched sweep.
void add_items(const ReqPlan& P, int req, std::vector<SweepItem>& items, std::vector<double>& cost) {
  if (P.empty || P.direct || P.fused) return;   // fused tiles are implicit (layout_batch)
  if (P.need_spec)
    for (int c = 0; c < P.fsp.n_chunks; ++c) {
      const int tris = std::min(P.nt, (c + 1) * P.fsp.per_chunk) - c * P.fsp.per_chunk;
      for (int64_t x0 = 0; x0 < P.nE; x0 += FWD_CHUNK) {
        items.push_back({0, req, (int)x0, c});
        cost.push_back((double)tris * (double)std::min<int64_t>(FWD_CHUNK, P.nE - x0));
      }
    }
  if (P.want_vjp && P.dV)
    for (int c = 0; c < P.vsp.n_chunks; ++c) {
      const int64_t ents = std::min<int64_t>(P.nE, (int64_t)(c + 1) * P.vsp.per_chunk) - (int64_t)c * P.vsp.per_chunk;
      for (int x0 = 0; x0 < P.nt; x0 += P.vsp.tpb) {
        items.push_back({1, req, x0, c});
        cost.push_back(1.3 * (double)ents * (double)std::min(P.vsp.tpb, P.nt - x0));
      }
    }
}

SweepReq sweep_req(const ReqPlan& P) {
  SweepReq q{};
  q.mode = P.mode;
  q.nE = (int)P.nE;
  q.nt = P.nt;
  q.tpc = P.fsp.per_chunk;
  q.epc = P.vsp.per_chunk;
  q.vsub = P.vsp.sub;
  q.vtpb = P.vsp.tpb;
  q.tpx = P.gc.two_pi_over_L[0];
  q.tpy = P.gc.two_pi_over_L[1];
  q.tpz = P.gc.two_pi_over_L[2];
  q.tile0 = 0;
  q.ntr = P.fsp.n_chunks;
  q.kf = P.b.kf;
  q.rec = P.empty ? nullptr : P.ptr<float>(P.o_rec);
  q.fpart = P.need_spec && !P.empty ? P.ptr<float2>(P.o_part) : nullptr;
  q.erec = P.want_vjp && P.dV && !P.empty ? P.ptr<float4>(P.o_erec) : nullptr;
  q.vpart = P.want_vjp && P.dV && !P.empty ? P.ptr<float>(P.o_vpart) : nullptr;
  return q;
}

// Spectrum, image, PSF gradient and vertex gradient from the sweep partials.
dm_status stage_post(dm_handle* h, ReqPlan& P, hipStream_t s) {
  if (P.empty) return DM_OK;
  MeshInfo* info = P.ptr<MeshInfo>(P.o_info);
  float2* xh = P.image ? P.ptr<float2>(P.o_x) : nullptr;
  if (P.need_spec) {
    float2* sp = P.spec_out ? reinterpret_cast<float2*>(P.spec_out) : P.ptr<float2>(P.o_spec);
    HIP_TRY(launch_fwd_finalize(P.mode, P.gc, P.b, P.ptr<float2>(P.o_part), P.fsp.n_chunks, info, sp, xh, s));
  } else if (P.image) {
    HIP_TRY(launch_spec_scatter(P.gc, P.b, reinterpret_cast<const float2*>(P.spec_in), xh, s));
  }
  if (P.image) DM_TRY(run_fft(h, P.fp->c2r, xh, P.image, P.ptr<char>(P.o_fftw), P.fp->work_c2r, s));
  if (P.want_vjp && P.dS) {
    double* dsp = P.ptr<double>(P.o_dsp);
    HIP_TRY(launch_dsig(P.gc, P.b, P.ptr<float2>(P.o_ghat), spectrum_of(P), dsp, P.adj_blocks, s));
    HIP_TRY(launch_dsig_final(dsp, P.adj_blocks, P.dS, s));
  }
  if (P.want_vjp && P.dV) {
    float* red = P.ptr<float>(P.o_red);
    HIP_TRY(launch_vjp_reduce(P.mode, P.ptr<float>(P.o_vpart), P.vsp.n_chunks, P.nt, P.ptr<float>(P.o_rtmp), red, s));
    double* R = P.ptr<double>(P.o_R);
    if (P.mode == DM_SURFACE) HIP_TRY(launch_surface_scalar(red, P.ptr<float>(P.o_rec), P.nt, info, R, s));
    HIP_TRY(launch_vertex_gather(P.mode, P.m->verts_dev, P.nv, P.m->topo->faces, P.m->topo->flags, P.m->topo->weights,
                                 P.nt, P.m->topo->csr_off,
                                 P.m->topo->csr_ent, red, R, P.dV, s));
  }
  return DM_OK;
}

dm_status render_impl(dm_handle* h, const dm_mesh* m, const dm_psf* psf, const dm_grid* g, float* image,
                      float* spec_out, const float* dLdI, float* dV, float* dS, const float* spec_in, hipStream_t s,
                      const float2* otf = nullptr) {
  CallScope call(h, s);
  DM_TRY(call.begin());
  ReqPlan P;
  P.m = m;
  P.g = *g;
  if (psf) P.psf = *psf;
  P.otf = otf;
  P.image = image;
  P.spec_out = spec_out;
  P.dLdI = dLdI;
  P.dV = dV;
  P.dS = dS;
  P.spec_in = spec_in;
  DM_TRY(plan_request(h, P, s, false));
  DM_TRY(ensure_ws(h, P.bytes));
  P.base = static_cast<char*>(h->ws);
  DM_TRY(stage_pre(h, P, s));
  DM_TRY(stage_sweeps(h, P, s));
  DM_TRY(stage_post(h, P, s));
  return call.end();
}

dm_status check_request(const dm_request& r, int i) {
  DM_TRY(check_grid(&r.grid));
  if (!r.otf_dev) DM_TRY(check_psf(&r.psf));
  DM_TRY(check_mesh(&r.mesh, r.grid.mode));
  if (!r.image_dev && !r.dL_dverts_dev && !r.dL_dsigma_dev) return fail(DM_ERR_ARG, "request %d: no output", i);
  if ((r.dL_dverts_dev || r.dL_dsigma_dev) && !r.dL_dimage_dev)
    return fail(DM_ERR_ARG, "request %d: gradients need dL_dimage", i);
  if (r.otf_dev && r.dL_dsigma_dev)
    return fail(DM_ERR_ARG, "request %d: no PSF gradient with a tabulated OTF", i);
  return DM_OK;
}

void fill_plan(ReqPlan& P, const dm_request& r) {
  P.m = &r.mesh;
  P.g = r.grid;
  P.psf = r.psf;
  P.dLdI = r.dL_dimage_dev;
  P.image = r.image_dev;
  P.dV = r.dL_dimage_dev ? r.dL_dverts_dev : nullptr;
  P.dS = r.dL_dimage_dev ? r.dL_dsigma_dev : nullptr;
  P.otf = static_cast<const float2*>(r.otf_dev);
}

// Device layout of a batch: request regions, then the sorted work list, the
// per-request sweep descriptors and the queue counter.
struct BatchLayout {
  std::vector<size_t> off;
  std::vector<SweepItem> items;   // grouped by (kind, mode), each group longest first
  std::vector<SweepReq> reqs;
  int group_end[BATCH_GROUPS] = {};
  // fused requests of the shared launch per density, in queue order (largest
  // tiles first), with their first tiles; the descriptors are filled in when
  // the batch's memory is known
  std::vector<int> fused_order[2], fused_tile0[2];
  int fused_tiles[2] = {0, 0};
  std::vector<SweepReq> fused_reqs[2];
  size_t o_fused[2] = {0, 0};
  size_t o_items = 0, o_reqs = 0, o_counter = 0, total = 0;
  double pairs = 0.0;
};

void layout_batch(std::vector<ReqPlan>& P, BatchLayout& L) {
  const size_t n = P.size();
  std::vector<SweepItem> items;
  std::vector<double> cost;
  L.off.assign(n, 0);
  L.total = 0;
  L.pairs = 0.0;
  for (size_t i = 0; i < n; ++i) {
    L.off[i] = L.total;
    L.total += align_up(P[i].bytes);
    add_items(P[i], (int)i, items, cost);
    if (!P[i].direct) L.pairs += (double)P[i].nE * P[i].nt;
  }
  std::vector<size_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  auto group = [&](size_t i) { return 2 * items[i].kind + P[(size_t)items[i].req].mode; };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    if (group(a) != group(b)) return group(a) < group(b);
    return cost[a] > cost[b];
  });
  L.items.resize(items.size());
  int count[BATCH_GROUPS] = {};
  for (size_t i = 0; i < order.size(); ++i) {
    L.items[i] = items[order[i]];
    count[group(order[i])]++;
  }
  for (int g = 0, acc = 0; g < BATCH_GROUPS; ++g) {
    acc += count[g];
    L.group_end[g] = acc;
  }
  for (int m = 0; m < 2; ++m) {
    std::vector<int>& ord = L.fused_order[m];
    ord.clear();
    L.fused_tile0[m].clear();
    for (size_t i = 0; i < n; ++i)
      if (P[i].fused && !P[i].direct && !P[i].empty && P[i].mode == m) ord.push_back((int)i);
    // largest tiles first (longest-processing-time order), then request order
    auto tile_pairs = [&](int i) { return (double)P[(size_t)i].vsp.per_chunk * P[(size_t)i].vsp.tpb; };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return tile_pairs(a) > tile_pairs(b); });
    int acc = 0;
    for (int i : ord) {
      L.fused_tile0[m].push_back(acc);
      acc += P[(size_t)i].vsp.n_chunks * P[(size_t)i].fsp.n_chunks;
    }
    L.fused_tiles[m] = acc;
    L.o_fused[m] = L.total;
    L.total += align_up(std::max<size_t>(1, ord.size()) * sizeof(SweepReq));
  }
  L.o_items = L.total;
  L.total += align_up(std::max<size_t>(1, L.items.size()) * sizeof(SweepItem));
  L.o_reqs = L.total;
  L.total += align_up(std::max<size_t>(1, n) * sizeof(SweepReq));
  L.o_counter = L.total;
  L.total += 256;
}

// The part of a batch after the pre-steps: the shared persistent launch and
// its requests' post-steps on s, then the large requests, alternating between
// s and s2 (the same stream when there is no second one).
template <typename Done, typename Fork, typename Join>
dm_status enqueue_batch_rest(dm_handle* h, std::vector<ReqPlan>& P, BatchLayout& L, char* base, hipStream_t s,
                             hipStream_t s2, Done& done, const std::vector<hipStream_t>& lanes, Fork& lanes_fork,
                             Join& lanes_join) {
  const size_t n = P.size();
  if (!L.items.empty() || L.fused_tiles[0] > 0 || L.fused_tiles[1] > 0) {
    if (!L.items.empty())
      HIP_TRY(hipMemcpyAsync(base + L.o_items, L.items.data(), L.items.size() * sizeof(SweepItem),
                             hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(base + L.o_reqs, L.reqs.data(), n * sizeof(SweepReq), hipMemcpyHostToDevice, s));
    const SweepReq* freqs[2];
    int n_freqs[2];
    for (int m = 0; m < 2; ++m) {
      freqs[m] = reinterpret_cast<const SweepReq*>(base + L.o_fused[m]);
      n_freqs[m] = (int)L.fused_reqs[m].size();
      if (n_freqs[m] > 0)
        HIP_TRY(hipMemcpyAsync(base + L.o_fused[m], L.fused_reqs[m].data(), L.fused_reqs[m].size() * sizeof(SweepReq),
                               hipMemcpyHostToDevice, s));
    }
    SweepTimer tm(h, s, 2, L.pairs);
    HIP_TRY(launch_batch_sweep(reinterpret_cast<const SweepItem*>(base + L.o_items), L.group_end,
                               reinterpret_cast<const SweepReq*>(base + L.o_reqs), freqs, n_freqs, L.fused_tiles,
                               reinterpret_cast<int*>(base + L.o_counter), s));
    tm.done();
  }
  DM_TRY(lanes_fork());
  // the post-steps of the shared launch's requests, spread over the lanes
  int j = 0;
  for (size_t i = 0; i < n; ++i)
    if (!P[i].direct) {
      const hipStream_t st = lanes[(size_t)(j++) % lanes.size()];
      DM_TRY(stage_post(h, P[i], st));
      DM_TRY(done(i, st));
    }
  DM_TRY(lanes_join());
  int k = 0;
  for (size_t i = 0; i < n; ++i)
    if (P[i].direct) {
      const hipStream_t st = (k++ & 1) ? s : s2;
      DM_TRY(stage_sweeps(h, P[i], st));
      DM_TRY(stage_post(h, P[i], st));
      DM_TRY(done(i, st));
    }
  return DM_OK;
}

// Enqueues a planned batch on s: every request's pre-steps, the shared
// persistent launch and the post-steps of the requests in it, then each large
// request's own sweeps and post-steps.  Large requests alternate between s
// and the second stream aux (forked after the pre-steps, joined back into s
// at the end), so one request's post-steps and the tail of its sweeps
// overlap the next one's sweeps; each request works in its own region of the
// batch memory, and its FFTs get its own work buffer.  With req_done, an
// event is recorded after each request's last step (req_done[i] for request
// i, on the stream that ran it), so that a caller can hand out results as
// they complete.
dm_status enqueue_batch(dm_handle* h, std::vector<ReqPlan>& P, BatchLayout& L, char* base, hipStream_t s,
                        AuxStream* aux, const std::vector<hipEvent_t>* req_done = nullptr) {
  const size_t n = P.size();
  L.reqs.resize(n);
  int n_direct = 0;
  for (size_t i = 0; i < n; ++i) {
    P[i].base = base + L.off[i];
    bind_band(P[i]);
    L.reqs[i] = sweep_req(P[i]);
    if (P[i].direct && !P[i].empty) ++n_direct;
  }
  for (int m = 0; m < 2; ++m) {
    L.fused_reqs[m].clear();
    for (size_t k = 0; k < L.fused_order[m].size(); ++k) {
      SweepReq q = L.reqs[(size_t)L.fused_order[m][k]];
      q.tile0 = L.fused_tile0[m][k];
      L.fused_reqs[m].push_back(q);
    }
  }
  auto done = [&](size_t i, hipStream_t st) -> dm_status {
    if (req_done && (*req_done)[i]) HIP_TRY(hipEventRecord((*req_done)[i], st));
    return DM_OK;
  };
  // The requests' small steps (pre-steps before the shared launch, post-steps
  // after it) do not fill the GPU one request at a time: they are dealt over
  // up to 1 + AUX_STREAMS lanes (s and aux streams forked from it, joined back
  // into s before the shared launch and after the post-steps).  Every request
  // works in its own region of the batch memory with its own FFT buffers, so
  // requests on different lanes share nothing but read-only inputs.
  const int n_aux = (int)std::min<size_t>(AUX_STREAMS, n > 0 ? n - 1 : 0);
  if (n_aux > 0 || n_direct >= 2) DM_TRY(ensure_aux(aux));
  std::vector<hipStream_t> lanes{s};
  for (int k = 0; k < n_aux; ++k) lanes.push_back(aux->s[k]);
  bool forked = false;
  auto lanes_fork = [&]() -> dm_status {
    DM_TRY(aux_fork(aux, n_aux, s));
    forked = n_aux > 0;
    return DM_OK;
  };
  auto lanes_join = [&]() -> dm_status {
    if (!forked) return DM_OK;
    forked = false;
    return aux_join(aux, n_aux, s);
  };
  dm_status st = lanes_fork();
  for (size_t i = 0; i < n && st == DM_OK; ++i) st = stage_pre(h, P[i], lanes[i % lanes.size()]);
  // join even after a failed enqueue, so that s never runs ahead of an aux stream
  const dm_status jst = lanes_join();
  if (st != DM_OK) return st;
  DM_TRY(jst);
  hipStream_t s2 = s;
  if (n_direct >= 2) {
    DM_TRY(aux_fork(aux, 1, s));
    s2 = aux->s[0];
  }
  st = enqueue_batch_rest(h, P, L, base, s, s2, done, lanes, lanes_fork, lanes_join);
  const dm_status jst2 = lanes_join();
  if (s2 != s) DM_TRY(aux_join(aux, 1, s));
  if (st != DM_OK) return st;
  return jst2;
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
  // the allocation-free entry point's scratch: its address on this device
  HIP_TRY(scratch_init(device));
  *out = h.release();
  return DM_OK;
}

dm_status dm_destroy(dm_handle* h) {
  g_err.clear();
  if (!h) return DM_OK;
  DeviceGuard dg(h->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : h->bands) (void)hipFree(kv.second.mem);
  if (h->otf_band.mem) (void)hipFree(h->otf_band.mem);
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
  destroy_aux(&h->aux);
  delete h;
  return DM_OK;
}

dm_status dm_timing_enable(dm_handle* h, int enable) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  h->timing = enable != 0;
  return DM_OK;
}

dm_status dm_timing_read(dm_handle* h, dm_kernel_time* fwd_sweep, dm_kernel_time* vjp_sweep,
                         dm_kernel_time* batch_sweep, dm_kernel_time* fused_sweep, int reset) {
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
  if (batch_sweep) *batch_sweep = h->acc[2];
  if (fused_sweep) *fused_sweep = h->acc[3];
  if (reset) h->acc[0] = h->acc[1] = h->acc[2] = h->acc[3] = dm_kernel_time{0, 0.0, 0.0};
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
  TopoTables T;
  const Check c = build_topology(F, n_verts, &T);
  if (c.st != DM_OK) return fail(c.st, "%s", c.msg.c_str());
  auto t = std::make_unique<dm_topology>();
  t->h = h;
  t->nt = n_faces;
  t->nv = n_verts;
  t->closed = T.closed ? 1 : 0;
  t->closed_plain = t->closed;
  t->n_strips = T.n_strips;
  t->lap_mu = T.lap_mu;
  t->faces_in.swap(F);
  t->src.swap(T.src);
  const std::vector<int32_t>& Fs = T.faces;
  const size_t bf = align_up(Fs.size() * 4), bo = align_up(T.csr_off.size() * 4), be = align_up(T.csr_ent.size() * 4),
               bl = align_up(T.flags.size() * 4), bao = align_up(T.adj_off.size() * 4),
               ban = align_up(T.adj_nbr.size() * 4), bat = align_up(T.adj_tab.size() * 4);
  void* mem = nullptr;
  DM_TRY(dev_alloc(h, &mem, bf + bo + be + bl + bao + ban + bat));
  t->bytes = bf + bo + be + bl + bao + ban + bat;
  char* base = static_cast<char*>(mem);
  t->faces = reinterpret_cast<int32_t*>(base);
  t->csr_off = reinterpret_cast<int32_t*>(base + bf);
  t->csr_ent = reinterpret_cast<int32_t*>(base + bf + bo);
  t->flags = reinterpret_cast<int32_t*>(base + bf + bo + be);
  t->adj_off = reinterpret_cast<int32_t*>(base + bf + bo + be + bl);
  t->adj_nbr = reinterpret_cast<int32_t*>(base + bf + bo + be + bl + bao);
  t->adj_tab = T.adj_tab.empty() ? nullptr : reinterpret_cast<int32_t*>(base + bf + bo + be + bl + bao + ban);
  hipError_t err = hipSuccess;
  auto up = [&](int32_t* dst, const std::vector<int32_t>& v) {
    if (err == hipSuccess && !v.empty()) err = hipMemcpy(dst, v.data(), v.size() * 4, hipMemcpyHostToDevice);
  };
  up(t->faces, Fs);
  up(t->csr_off, T.csr_off);
  up(t->csr_ent, T.csr_ent);
  up(t->flags, T.flags);
  up(t->adj_off, T.adj_off);
  up(t->adj_nbr, T.adj_nbr);
  if (t->adj_tab) up(t->adj_tab, T.adj_tab);
  if (err != hipSuccess) {
    dev_free(h, mem, t->bytes);
    return fail(DM_ERR_DEVICE, "topology upload: %s", hipGetErrorString(err));
  }
  h->topo_count++;
  *out = t.release();
  return DM_OK;
}

dm_status dm_topology_strips(const int32_t* faces, int32_t n_faces, int32_t* faces_out, int32_t* flags_out,
                             int32_t* n_strips) {
  g_err.clear();
  if (n_faces < 0) return fail(DM_ERR_ARG, "negative face count");
  if (n_faces > 0 && (!faces || !faces_out || !flags_out)) return fail(DM_ERR_ARG, "NULL array");
  if ((int64_t)n_faces * 3 >= ((int64_t)1 << 31)) return fail(DM_ERR_ARG, "too many faces");
  std::vector<int32_t> F(faces, faces + (size_t)n_faces * 3), Fs, fl;
  const int ns = build_strips(F, Fs, fl);
  if (n_faces > 0) {
    memcpy(faces_out, Fs.data(), Fs.size() * sizeof(int32_t));
    memcpy(flags_out, fl.data(), fl.size() * sizeof(int32_t));
  }
  if (n_strips) *n_strips = ns;
  return DM_OK;
}

dm_status dm_topology_destroy(dm_topology* t) {
  g_err.clear();
  if (!t) return DM_OK;
  DeviceGuard dg(t->h->device);
  (void)hipDeviceSynchronize();
  dev_free(t->h, t->faces, t->bytes);
  dev_free(t->h, t->smooth_ws, t->smooth_bytes);
  dev_free(t->h, t->weights, align_up((size_t)t->nt * 4));
  t->h->topo_count--;
  delete t;
  return DM_OK;
}

dm_status dm_laplace_smooth(dm_handle* h, dm_topology* t, float lambda, const float* grad, float* out,
                            int32_t max_iter, float tol, float* info, void* stream) {
  g_err.clear();
  if (!h || !t || !grad || !out) return fail(DM_ERR_ARG, "NULL argument");
  if (t->h != h) return fail(DM_ERR_ARG, "topology belongs to another handle");
  if (!(lambda >= 0.0f) || !std::isfinite(lambda)) return fail(DM_ERR_ARG, "lambda must be finite and >= 0");
  if (max_iter < 1) return fail(DM_ERR_ARG, "max_iter must be at least 1");
  if (!(tol > 0.0f)) return fail(DM_ERR_ARG, "tol must be > 0");
  if (t->nv == 0) return DM_OK;
  DeviceGuard dg(h->device);
  const size_t need = laplace_smooth_workspace(t->nv);
  if (t->smooth_bytes < need) {
    void* mem = nullptr;
    DM_TRY(dev_alloc(h, &mem, need));
    dev_free(h, t->smooth_ws, t->smooth_bytes);
    t->smooth_ws = static_cast<float*>(mem);
    t->smooth_bytes = need;
  }
  HIP_TRY(launch_laplace_smooth(t->nv, t->adj_off, t->adj_nbr, t->adj_tab, t->lap_mu, lambda, grad, out,
                                t->smooth_ws, max_iter, tol, info, static_cast<hipStream_t>(stream)));
  return DM_OK;
}

dm_status dm_topology_set_weights(dm_topology* t, const float* weights) {
  g_err.clear();
  if (!t) return fail(DM_ERR_ARG, "topology is NULL");
  DeviceGuard dg(t->h->device);
  if (!weights) {
    (void)hipDeviceSynchronize();
    dev_free(t->h, t->weights, align_up((size_t)t->nt * 4));
    t->weights = nullptr;
    t->closed = t->closed_plain;
    return DM_OK;
  }
  bool closed = false;
  const Check c = weights_close(t->faces_in, weights, t->nt, &closed);
  if (c.st != DM_OK) return fail(c.st, "%s", c.msg.c_str());
  std::vector<float> ws((size_t)t->nt);
  for (int i = 0; i < t->nt; ++i) ws[(size_t)i] = weights[t->src[(size_t)i]];
  if (!t->weights) {
    void* mem = nullptr;
    DM_TRY(dev_alloc(t->h, &mem, align_up((size_t)t->nt * 4)));
    t->weights = static_cast<float*>(mem);
  }
  (void)hipDeviceSynchronize();
  if (t->nt > 0) HIP_TRY(hipMemcpy(t->weights, ws.data(), ws.size() * 4, hipMemcpyHostToDevice));
  t->closed = closed ? 1 : 0;
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
  CallScope call(h, s);
  DM_TRY(call.begin());
  BandDev b;
  DM_TRY(get_band(h, g, psf, s, &b));
  DM_TRY(call.end());
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
  CallScope call(h, s);
  DM_TRY(call.begin());
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
  DM_TRY(call.end());
  return DM_OK;
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

dm_status dm_render_otf(dm_handle* h, const dm_mesh* mesh, const void* otf_dev, const dm_grid* g, float* image_dev,
                        void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_mesh(mesh, g->mode));
  if (!otf_dev) return fail(DM_ERR_ARG, "otf is NULL");
  if (!image_dev) return fail(DM_ERR_ARG, "no output requested");
  DeviceGuard dg(h->device);
  return render_impl(h, mesh, nullptr, g, image_dev, nullptr, nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream,
                     static_cast<const float2*>(otf_dev));
}

dm_status dm_render_otf_vjp(dm_handle* h, const dm_mesh* mesh, const void* otf_dev, const dm_grid* g,
                            const float* dL_dimage_dev, float* dL_dverts_dev, float* image_dev, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_mesh(mesh, g->mode));
  if (!otf_dev) return fail(DM_ERR_ARG, "otf is NULL");
  if (!dL_dimage_dev) return fail(DM_ERR_ARG, "dL_dimage is NULL");
  if (!dL_dverts_dev && !image_dev) return fail(DM_ERR_ARG, "no output requested");
  DeviceGuard dg(h->device);
  return render_impl(h, mesh, nullptr, g, image_dev, nullptr, dL_dimage_dev, dL_dverts_dev, nullptr, nullptr,
                     (hipStream_t)stream, static_cast<const float2*>(otf_dev));
}

dm_status dm_batch_run(dm_handle* h, int32_t n, const dm_request* reqs, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  if (n < 0 || (n > 0 && !reqs)) return fail(DM_ERR_ARG, "bad request list");
  for (int i = 0; i < n; ++i) DM_TRY(check_request(reqs[i], i));
  if (n == 0) return DM_OK;
  DeviceGuard dg(h->device);
  hipStream_t s = (hipStream_t)stream;
  CallScope call(h, s);
  DM_TRY(call.begin());
  std::vector<ReqPlan> P((size_t)n);
  dm_status st = DM_OK;
  for (int i = 0; i < n && st == DM_OK; ++i) {
    fill_plan(P[i], reqs[i]);
    st = plan_request(h, P[i], s, true);
  }
  BatchLayout L;
  if (st == DM_OK) {
    layout_batch(P, L);
    st = ensure_ws(h, L.total);
  }
  if (st == DM_OK) st = enqueue_batch(h, P, L, static_cast<char*>(h->ws), s, &h->aux);
  for (auto& pl : P) release_band(h, pl);
  if (st != DM_OK) return st;
  return call.end();
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
  CallScope call(h, s);
  DM_TRY(call.begin());
  if (nt == 0) {
    DM_TRY(zero_fill(out_dev, 2 * n, s));
    return call.end();
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
  HIP_TRY(launch_mesh_prep(mode, gc, mesh->verts_dev, mesh->n_verts, mesh->topo->faces, mesh->topo->flags,
                           mesh->topo->weights, nt, rec, info,
                           at<double>(h, o_ptmp), prep_blocks, s));
  float4* kf = at<float4>(h, o_kf);
  HIP_TRY(launch_points_prepare(gc, k_dev, n, kf, s));
  float2* part = at<float2>(h, o_part);
  SweepTimer tm(h, s, 0, (double)n * nt);
  HIP_TRY(launch_fwd_lanes(mode, kf, n, rec, nt, sp.per_chunk, sp.n_chunks, part, s));
  tm.done();
  HIP_TRY(launch_points_finalize(mode, gc, kf, n, part, sp.n_chunks, info, reinterpret_cast<float2*>(out_dev), s));
  return call.end();
}

dm_status dm_mesh_transform_noalloc(dm_handle* h, const dm_mesh* mesh, const dm_grid* g, const int32_t* k_dev,
                                    int64_t n, float* out_dev, void* stream) {
  g_err.clear();
  if (!h) return fail(DM_ERR_ARG, "NULL handle");
  DM_TRY(check_grid(g));
  DM_TRY(check_mesh(mesh, g->mode));
  if (n < 0 || (n > 0 && (!k_dev || !out_dev))) return fail(DM_ERR_ARG, "bad frequency list");
  if (n >= ((int64_t)1 << 31)) return fail(DM_ERR_ARG, "too many frequencies");
  if (n == 0) return DM_OK;
  DeviceGuard dg(h->device);
  char* base = static_cast<char*>(scratch_ptr(h->device));
  if (!base) return fail(DM_ERR_DEVICE, "scratch of device %d not resolved", h->device);
  hipStream_t s = (hipStream_t)stream;
  const int mode = g->mode;
  const GridC gc = make_gridc(g);
  const int nt = mesh->topo->nt;
  // the same triangle chunking as dm_mesh_transform when it fits, else fewer chunks
  SweepPlan sp = plan_fwd(n, nt);
  const int prep_blocks = mesh_prep_blocks(nt);
  size_t o_rec = 0, o_info = 0, o_ptmp = 0, o_kf = 0, o_part = 0, need = 0;
  for (;;) {
    Carver cv;
    o_rec = cv.take<float>((size_t)std::max(nt, 1) * TRI_REC);
    o_info = cv.take<MeshInfo>(1);
    o_ptmp = cv.take<double>(2 * (size_t)prep_blocks);
    o_kf = cv.take<float4>(n);
    o_part = cv.take<float2>((size_t)sp.n_chunks * n);
    need = cv.off;
    if (need <= DM_NOALLOC_SCRATCH_BYTES || sp.n_chunks == 1) break;
    const int64_t fixed = (int64_t)o_part;
    const int64_t fit = ((int64_t)DM_NOALLOC_SCRATCH_BYTES - fixed) / (8 * n);
    const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(sp.n_chunks - 1, fit));
    sp.per_chunk = std::max(1, (nt + chunks - 1) / chunks);
    sp.n_chunks = std::max(1, (nt + sp.per_chunk - 1) / sp.per_chunk);
  }
  if (need > DM_NOALLOC_SCRATCH_BYTES)
    return fail(DM_ERR_BUDGET, "%d triangles and %lld frequencies need %zu bytes of scratch; it holds %zu", nt,
                (long long)n, need, (size_t)DM_NOALLOC_SCRATCH_BYTES);
  CallScope call(h, s);
  DM_TRY(call.begin());
  if (nt == 0) {
    DM_TRY(zero_fill(out_dev, 2 * n, s));
    return call.end();
  }
  float* rec = reinterpret_cast<float*>(base + o_rec);
  MeshInfo* info = reinterpret_cast<MeshInfo*>(base + o_info);
  HIP_TRY(launch_mesh_prep(mode, gc, mesh->verts_dev, mesh->n_verts, mesh->topo->faces, mesh->topo->flags,
                           mesh->topo->weights, nt, rec, info, reinterpret_cast<double*>(base + o_ptmp), prep_blocks,
                           s));
  float4* kf = reinterpret_cast<float4*>(base + o_kf);
  HIP_TRY(launch_points_prepare(gc, k_dev, n, kf, s));
  float2* part = reinterpret_cast<float2*>(base + o_part);
  HIP_TRY(launch_fwd_lanes(mode, kf, n, rec, nt, sp.per_chunk, sp.n_chunks, part, s));
  HIP_TRY(launch_points_finalize(mode, gc, kf, n, part, sp.n_chunks, info, reinterpret_cast<float2*>(out_dev), s));
  return call.end();
}

}  // extern "C"

// =============================================================== serving
namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct ResidentMesh {
  float* verts = nullptr;
  int32_t nv = 0;
  dm_topology* topo = nullptr;
  int pending = 0;
};

struct ServeReq {
  dm_serve_request r{};
  dm_request req{};       // expanded form handed to the batch engine
  dm_status status = DM_ERR_BUSY;   // DM_ERR_BUSY while pending
  int32_t batch = 0;
  double t_submit = 0.0, t_launch = 0.0, t_done = 0.0;
  bool large = false;     // planned once: runs its own sweep launches
};

struct Inflight {
  std::vector<uint64_t> tickets;
  std::vector<hipEvent_t> req_ev;   // per ticket: its outputs are complete
  std::vector<char> finished;       // per ticket: already handed out
  hipEvent_t ev = nullptr;          // the whole batch (slot and memory free)
  size_t bytes = 0;
  int slot = 0;
  void* mem = nullptr;    // fallback allocation when the stream-ordered pool is unavailable
  bool solo = false;      // holds a request that runs its own sweep launches
};

}  // namespace

struct dm_server {
  dm_handle* h = nullptr;
  dm_server_config cfg{};
  bool pools = true;
  std::vector<hipStream_t> streams;
  std::vector<AuxStream> aux;              // each slot's second stream (large requests)
  std::vector<bool> busy;
  std::vector<hipEvent_t> event_pool;
  std::mutex hmu;                          // serialises use of the handle
  std::mutex mu;                           // queue, requests, in-flight list, stats
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, ServeReq> reqs;
  std::unordered_map<int32_t, ResidentMesh> meshes;
  std::vector<Inflight> inflight;
  size_t inflight_bytes = 0;
  uint64_t next_ticket = 1;
  int32_t next_mesh = 1;
  bool stop = false;
  dm_server_stats stats{};
  std::thread worker;
};

namespace {

void finish_locked(dm_server* S, uint64_t t, dm_status st, int32_t batch) {
  auto it = S->reqs.find(t);
  if (it == S->reqs.end()) return;
  it->second.status = st;
  it->second.batch = batch;
  it->second.t_done = now_ms();
  auto m = S->meshes.find(it->second.r.mesh_id);
  if (m != S->meshes.end()) m->second.pending--;
  if (st == DM_OK)
    S->stats.completed++;
  else
    S->stats.rejected++;
}

// Hands out finished requests and retires finished batches (mu held).
void retire_locked(dm_server* S) {
  bool any = false;
  for (size_t i = 0; i < S->inflight.size();) {
    Inflight& b = S->inflight[i];
    for (size_t k = 0; k < b.tickets.size(); ++k) {
      if (b.finished[k] || !b.req_ev[k]) continue;
      const hipError_t qk = hipEventQuery(b.req_ev[k]);
      if (qk == hipErrorNotReady) continue;
      finish_locked(S, b.tickets[k], qk == hipSuccess ? DM_OK : DM_ERR_DEVICE, (int32_t)b.tickets.size());
      b.finished[k] = 1;
      any = true;
    }
    const hipError_t q = hipEventQuery(b.ev);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    const dm_status st = q == hipSuccess ? DM_OK : DM_ERR_DEVICE;
    for (size_t k = 0; k < b.tickets.size(); ++k)
      if (!b.finished[k]) finish_locked(S, b.tickets[k], st, (int32_t)b.tickets.size());
    if (b.mem) (void)hipFree(b.mem);
    S->event_pool.push_back(b.ev);
    for (hipEvent_t e : b.req_ev)
      if (e) S->event_pool.push_back(e);
    S->busy[b.slot] = false;
    S->inflight_bytes -= std::min(S->inflight_bytes, b.bytes);
    S->inflight.erase(S->inflight.begin() + (long)i);
    any = true;
  }
  if (any) S->cv_done.notify_all();
}

// Plans and launches one batch from `take` on stream slot `slot`.  Requests
// that do not fit the budget next to the in-flight batches go back to the
// front of the queue.  Unless there is a backlog, a large request runs in a
// batch of its own on an idle device: one first in `take` on an idle device
// is launched alone, otherwise the batch ends before it; what follows it in
// `take` goes back.
size_t launch_batch(dm_server* S, int slot, std::vector<uint64_t> take, bool idle, bool backlog) {
  hipStream_t s = S->streams[(size_t)slot];
  std::vector<ReqPlan> P;
  std::vector<uint64_t> ids;
  std::vector<uint64_t> back;
  std::vector<std::pair<uint64_t, dm_status>> failed;
  size_t used = 0, inflight_bytes;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    inflight_bytes = S->inflight_bytes;
  }
  std::lock_guard<std::mutex> hl(S->hmu);
  dm_handle* h = S->h;
  const size_t budget = S->cfg.hbm_budget_bytes;
  P.reserve(take.size());
  for (size_t i = 0; i < take.size(); ++i) {
    const dm_request* rq;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      rq = &S->reqs[take[i]].req;
    }
    ReqPlan pl;
    fill_plan(pl, *rq);
    dm_status st = plan_request(h, pl, s, true, BATCH_DIRECT_PAIRS);
    if (st != DM_OK) {
      failed.push_back({take[i], st});
      continue;
    }
    bool last = false;
    if (pl.direct) {
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->reqs[take[i]].large = true;
      }
      if (!backlog) {
        if (!idle || !P.empty()) {
          release_band(h, pl);
          back.assign(take.begin() + (long)i, take.end());
          break;
        }
        last = true;
      }
    }
    const size_t need = align_up(pl.bytes) + 4096;
    if (budget && need > budget) {
      release_band(h, pl);
      failed.push_back({take[i], DM_ERR_BUDGET});
      continue;
    }
    if (budget && inflight_bytes + used + need > budget && !P.empty()) {
      release_band(h, pl);
      back.assign(take.begin() + (long)i, take.end());
      break;
    }
    if (budget && inflight_bytes + used + need > budget) {   // wait for memory to free up
      release_band(h, pl);
      back.assign(take.begin() + (long)i, take.end());
      break;
    }
    used += need;
    P.push_back(pl);
    ids.push_back(take[i]);
    if (last) {
      back.assign(take.begin() + (long)i + 1, take.end());
      break;
    }
  }
  Inflight b;
  dm_status st = DM_OK;
  if (!P.empty()) {
    BatchLayout L;
    layout_batch(P, L);
    b.bytes = L.total;
    // one completion event per request (events come from the server's pool)
    {
      std::lock_guard<std::mutex> lk(S->mu);
      b.req_ev.assign(P.size(), nullptr);
      for (size_t i = 0; i < P.size(); ++i) {
        if (S->event_pool.empty()) {
          hipEvent_t ev;
          if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) S->event_pool.push_back(ev);
        }
        if (!S->event_pool.empty()) {
          b.req_ev[i] = S->event_pool.back();
          S->event_pool.pop_back();
        }
      }
      b.finished.assign(P.size(), 0);
    }
    void* mem = nullptr;
    hipError_t e = S->pools ? hipMallocAsync(&mem, L.total, s) : hipMalloc(&mem, L.total);
    if (e != hipSuccess) st = fail(DM_ERR_DEVICE, "workspace allocation: %s", hipGetErrorString(e));
    if (st == DM_OK) st = enqueue_batch(h, P, L, static_cast<char*>(mem), s, &S->aux[(size_t)slot], &b.req_ev);
    if (S->pools && mem) (void)hipFreeAsync(mem, s);
    if (!S->pools) b.mem = mem;
    if (S->event_pool.empty()) {
      hipEvent_t ev;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) S->event_pool.push_back(ev);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->event_pool.empty()) {
      b.ev = S->event_pool.back();
      S->event_pool.pop_back();
    }
    if (st == DM_OK && b.ev) st = hipEventRecord(b.ev, s) == hipSuccess ? DM_OK : DM_ERR_DEVICE;
    for (auto& pl : P) release_band(h, pl);
    const double t = now_ms();
    if (st == DM_OK && b.ev) {
      b.tickets = ids;
      b.slot = slot;
      for (const auto& pl : P) b.solo = b.solo || pl.direct;
      for (uint64_t id : ids) S->reqs[id].t_launch = t;
      S->inflight.push_back(b);
      S->busy[(size_t)slot] = true;
      S->inflight_bytes += b.bytes;
      S->stats.peak_inflight_bytes = std::max(S->stats.peak_inflight_bytes, S->inflight_bytes);
      S->stats.batches++;
    } else {
      if (b.ev) S->event_pool.push_back(b.ev);
      for (hipEvent_t ev : b.req_ev)
        if (ev) S->event_pool.push_back(ev);
      if (b.mem) (void)hipFree(b.mem);
      for (uint64_t id : ids) finish_locked(S, id, st == DM_OK ? DM_ERR_DEVICE : st, (int32_t)ids.size());
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& f : failed) finish_locked(S, f.first, f.second, 0);
  for (auto it = back.rbegin(); it != back.rend(); ++it) S->queue.push_front(*it);
  if (!failed.empty() || st != DM_OK) S->cv_done.notify_all();
  return P.size() + failed.size();
}

void serve_loop(dm_server* S) {
  (void)hipSetDevice(S->h->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    retire_locked(S);
    if (S->stop && S->queue.empty() && S->inflight.empty()) break;
    int slot = -1;
    for (size_t i = 0; i < S->busy.size(); ++i)
      if (!S->busy[i]) {
        slot = (int)i;
        break;
      }
    const bool mem_free = !S->cfg.hbm_budget_bytes || S->inflight.empty() ||
                          S->inflight_bytes < S->cfg.hbm_budget_bytes;
    // Large requests (their own sweep launches) run alone unless a backlog of
    // a full batch has built up: nothing new starts beside one, and one starts
    // only on an idle device.  Work sharing the compute units with a large
    // request stretches the longest latencies, and a large request started
    // beside a batch stretches that batch; requests that wait are batched
    // afterwards.
    bool solo = false;
    for (const Inflight& b : S->inflight) solo = solo || b.solo;
    const bool backlog = (int)S->queue.size() >= S->cfg.max_batch;
    const bool idle = S->inflight.empty();
    bool head_large = false;
    if (!S->queue.empty()) {
      auto it = S->reqs.find(S->queue.front());
      head_large = it != S->reqs.end() && it->second.large;
    }
    if (slot >= 0 && !S->queue.empty() && mem_free && (!solo || backlog) && (!head_large || idle || backlog)) {
      std::vector<uint64_t> take;
      while ((int)take.size() < S->cfg.max_batch && !S->queue.empty()) {
        take.push_back(S->queue.front());
        S->queue.pop_front();
      }
      lk.unlock();
      const size_t handled = launch_batch(S, slot, std::move(take), idle, backlog);
      lk.lock();
      // nothing fitted next to the in-flight work: wait for a batch to finish
      if (handled == 0) S->cv_work.wait_for(lk, std::chrono::microseconds(20));
      continue;
    }
    if (S->inflight.empty())
      S->cv_work.wait(lk);
    else
      S->cv_work.wait_for(lk, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

dm_status dm_server_create(int device, const dm_server_config* cfg, dm_server** out) {
  g_err.clear();
  if (!cfg || !out) return fail(DM_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_inflight > 8 || cfg->queue_capacity < 1)
    return fail(DM_ERR_ARG, "bad server configuration");
  dm_handle* h = nullptr;
  DM_TRY(dm_create(&h, device, 0));
  auto S = std::make_unique<dm_server>();
  S->h = h;
  S->cfg = *cfg;
  DeviceGuard dg(device);
  int pools = 0;
  if (hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device) != hipSuccess) pools = 0;
  S->pools = pools != 0;
  for (int i = 0; i < cfg->max_inflight; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
      dm_destroy(h);
      return fail(DM_ERR_DEVICE, "stream creation failed");
    }
    S->streams.push_back(st);
    S->aux.push_back(AuxStream{});
    S->busy.push_back(false);
  }
  dm_server* raw = S.release();
  raw->worker = std::thread(serve_loop, raw);
  *out = raw;
  return DM_OK;
}

dm_status dm_server_destroy(dm_server* S) {
  g_err.clear();
  if (!S) return DM_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  {
    DeviceGuard dg(S->h->device);
    (void)hipDeviceSynchronize();
    for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
    for (AuxStream& a : S->aux) destroy_aux(&a);
    for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
    for (auto& kv : S->meshes) {
      dm_topology_destroy(kv.second.topo);
      (void)hipFree(kv.second.verts);
    }
  }
  dm_destroy(S->h);
  delete S;
  return DM_OK;
}

dm_status dm_server_mesh_add(dm_server* S, const float* verts_host, int32_t n_verts, const int32_t* faces_host,
                             int32_t n_faces, int32_t* mesh_id) {
  g_err.clear();
  if (!S || !mesh_id || (n_verts > 0 && !verts_host)) return fail(DM_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> hl(S->hmu);
  DeviceGuard dg(S->h->device);
  ResidentMesh m;
  m.nv = n_verts;
  DM_TRY(dm_topology_create(S->h, faces_host, n_faces, n_verts, 0, &m.topo));
  hipError_t e = hipMalloc(&m.verts, std::max<size_t>(4, (size_t)n_verts * 3 * sizeof(float)));
  if (e == hipSuccess && n_verts > 0)
    e = hipMemcpy(m.verts, verts_host, (size_t)n_verts * 3 * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dm_topology_destroy(m.topo);
    if (m.verts) (void)hipFree(m.verts);
    return fail(DM_ERR_DEVICE, "mesh upload: %s", hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(S->mu);
  *mesh_id = S->next_mesh++;
  S->meshes[*mesh_id] = m;
  return DM_OK;
}

dm_status dm_server_mesh_remove(dm_server* S, int32_t mesh_id) {
  g_err.clear();
  if (!S) return fail(DM_ERR_ARG, "NULL server");
  ResidentMesh m;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->meshes.find(mesh_id);
    if (it == S->meshes.end()) return fail(DM_ERR_STATE, "unknown mesh %d", mesh_id);
    if (it->second.pending > 0) return fail(DM_ERR_STATE, "mesh %d has pending requests", mesh_id);
    m = it->second;
    S->meshes.erase(it);
  }
  std::lock_guard<std::mutex> hl(S->hmu);
  DeviceGuard dg(S->h->device);
  dm_topology_destroy(m.topo);
  (void)hipFree(m.verts);
  return DM_OK;
}

dm_status dm_submit(dm_server* S, const dm_serve_request* r, uint64_t* ticket) {
  g_err.clear();
  if (!S || !r || !ticket) return fail(DM_ERR_ARG, "NULL argument");
  DM_TRY(check_grid(&r->grid));
  if (!r->otf_dev) DM_TRY(check_psf(&r->psf));
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->stop) return fail(DM_ERR_STATE, "server is shutting down");
  auto it = S->meshes.find(r->mesh_id);
  if (it == S->meshes.end()) return fail(DM_ERR_ARG, "unknown mesh %d", r->mesh_id);
  ServeReq q;
  q.r = *r;
  q.req.mesh.verts_dev = it->second.verts;
  q.req.mesh.n_verts = it->second.nv;
  q.req.mesh.topo = it->second.topo;
  q.req.psf = r->psf;
  q.req.grid = r->grid;
  q.req.dL_dimage_dev = r->dL_dimage_dev;
  q.req.image_dev = r->image_dev;
  q.req.dL_dverts_dev = r->dL_dverts_dev;
  q.req.dL_dsigma_dev = r->dL_dsigma_dev;
  q.req.otf_dev = r->otf_dev;
  DM_TRY(check_request(q.req, 0));
  if ((int)S->queue.size() >= S->cfg.queue_capacity) return fail(DM_ERR_BUSY, "queue full");
  q.t_submit = now_ms();
  const uint64_t t = S->next_ticket++;
  S->reqs[t] = q;
  it->second.pending++;
  S->queue.push_back(t);
  S->stats.submitted++;
  *ticket = t;
  lk.unlock();
  S->cv_work.notify_one();
  return DM_OK;
}

dm_status dm_poll(dm_server* S, uint64_t ticket, int blocking, dm_serve_result* out) {
  g_err.clear();
  if (!S) return fail(DM_ERR_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(DM_ERR_STATE, "unknown ticket");
  while (it->second.status == DM_ERR_BUSY) {
    if (!blocking) return DM_ERR_BUSY;
    S->cv_done.wait(lk);
    it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(DM_ERR_STATE, "ticket vanished");
  }
  if (out) {
    out->status = it->second.status;
    out->batch_size = it->second.batch;
    out->queue_ms = it->second.t_launch > 0 ? it->second.t_launch - it->second.t_submit : 0.0;
    out->total_ms = it->second.t_done - it->second.t_submit;
  }
  S->reqs.erase(it);
  return DM_OK;
}

dm_status dm_server_stats_read(dm_server* S, dm_server_stats* out) {
  if (!S || !out) return fail(DM_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->mean_batch = S->stats.batches ? (double)(S->stats.completed) / (double)S->stats.batches : 0.0;
  return DM_OK;
}

}  // extern "C"
