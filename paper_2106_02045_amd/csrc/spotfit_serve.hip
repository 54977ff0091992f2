// spotfit_serve.hip -- real-time serving loop for camera frames of fiducial
// spots (the paper's use: tracking markers at hundreds to thousands of frames
// per second for sample stabilisation, Introduction).
//
// A frame is submitted from host memory and copied into pinned staging rings;
// it is admitted only if the device-memory budget (pixel ring + per-spot ring)
// and a frame slot have room, otherwise submit returns SPOTFIT_E_AGAIN.  A
// dispatcher thread continuously folds every admitted frame into the next
// launch (continuous batching): copy in, fit, copy out on one of several
// streams, each with its own context, so batches overlap on the device.  When a
// batch's event completes its results are copied to the callers' host arrays
// and the frames' ring space is released (oldest first).  Latency is measured
// from the frame's arrival (submit time, or the scheduled arrival in replay) to
// the moment its results are in the caller's arrays.
//
// Drift tracking (optional): after a launch's fit, the drift pass of its
// tracked frames runs on the same stream (spotfit_track.hip), chained behind
// the previous launch's pass by an event so the history is written in
// submission order; its per-frame records come back with the fit results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "spotfit_track.h"

namespace {

using Clock = std::chrono::steady_clock;

inline uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             Clock::now().time_since_epoch())
      .count();
}

enum FrameState : int { kFree = 0, kAdmitted = 1, kLaunched = 2, kDone = 3, kFailed = 4 };

struct FrameRec {
  uint64_t ticket = 0;
  int state = kFree;
  int dtype = 0;
  bool dev_init = false;   // start values computed on the device
  int64_t n = 0;           // spots
  int64_t spot0 = 0;       // first index in the spot ring
  int64_t pix_off = 0;     // byte offset in the pixel ring
  int64_t pix_bytes = 0;   // bytes reserved in the pixel ring (incl. skipped tail)
  int64_t pix_alloc = 0;   // aligned bytes of the frame's pixels and records
  int64_t meta_off = 0;    // byte offset in the pixel ring of the frame's records
  int64_t spot_res = 0;    // spots reserved in the spot ring (incl. skipped tail)
  uint64_t t_arrival = 0;  // ns
  uint64_t t_done = 0;
  float* params = nullptr;
  float* chi2 = nullptr;
  int32_t* iters = nullptr;
  int32_t* status = nullptr;
  int64_t track_q = -1;               // sequence number among tracked frames, or -1
  spotfit_drift_t* drift = nullptr;   // caller's record for a tracked frame
};

struct Batch {
  int stream = 0;
  hipEvent_t ev = nullptr;
  uint64_t first_ticket = 0;  // frames [first_ticket, first_ticket + n_frames)
  int n_frames = 0;
  int64_t spot0 = 0, n_spots = 0;
  int n_tracked = 0;  // tracked frames of the batch, in ticket order
  bool failed = false;
};

}  // namespace

struct spotfit_serve {
  int device = 0;
  spotfit_options_t opt{};
  int n_streams = 0;
  std::vector<hipStream_t> streams;
  std::vector<spotfit_ctx_t*> ctxs;
  std::vector<bool> stream_busy;

  // rings indexed by spot position: pixels (bytes, device and pinned host
  // mirror); per-spot records staged on the host as frames arrive (h_sizes,
  // h_offs, h_init); a batch's records packed into its slice of the meta ring,
  // kMetaBytes per spot (offsets, shapes, start values: one copy in), and its
  // results into its slice of the result ring, kResBytes per spot (params, chi2,
  // iterations, status: one copy out)
  static constexpr int64_t kMetaBytes = 32, kResBytes = 36;
  int64_t pix_cap = 0, spot_cap = 0;
  unsigned char* d_pix = nullptr;
  unsigned char* h_pix = nullptr;
  spotfit_shape_t* h_sizes = nullptr;
  int64_t* h_offs = nullptr;
  float* h_init = nullptr;
  unsigned char *d_meta = nullptr, *h_meta = nullptr;
  unsigned char *d_res = nullptr, *h_res = nullptr;
  int64_t pix_head = 0, pix_used = 0, spot_head = 0, spot_used = 0;

  // frame slots, FIFO by ticket
  int max_frames = 0;
  std::vector<FrameRec> frames;
  uint64_t next_ticket = 1;   // next ticket to hand out
  uint64_t oldest_ticket = 1; // oldest ticket still holding ring space
  uint64_t next_launch = 1;   // oldest admitted ticket not yet launched

  std::deque<Batch> inflight;
  std::vector<hipEvent_t> event_pool;  // completion events, reused
  std::mutex mu;
  std::condition_variable cv_done;
  std::thread worker;
  std::atomic<bool> stop{false};
  // tickets below this are admitted: the dispatcher polls it without the lock
  std::atomic<uint64_t> admitted_end{1};

  // drift tracking: reference positions and history ring on the device; per
  // stream, staging for one batch's tracked frames and their drift records
  int track_markers = 0, track_window = 0;
  int64_t track_next = 0;  // sequence number of the next tracked frame
  float* d_ref = nullptr;
  sf::TrackHist* d_hist = nullptr;
  std::vector<sf::TrackFrame*> h_tf, d_tf;
  std::vector<spotfit_drift_t*> h_drift, d_drift;
  hipEvent_t track_ev = nullptr;  // the last launched drift pass
  bool track_ev_live = false;

  // failed frames keep their failure after their ring space is released
  std::unordered_set<uint64_t> failed_tickets;
  // failure handling test hook: batch number fail_batch (1-based; 0 = never)
  // fails on the host without enqueueing anything
  int64_t fail_batch = 0;
  int64_t batches_started = 0;

  // statistics
  std::vector<uint64_t> lat_ns;
  uint64_t frames_done = 0, spots_done = 0, batches = 0, rejected = 0, frames_failed = 0;
  uint64_t t_first = 0, t_last = 0;
  std::string error;

  FrameRec& rec(uint64_t t) { return frames[t % (uint64_t)max_frames]; }
  void run();
  bool launch_ready();
  bool reap();
  void free_tracking();
};

namespace {

thread_local std::string g_serve_error;

int serve_fail(int code, const std::string& what) {
  g_serve_error = what;
  return code;
}

template <typename T>
hipError_t alloc_pair(T** d, T** h, int64_t n) {
  hipError_t e = hipMalloc((void**)d, sizeof(T) * (size_t)n);
  if (e != hipSuccess) return e;
  return hipHostMalloc((void**)h, sizeof(T) * (size_t)n, hipHostMallocDefault);
}

template <typename T>
hipError_t alloc_host(T** h, int64_t n) {
  return hipHostMalloc((void**)h, sizeof(T) * (size_t)n, hipHostMallocDefault);
}

// A frame's own records, staged right after its pixels in the pixel ring so that
// a batch of one frame moves them in with its pixels: offsets (8 B per spot),
// shapes (4 B), start values (16 B, after 4 B of padding), the size-class lists
// (3 x 4 B: class c's spot indices from c * n) and the eight counters of a
// mixed-size launch (class sizes, then zeros).
int64_t frame_meta_bytes(int64_t n) { return n > 0 ? (44 * n + 32 + 255) & ~(int64_t)255 : 0; }

struct FrameMeta {
  int64_t* offs;
  spotfit_shape_t* sizes;
  float* init;
  int32_t* lists;
  int32_t* counters;
};

FrameMeta frame_meta(unsigned char* m, int64_t n) {
  return FrameMeta{reinterpret_cast<int64_t*>(m), reinterpret_cast<spotfit_shape_t*>(m + 8 * n),
                   reinterpret_cast<float*>(m + 16 * n), reinterpret_cast<int32_t*>(m + 32 * n),
                   reinterpret_cast<int32_t*>(m + 44 * n)};
}

// Size class of a spot in a mixed-size launch (largest side <= 8, <= 16, <= 32),
// as the device's classify pass assigns it.
int size_class_of(const spotfit_shape_t& sh) {
  const int m = sh.w > sh.h ? sh.w : sh.h;
  return m <= 8 ? 0 : m <= 16 ? 1 : 2;
}

// A batch of n spots in its slices of the meta and result rings.
struct BatchView {
  int64_t* offs;
  spotfit_shape_t* sizes;
  float* init;
  float* params;
  float* chi2;
  int32_t* iters;
  int32_t* status;
};

BatchView batch_view(unsigned char* meta, unsigned char* res, int64_t n) {
  BatchView v;
  v.offs = reinterpret_cast<int64_t*>(meta);
  v.sizes = reinterpret_cast<spotfit_shape_t*>(meta + 8 * n);
  v.init = reinterpret_cast<float*>(meta + 16 * n);
  v.params = reinterpret_cast<float*>(res);
  v.chi2 = reinterpret_cast<float*>(res + 24 * n);
  v.iters = reinterpret_cast<int32_t*>(res + 28 * n);
  v.status = reinterpret_cast<int32_t*>(res + 32 * n);
  return v;
}

template <typename T>
void free_pair(T* d, T* h) {
  if (d) (void)hipFree(d);
  if (h) (void)hipHostFree(h);
}

}  // namespace

// Launch one batch of the oldest admitted frames on a free stream.  Returns true
// if something was launched.
bool spotfit_serve::launch_ready() {
  int si = -1;
  uint64_t t0, t1;
  int64_t spot0, nsp = 0;
  int dtype;
  bool dev_init = false;
  // nothing new to launch, or no stream free: return without taking the lock
  if (next_launch >= admitted_end.load(std::memory_order_acquire)) return false;
  {
    bool any_free = false;
    for (int i = 0; i < n_streams; ++i) any_free = any_free || !stream_busy[i];
    if (!any_free) return false;
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    while (next_launch < next_ticket && rec(next_launch).state == kDone) ++next_launch;
    if (next_launch >= next_ticket) return false;
    FrameRec& f0 = rec(next_launch);
    if (f0.state != kAdmitted) return false;
    for (int i = 0; i < n_streams; ++i)
      if (!stream_busy[i]) {
        si = i;
        break;
      }
    if (si < 0) return false;
    // the batch: consecutive admitted frames of one dtype and one source of
    // start values that are contiguous in the spot ring
    t0 = next_launch;
    spot0 = f0.spot0;
    dtype = f0.dtype;
    dev_init = f0.dev_init;
    t1 = t0;
    while (t1 < next_ticket) {
      FrameRec& f = rec(t1);
      if (f.state != kAdmitted || f.dtype != dtype || f.dev_init != dev_init ||
          f.spot0 != spot0 + nsp)
        break;
      nsp += f.n;
      ++t1;
    }
    for (uint64_t t = t0; t < t1; ++t) rec(t).state = kLaunched;
    next_launch = t1;
    stream_busy[si] = true;
  }
  hipStream_t st = streams[si];
  const bool injected = fail_batch > 0 && ++batches_started == fail_batch;
  // pixel bytes of the batch: frames are consecutive in the pixel ring except
  // where it wrapped, so copy maximal contiguous runs
  hipError_t e = injected ? hipErrorUnknown : hipSuccess;
  if (!injected) {
    int64_t run0 = -1, run1 = -1;
    for (uint64_t t = t0; t <= t1 && e == hipSuccess; ++t) {
      const bool last = t == t1;
      if (!last) {
        const FrameRec& f = rec(t);
        if (run0 >= 0 && f.pix_off == run1) {
          run1 = f.pix_off + f.pix_alloc;
          continue;
        }
      }
      if (run0 >= 0)
        e = hipMemcpyAsync(d_pix + run0, h_pix + run0, (size_t)(run1 - run0), hipMemcpyHostToDevice, st);
      if (!last) {
        const FrameRec& f = rec(t);
        run0 = f.pix_off;
        run1 = f.pix_off + f.pix_alloc;
      }
    }
  }
  const BatchView hv = batch_view(h_meta + kMetaBytes * spot0, h_res + kResBytes * spot0, nsp);
  const BatchView dv = batch_view(d_meta + kMetaBytes * spot0, d_res + kResBytes * spot0, nsp);
  int rc = SPOTFIT_OK;
  if (t1 == t0 + 1 && opt.precision == SPOTFIT_PREC_FP64 && opt.schedule == SPOTFIT_SCHEDULE_MIXED) {
    // one frame: its records and class lists came in with its pixels, and the
    // fit starts without a classify pass: two API calls fewer per frame, which
    // the dispatcher thread otherwise spends while the GPU waits
    const FrameMeta m = frame_meta(d_pix + rec(t0).meta_off, nsp);
    const sf::MixedWs ws{m.counters, m.lists, nsp};
    if (e == hipSuccess)
      rc = sf::fit_preclassified(ctxs[si], d_pix, dtype, m.sizes, m.offs, dev_init ? nullptr : m.init,
                                 dev_init ? m.init : nullptr, nsp, opt, ws, dv.params, dv.chi2,
                                 dv.iters, dv.status, st);
  } else {
    // the batch's records, packed on the host into its meta slice: one copy (the
    // ring space of these spot positions is not in use by any other batch)
    std::memcpy(hv.offs, h_offs + spot0, sizeof(int64_t) * nsp);
    std::memcpy(hv.sizes, h_sizes + spot0, sizeof(spotfit_shape_t) * nsp);
    if (!dev_init) std::memcpy(hv.init, h_init + 4 * spot0, sizeof(float) * 4 * nsp);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dv.offs, hv.offs, (size_t)(dev_init ? 12 : kMetaBytes) * nsp,
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess && dev_init)  // start values on the device, in the fit's own launch
      rc = spotfit_fit_raw(ctxs[si], d_pix, dtype, dv.sizes, dv.offs, nsp, &opt, dv.init,
                           dv.params, dv.chi2, dv.iters, dv.status, nullptr, st);
    else if (e == hipSuccess)
      rc = spotfit_fit_spots(ctxs[si], d_pix, dtype, dv.sizes, dv.offs, dv.init, nsp, &opt,
                             dv.params, dv.chi2, dv.iters, dv.status, nullptr, st);
  }
  int n_tracked = 0;
  if (e == hipSuccess && rc == SPOTFIT_OK && track_markers > 0) {
    sf::TrackFrame* tf = h_tf[si];
    for (uint64_t t = t0; t < t1; ++t) {
      const FrameRec& f = rec(t);
      if (f.track_q >= 0) tf[n_tracked++] = sf::TrackFrame{f.spot0 - spot0, f.track_q};
    }
    if (n_tracked > 0) {
      e = hipMemcpyAsync(d_tf[si], tf, sizeof(sf::TrackFrame) * n_tracked, hipMemcpyHostToDevice, st);
      if (e == hipSuccess && track_ev_live) e = hipStreamWaitEvent(st, track_ev, 0);
      if (e == hipSuccess)
        e = sf::launch_drift_track(d_tf[si], n_tracked, dv.params, dv.status, d_ref, track_markers,
                                   d_hist, track_window, d_drift[si], st);
      if (e == hipSuccess) e = hipEventRecord(track_ev, st);
      track_ev_live = track_ev_live || e == hipSuccess;
      if (e == hipSuccess)
        e = hipMemcpyAsync(h_drift[si], d_drift[si], sizeof(spotfit_drift_t) * n_tracked,
                           hipMemcpyDeviceToHost, st);
    }
  }
  if (e == hipSuccess && rc == SPOTFIT_OK)
    e = hipMemcpyAsync(hv.params, dv.params, (size_t)kResBytes * nsp, hipMemcpyDeviceToHost, st);
  Batch b;
  b.stream = si;
  b.first_ticket = t0;
  b.n_frames = (int)(t1 - t0);
  b.spot0 = spot0;
  b.n_spots = nsp;
  b.n_tracked = n_tracked;
  b.failed = !(e == hipSuccess && rc == SPOTFIT_OK);
  if (!b.failed) {
    if (!event_pool.empty()) {
      b.ev = event_pool.back();
      event_pool.pop_back();
      e = hipSuccess;
    } else {
      e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventRecord(b.ev, st);
    b.failed = e != hipSuccess;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (b.failed && error.empty())
    error = injected ? std::string("serve batch failed: injected failure (test hook)")
                     : std::string("serve batch failed: ") +
                           (rc != SPOTFIT_OK ? spotfit_last_error() : hipGetErrorString(e));
  inflight.push_back(b);
  ++batches;
  return true;
}

// Complete finished batches: copy results out, release ring space.
bool spotfit_serve::reap() {
  bool any = false;
  for (auto it = inflight.begin(); it != inflight.end();) {
    Batch& b = *it;
    bool done = b.failed;
    if (!done) {
      const hipError_t q = hipEventQuery(b.ev);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      if (q != hipSuccess) b.failed = true;
      done = true;
      if (!b.failed) (void)hipEventSynchronize(b.ev);
    }
    if (b.ev) event_pool.push_back(b.ev);
    const uint64_t tnow = now_ns();
    std::lock_guard<std::mutex> lk(mu);
    int tracked = 0;
    for (int k = 0; k < b.n_frames; ++k) {
      FrameRec& f = rec(b.first_ticket + k);
      if (!b.failed) {
        if (f.track_q >= 0) {
          if (f.drift) *f.drift = h_drift[b.stream][tracked];
          ++tracked;
        }
        const BatchView hv = batch_view(h_meta + kMetaBytes * b.spot0, h_res + kResBytes * b.spot0,
                                        b.n_spots);
        const int64_t rel = f.spot0 - b.spot0;
        std::memcpy(f.params, hv.params + 6 * rel, sizeof(float) * 6 * f.n);
        std::memcpy(f.chi2, hv.chi2 + rel, sizeof(float) * f.n);
        if (f.iters) std::memcpy(f.iters, hv.iters + rel, sizeof(int32_t) * f.n);
        if (f.status) std::memcpy(f.status, hv.status + rel, sizeof(int32_t) * f.n);
        f.state = kDone;
        ++frames_done;
        spots_done += (uint64_t)f.n;
      } else {
        f.state = kFailed;
        failed_tickets.insert(f.ticket);
        ++frames_failed;
      }
      f.t_done = tnow;
      lat_ns.push_back(tnow > f.t_arrival ? tnow - f.t_arrival : 0);
    }
    t_last = tnow;
    stream_busy[b.stream] = false;
    // release ring space of the oldest finished frames
    while (oldest_ticket < next_ticket) {
      FrameRec& f = rec(oldest_ticket);
      if (f.state != kDone && f.state != kFailed) break;
      pix_used -= f.pix_bytes;
      spot_used -= f.spot_res;
      ++oldest_ticket;
    }
    it = inflight.erase(it);
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

void spotfit_serve::run() {
  (void)hipSetDevice(device);
  while (!stop.load(std::memory_order_acquire)) {
    bool busy = inflight.empty() ? false : reap();
    busy = launch_ready() || busy;
    if (!busy) __builtin_ia32_pause();
  }
  // drain: wait for everything launched
  for (auto& b : inflight)
    if (b.ev) (void)hipEventSynchronize(b.ev);
  reap();
}

void spotfit_serve::free_tracking() {
  if (d_ref) (void)hipFree(d_ref);
  if (d_hist) (void)hipFree(d_hist);
  for (auto p : d_tf) (void)hipFree(p);
  for (auto p : h_tf) (void)hipHostFree(p);
  for (auto p : d_drift) (void)hipFree(p);
  for (auto p : h_drift) (void)hipHostFree(p);
  if (track_ev) (void)hipEventDestroy(track_ev);
  d_ref = nullptr;
  d_hist = nullptr;
  d_tf.clear();
  h_tf.clear();
  d_drift.clear();
  h_drift.clear();
  track_ev = nullptr;
  track_ev_live = false;
  track_markers = 0;
  track_window = 0;
}

extern "C" {

int spotfit_serve_track(spotfit_serve_t* sv, int32_t n_markers, const float* ref_xy,
                        int32_t window) {
  if (!sv) return serve_fail(SPOTFIT_E_NULL, "serve_track: NULL serving loop");
  if (n_markers < 0 || n_markers > 65536 || (n_markers > 0 && (window < 1 || window > 65536)))
    return serve_fail(SPOTFIT_E_ARG, "serve_track: n_markers in [0, 65536], window in [1, 65536]");
  if (n_markers > 0 && !ref_xy) return serve_fail(SPOTFIT_E_NULL, "serve_track: NULL reference");
  std::lock_guard<std::mutex> lk(sv->mu);
  for (uint64_t t = sv->oldest_ticket; t < sv->next_ticket; ++t)  // frames in flight
    if (sv->rec(t).state != kDone && sv->rec(t).state != kFailed) return SPOTFIT_E_AGAIN;
  // the caller's current device is restored on return
  struct Restore {
    int dev = -1;
    ~Restore() {
      if (dev >= 0) (void)hipSetDevice(dev);
    }
  } restore;
  (void)hipGetDevice(&restore.dev);
  (void)hipSetDevice(sv->device);
  sv->free_tracking();
  sv->track_next = 0;
  if (n_markers == 0) return SPOTFIT_OK;
  const size_t nf = (size_t)sv->max_frames;
  hipError_t e = hipMalloc((void**)&sv->d_ref, sizeof(float) * 2 * (size_t)n_markers);
  if (e == hipSuccess) e = hipMalloc((void**)&sv->d_hist, sizeof(sf::TrackHist) * (size_t)window);
  for (int i = 0; i < sv->n_streams && e == hipSuccess; ++i) {
    sf::TrackFrame *dt = nullptr, *ht = nullptr;
    spotfit_drift_t *dd = nullptr, *hd = nullptr;
    e = hipMalloc((void**)&dt, sizeof(sf::TrackFrame) * nf);
    if (e == hipSuccess) sv->d_tf.push_back(dt);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ht, sizeof(sf::TrackFrame) * nf, hipHostMallocDefault);
    if (e == hipSuccess) sv->h_tf.push_back(ht);
    if (e == hipSuccess) e = hipMalloc((void**)&dd, sizeof(spotfit_drift_t) * nf);
    if (e == hipSuccess) sv->d_drift.push_back(dd);
    if (e == hipSuccess) e = hipHostMalloc((void**)&hd, sizeof(spotfit_drift_t) * nf, hipHostMallocDefault);
    if (e == hipSuccess) sv->h_drift.push_back(hd);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->track_ev, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipMemcpy(sv->d_ref, ref_xy, sizeof(float) * 2 * (size_t)n_markers, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sv->free_tracking();
    return serve_fail(SPOTFIT_E_HIP, std::string("serve_track: ") + hipGetErrorString(e));
  }
  sv->track_markers = n_markers;
  sv->track_window = window;
  return SPOTFIT_OK;
}

int spotfit_serve_create(spotfit_serve_t** out, int device, const spotfit_options_t* opt,
                         size_t budget, int32_t max_frames, int32_t n_streams) {
  if (!out) return serve_fail(SPOTFIT_E_NULL, "serve_create: NULL out pointer");
  *out = nullptr;
  if (max_frames < 1 || max_frames > (1 << 20) || n_streams < 1 || n_streams > 16 ||
      budget < ((size_t)1 << 20))
    return serve_fail(SPOTFIT_E_ARG, "serve_create: max_frames in [1, 2^20], n_streams in [1, 16], budget >= 1 MiB");
  spotfit_options_t o;
  if (opt)
    o = *opt;
  else
    spotfit_default_options(&o);
  int rc = spotfit_validate_options(&o);
  if (rc != SPOTFIT_OK) return serve_fail(rc, spotfit_last_error());
  spotfit_serve* sv = new (std::nothrow) spotfit_serve();
  if (!sv) return serve_fail(SPOTFIT_E_ARG, "serve_create: out of host memory");
  sv->device = device;
  sv->opt = o;
  if (const char* env = std::getenv("SPOTFIT_SERVE_FAIL_BATCH")) sv->fail_batch = std::atoll(env);
  sv->n_streams = n_streams;
  sv->max_frames = max_frames;
  sv->frames.resize((size_t)max_frames);
  // budget split: 3/4 pixels, 1/4 per-spot records (32 B in + 36 B out)
  sv->pix_cap = (int64_t)(budget / 4 * 3) & ~(int64_t)255;
  sv->spot_cap = (int64_t)(budget / 4) / (spotfit_serve::kMetaBytes + spotfit_serve::kResBytes);
  hipError_t e = hipSetDevice(device);
  auto cleanup = [&](hipError_t err, const char* where) {
    spotfit_serve_destroy(sv);
    return serve_fail(SPOTFIT_E_HIP, std::string(where) + ": " + hipGetErrorString(err));
  };
  if (e != hipSuccess) return cleanup(e, "hipSetDevice");
  if ((e = alloc_pair(&sv->d_pix, &sv->h_pix, sv->pix_cap)) != hipSuccess) return cleanup(e, "pixel ring");
  if ((e = alloc_host(&sv->h_sizes, sv->spot_cap)) != hipSuccess) return cleanup(e, "sizes ring");
  if ((e = alloc_host(&sv->h_offs, sv->spot_cap)) != hipSuccess) return cleanup(e, "offsets ring");
  if ((e = alloc_host(&sv->h_init, 4 * sv->spot_cap)) != hipSuccess) return cleanup(e, "init ring");
  if ((e = alloc_pair(&sv->d_meta, &sv->h_meta, spotfit_serve::kMetaBytes * sv->spot_cap)) != hipSuccess)
    return cleanup(e, "record ring");
  if ((e = alloc_pair(&sv->d_res, &sv->h_res, spotfit_serve::kResBytes * sv->spot_cap)) != hipSuccess)
    return cleanup(e, "result ring");
  for (int i = 0; i < n_streams; ++i) {
    hipStream_t st = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return cleanup(e, "stream");
    sv->streams.push_back(st);
    spotfit_ctx_t* c = nullptr;
    rc = spotfit_ctx_create(&c, device);
    if (rc != SPOTFIT_OK) {
      std::string m = spotfit_last_error();
      spotfit_serve_destroy(sv);
      return serve_fail(rc, m);
    }
    sv->ctxs.push_back(c);
    if (o.precision == SPOTFIT_PREC_FP64 && o.schedule == SPOTFIT_SCHEDULE_MIXED) {
      rc = spotfit_ctx_reserve(c, sv->spot_cap);
      if (rc != SPOTFIT_OK) {
        std::string m = spotfit_last_error();
        spotfit_serve_destroy(sv);
        return serve_fail(rc, m);
      }
    }
  }
  sv->stream_busy.assign((size_t)n_streams, false);
  sv->lat_ns.reserve(1 << 16);
  sv->worker = std::thread([sv] { sv->run(); });
  *out = sv;
  return SPOTFIT_OK;
}

int spotfit_serve_submit(spotfit_serve_t* sv, const spotfit_frame_t* fr, uint64_t arrival_ns,
                         uint64_t* ticket) {
  if (!sv || !fr || !ticket) return serve_fail(SPOTFIT_E_NULL, "serve_submit: NULL argument");
  if (fr->n_spots < 0 || (fr->n_spots > 0 && (!fr->data || !fr->sizes || !fr->params_out ||
                                               !fr->chi2_out)))
    return serve_fail(SPOTFIT_E_ARG, "serve_submit: bad frame");
  if (fr->dtype != SPOTFIT_U16 && fr->dtype != SPOTFIT_F32) return serve_fail(SPOTFIT_E_ARG, "serve_submit: dtype");
  const int64_t n = fr->n_spots;
  const int64_t esz = fr->dtype == SPOTFIT_U16 ? 2 : 4;
  int64_t npx = 0;
  for (int64_t i = 0; i < n; ++i) npx += (int64_t)fr->sizes[i].w * fr->sizes[i].h;
  const int64_t px_bytes = ((npx * esz) + 255) & ~(int64_t)255;
  const int64_t bytes = px_bytes + frame_meta_bytes(n);
  std::unique_lock<std::mutex> lk(sv->mu);
  if (fr->drift_out && (sv->track_markers == 0 || n != sv->track_markers))
    return serve_fail(SPOTFIT_E_ARG, "serve_submit: a tracked frame needs tracking on and one spot per marker");
  const uint64_t t = sv->next_ticket;
  // a free slot, and room in both rings (skipping a ring's tail when the frame
  // does not fit before the wrap)
  const bool slot_ok = t - sv->oldest_ticket < (uint64_t)sv->max_frames;
  int64_t pix_skip = sv->pix_cap - sv->pix_head < bytes ? sv->pix_cap - sv->pix_head : 0;
  int64_t spot_skip = sv->spot_cap - sv->spot_head < n ? sv->spot_cap - sv->spot_head : 0;
  const bool pix_ok = bytes <= sv->pix_cap && sv->pix_used + pix_skip + bytes <= sv->pix_cap;
  const bool spot_ok = n <= sv->spot_cap && sv->spot_used + spot_skip + n <= sv->spot_cap;
  if (!slot_ok || !pix_ok || !spot_ok) {
    ++sv->rejected;
    return SPOTFIT_E_AGAIN;
  }
  if (pix_skip) sv->pix_head = 0;
  if (spot_skip) sv->spot_head = 0;
  FrameRec& f = sv->rec(t);
  f = FrameRec();
  f.ticket = t;
  f.dtype = fr->dtype;
  f.dev_init = fr->init == nullptr;
  f.n = n;
  f.spot0 = sv->spot_head;
  f.pix_off = sv->pix_head;
  f.pix_bytes = bytes + pix_skip;
  f.pix_alloc = bytes;
  f.meta_off = f.pix_off + px_bytes;
  f.spot_res = n + spot_skip;
  f.t_arrival = arrival_ns ? arrival_ns : now_ns();
  f.params = fr->params_out;
  f.chi2 = fr->chi2_out;
  f.iters = fr->iters_out;
  f.status = fr->status_out;
  if (fr->drift_out) {
    f.track_q = sv->track_next++;
    f.drift = fr->drift_out;
  }
  sv->pix_head = (sv->pix_head + bytes) % sv->pix_cap;
  sv->spot_head = (sv->spot_head + n) % sv->spot_cap;
  sv->pix_used += f.pix_bytes;
  sv->spot_used += f.spot_res;
  // stage the frame (pinned mirrors); element offsets into the pixel ring
  std::memcpy(sv->h_pix + f.pix_off, fr->data, (size_t)(npx * esz));
  std::memcpy(sv->h_sizes + f.spot0, fr->sizes, sizeof(spotfit_shape_t) * n);
  if (fr->init) std::memcpy(sv->h_init + 4 * f.spot0, fr->init, sizeof(float) * 4 * n);
  int64_t o = f.pix_off / esz;
  for (int64_t i = 0; i < n; ++i) {
    sv->h_offs[f.spot0 + i] = o;
    o += (int64_t)fr->sizes[i].w * fr->sizes[i].h;
  }
  if (n > 0) {
    // the frame's own records after its pixels (a batch of this frame alone
    // reads them from there)
    const FrameMeta m = frame_meta(sv->h_pix + f.meta_off, n);
    std::memcpy(m.offs, sv->h_offs + f.spot0, sizeof(int64_t) * n);
    std::memcpy(m.sizes, fr->sizes, sizeof(spotfit_shape_t) * n);
    if (fr->init) std::memcpy(m.init, fr->init, sizeof(float) * 4 * n);
    int32_t cnt[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
      const int c = size_class_of(fr->sizes[i]);
      m.lists[c * n + cnt[c]++] = (int32_t)i;
    }
    for (int c = 0; c < 8; ++c) m.counters[c] = c < 3 ? cnt[c] : 0;
  }
  if (sv->t_first == 0) sv->t_first = f.t_arrival;
  sv->next_ticket = t + 1;
  f.state = n > 0 ? kAdmitted : kDone;
  sv->admitted_end.store(t + 1, std::memory_order_release);
  if (n == 0) {
    // nothing to fit: complete at once (keeps FIFO order of tickets)
    f.t_done = now_ns();
    ++sv->frames_done;
  }
  *ticket = t;
  return SPOTFIT_OK;
}

int spotfit_serve_poll(spotfit_serve_t* sv, uint64_t ticket) {
  if (!sv) return serve_fail(SPOTFIT_E_NULL, "serve_poll: NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket == 0 || ticket >= sv->next_ticket) return serve_fail(SPOTFIT_E_ARG, "serve_poll: unknown ticket");
  if (ticket < sv->oldest_ticket)  // finished and released
    return sv->failed_tickets.count(ticket) ? serve_fail(SPOTFIT_E_HIP, sv->error) : SPOTFIT_OK;
  const FrameRec& f = sv->rec(ticket);
  if (f.state == kDone) return SPOTFIT_OK;
  if (f.state == kFailed) return serve_fail(SPOTFIT_E_HIP, sv->error);
  return 1;
}

int spotfit_serve_wait(spotfit_serve_t* sv, uint64_t ticket) {
  if (!sv) return serve_fail(SPOTFIT_E_NULL, "serve_wait: NULL");
  for (;;) {
    const int r = spotfit_serve_poll(sv, ticket);
    if (r != 1) return r;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait_for(lk, std::chrono::microseconds(200));
  }
}

int spotfit_serve_stats(spotfit_serve_t* sv, spotfit_serve_stats_t* out) {
  if (!sv || !out) return serve_fail(SPOTFIT_E_NULL, "serve_stats: NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(out, 0, sizeof *out);
  out->frames_done = sv->frames_done;
  out->frames_failed = sv->frames_failed;
  out->spots_done = sv->spots_done;
  out->batches = sv->batches;
  out->rejected = sv->rejected;
  if (!sv->lat_ns.empty()) {
    std::vector<uint64_t> v = sv->lat_ns;
    auto q = [&](double p) {
      const size_t k = (size_t)(p * (double)(v.size() - 1));
      std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
      return (double)v[k] / 1e3;
    };
    out->latency_p50_us = q(0.50);
    out->latency_p99_us = q(0.99);
    out->latency_max_us = (double)*std::max_element(v.begin(), v.end()) / 1e3;
  }
  out->mean_frames_per_batch = sv->batches ? (double)sv->lat_ns.size() / (double)sv->batches : 0.0;
  out->wall_s = sv->t_last > sv->t_first ? (double)(sv->t_last - sv->t_first) / 1e9 : 0.0;
  return SPOTFIT_OK;
}

void spotfit_serve_destroy(spotfit_serve_t* sv) {
  if (!sv) return;
  if (sv->worker.joinable()) {
    sv->stop.store(true, std::memory_order_release);
    sv->worker.join();
  }
  (void)hipSetDevice(sv->device);
  for (auto s : sv->streams) (void)hipStreamSynchronize(s);
  for (auto ev : sv->event_pool) (void)hipEventDestroy(ev);
  sv->free_tracking();
  for (auto c : sv->ctxs) spotfit_ctx_destroy(c);
  for (auto s : sv->streams) (void)hipStreamDestroy(s);
  free_pair(sv->d_pix, sv->h_pix);
  free_pair<spotfit_shape_t>(nullptr, sv->h_sizes);
  free_pair<int64_t>(nullptr, sv->h_offs);
  free_pair<float>(nullptr, sv->h_init);
  free_pair(sv->d_meta, sv->h_meta);
  free_pair(sv->d_res, sv->h_res);
  delete sv;
}

int spotfit_serve_replay(spotfit_serve_t* sv, const spotfit_frame_t* frames, int64_t n_frames,
                         const uint64_t* arrival_offset_ns) {
  if (!sv || (n_frames > 0 && (!frames || !arrival_offset_ns)))
    return serve_fail(SPOTFIT_E_NULL, "serve_replay: NULL argument");
  std::vector<uint64_t> tickets((size_t)n_frames, 0);
  const uint64_t t0 = now_ns() + 1000000;  // start 1 ms from now
  for (int64_t f = 0; f < n_frames; ++f) {
    const uint64_t ta = t0 + arrival_offset_ns[f];
    while (now_ns() < ta) {
    }
    for (;;) {  // a frame that is not admitted waits for space; its latency keeps counting
      const int r = spotfit_serve_submit(sv, &frames[f], ta, &tickets[(size_t)f]);
      if (r == SPOTFIT_OK) break;
      if (r != SPOTFIT_E_AGAIN) return r;
      std::this_thread::yield();
    }
  }
  for (int64_t f = 0; f < n_frames; ++f) {
    const int r = spotfit_serve_wait(sv, tickets[(size_t)f]);
    if (r != SPOTFIT_OK) return r;
  }
  return SPOTFIT_OK;
}

const char* spotfit_serve_last_error(void) { return g_serve_error.c_str(); }

}  // extern "C"
