// C ABI of the H-matrix library: validation, handle lifetime, build
// orchestration (plan -> K1 -> K2 -> compaction -> product plan), the product,
// GMRES and the inspection entry points.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "hmat_internal.hpp"

namespace hm {
hipError_t launch_self(const DevGeo&, const SelfTask*, double*, hipStream_t);
hipError_t launch_near_only(const DevGeo&, const NearTask*, int, double*, hipStream_t);
hipError_t launch_entries(const DevGeo&, int64_t, const int64_t*, const int64_t*, double*, hipStream_t);
hipError_t launch_aca(const DevGeo&, const AcaTask*, int, int, size_t, size_t, bool, bool, int32_t*, int32_t*,
                      double*, hipStream_t);
hipError_t launch_compact(const CopyTask*, int, hipStream_t);
hipError_t launch_exact(const DevGeo&, const ExactTask*, int, bool, hipStream_t);
hipError_t launch_compact32(const CopyTask32*, int, hipStream_t);
hipError_t launch_copy_spans(const SpanCopy*, int, hipStream_t);
hipError_t launch_to_stream(const StreamTask*, int, double*, hipStream_t);
hipError_t launch_from_stream(const StreamTask*, int, const double*, hipStream_t);
hipError_t launch_from_stream32(const StreamTask*, int, const float*, hipStream_t);
hipError_t launch_gather(int, const double*, int64_t, const int32_t*, int64_t, double*, int64_t, hipStream_t);
hipError_t launch_matvec_group(const ProductPlanDev&, int, int, const double*, int64_t, double*, int64_t,
                               double*, double*, int64_t, hipStream_t, hipEvent_t*, int);
hipError_t launch_to_f32(const double*, float*, int64_t, hipStream_t);
size_t dots_part_size(int64_t, int);
size_t norm_part_size(int64_t);
hipError_t launch_cgs_pass(const double*, int64_t, int64_t, int, double*, double*, double*, double*, int, double*, hipStream_t);
hipError_t launch_norm(const double*, int64_t, double*, double*, hipStream_t);
hipError_t launch_scale_norm(const double*, int64_t, const double*, double*, double*, const int32_t*, double*,
                             const double*, int, double*, hipStream_t);
hipError_t launch_scale(const double*, int64_t, const double*, double*, hipStream_t);
hipError_t launch_add_comb(const double*, int64_t, int64_t, int, const double*, double*, hipStream_t);
hipError_t launch_residual(const double*, int64_t, double*, hipStream_t);
hipError_t launch_fill(double*, int64_t, double, hipStream_t);
hipError_t launch_axpy(double, const double*, int64_t, double*, hipStream_t);
hipError_t launch_dense_mv(const DenseMvTask*, int, const double*, const double*, double*, hipStream_t);
hipError_t launch_lowrank_delta(const DeltaTask*, const int4*, int, const int32_t*, const int32_t*, int,
                                const double*, double*, char*, hipStream_t);
hipError_t launch_amvm_aca_tasks(const AcaTask*, const int2*, int, AcaTask*, hipStream_t);
size_t amvm_sort_bytes(int64_t, int);
size_t amvm_leaf_shmem(int);
hipError_t launch_amvm_estimate(const AmvmDev&, double, double, hipStream_t);
hipError_t launch_amvm_stop(const AmvmDev&, double, int32_t, hipStream_t);
hipError_t launch_amvm_update(const AmvmDev&, int32_t, hipStream_t);
hipError_t launch_amvm_out(const double*, const int32_t*, int64_t, double*, hipStream_t);
hipError_t noalloc_workspace(double**);
}  // namespace hm

using namespace hm;

namespace {

thread_local std::string g_err;

hmat_status fail(hmat_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipError {
  hmat_status st;
  std::string msg;
};

void check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const bool oom = (e == hipErrorOutOfMemory);
  (void)hipGetLastError();
  throw HipError{oom ? HMAT_ENOMEM : HMAT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

// Device memory is stream-ordered on the stream of the entry point being
// served, so allocating or freeing never waits for work of other streams --
// concurrent requests on their own streams do not serialise on each other's
// allocations. Every entry point sets the stream with a StreamScope; a buffer
// is used only on that stream (calls on one handle are serialised by the
// caller).
thread_local hipStream_t g_alloc_stream = nullptr;

struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(g_alloc_stream) { g_alloc_stream = s; }
  ~StreamScope() { g_alloc_stream = prev; }
};

// Release threshold of the device's default pool (freed memory beyond it
// goes back to the device at the next synchronisation): 4 GiB, and 64 GiB
// (at most a quarter of the device memory) while a request server runs.
// Handing memory back while other streams run stalled concurrent builds
// (measured with four to eight at once); a single large build, on the other
// hand, needs its freed staging back for its arenas. An allocation that runs
// out of memory empties the pool and the library's caches and tries again
// (mem_trim).
std::mutex g_pool_mu;
int g_pool_servers = 0;  // request servers alive

void apply_pool_threshold() {  // with g_pool_mu held
  int dev = 0;
  hipMemPool_t pool = nullptr;
  size_t fr = 0, tot = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess &&
      hipMemGetInfo(&fr, &tot) == hipSuccess) {
    uint64_t thr = g_pool_servers > 0 ? std::min<uint64_t>((uint64_t)64 << 30, tot / 4) : (uint64_t)4 << 30;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
}

void init_pool() {
  static std::once_flag once;
  std::call_once(once, [] {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    apply_pool_threshold();
  });
}

// Device memory cache. A stream-ordered hipMallocAsync / hipFreeAsync pair
// costs about 0.3 ms on an idle device and far more when several threads
// allocate at once, and a build makes dozens of allocations; so blocks the
// library releases are kept per device and handed to later allocations. Sizes
// are rounded up to classes of an eighth of a power of two (at least 256 B)
// up to 64 MiB and to multiples of 2 MiB above; an allocation takes the
// smallest cached block of at least its class and at most 1.25 times it. A released block carries an event recorded on the
// releasing stream (the stream of its last use), and the allocating stream
// waits for it, so reuse on any stream is ordered after the last use. The
// cache holds at most a sixteenth of the device memory (the largest blocks go
// first beyond that) and is emptied when an allocation runs out of memory.
constexpr int MAX_DEVICES = 64;
struct CachedBlock {
  void* p;
  size_t bytes;
  hipEvent_t ev;
};
struct MemCache {
  std::mutex mu;
  std::multimap<size_t, CachedBlock> blocks;  // by size
  size_t cached = 0, limit = 0;
  std::vector<hipEvent_t> spare;  // events of reused blocks
};
MemCache g_mem[MAX_DEVICES];

size_t size_class(size_t b) {
  if (b <= 256) return 256;
  if (b > ((size_t)64 << 20)) return (b + ((size_t)2 << 20) - 1) / ((size_t)2 << 20) * ((size_t)2 << 20);
  const int lg = 63 - __builtin_clzll((unsigned long long)(b - 1));  // 2^lg <= b-1 < 2^(lg+1)
  const size_t step = (size_t)1 << (lg - 3);
  return (b + step - 1) / step * step;
}

int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  return dev < MAX_DEVICES ? dev : -1;
}

// Device memory the library holds per device: live buffers, cached blocks
// and kept ACA panel buffers (what it has allocated and not handed back), and
// the cap hmat_set_mem_budget sets on it (0: none). An allocation that would
// pass the cap fails as if the device were full, so the release-and-retry
// path runs first and HMAT_ENOMEM follows if that does not make room.
std::atomic<int64_t> g_held[MAX_DEVICES];
std::atomic<int64_t> g_peak[MAX_DEVICES];  // largest g_held after an allocation since hmat_mem_held
std::atomic<int64_t> g_budget{0};

bool over_budget(int dev, size_t bytes) {
  const int64_t b = g_budget.load();
  return b > 0 && dev >= 0 && g_held[dev].load() + (int64_t)bytes > b;
}
hipError_t dev_malloc(void** p, size_t bytes, hipStream_t s, int dev) {
  if (over_budget(dev, bytes)) return hipErrorOutOfMemory;
  const hipError_t e = hipMallocAsync(p, bytes, s);
  if (e == hipSuccess && dev >= 0) {
    const int64_t now = g_held[dev] += (int64_t)bytes;
    int64_t pk = g_peak[dev].load();
    while (now > pk && !g_peak[dev].compare_exchange_weak(pk, now)) {
    }
  }
  return e;
}
void dev_free(void* p, size_t bytes, hipStream_t s, int dev) {
  (void)hipFreeAsync(p, s);
  if (dev >= 0) g_held[dev] -= (int64_t)bytes;
}
// The error of an allocation that still failed after the retry.
void check_alloc(hipError_t e, int dev, size_t bytes, const char* what) {
  if (e == hipErrorOutOfMemory && over_budget(dev, bytes)) {
    (void)hipGetLastError();
    throw HipError{HMAT_ENOMEM, std::string(what) + ": the device memory budget (hmat_set_mem_budget) is exceeded"};
  }
  check(e, what);
}

// Frees every cached block of device dev, ordered on stream s, and hands the
// default pool's unused memory back to the device.
void mem_trim(int dev, hipStream_t s) {
  if (dev < 0) return;
  MemCache& c = g_mem[dev];
  std::vector<CachedBlock> all;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto& kv : c.blocks) all.push_back(kv.second);
    c.blocks.clear();
    c.cached = 0;
  }
  for (const CachedBlock& b : all) {
    (void)hipStreamWaitEvent(s, b.ev, 0);
    dev_free(b.p, b.bytes, s, dev);
    (void)hipEventDestroy(b.ev);
  }
  (void)hipStreamSynchronize(s);
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  (void)hipGetLastError();
}

// A build whose staging buffers are a large share of the device memory hands
// them back to the device once freed (after the stream has passed their last
// use): kept in the pool, they would crowd out the build's next, differently
// sized arenas. Builds of serving size stay below the bar and trim nothing.
void trim_pool_after(int64_t freed_bytes, hipStream_t s) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  const int dev = current_device();
  if (dev < 0 || (size_t)freed_bytes <= tot / 16) return;
  (void)hipStreamSynchronize(s);
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, (size_t)4 << 30);
  (void)hipGetLastError();
}

void drop_idle_panels(int dev, hipStream_t s);  // idle ACA panel buffers (below)

// At least b bytes for use on stream s; *cls and *dev receive what mem_free needs.
void* mem_alloc(size_t b, hipStream_t s, size_t* cls, int* dev, const char* what) {
  const size_t cl = size_class(b);
  const int d = current_device();
  *dev = d;
  if (d >= 0) {
    MemCache& c = g_mem[d];
    CachedBlock blk{nullptr, 0, nullptr};
    {
      std::lock_guard<std::mutex> lk(c.mu);
      auto it = c.blocks.lower_bound(cl);
      if (it != c.blocks.end() && it->first <= cl + cl / 4) {
        blk = it->second;
        c.cached -= blk.bytes;
        c.blocks.erase(it);
      }
    }
    if (blk.p) {
      const hipError_t e = hipStreamWaitEvent(s, blk.ev, 0);
      {
        std::lock_guard<std::mutex> lk(c.mu);
        c.spare.push_back(blk.ev);
      }
      if (e != hipSuccess) {  // cannot order the reuse: give the block back to the pool
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        (void)hipFree(blk.p);
        g_held[d] -= (int64_t)blk.bytes;
      } else {
        *cls = blk.bytes;
        return blk.p;
      }
    }
  }
  void* p = nullptr;
  hipError_t e = dev_malloc(&p, cl, s, d);
  if (e == hipErrorOutOfMemory) {  // hand everything kept back, then try again
    (void)hipGetLastError();
    const auto t0 = std::chrono::steady_clock::now();
    drop_idle_panels(d, s);
    mem_trim(d, s);
    e = dev_malloc(&p, cl, s, d);
    if (std::getenv("HMAT_TRACE_BUILD"))
      std::fprintf(stderr, "hmat memory: %s (%zu bytes) found the device full; releasing kept memory and retrying took %.1f ms\n",
                   what, cl, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  }
  check_alloc(e, d, cl, what);
  *cls = cl;
  return p;
}

// Releases a block of class cls (from mem_alloc on device dev) whose last use
// is on stream s.
void mem_free(void* p, size_t cls, int dev, hipStream_t s) {
  if (dev < 0 || dev != current_device()) {
    dev_free(p, cls, s, dev);
    return;
  }
  MemCache& c = g_mem[dev];
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.limit == 0) {
      size_t fr = 0, tot = 0;
      c.limit = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 16 : (size_t)1 << 30;
      (void)hipGetLastError();
    }
    if (!c.spare.empty()) {
      ev = c.spare.back();
      c.spare.pop_back();
    }
  }
  if ((!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ||
      hipEventRecord(ev, s) != hipSuccess) {
    (void)hipGetLastError();
    if (ev) (void)hipEventDestroy(ev);
    dev_free(p, cls, s, dev);
    return;
  }
  std::vector<CachedBlock> evict;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    c.blocks.emplace(cls, CachedBlock{p, cls, ev});
    c.cached += cls;
    while (c.cached > c.limit && !c.blocks.empty()) {
      auto it = std::prev(c.blocks.end());
      evict.push_back(it->second);
      c.cached -= it->first;
      c.blocks.erase(it);
    }
  }
  for (const CachedBlock& b : evict) {
    (void)hipStreamWaitEvent(s, b.ev, 0);
    dev_free(b.p, b.bytes, s, dev);
    std::lock_guard<std::mutex> lk(c.mu);
    c.spare.push_back(b.ev);
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;  // requested
  size_t cls = 0;    // held (size class)
  int dev = -1;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) mem_free(p, cls, dev, g_alloc_stream);
    p = nullptr;
    bytes = 0;
    cls = 0;
  }
  void alloc(size_t b, const char* what) {
    release();
    if (b == 0) return;
    p = mem_alloc(b, g_alloc_stream, &cls, &dev, what);
    bytes = b;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

template <class T>
void upload(DevBuf& d, const std::vector<T>& h, hipStream_t s, const char* what) {
  d.alloc(h.size() * sizeof(T), what);
  if (!h.empty()) check(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), what);
}

constexpr int KCAP_FIRST = 128;  // largest first-pass panel capacity (columns) of ACA

// First-pass capacity for accuracy eps: about twice the largest rank that
// ACA reaches at that accuracy on the surface meshes here (ranks grow by
// about six per decade of eps), in multiples of 16, at most KCAP_FIRST. A
// block that reaches it continues in a later pass with a larger capacity, so
// the factors do not depend on this choice; only the panel memory and the
// number of passes do. HMAT_ACA_KCAP_FIRST (>= 2) overrides it.
int32_t kcap_first(double eps) {
  if (const char* e = std::getenv("HMAT_ACA_KCAP_FIRST")) return std::max(2, std::atoi(e));
  const double d = -std::log10(eps);
  const int32_t c = 16 * (int32_t)std::ceil((24.0 + 12.0 * d) / 16.0);
  return std::min<int32_t>(KCAP_FIRST, std::max<int32_t>(32, c));
}

// First-pass ACA panels (several GB for a mesh of 10^5 DOF) are not
// allocated per build: each device keeps the panel buffers of finished ACA
// passes (each up to a sixteenth of the device memory, together up to an
// eighth; the smallest go first beyond that). A pass borrows the smallest
// idle buffer that is large enough and allocates a new one only if none is;
// a pass that needs more than a sixteenth uses a buffer of its own, released
// after its build's ACA phase. Allocating and releasing buffers of that size
// on every build stalled builds for up to seconds, the more so with several
// builds at once. Kept buffers are held until the process ends.
struct PanelCache {
  std::mutex mu;
  std::vector<std::pair<void*, size_t>> idle;  // buffers not lent
  size_t keep_max = 0;                         // largest buffer kept (0: not known yet)
};
PanelCache g_panel_cache[MAX_DEVICES];

// Frees the idle ACA panel buffers of device dev, ordered on stream s.
void drop_idle_panels(int dev, hipStream_t s) {
  if (dev < 0) return;
  std::vector<std::pair<void*, size_t>> idle;
  {
    std::lock_guard<std::mutex> lk(g_panel_cache[dev].mu);
    idle.swap(g_panel_cache[dev].idle);
  }
  for (const auto& q : idle) dev_free(q.first, q.second, s, dev);
}

class PanelLease {
 public:
  PanelLease(int dev, hipStream_t s) : s_(s), dev_(dev < MAX_DEVICES ? dev : -1) {
    if (dev < 0 || dev >= MAX_DEVICES) return;
    PanelCache& c = g_panel_cache[dev];
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.keep_max == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return;
      }
      c.keep_max = tot / 16;
    }
    cache_ = &c;
    keep_max_ = c.keep_max;
  }
  PanelLease(const PanelLease&) = delete;
  PanelLease& operator=(const PanelLease&) = delete;
  // At least `need` bytes, on the lease's stream. Every kernel that used the
  // previous buffer of this lease has finished (the build synchronises its
  // stream after each ACA pass).
  double* get(size_t need) {
    if (p_ && bytes_ >= need) return static_cast<double*>(p_);
    if (!cache_ || need > keep_max_) {
      if (own_.bytes < need) own_.alloc(need, "ACA panels");
      return own_.as<double>();
    }
    void* had = p_;
    const size_t had_bytes = bytes_;
    p_ = nullptr;
    bytes_ = 0;
    {
      std::lock_guard<std::mutex> lk(cache_->mu);
      if (had) cache_->idle.emplace_back(had, had_bytes);
      auto best = cache_->idle.end();
      for (auto it = cache_->idle.begin(); it != cache_->idle.end(); ++it)
        if (it->second >= need && (best == cache_->idle.end() || it->second < best->second)) best = it;
      if (best != cache_->idle.end()) {
        p_ = best->first;
        bytes_ = best->second;
        cache_->idle.erase(best);
      }
    }
    if (!p_) {
      hipError_t e = dev_malloc(&p_, need, s_, dev_);
      if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        drop_idle(0);
        mem_trim(dev_, s_);
        e = dev_malloc(&p_, need, s_, dev_);
      }
      if (e != hipSuccess) p_ = nullptr;
      check_alloc(e, dev_, need, "ACA panels");
      bytes_ = need;
    }
    return static_cast<double*>(p_);
  }
  // Returned (at the latest by the destructor) once the stream has finished
  // every kernel that used it.
  void give_back() {
    own_.release();
    if (!cache_) return;
    if (p_) {
      (void)hipStreamSynchronize(s_);
      std::lock_guard<std::mutex> lk(cache_->mu);
      cache_->idle.emplace_back(p_, bytes_);
    }
    p_ = nullptr;
    bytes_ = 0;
    drop_idle(2 * keep_max_);
    cache_ = nullptr;
  }
  ~PanelLease() { give_back(); }

 private:
  // Frees idle buffers, smallest first, until at most `keep` bytes are idle.
  void drop_idle(size_t keep) {
    std::vector<std::pair<void*, size_t>> drop;
    {
      std::lock_guard<std::mutex> lk(cache_->mu);
      size_t total = 0;
      for (const auto& q : cache_->idle) total += q.second;
      while (total > keep && !cache_->idle.empty()) {
        auto it = std::min_element(cache_->idle.begin(), cache_->idle.end(),
                                   [](const std::pair<void*, size_t>& x, const std::pair<void*, size_t>& y) {
                                     return x.second < y.second;
                                   });
        total -= it->second;
        drop.push_back(*it);
        cache_->idle.erase(it);
      }
    }
    for (const auto& q : drop) dev_free(q.first, q.second, s_, dev_);
  }

  hipStream_t s_;
  int dev_ = -1;
  PanelCache* cache_ = nullptr;
  void* p_ = nullptr;
  size_t bytes_ = 0;
  size_t keep_max_ = 0;
  DevBuf own_;
};
constexpr int MV_TILE = 128;     // rows per product tile (one wave, two rows per lane)
constexpr int MV_SEG_COLS = 128; // columns per product segment
constexpr int64_t MV_CHUNK_BYTES = 16 * 1024;         // nrhs = 1; HMAT_MV_CHUNK_KB overrides
// nrhs > 1: 64 KB while the stream holds under 32768 such chunks of 128 KB
// (so there are several rounds of waves and no long tail), else 128 KB (the
// partial sums, 16 KB per chunk, stay an eighth of the stream)
constexpr int64_t MV_CHUNK_BYTES_MULTI = 128 * 1024;
constexpr int64_t MV_CHUNK_BYTES_MULTI_SMALL = 64 * 1024;
constexpr int64_t MV_CHUNK_MULTI_SMALL_BELOW = 32768 * MV_CHUNK_BYTES_MULTI;  // stream bytes

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Panel layout of a block matrix whose rows are the global DOFs [R0, R0 + M).
struct PanelShape {
  int32_t fp, ld;
};
inline PanelShape panel_shape(int64_t R0, int64_t M) {
  const int32_t fp = (int32_t)(R0 % PANEL_ALIGN);
  return PanelShape{fp, (int32_t)round_up(fp + M, PANEL_ALIGN)};
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

namespace {
// Pinned host buffers for GMRES's Hessenberg columns (3 x 1026 doubles),
// recycled across handles: allocating pinned memory synchronises the device.
// Coherent, since a kernel writes the columns into them directly.
std::mutex g_pin_mu;
std::vector<double*> g_pin_free;
constexpr size_t PIN_DOUBLES = 3 * 1026;
double* pinned_acquire() {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin_free.empty()) {
      double* p = g_pin_free.back();
      g_pin_free.pop_back();
      return p;
    }
  }
  double* p = nullptr;
  if (hipHostMalloc((void**)&p, sizeof(double) * PIN_DOUBLES, hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}
void pinned_release(double* p) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(p);
}
}  // namespace

struct hmat {
  int device = 0;
  hipStream_t last_stream = nullptr;  // stream of the latest call (hmat_free syncs it)
  // Captured products (hmat_matvec_graph): one executable graph per argument
  // set, replayed on an internal stream ordered after and before the caller's.
  struct GraphKey {
    int prec, nrhs;
    const double* x;
    int64_t ldx;
    double* y;
    int64_t ldy;
    bool operator==(const GraphKey& o) const {
      return prec == o.prec && nrhs == o.nrhs && x == o.x && ldx == o.ldx && y == o.y && ldy == o.ldy;
    }
  };
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
  hipStream_t graph_stream = nullptr;
  hipEvent_t graph_done = nullptr;  // recorded after every replay
  bool graph_live = false;          // graph_done marks a replay
  Plan plan;
  double eta = 0;
  int32_t leaf = 0;
  int64_t N = 0;
  // Bodies: one H-matrix per body, laid out block-diagonally in one handle.
  // Body b owns triangles [tri_off, tri_off + nt) and DOFs [3 tri_off, ...)
  // both in the caller's numbering and in cluster order.
  struct Body {
    int32_t tri_off, nt;
    double E, nu, eps;
  };
  std::vector<Body> bodies;
  std::vector<int32_t> pos_body;  // cluster position -> body
  DevBuf d_cen, d_q, d_vtx, d_gl, d_order, d_kc;
  DevBuf d_cen32, d_q32;  // FP32 copies of d_cen, d_q (FP32 ACA only)
  DevGeo G{};
  std::vector<int32_t> inv_order;  // caller's triangle -> cluster position
  // block bookkeeping (canonical order)
  std::vector<int32_t> kind_index;  // far index or near index of block b
  std::vector<int32_t> far_blocks, near_blocks;
  std::vector<int32_t> rank, stop;
  std::vector<double> ratio;
  std::vector<int64_t> far_voff;    // per far block: V panel base in the far arena
  std::vector<PanelShape> far_vshape;
  DevBuf far_arena;                 // V factors (panel layout)
  DevBuf stream;                    // U factors and dense blocks in product order
  DevBuf far32, stream32;           // FP32 copies of both (hmat_set_precision), same layout
  std::deque<DevBuf> piv_bufs;          // ACA pivots, one buffer per pass and group
  std::vector<const int32_t*> piv_ptr;  // per far block: device [2][cap]
  std::vector<int32_t> piv_cap;
  int aca_passes = 0;
  int32_t n_exact = 0;  // admissible blocks stored exactly (ACA reached full rank)
  bool fp32_only = false;    // entries stored in FP32 only (hmat_build_ex precision 1)
  bool fp32_aca = false;     // ACA in FP32 (FP32 builds with eps >= 1e-5)
  double stop_factor = 1.0;  // ACA stop test |u||v| <= stop_factor eps ||S||
  int32_t aca_small_tri = ACA_SMALL_TRI;  // ACA schedule: one wave per block up to this size
  bool aca_wide = false;                  // ACA schedule: 512-thread first pass
  // product plan
  DevBuf d_seg;
  // Work lists: [0] for single right-hand sides (8-column phase-A items,
  // small chunks, short tail), [1] for several (64-column items for the
  // matrix cores; larger chunks, as the partial sums grow with the number of
  // vectors). Both chunk lists are cut from the same segment order.
  struct ChunkList {
    DevBuf d_items, d_chunk, d_tile_near, d_tile_far;
    int nA = 0, n = 0, n_near = 0;
    int64_t target = 0;  // chunk size in bytes the list was cut for
  } cl[2];
  int nSeg = 0, nTiles = 0;
  int64_t Ztot = 0, ldxp = 0, stream_n = 0;
  std::vector<MvSeg> segs;                       // host copy, product order
  std::vector<int32_t> seg_tile;                 // tile of each segment
  // Where each block's matrix lives in the stream: pieces (block columns
  // [bc0, bc1) inside segment `seg`, starting at stream offset so).
  struct Piece {
    int32_t seg, bc0, bc1;
    int64_t so;
  };
  std::vector<std::vector<Piece>> block_pieces;  // canonical block -> its pieces
  int64_t mv_chunk_bytes = MV_CHUNK_BYTES;       // product tuning (HMAT_MV_CHUNK_KB)
  int64_t mv_chunk_bytes_multi = 0;  // 0: by stream size (multi_chunk_bytes)
  int mv_unroll = 16;                            // columns per batch in phase B (HMAT_MV_UNROLL)
  DevBuf d_xp, d_z, d_part, d_dotpart;
  DevBuf d_ir;  // iterative refinement: residual and correction
  // GMRES workspace
  DevBuf d_Q, d_w, d_small;
  int q_cols = 0;
  double* h_pinned = nullptr;  // [2][1026] Hessenberg columns read back; [1026..] Givens solution
  hipEvent_t col_ev[2] = {nullptr, nullptr};
  // product profiling: 5 events per recorded group (start, gathered, V^T x, U z + D x, done)
  bool prof = false;
  std::vector<std::array<hipEvent_t, 5>> prof_pending;
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_calls = 0;
  hmat_stats st{};
  ~hmat() {
    for (auto& e : prof_pending)
      for (hipEvent_t x : e) (void)hipEventDestroy(x);
    for (hipEvent_t e : col_ev)
      if (e) (void)hipEventDestroy(e);
    if (graph_live) (void)hipEventSynchronize(graph_done);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    if (graph_done) (void)hipEventDestroy(graph_done);
    if (graph_stream) {
      (void)hipStreamSynchronize(graph_stream);
      (void)hipStreamDestroy(graph_stream);
    }
    if (h_pinned) pinned_release(h_pinned);
  }
};

namespace {

int64_t block_m(const hmat* h, int32_t b) { return 3 * (int64_t)h->plan.cl[h->plan.blk[b].t].len; }
int64_t block_n(const hmat* h, int32_t b) { return 3 * (int64_t)h->plan.cl[h->plan.blk[b].s].len; }

// Panel layout of the V factors for the current ranks. Returns the arena size in doubles.
int64_t far_layout(hmat* h) {
  const Plan& P = h->plan;
  const size_t nf = h->far_blocks.size();
  h->far_voff.assign(nf, 0);
  h->far_vshape.assign(nf, PanelShape{0, 0});
  int64_t fo = 0;
  for (size_t f = 0; f < nf; f++) {
    const BlockRec& B = P.blk[h->far_blocks[f]];
    h->far_vshape[f] = panel_shape(3 * (int64_t)P.cl[B.s].off, 3 * (int64_t)P.cl[B.s].len);
    h->far_voff[f] = fo;
    fo += (int64_t)h->far_vshape[f].ld * h->rank[f];
  }
  return fo;
}

// Product plan for the current ranks and V layout: phase-A items, phase-B
// segments in product order with their stream offsets, chunks of about
// MV_CHUNK_BYTES per tile. Sets stream_n; uploads the plan.
// Build phase timing on stderr when HMAT_TRACE_BUILD is set (synchronises
// the stream at every mark, so device work is charged to its phase).
struct BuildTrace {
  bool on = std::getenv("HMAT_TRACE_BUILD") != nullptr;
  std::chrono::steady_clock::time_point last = std::chrono::steady_clock::now();
  void mark(const char* what, hipStream_t s) {
    if (!on) return;
    (void)hipStreamSynchronize(s);
    std::fprintf(stderr, "hmat build: %-28s %9.1f ms\n", what, ms_since(last));
    last = std::chrono::steady_clock::now();
  }
};

// Captured product graphs hold the plan's and arenas' device pointers:
// drop them whenever those change (after the graphs' last replay finished).
void drop_graphs(hmat* h) {
  if (h->graphs.empty()) return;
  if (h->graph_live) (void)hipEventSynchronize(h->graph_done);
  h->graph_live = false;
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
  h->graphs.clear();
}

// Phase-B chunk list l: runs of consecutive segments of one tile and kind
// (dense first, then low-rank) holding about `target` bytes, checked and
// uploaded; the partial-sum workspace grows to fit ([chunk][NR][128], NR = 1
// for list 0, up to 16 for list 1).
void set_chunk_list(hmat* h, int l, int64_t target, hipStream_t s) {
  drop_graphs(h);
  std::vector<MvChunk> chunks;
  std::vector<int32_t> tile_near(h->nTiles + 1, 0), tile_far(h->nTiles + 1, 0);
  int n_near = 0;
  const size_t ns = h->segs.size();
  size_t i = 0;
  for (int32_t group = 0; group < 2; group++) {
    std::vector<int32_t>& tc = group == 0 ? tile_near : tile_far;
    for (int32_t T = 0; T < h->nTiles; T++) {
      tc[T] = (int32_t)chunks.size();
      while (i < ns && h->segs[i].far == group && h->seg_tile[i] == T) {
        MvChunk c{T, (int32_t)i, (int32_t)i, 0};
        int64_t bytes = 0;
        while (i < ns && h->segs[i].far == group && h->seg_tile[i] == T &&
               (bytes < target || c.seg_hi == c.seg_lo)) {
          bytes += 8 * (int64_t)(h->segs[i].row_hi - h->segs[i].row_lo) * (h->segs[i].c1 - h->segs[i].c0);
          i++;
          c.seg_hi = (int32_t)i;
        }
        chunks.push_back(c);
      }
    }
    tc[h->nTiles] = (int32_t)chunks.size();
    if (group == 0) n_near = (int32_t)chunks.size();
  }
  auto bad = [](const char* what) { throw HipError{HMAT_EDEVICE, std::string("internal: product plan: ") + what}; };
  if (i != ns) bad("segments left over");
  for (const MvChunk& c : chunks)
    if (c.tile < 0 || c.tile >= h->nTiles || c.seg_lo >= c.seg_hi || c.seg_hi > (int32_t)ns) bad("chunks");
  for (int32_t T = 0; T < h->nTiles; T++)
    if (tile_near[T + 1] <= tile_near[T] || tile_far[T + 1] < tile_far[T]) bad("tile chunk ranges");
  hmat::ChunkList& CL = h->cl[l];
  upload(CL.d_chunk, chunks, s, "product plan");
  upload(CL.d_tile_near, tile_near, s, "product plan");
  upload(CL.d_tile_far, tile_far, s, "product plan");
  CL.n = (int)chunks.size();
  CL.n_near = n_near;
  CL.target = target;
  const size_t need = sizeof(double) * MV_TILE *
                      std::max<int64_t>(std::max(1, h->cl[0].n), (int64_t)MV_MAX_NR * std::max(1, h->cl[1].n));
  if (h->d_part.bytes < need) h->d_part.alloc(need, "product workspace");
}

// Chunk size of the several-vector product: the tuned one, else by stream size.
int64_t multi_chunk_bytes(const hmat* h) {
  if (h->mv_chunk_bytes_multi > 0) return h->mv_chunk_bytes_multi;
  return (int64_t)sizeof(double) * h->stream_n < MV_CHUNK_MULTI_SMALL_BELOW ? MV_CHUNK_BYTES_MULTI_SMALL
                                                                           : MV_CHUNK_BYTES_MULTI;
}

void build_product_plan(hmat* h, hipStream_t s) {
  const Plan& P = h->plan;
  BuildTrace tr;
  // Phase-A items: groups of <= 8 columns of one V panel for one vector, of
  // <= 64 (four matrix-core tiles, sharing each load of the vectors) for
  // several; largest first (several vectors), by column window and XCD (one).
  std::vector<MvA> items_l[2];
  std::vector<int64_t> zoff(h->far_blocks.size(), 0);
  int64_t z = 0;
  for (size_t f = 0; f < h->far_blocks.size(); f++) {
    const int32_t b = h->far_blocks[f];
    const int32_t k = h->rank[f];
    zoff[f] = z;
    if (k == 0) continue;
    const int64_t R0 = 3 * (int64_t)P.cl[P.blk[b].s].off;
    const PanelShape& V = h->far_vshape[f];
    for (int l = 0; l < 2; l++) {
      const int32_t w = l == 0 ? 8 : 64;
      for (int32_t l0 = 0; l0 < k; l0 += w)
        items_l[l].push_back(MvA{h->far_voff[f], V.ld, l0, std::min(k, l0 + w), (int32_t)(R0 - V.fp),
                                 (int32_t)(z + l0), 0});
    }
    z += k;
  }
  for (auto& items : items_l) {
    // largest first; equal sizes keep their canonical order
    std::vector<uint64_t> key(items.size());
    for (size_t t = 0; t < items.size(); t++) key[t] = (uint64_t)items[t].ld * (uint64_t)(items[t].l1 - items[t].l0);
    const std::vector<int32_t> ord = order_desc_stable(key);
    std::vector<MvA> sorted(items.size());
    for (size_t t = 0; t < items.size(); t++) sorted[t] = items[ord[t]];
    items.swap(sorted);
  }
  {
    // Single vector: the items of one column window together, and each of
    // the 8 XCDs (workgroup b runs on XCD b mod 8) given a contiguous eighth
    // of them by work, so the window's x entries stay in that XCD's L2 while
    // its items run (0.628 -> 0.612 ms per product at icosphere L5; no gain
    // for the matrix-core list). Ranges are padded to equal counts with empty
    // items (ld = 0, no columns).
    constexpr int NX = 8;
    std::vector<MvA>& items = items_l[0];
    std::stable_sort(items.begin(), items.end(), [](const MvA& a, const MvA& b) { return a.a0 < b.a0; });
    int64_t tot = 0;
    for (const MvA& I : items) tot += (int64_t)I.ld * (I.l1 - I.l0);
    std::vector<size_t> start(NX + 1, items.size());
    start[0] = 0;
    int64_t acc = 0;
    int x = 1;
    for (size_t t = 0; t < items.size() && x < NX; t++) {
      acc += (int64_t)items[t].ld * (items[t].l1 - items[t].l0);
      while (x < NX && acc * NX >= tot * x) start[x++] = t + 1;
    }
    size_t most = 0;
    for (int q = 0; q < NX; q++) most = std::max(most, start[q + 1] - start[q]);
    std::vector<MvA> spread(most * NX, MvA{0, 0, 0, 0, 0, 0, 0});
    for (int q = 0; q < NX; q++)
      for (size_t j = 0; j < start[q + 1] - start[q]; j++) spread[j * NX + q] = items[start[q] + j];
    items.swap(spread);
  }
  tr.mark("  plan: phase-A items", s);
  h->Ztot = std::max<int64_t>(round_up(z, 2), 2);
  // Column groups: the low-rank blocks of one row cluster (consecutive in
  // canonical order, so their z entries are contiguous) form one group whose
  // columns are the concatenation of their ranks; each dense block is a group
  // of its own. A group's rows are its row cluster's.
  struct Group {
    std::vector<int32_t> members;  // canonical blocks, all far or all near, same row cluster
    int64_t ncols, soff;
    int32_t far;
  };
  std::vector<Group> groups;
  std::vector<int64_t> gcol(P.blk.size(), 0);  // block's first column inside its group
  int32_t last_far_group = -1;
  for (size_t b = 0; b < P.blk.size(); b++) {
    const BlockRec& B = P.blk[b];
    if (B.far) {
      const int32_t f = h->kind_index[b];
      if (h->rank[f] == 0) continue;
      Group* g = last_far_group >= 0 ? &groups[last_far_group] : nullptr;
      if (g && P.blk[g->members[0]].t == B.t && g->soff + g->ncols == zoff[f]) {
        gcol[b] = g->ncols;
        g->ncols += h->rank[f];
        g->members.push_back((int32_t)b);
      } else {
        groups.push_back(Group{{(int32_t)b}, h->rank[f], zoff[f], 1});
        last_far_group = (int32_t)groups.size() - 1;
      }
    } else {
      groups.push_back(Group{{(int32_t)b}, block_n(h, (int32_t)b), 3 * (int64_t)P.cl[B.s].off, 0});
    }
  }
  struct SegT {
    int32_t tile, group;
    MvSeg seg;
  };
  std::vector<SegT> segs;
  for (size_t gi = 0; gi < groups.size(); gi++) {
    const Group& g = groups[gi];
    const BlockRec& B = P.blk[g.members[0]];
    const int64_t R0 = 3 * (int64_t)P.cl[B.t].off, m = block_m(h, g.members[0]);
    // rows [R0, R0 + m) widened to even rows (zero rows in the stream)
    const int64_t A0 = R0 / STREAM_ALIGN * STREAM_ALIGN, A1 = round_up(R0 + m, STREAM_ALIGN);
    for (int64_t T = A0 / MV_TILE; T * MV_TILE < A1; T++) {
      const int64_t lo = std::max(A0, T * MV_TILE) - T * MV_TILE;
      const int64_t hi = std::min(A1, (T + 1) * MV_TILE) - T * MV_TILE;
      for (int64_t c0 = 0; c0 < g.ncols; c0 += MV_SEG_COLS) {
        MvSeg sg{};
        sg.c0 = (int32_t)c0;
        sg.c1 = (int32_t)std::min<int64_t>(g.ncols, c0 + MV_SEG_COLS);
        sg.soff = (int32_t)g.soff;
        sg.row_lo = (int16_t)lo;
        sg.row_hi = (int16_t)hi;
        sg.far = g.far;
        segs.push_back(SegT{(int32_t)T, (int32_t)gi, sg});
      }
    }
  }
  // dense-block segments first (launch 1 reads them with the phase-A items),
  // then low-rank segments; tile order within each group
  {
    // stable counting sort by (far, tile)
    const int64_t nT = (h->N + MV_TILE - 1) / MV_TILE;
    std::vector<int64_t> cnt(2 * nT + 1, 0);
    for (const SegT& t : segs) cnt[t.seg.far * nT + t.tile + 1]++;
    for (size_t b = 1; b < cnt.size(); b++) cnt[b] += cnt[b - 1];
    std::vector<SegT> sorted(segs.size());
    for (const SegT& t : segs) sorted[cnt[t.seg.far * nT + t.tile]++] = t;
    segs.swap(sorted);
  }
  tr.mark("  plan: groups, segments", s);
  h->nTiles = (int)((h->N + MV_TILE - 1) / MV_TILE);
  h->segs.assign(segs.size(), MvSeg{});
  h->seg_tile.assign(segs.size(), 0);
  h->block_pieces.assign(P.blk.size(), {});
  // stream offsets in segment order; every segment starts on a 128-byte line
  int64_t so = 0;
  for (size_t i = 0; i < segs.size(); i++) {
    MvSeg sg = segs[i].seg;
    const int64_t len = sg.row_hi - sg.row_lo;
    so = round_up(so, SEG_START_ALIGN);
    sg.so = so;
    so += len * (sg.c1 - sg.c0);
    h->segs[i] = sg;
    h->seg_tile[i] = segs[i].tile;
    const Group& g = groups[segs[i].group];
    for (int32_t b : g.members) {
      const int64_t nb = P.blk[b].far ? h->rank[h->kind_index[b]] : block_n(h, b);
      const int64_t lo_c = std::max<int64_t>(sg.c0, gcol[b]);
      const int64_t hi_c = std::min<int64_t>(sg.c1, gcol[b] + nb);
      if (lo_c >= hi_c) continue;
      h->block_pieces[b].push_back(hmat::Piece{(int32_t)i, (int32_t)(lo_c - gcol[b]),
                                               (int32_t)(hi_c - gcol[b]), sg.so + (lo_c - sg.c0) * len});
    }
  }
  tr.mark("  plan: offsets, pieces", s);

  h->stream_n = std::max<int64_t>(so, PANEL_ALIGN);
  h->ldxp = round_up(h->N, PANEL_ALIGN);
  // Host-side bounds check of every access the product kernels will make.
  {
    const int64_t far_n = (int64_t)(h->far_arena.bytes / sizeof(double));
    auto bad = [](const char* what) { throw HipError{HMAT_EDEVICE, std::string("internal: product plan: ") + what}; };
    for (const auto& items : items_l)
      for (const MvA& I : items) {
        if (I.ld == 0 && I.l1 == I.l0) continue;  // padding (no work)
        if (I.v_off < 0 || I.v_off % 2 || I.ld % 2 || I.a0 % 2 || I.a0 < 0) bad("phase A alignment");
        if (I.l0 < 0 || I.l1 <= I.l0 || I.l1 - I.l0 > 64) bad("phase A columns");
        if (I.v_off + (int64_t)I.l1 * I.ld > far_n) bad("phase A matrix range");
        if ((int64_t)I.a0 + I.ld > h->ldxp) bad("phase A vector range");
        if ((int64_t)I.zoff + (I.l1 - I.l0) > h->Ztot) bad("phase A output range");
      }
    for (const MvSeg& sg : h->segs) {
      if (sg.row_lo < 0 || sg.row_hi > MV_TILE || sg.row_lo >= sg.row_hi || sg.row_lo % 2) bad("phase B rows");
      if (sg.so % 2 || sg.so < 0) bad("phase B alignment");
      if (sg.so + (int64_t)(sg.row_hi - sg.row_lo) * (sg.c1 - sg.c0) > h->stream_n) bad("phase B matrix range");
      if ((int64_t)sg.soff + sg.c1 > (sg.far ? h->Ztot : h->N)) bad("phase B vector range");
    }
  }
  h->nSeg = (int)h->segs.size();
  tr.mark("  plan: chunks, checks", s);
  upload(h->d_seg, h->segs, s, "product plan");
  for (int l = 0; l < 2; l++) {
    upload(h->cl[l].d_items, items_l[l], s, "product plan");
    h->cl[l].nA = (int)items_l[l].size();
    set_chunk_list(h, l, l == 0 ? h->mv_chunk_bytes : multi_chunk_bytes(h), s);
  }

  if (h->d_xp.bytes < sizeof(double) * (MV_MAX_NR + 1) * h->ldxp) {
    // one vector at [0, ldxp), several side by side at [ldxp, (MV_MAX_NR + 1) ldxp);
    // rows [N, ldxp) of either stay zero: they meet only zero pad rows of V panels
    h->d_xp.alloc(sizeof(double) * (MV_MAX_NR + 1) * h->ldxp, "product workspace");
    check(hipMemsetAsync(h->d_xp.p, 0, h->d_xp.bytes, s), "product workspace");
  }
  h->d_z.alloc(sizeof(double) * MV_MAX_NR * h->Ztot, "product workspace");
  check(hipStreamSynchronize(s), "product plan");
}

// Stream tasks for every piece of the blocks selected by `want`, with the
// plain column-major source/destination of each block given by `mat(b)`.
template <class Want, class Mat>
std::vector<StreamTask> stream_tasks(const hmat* h, Want want, Mat mat) {
  std::vector<StreamTask> t;
  const Plan& P = h->plan;
  for (size_t b = 0; b < P.blk.size(); b++) {
    if (!want((int32_t)b)) continue;
    const int64_t R0 = 3 * (int64_t)P.cl[P.blk[b].t].off, m = block_m(h, (int32_t)b);
    double* ptr = mat((int32_t)b);
    for (const hmat::Piece& pc : h->block_pieces[b]) {
      const MvSeg& sg = h->segs[pc.seg];
      StreamTask st{};
      st.src = ptr;
      st.dst = ptr;
      st.so = pc.so;
      st.ld = (int32_t)m;
      st.r0 = (int32_t)((int64_t)h->seg_tile[pc.seg] * MV_TILE - R0);
      st.row_lo = sg.row_lo;
      st.row_hi = sg.row_hi;
      st.c0 = pc.bc0;
      st.c1 = pc.bc1;
      t.push_back(st);
    }
  }
  return t;
}

void fill_stats(hmat* h) {
  hmat_stats& st = h->st;
  const Plan& P = h->plan;
  st.n_dof = h->N;
  st.n_triangles = P.nt;
  st.n_clusters = (int32_t)P.cl.size();
  st.depth = P.depth;
  st.n_blocks = (int32_t)P.blk.size();
  st.n_far = (int32_t)h->far_blocks.size();
  st.n_near = (int32_t)h->near_blocks.size();
  st.c_sp = P.csp;
  st.rank_min = INT32_MAX;
  st.rank_max = 0;
  double rs = 0;
  st.far_scalars = 0;
  st.near_scalars = 0;
  st.far_u_scalars = 0;
  st.far_v_scalars = 0;
  st.n_rank_full = 0;
  st.n_near_threshold = 0;
  for (size_t f = 0; f < h->far_blocks.size(); f++) {
    const int32_t b = h->far_blocks[f], k = h->rank[f];
    st.rank_min = std::min(st.rank_min, k);
    st.rank_max = std::max(st.rank_max, k);
    rs += k;
    st.far_scalars += (int64_t)k * (block_m(h, b) + block_n(h, b));
    st.far_u_scalars += (int64_t)k * block_m(h, b);
    st.far_v_scalars += (int64_t)k * block_n(h, b);
    if (h->stop[f] == 2) st.n_rank_full++;
    if (h->ratio[f] >= 1.0 - 1e-9 && h->ratio[f] <= 1.0) st.n_near_threshold++;
  }
  if (h->far_blocks.empty()) st.rank_min = 0;
  st.rank_mean = h->far_blocks.empty() ? 0.0 : rs / h->far_blocks.size();
  for (int32_t b : h->near_blocks) st.near_scalars += block_m(h, b) * block_n(h, b);
  double dense = 0.0;  // sum over bodies of n_dof^2
  for (const hmat::Body& B : h->bodies) dense += 9.0 * (double)B.nt * (double)B.nt;
  st.compression = (double)(st.far_scalars + st.near_scalars) / dense;
  st.aca_passes = h->aca_passes;
  st.n_exact = h->n_exact;
  st.precision = h->fp32_only ? 1 : 0;
  st.aca_fp32 = h->fp32_aca ? 1 : 0;
  st.n_bodies = (int32_t)h->bodies.size();
  size_t piv_bytes = 0;
  for (const DevBuf& d : h->piv_bufs) piv_bytes += d.bytes;
  st.device_bytes = (int64_t)(h->d_cen.bytes + h->d_q.bytes + h->d_vtx.bytes + h->d_gl.bytes +
                              h->d_order.bytes + h->far_arena.bytes + h->stream.bytes +
                              piv_bytes + h->d_kc.bytes + h->cl[0].d_items.bytes + h->cl[1].d_items.bytes + h->d_seg.bytes +
                              h->cl[0].d_chunk.bytes + h->cl[0].d_tile_near.bytes + h->cl[0].d_tile_far.bytes +
                              h->cl[1].d_chunk.bytes + h->cl[1].d_tile_near.bytes + h->cl[1].d_tile_far.bytes + h->d_xp.bytes +
                              h->d_z.bytes + h->d_part.bytes + h->d_dotpart.bytes + h->d_Q.bytes +
                              h->d_w.bytes + h->d_small.bytes + h->far32.bytes + h->stream32.bytes +
                              h->d_ir.bytes);
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    check(hipEventCreate(&a), "event");
    check(hipEventCreate(&b), "event");
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  double ms() const {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    return t;
  }
};

// One ACA pass over the far blocks listed in `fidx` (largest first) with
// per-block capacity cap(f); panels in `panels`, pivots in `piv`. Each block
// resumes from and saves to states[f] and its row set at zbits + zoff[f]
// (zeroed state: a fresh start). prep(tasks) enqueues what must precede the
// launch. `wide`: 512-thread workgroups for the large blocks (later passes,
// which hold few).
template <class CapFn, class PanelFn, class PrepFn>
void run_aca_pass(hmat* h, const std::vector<int32_t>& fidx, CapFn cap, PanelFn get_panels, DevBuf& piv,
                  DevBuf& d_rank, DevBuf& d_stop, DevBuf& d_ratio,
                  std::vector<const void*>& panel_ptr, AcaState* states, uint32_t* zbits,
                  const std::vector<int64_t>& zoff, PrepFn prep, bool wide, hipStream_t s) {
  const Plan& P = h->plan;
  // largest blocks first (|t| + |s|), equal sizes in the given order
  std::vector<uint64_t> size(fidx.size());
  for (size_t q = 0; q < fidx.size(); q++) {
    const BlockRec& B = P.blk[h->far_blocks[fidx[q]]];
    size[q] = (uint64_t)P.cl[B.t].len + (uint64_t)P.cl[B.s].len;
  }
  const std::vector<int32_t> by_size = order_desc_stable(size);
  std::vector<int32_t> ord(fidx.size());
  for (size_t q = 0; q < fidx.size(); q++) ord[q] = fidx[by_size[q]];
  // blocks for the 256-thread kernel first, then the one-wave ones
  auto big = [&](int32_t f) {
    const BlockRec& B = P.blk[h->far_blocks[f]];
    return std::max(P.cl[B.t].len, P.cl[B.s].len) > h->aca_small_tri;
  };
  const int n_big = (int)(std::stable_partition(ord.begin(), ord.end(), big) - ord.begin());
  const int esize = h->fp32_aca ? 4 : 8;  // bytes per panel entry
  int64_t panel_total = 0, piv_total = 0;
  size_t shmem[2] = {0, 0};  // 256-thread part, one-wave part
  for (size_t q = 0; q < ord.size(); q++) {
    const int32_t b = h->far_blocks[ord[q]];
    const int64_t m = block_m(h, b), n = block_n(h, b);
    const int32_t kc = cap(ord[q]);
    panel_total += (m + n) * kc;
    piv_total += 2 * (int64_t)kc;
    size_t& sh = shmem[(int)q < n_big ? 0 : 1];
    sh = std::max(sh, aca_shmem(kc, m, n, (int)q < n_big ? (wide ? ACA_WIDE_NWV : ACA_NWV) : 1, esize));
  }
  if (std::max(shmem[0], shmem[1]) > 160 * 1024)
    throw HipError{HMAT_ENOTSUP, "ACA panel row exceeds LDS capacity"};
  char* const panels = static_cast<char*>(get_panels((size_t)esize * std::max<int64_t>(panel_total, 1)));
  piv.alloc(sizeof(int32_t) * piv_total, "ACA pivots");
  std::vector<AcaTask> tasks;
  tasks.reserve(ord.size());
  int64_t po = 0, vo = 0;
  for (int32_t f : ord) {
    const int32_t b = h->far_blocks[f];
    const BlockRec& B = P.blk[b];
    const int64_t m = block_m(h, b), n = block_n(h, b);
    const int32_t kc = cap(f);
    AcaTask t{};
    t.t_off = P.cl[B.t].off;
    t.t_len = P.cl[B.t].len;
    t.s_off = P.cl[B.s].off;
    t.s_len = P.cl[B.s].len;
    t.panel = panels + (size_t)esize * po;
    t.piv = piv.as<int32_t>() + vo;
    t.kcap = kc;
    t.blk = f;
    t.eps = h->bodies[h->pos_body[t.t_off]].eps * h->stop_factor;
    t.st = states + f;
    t.zbits = zbits + zoff[f];
    tasks.push_back(t);
    h->piv_ptr[f] = t.piv;
    h->piv_cap[f] = kc;
    panel_ptr[f] = t.panel;
    po += (m + n) * kc;
    vo += 2 * (int64_t)kc;
  }
  DevBuf d_tasks;
  upload(d_tasks, tasks, s, "ACA tasks");
  prep(tasks);
  EventPair ev;
  check(hipEventRecord(ev.a, s), "event");
  check(launch_aca(h->G, d_tasks.as<AcaTask>(), (int)tasks.size(), n_big, shmem[0], shmem[1], wide, h->fp32_aca,
                   d_rank.as<int32_t>(), d_stop.as<int32_t>(), d_ratio.as<double>(), s),
        "ACA launch");
  check(hipEventRecord(ev.b, s), "event");
  check(hipStreamSynchronize(s), "ACA");
  h->st.t_aca_kernel_ms += ev.ms();
}

// Fill the stream arena from plain column-major sources of the dense blocks
// (near_src + near_off[i]) and of the U factors (u_ptr[f], leading dimension m).
void fill_stream(hmat* h, const double* near_src, const std::vector<int64_t>& near_off,
                 const std::vector<const double*>& u_ptr, hipStream_t s, BuildTrace* tr = nullptr) {
  h->stream.alloc(sizeof(double) * h->stream_n, "product stream");
  if (tr) tr->mark("  stream: allocation", s);
  // the gaps that align segment starts are never read; keep them zero anyway
  check(hipMemsetAsync(h->stream.p, 0, h->stream.bytes, s), "product stream");
  if (tr) tr->mark("  stream: zero fill", s);
  auto tasks = stream_tasks(
      h, [&](int32_t b) { return !h->plan.blk[b].far || h->rank[h->kind_index[b]] > 0; },
      [&](int32_t b) -> double* {
        const int32_t idx = h->kind_index[b];
        return const_cast<double*>(h->plan.blk[b].far ? u_ptr[idx] : near_src + near_off[idx]);
      });
  DevBuf d_t;
  upload(d_t, tasks, s, "stream tasks");
  if (tr) tr->mark("  stream: tasks", s);
  check(launch_to_stream(d_t.as<StreamTask>(), (int)tasks.size(), h->stream.as<double>(), s), "stream fill");
  check(hipStreamSynchronize(s), "stream fill");
  if (tr) tr->mark("  stream: copies", s);
}

// One body of a build: mesh (HOST, borrowed) and its material and accuracy.
struct BodyIn {
  const hmat_mesh* mesh;
  double E, nu, eps;
};

// Plans of all bodies merged into one: triangles, clusters and blocks of body
// b follow those of bodies 0..b-1, offsets shifted; the block list stays in
// canonical (row_off, col_off) order. The meshes are concatenated likewise.
void merge_bodies(hmat* h, const std::vector<BodyIn>& in, double eta, int32_t leaf,
                  std::vector<double>& allV, std::vector<int32_t>& allT) {
  Plan& P = h->plan;
  P = Plan{};
  int32_t vtx_off = 0;
  for (const BodyIn& B : in) {
    Plan pb;
    make_plan(B.mesh, eta, leaf, pb);
    const int32_t tri_off = P.nt, cl_off = (int32_t)P.cl.size();
    for (int32_t o : pb.order) P.order.push_back(o + tri_off);
    for (Cluster c : pb.cl) {
      c.off += tri_off;
      if (c.son0 >= 0) {
        c.son0 += cl_off;
        c.son1 += cl_off;
      }
      P.cl.push_back(c);
    }
    for (BlockRec r : pb.blk) {
      r.t += cl_off;
      r.s += cl_off;
      P.blk.push_back(r);
    }
    P.csp = std::max(P.csp, pb.csp);
    P.depth = std::max(P.depth, pb.depth);
    P.nt += pb.nt;
    allV.insert(allV.end(), B.mesh->vertices, B.mesh->vertices + 3 * (size_t)B.mesh->n_vertices);
    for (int64_t e = 0; e < 3 * (int64_t)B.mesh->n_triangles; e++) allT.push_back(B.mesh->triangles[e] + vtx_off);
    vtx_off += B.mesh->n_vertices;
    h->bodies.push_back(hmat::Body{tri_off, pb.nt, B.E, B.nu, B.eps});
  }
  h->pos_body.assign(P.nt, 0);
  for (size_t b = 0; b < h->bodies.size(); b++)
    std::fill(h->pos_body.begin() + h->bodies[b].tri_off,
              h->pos_body.begin() + h->bodies[b].tri_off + h->bodies[b].nt, (int32_t)b);
}

thread_local int64_t g_aca_budget = 0;  // per-thread override (hm::set_thread_aca_budget)

// Bytes of first-pass ACA panels that one group may hold at once: the
// calling thread's override if set, else HMAT_ACA_BUDGET_MB, else a quarter
// of the free device memory (>= 1 GiB).
int64_t aca_budget() {
  if (g_aca_budget > 0) return g_aca_budget;
  if (const char* e = std::getenv("HMAT_ACA_BUDGET_MB")) return std::max(1L, std::atol(e)) << 20;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return (int64_t)1 << 30;
  }
  return std::max<int64_t>((int64_t)1 << 30, (int64_t)(fr / 4));
}

// Plan (tree, partition; several bodies merged), geometry upload and the
// dense blocks (K1) into a plain column-major staging arena: dense block i
// at near_off[i], m x n. Shared by the build and the adaptive multiplication.
void setup_dense(hmat* h, const std::vector<BodyIn>& in, double eta, int32_t leaf, hipStream_t s,
                 std::chrono::steady_clock::time_point t0, DevBuf& near_stage,
                 std::vector<int64_t>& near_off, EventPair& evn) {
  h->eta = eta;
  h->leaf = leaf;
  std::vector<double> allV;
  std::vector<int32_t> allT;
  merge_bodies(h, in, eta, leaf, allV, allT);
  const Plan& P = h->plan;
  const int32_t nt = P.nt;
  h->N = 3 * (int64_t)nt;
  h->inv_order.assign(nt, 0);
  for (int32_t p = 0; p < nt; p++) h->inv_order[P.order[p]] = p;
  HostGeometry hg;
  const hmat_mesh all{(int32_t)(allV.size() / 3), nt, allV.data(), allT.data()};
  make_geometry(&all, P, hg);
  upload(h->d_cen, hg.cen, s, "geometry");
  upload(h->d_q, hg.q, s, "geometry");
  upload(h->d_vtx, hg.vtx, s, "geometry");
  upload(h->d_gl, hg.gl, s, "geometry");
  upload(h->d_order, P.order, s, "geometry");
  std::vector<double> kc(2 * (size_t)nt);
  for (int32_t p = 0; p < nt; p++) {
    const hmat::Body& B = h->bodies[h->pos_body[p]];
    const double cK = (1.0 + B.nu) / (8.0 * M_PI * B.E * (1.0 - B.nu));
    kc[p] = cK * (3.0 - 4.0 * B.nu);
    kc[nt + p] = cK;
  }
  upload(h->d_kc, kc, s, "geometry");
  if (h->fp32_aca) {  // FP32 copies of the centroids and quadrature nodes for the FP32 ACA
    upload(h->d_cen32, std::vector<float>(hg.cen.begin(), hg.cen.end()), s, "geometry");
    upload(h->d_q32, std::vector<float>(hg.q.begin(), hg.q.end()), s, "geometry");
  }
  h->G = DevGeo{h->d_cen.as<double>(), h->d_q.as<double>(), h->d_vtx.as<double>(),
                h->d_gl.as<double>(), h->d_kc.as<double>(), h->d_cen32.as<float>(), h->d_q32.as<float>(),
                nt, 0, 0.0, 0.0};
  h->kind_index.assign(P.blk.size(), -1);
  for (size_t b = 0; b < P.blk.size(); b++) {
    if (P.blk[b].far) {
      h->kind_index[b] = (int32_t)h->far_blocks.size();
      h->far_blocks.push_back((int32_t)b);
    } else {
      h->kind_index[b] = (int32_t)h->near_blocks.size();
      h->near_blocks.push_back((int32_t)b);
    }
  }
  // K1 into a plain column-major staging arena (m x n per dense block)
  std::vector<NearTask> ntasks;
  std::vector<SelfTask> stasks(nt);
  int64_t noff = 0;
  for (int32_t b : h->near_blocks) {
    const BlockRec& B = P.blk[b];
    const Cluster& T = P.cl[B.t];
    const Cluster& S = P.cl[B.s];
    near_off.push_back(noff);
    ntasks.push_back(NearTask{T.off, T.len, S.off, S.len, noff, 3 * T.len, 0});
    if (B.t == B.s)
      for (int32_t p = 0; p < T.len; p++) stasks[T.off + p] = SelfTask{noff, 3 * T.len, 0, p, 0};
    noff += 9 * (int64_t)T.len * S.len;
  }
  {
    std::vector<char> seen(nt, 0);
    for (int32_t b : h->near_blocks)
      if (P.blk[b].t == P.blk[b].s)
        for (int32_t p = 0; p < P.cl[P.blk[b].t].len; p++) seen[P.cl[P.blk[b].t].off + p] = 1;
    for (int32_t p = 0; p < nt; p++)
      if (!seen[p]) throw HipError{HMAT_EDEVICE, "internal: triangle without diagonal dense block"};
  }
  for (const NearTask& t : ntasks)
    if (t.d_off + (int64_t)(3 * t.s_len) * t.ld > noff) throw HipError{HMAT_EDEVICE, "internal: dense block out of range"};
  h->st.t_plan_ms = ms_since(t0);
  near_stage.alloc(sizeof(double) * std::max<int64_t>(noff, 1), "dense blocks");
  DevBuf d_ntasks, d_stasks;
  upload(d_ntasks, ntasks, s, "dense tasks");
  upload(d_stasks, stasks, s, "self tasks");
  check(hipEventRecord(evn.a, s), "event");
  check(launch_near_only(h->G, d_ntasks.as<NearTask>(), (int)ntasks.size(), near_stage.as<double>(), s), "K1 launch");
  check(launch_self(h->G, d_stasks.as<SelfTask>(), near_stage.as<double>(), s), "K1 self launch");
  check(hipEventRecord(evn.b, s), "event");
}

struct BuildOpts {
  int precision = 0;         // 1: store the entries in FP32 only
  double stop_factor = 1.0;  // constant of the ACA stop test
  int32_t small_tri = ACA_SMALL_TRI;  // ACA schedule (see hmat_opts)
  bool wide = false;
};

hmat_status parse_opts(const hmat_opts* opts, double eps, BuildOpts& o, std::string& err) {
  if (!opts) return HMAT_OK;
  if (opts->precision != 0 && opts->precision != 1) {
    err = "precision must be 0 (FP64) or 1 (FP32)";
    return HMAT_EINVAL;
  }
  if (!(opts->aca_stop_factor > 0.0) || !(opts->aca_stop_factor * eps < 1.0)) {
    err = "aca_stop_factor must be > 0 with aca_stop_factor * eps < 1";
    return HMAT_EINVAL;
  }
  if (opts->aca_small_tri < 0 || opts->aca_small_tri > 1024) {
    err = "aca_small_tri must lie in 0..1024";
    return HMAT_EINVAL;
  }
  if (opts->aca_wide != 0 && opts->aca_wide != 1) {
    err = "aca_wide must be 0 or 1";
    return HMAT_EINVAL;
  }
  o.precision = opts->precision;
  o.stop_factor = opts->aca_stop_factor;
  o.small_tri = opts->aca_small_tri > 0 ? opts->aca_small_tri : ACA_SMALL_TRI;
  o.wide = opts->aca_wide == 1;
  return HMAT_OK;
}

hmat_status build_impl(const std::vector<BodyIn>& in, double eta, int32_t leaf, hipStream_t s,
                       hmat** out, const BuildOpts& opt = BuildOpts{}) {
  auto t0 = std::chrono::steady_clock::now();
  StreamScope scope(s);
  init_pool();
  hmat* h = new (std::nothrow) hmat();
  if (!h) return fail(HMAT_ENOMEM, "host allocation failed");
  h->last_stream = s;
  try {
    check(hipGetDevice(&h->device), "hipGetDevice");
    if (const char* e = std::getenv("HMAT_MV_CHUNK_KB")) h->mv_chunk_bytes = std::max(1L, std::atol(e)) * 1024;
    if (const char* e = std::getenv("HMAT_MV_UNROLL")) h->mv_unroll = std::atoi(e);
    h->eta = eta;
    h->leaf = leaf;
    h->fp32_only = opt.precision == 1;
    h->stop_factor = opt.stop_factor;
    h->aca_small_tri = opt.small_tri;
    h->aca_wide = opt.wide;
    // FP32 arithmetic resolves ACA remainders down to about 1e-6 of a block
    double eps_min = 1.0;
    for (const BodyIn& b : in) eps_min = std::min(eps_min, b.eps * opt.stop_factor);
    h->fp32_aca = h->fp32_only && eps_min >= 1e-5;
    DevBuf near_stage;
    std::vector<int64_t> near_off;
    EventPair evn;
    setup_dense(h, in, eta, leaf, s, t0, near_stage, near_off, evn);
    // K2: ACA in groups of far blocks (canonical order) whose first-pass
    // panels fit the budget; each group's factors are compacted into a plain
    // column-major staging buffer (U m x k, then V n x k) and its panels freed.
    const size_t nf = h->far_blocks.size();
    h->rank.assign(nf, 0);
    h->stop.assign(nf, 0);
    h->ratio.assign(nf, 0.0);
    h->piv_ptr.assign(nf, nullptr);
    h->piv_cap.assign(nf, 0);
    DevBuf d_rank, d_stop, d_ratio;
    d_rank.alloc(sizeof(int32_t) * std::max<size_t>(nf, 1), "ACA ranks");
    d_stop.alloc(sizeof(int32_t) * std::max<size_t>(nf, 1), "ACA ranks");
    d_ratio.alloc(sizeof(double) * std::max<size_t>(nf, 1), "ACA ranks");
    EventPair eva;
    check(hipEventRecord(eva.a, s), "event");
    std::vector<int32_t> kfirst(h->bodies.size());  // first-pass capacity of each body's blocks
    for (size_t q = 0; q < h->bodies.size(); q++) kfirst[q] = kcap_first(h->bodies[q].eps);
    auto cap1 = [&](int32_t f) {
      const int32_t b = h->far_blocks[f];
      const int32_t kf = kfirst[h->pos_body[h->plan.cl[h->plan.blk[b].t].off]];
      return (int32_t)std::min<int64_t>(std::min(block_m(h, b), block_n(h, b)), kf);
    };
    std::vector<int32_t> capv(nf, 0);
    // later passes: four times the previous capacity, at most min(m, n)
    auto cap_next = [&](int32_t f) {
      const int32_t b = h->far_blocks[f];
      return (int32_t)std::min<int64_t>(std::min(block_m(h, b), block_n(h, b)), 4 * (int64_t)capv[f]);
    };
    std::vector<const void*> panel_ptr(nf, nullptr);  // in the ACA precision
    std::vector<const double*> u_ptr(nf, nullptr), v_ptr(nf, nullptr);
    const int esize = h->fp32_aca ? 4 : 8;  // bytes per panel entry
    // ACA state of every far block (a block that fills its panels is
    // resumed from it in the next pass), zeroed: the first pass starts fresh
    std::vector<int64_t> zoff(nf, 0);
    int64_t ztot = 0;
    for (size_t f = 0; f < nf; f++) {
      zoff[f] = ztot;
      ztot += (block_m(h, h->far_blocks[f]) + 31) / 32;
    }
    DevBuf d_states, d_zbits, d_spans;
    d_states.alloc(sizeof(AcaState) * std::max<size_t>(nf, 1), "ACA state");
    d_zbits.alloc(sizeof(uint32_t) * std::max<int64_t>(ztot, 1), "ACA state");
    check(hipMemsetAsync(d_states.p, 0, d_states.bytes, s), "ACA state");
    check(hipMemsetAsync(d_zbits.p, 0, d_zbits.bytes, s), "ACA state");
    AcaState* const states = d_states.as<AcaState>();
    uint32_t* const zbits = d_zbits.as<uint32_t>();
    std::deque<DevBuf> ustage, vstage;
    int64_t staged_u = 0, staged_v = 0;  // bytes
    const int64_t budget = aca_budget();
    h->aca_passes = 0;
    PanelLease panels1(h->device, s);  // first-pass panels, reused by every group
    BuildTrace tr;
    tr.mark("plan, geometry, K1", s);
    for (size_t f0 = 0; f0 < nf;) {
      size_t f1 = f0;
      int64_t bytes = 0;
      while (f1 < nf) {
        const int32_t b = h->far_blocks[f1];
        const int64_t bb = esize * (block_m(h, b) + block_n(h, b)) * cap1((int32_t)f1);
        if (f1 > f0 && bytes + bb > budget) break;
        bytes += bb;
        f1++;
      }
      std::vector<int32_t> grp(f1 - f0);
      std::iota(grp.begin(), grp.end(), (int32_t)f0);
      for (int32_t f : grp) capv[f] = cap1(f);
      std::deque<DevBuf> panels_more;  // panels of the later passes (read by the compaction)
      int64_t later_bytes = 0;         // their bytes
      h->piv_bufs.emplace_back();
      run_aca_pass(h, grp, cap1, [&](size_t b) { return static_cast<void*>(panels1.get(b)); }, h->piv_bufs.back(), d_rank,
                   d_stop, d_ratio, panel_ptr, states, zbits, zoff, [](const std::vector<AcaTask>&) {},
                   h->aca_wide, s);
      h->aca_passes = std::max(h->aca_passes, 1);
      auto fetch = [&]() {
        check(hipMemcpyAsync(h->rank.data() + f0, d_rank.as<int32_t>() + f0, sizeof(int32_t) * (f1 - f0),
                             hipMemcpyDeviceToHost, s), "ranks");
        check(hipMemcpyAsync(h->stop.data() + f0, d_stop.as<int32_t>() + f0, sizeof(int32_t) * (f1 - f0),
                             hipMemcpyDeviceToHost, s), "ranks");
        check(hipStreamSynchronize(s), "ranks");
      };
      fetch();
      // blocks that filled their panels continue from their saved state with
      // a larger capacity (their panel columns and pivots so far are copied
      // over first; ACA is sequential, so the factors are those of an
      // uninterrupted run), until none fills its panels
      for (int pass = 2;; pass++) {
        std::vector<int32_t> again;
        for (int32_t f : grp)
          if (h->stop[f] == 4) again.push_back(f);
        if (again.empty()) break;
        std::vector<const char*> old_panel(nf, nullptr);
        std::vector<const int32_t*> old_piv(nf, nullptr);
        std::vector<int32_t> old_cap(nf, 0);
        for (int32_t f : again) {
          old_panel[f] = static_cast<const char*>(panel_ptr[f]);
          old_piv[f] = h->piv_ptr[f];
          old_cap[f] = capv[f];
          capv[f] = cap_next(f);
        }
        auto carry = [&](const std::vector<AcaTask>& tasks) {
          std::vector<SpanCopy> sp;
          sp.reserve(4 * tasks.size());
          auto span = [&](const void* src, void* dst, int64_t words) {
            sp.push_back(SpanCopy{static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst), words});
          };
          for (const AcaTask& t : tasks) {
            const int32_t f = t.blk, kc = old_cap[f];  // stop 4: k == kc columns so far
            const int64_t m = 3 * (int64_t)t.t_len, n = 3 * (int64_t)t.s_len, w = esize / 4;
            char* dst = static_cast<char*>(t.panel);
            span(old_panel[f], dst, w * m * kc);                                            // U
            span(old_panel[f] + esize * m * kc, dst + esize * m * t.kcap, w * n * kc);      // V
            span(old_piv[f], t.piv, kc);                                           // pivot rows
            span(old_piv[f] + kc, t.piv + t.kcap, kc);                             // pivot columns
          }
          upload(d_spans, sp, s, "ACA carry");
          check(launch_copy_spans(d_spans.as<SpanCopy>(), (int)sp.size(), s), "ACA carry");
        };
        // in sub-groups whose panels fit what is left of the ACA budget beside
        // the later-pass panels this group already holds (one block at least)
        for (size_t a0 = 0; a0 < again.size();) {
          size_t a1 = a0;
          int64_t bytes = 0;
          const int64_t avail = std::max<int64_t>(budget - later_bytes, 0);
          while (a1 < again.size()) {
            const int32_t b = h->far_blocks[again[a1]];
            const int64_t bb = esize * ((block_m(h, b) + block_n(h, b)) * (int64_t)capv[again[a1]]);
            if (a1 > a0 && bytes + bb > avail) break;
            bytes += bb;
            a1++;
          }
          const std::vector<int32_t> sub(again.begin() + a0, again.begin() + a1);
          panels_more.emplace_back();
          DevBuf& pb = panels_more.back();
          h->piv_bufs.emplace_back();
          run_aca_pass(h, sub, [&](int32_t f) { return capv[f]; },
                       [&](size_t b) {
                         if (pb.bytes < b) pb.alloc(b, "ACA panels");
                         return pb.p;
                       },
                       h->piv_bufs.back(), d_rank, d_stop, d_ratio, panel_ptr, states, zbits, zoff, carry,
                       true, s);
          later_bytes += (int64_t)pb.bytes;
          a0 = a1;
        }
        h->aca_passes = std::max(h->aca_passes, pass);
        fetch();
      }
      // blocks whose ACA reached full rank are stored exactly (U = B, V = I or
      // U = I, V = B^T) in their panels before the compaction
      {
        std::vector<ExactTask> ex;
        for (int32_t f : grp) {
          const int32_t b = h->far_blocks[f];
          const BlockRec& B = h->plan.blk[b];
          const auto& CL = h->plan.cl;
          if (h->rank[f] == std::min(block_m(h, b), block_n(h, b)))
            ex.push_back(ExactTask{CL[B.t].off, CL[B.t].len, CL[B.s].off, CL[B.s].len,
                                   const_cast<void*>(panel_ptr[f]), capv[f], 0});
        }
        if (!ex.empty()) {
          DevBuf d_ex;
          upload(d_ex, ex, s, "exact factors");
          check(launch_exact(h->G, d_ex.as<ExactTask>(), (int)ex.size(), h->fp32_aca, s), "exact factors");
          h->n_exact += (int32_t)ex.size();
        }
      }
      // U and V staged in separate buffers: the V staging is freed as soon as
      // the V arena is filled, before the stream arena is allocated
      int64_t totu = 0, totv = 0;
      for (int32_t f : grp) {
        const int32_t b = h->far_blocks[f];
        if (h->rank[f] > capv[f]) throw HipError{HMAT_EDEVICE, "internal: ACA rank beyond capacity"};
        totu += block_m(h, b) * h->rank[f];
        totv += block_n(h, b) * h->rank[f];
      }
      ustage.emplace_back();
      vstage.emplace_back();
      DevBuf& us = ustage.back();
      DevBuf& vs = vstage.back();
      us.alloc(sizeof(double) * std::max<int64_t>(totu, 1), "low-rank factors");
      vs.alloc(sizeof(double) * std::max<int64_t>(totv, 1), "low-rank factors");
      staged_u += (int64_t)us.bytes;
      staged_v += (int64_t)vs.bytes;
      std::vector<CopyTask> ct;
      std::vector<CopyTask32> ct32;  // FP32 panels, widened to the FP64 staging
      int64_t ou = 0, ov = 0;
      for (int32_t f : grp) {
        const int32_t b = h->far_blocks[f];
        const int32_t m = (int32_t)block_m(h, b), n = (int32_t)block_n(h, b), k = h->rank[f];
        u_ptr[f] = us.as<double>() + ou;
        v_ptr[f] = vs.as<double>() + ov;
        if (k > 0 && h->fp32_aca) {
          const float* pf = static_cast<const float*>(panel_ptr[f]);
          ct32.push_back(CopyTask32{pf, us.as<double>() + ou, m, k, m, 0});
          ct32.push_back(CopyTask32{pf + (int64_t)m * capv[f], vs.as<double>() + ov, n, k, n, 0});
        } else if (k > 0) {
          const double* pd = static_cast<const double*>(panel_ptr[f]);
          ct.push_back(CopyTask{pd, us.as<double>() + ou, m, k, m, 0});
          ct.push_back(CopyTask{pd + (int64_t)m * capv[f], vs.as<double>() + ov, n, k, n, 0});
        }
        ou += (int64_t)m * k;
        ov += (int64_t)n * k;
      }
      DevBuf d_ct, d_ct32;
      upload(d_ct, ct, s, "compaction tasks");
      upload(d_ct32, ct32, s, "compaction tasks");
      check(launch_compact(d_ct.as<CopyTask>(), (int)ct.size(), s), "compaction launch");
      check(launch_compact32(d_ct32.as<CopyTask32>(), (int)ct32.size(), s), "compaction launch");
      check(hipStreamSynchronize(s), "compaction");
      h->st.aca_groups++;
      f0 = f1;
      tr.mark("ACA group", s);
    }
    panels1.give_back();
    const auto t_layout = std::chrono::steady_clock::now();
    if (nf > 0) {
      check(hipMemcpyAsync(h->ratio.data(), d_ratio.p, sizeof(double) * nf, hipMemcpyDeviceToHost, s), "ranks");
      check(hipStreamSynchronize(s), "ranks");
      for (size_t f = 0; f < nf; f++)
        if (h->stop[f] == 5)
          throw HipError{HMAT_EINVAL, "non-finite matrix entries (overlapping or duplicate triangles?)"};
    }
    // V factors into the panel-layout arena
    const int64_t fo = far_layout(h);
    for (size_t f = 0; f < nf; f++)
      if (h->far_voff[f] + (int64_t)h->rank[f] * h->far_vshape[f].ld > fo)
        throw HipError{HMAT_EDEVICE, "internal: low-rank arena out of range"};
    h->far_arena.alloc(sizeof(double) * std::max<int64_t>(fo, PANEL_ALIGN), "low-rank arena");
    check(hipMemsetAsync(h->far_arena.p, 0, h->far_arena.bytes, s), "low-rank arena");
    std::vector<CopyTask> ct;
    for (size_t f = 0; f < nf; f++) {
      const int32_t b = h->far_blocks[f];
      const int32_t n = (int32_t)block_n(h, b), k = h->rank[f];
      if (k == 0) continue;
      ct.push_back(CopyTask{v_ptr[f], h->far_arena.as<double>() + h->far_voff[f], n, k,
                            h->far_vshape[f].ld, h->far_vshape[f].fp});
    }
    DevBuf d_ct;
    upload(d_ct, ct, s, "compaction tasks");
    check(launch_compact(d_ct.as<CopyTask>(), (int)ct.size(), s), "compaction launch");
    vstage.clear();  // stream-ordered: released after the compaction
    trim_pool_after(staged_v, s);
    tr.mark("V arena", s);
    // product plan, then U factors and dense blocks into the stream arena
    build_product_plan(h, s);
    tr.mark("product plan", s);
    fill_stream(h, near_stage.as<double>(), near_off, u_ptr, s, &tr);
    tr.mark("stream fill", s);
    check(hipEventRecord(eva.b, s), "event");
    check(hipStreamSynchronize(s), "build");
    h->st.t_layout_ms = ms_since(t_layout);
    ustage.clear();
    trim_pool_after(staged_u, s);
    if (h->fp32_only) {  // the FP32 arenas replace the FP64 ones (same layout)
      const int64_t nfar = (int64_t)(h->far_arena.bytes / sizeof(double));
      const int64_t nst = (int64_t)(h->stream.bytes / sizeof(double));
      h->far32.alloc(sizeof(float) * std::max<int64_t>(nfar, 2), "FP32 arenas");
      h->stream32.alloc(sizeof(float) * std::max<int64_t>(nst, 2), "FP32 arenas");
      check(launch_to_f32(h->far_arena.as<double>(), h->far32.as<float>(), nfar, s), "FP32 arenas");
      check(launch_to_f32(h->stream.as<double>(), h->stream32.as<float>(), nst, s), "FP32 arenas");
      h->far_arena.release();
      h->stream.release();
      check(hipStreamSynchronize(s), "FP32 arenas");
    }
    h->st.t_near_ms = evn.ms();
    h->st.t_aca_ms = eva.ms();
    fill_stats(h);
    h->st.t_build_ms = ms_since(t0);
    *out = h;
    return HMAT_OK;
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    delete h;
    return fail(e.st, e.msg);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    delete h;
    return fail(HMAT_ENOMEM, "host allocation failed");
  }
}

// Accumulate the elapsed times of recorded product groups (waits for them).
void prof_collect(hmat* h) {
  for (auto& e : h->prof_pending) {
    check(hipEventSynchronize(e[4]), "profile");
    for (int k = 0; k < 4; k++) {
      float t = 0.f;
      check(hipEventElapsedTime(&t, e[k], e[k + 1]), "profile");
      h->prof_ms[k] += t;
    }
    h->prof_calls++;
    for (hipEvent_t x : e) (void)hipEventDestroy(x);
  }
  h->prof_pending.clear();
}

// allow_prof = false: no per-phase events even while hmat_profile is on
// (the allocation-free solve creates no events). gathered = true (nrhs 1
// only): h->d_xp already holds x in cluster order, so the gather is skipped.
void matvec_impl(hmat* h, int prec, int32_t nrhs, const double* x, int64_t ldx, double* y,
                 int64_t ldy, hipStream_t s, bool allow_prof = true, bool gathered = false) {
  for (int32_t r0 = 0; r0 < nrhs; r0 += MV_MAX_NR) {
    const int nr = std::min<int32_t>(MV_MAX_NR, nrhs - r0);
    hipEvent_t* ev = nullptr;
    if (h->prof && allow_prof) {
      if (h->prof_pending.size() >= 4096) prof_collect(h);
      std::array<hipEvent_t, 5> e{};
      for (auto& q : e) check(hipEventCreate(&q), "profile");
      h->prof_pending.push_back(e);
      ev = h->prof_pending.back().data();
      check(hipEventRecord(ev[0], s), "profile");
    }
    if (!(gathered && nrhs == 1))
      check(launch_gather(nr, x + r0 * ldx, ldx, h->d_order.as<int32_t>(), h->N,
                          h->d_xp.as<double>(), h->ldxp, s),
            "gather");
    if (ev) check(hipEventRecord(ev[1], s), "profile");
    ProductPlanDev P{};

    const hmat::ChunkList& CL = h->cl[nr > 1 ? 1 : 0];
    P.items = CL.d_items.as<MvA>();
    P.chunks = CL.d_chunk.as<MvChunk>();
    P.segs = h->d_seg.as<MvSeg>();
    P.tile_near = CL.d_tile_near.as<int32_t>();
    P.tile_far = CL.d_tile_far.as<int32_t>();
    P.order = h->d_order.as<int32_t>();
    P.far = h->far_arena.as<double>();
    P.stream = h->stream.as<double>();
    P.far32 = h->far32.as<float>();
    P.stream32 = h->stream32.as<float>();
    P.nA = CL.nA;
    P.n_near_chunks = CL.n_near;
    P.n_far_chunks = CL.n - CL.n_near;
    P.ntiles = h->nTiles;
    P.N = h->N;
    check(launch_matvec_group(P, prec, nr, h->d_xp.as<double>(), h->ldxp, h->d_z.as<double>(), h->Ztot,
                              h->d_part.as<double>(), y + r0 * ldy, ldy, s, ev ? ev + 2 : nullptr,
                              h->mv_unroll),
          "product");
  }
}

// Copy the V panel of far block f into a plain column-major n x k host array.
void copy_v_out(const hmat* h, int32_t f, int64_t n, int64_t k, double* out) {
  if (k == 0) return;
  const PanelShape sh = h->far_vshape[f];
  std::vector<double> tmp((size_t)sh.ld * k);
  if (h->fp32_only) {
    std::vector<float> t32(tmp.size());
    check(hipMemcpy(t32.data(), h->far32.as<float>() + h->far_voff[f], sizeof(float) * t32.size(),
                    hipMemcpyDeviceToHost),
          "block copy");
    std::copy(t32.begin(), t32.end(), tmp.begin());
  } else {
    check(hipMemcpy(tmp.data(), h->far_arena.as<double>() + h->far_voff[f], sizeof(double) * tmp.size(),
                    hipMemcpyDeviceToHost),
          "block copy");
  }
  for (int64_t c = 0; c < k; c++) std::memcpy(out + c * n, tmp.data() + c * sh.ld + sh.fp, sizeof(double) * n);
}

// Copy block b's U factor or dense matrix (m x cols) out of the stream arena.
void copy_stream_out(const hmat* h, int32_t b, int64_t m, int64_t cols, double* out, hipStream_t s) {
  if (cols == 0) return;
  DevBuf tmp;
  tmp.alloc(sizeof(double) * m * cols, "block copy");
  auto tasks = stream_tasks(h, [&](int32_t bb) { return bb == b; }, [&](int32_t) { return tmp.as<double>(); });
  DevBuf d_t;
  upload(d_t, tasks, s, "block copy");
  if (h->fp32_only)
    check(launch_from_stream32(d_t.as<StreamTask>(), (int)tasks.size(), h->stream32.as<float>(), s), "block copy");
  else
    check(launch_from_stream(d_t.as<StreamTask>(), (int)tasks.size(), h->stream.as<double>(), s), "block copy");
  check(hipMemcpyAsync(out, tmp.p, sizeof(double) * m * cols, hipMemcpyDeviceToHost, s), "block copy");
  check(hipStreamSynchronize(s), "block copy");
}

// GMRES(m) for A_p x = b with x0 = 0, A_p the H-matrix with its entries
// stored in precision p (0: FP64, 1: FP32; FP64 arithmetic either way).
// Convergence on the explicit residual ||b - A_p x|| <= tol ||b||. Returns
// HMAT_OK or HMAT_ENOCONV; throws HipError on device errors.
constexpr int GM_COL = 1026;  // stride of a Hessenberg column buffer (restart <= 1024)

// Buffers of one GMRES(m) run: device Q (n_dof x (m+1)), w (n_dof), the
// partial sums (dots_part_size(n_dof, m+1) + norm_part_size(n_dof)) and the
// small buffer (4 GM_COL + 8); host: 3 GM_COL doubles for the Hessenberg
// columns and the update coefficients. With the two events the host reads
// column j while the device runs step j+1 (the host buffer is then pinned);
// without them every column copy is followed by a stream synchronisation.
struct GmresWs {
  double* Q = nullptr;
  double* w = nullptr;
  double* dotpart = nullptr;
  double* small = nullptr;
  double* host = nullptr;
  hipEvent_t* ev = nullptr;
};

size_t gmres_ws_doubles(int64_t N, int m, size_t* off) {
  auto up = [](size_t v) { return (v + 31) / 32 * 32; };  // 256-byte starts
  size_t o = 0;
  off[0] = o;  // Q
  o += up((size_t)N * (m + 1));
  off[1] = o;  // w
  o += up((size_t)N);
  off[2] = o;  // dot and norm partial sums
  o += up(dots_part_size(N, m + 1) + norm_part_size(N));
  off[3] = o;  // small
  o += up(4 * GM_COL + 8);
  return o;
}

// GMRES(m) workspace of the handle (grown, never shrunk). Allocation happens
// here, before any solve enqueues work, so no buffer is freed under a
// running kernel.
GmresWs ensure_gmres_ws(hmat* h, int m) {
  const int64_t N = h->N;
  if (h->q_cols < m + 1) {
    h->d_Q.alloc(sizeof(double) * N * (m + 1), "GMRES basis");
    h->q_cols = m + 1;
  }
  if (!h->d_w.p) h->d_w.alloc(sizeof(double) * N, "GMRES work");
  const size_t dp = dots_part_size(N, m + 1), np = norm_part_size(N);
  if (h->d_dotpart.bytes < sizeof(double) * (dp + np)) h->d_dotpart.alloc(sizeof(double) * (dp + np), "GMRES work");
  if (h->d_small.bytes < sizeof(double) * (4 * GM_COL + 8)) h->d_small.alloc(sizeof(double) * (4 * GM_COL + 8), "GMRES work");
  if (!h->h_pinned) {
    h->h_pinned = pinned_acquire();
    if (!h->h_pinned) throw HipError{HMAT_ENOMEM, "GMRES host buffer"};
  }
  for (hipEvent_t& e : h->col_ev)
    if (!e) check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "GMRES event");
  GmresWs ws;
  ws.Q = h->d_Q.as<double>();
  ws.w = h->d_w.as<double>();
  ws.dotpart = h->d_dotpart.as<double>();
  ws.small = h->d_small.as<double>();
  ws.host = h->h_pinned;
  ws.ev = h->col_ev;
  return ws;
}

hmat_status gmres_impl(hmat* h, int prec, const GmresWs& ws, const double* b, double* x, double tol,
                       int m, int maxit, hipStream_t s, int* used_out, int* restarts_out,
                       double* rel_out) {
  const int64_t N = h->N;
  constexpr int COL = GM_COL;
    const bool piped = ws.ev != nullptr;
    const size_t dp = dots_part_size(N, m + 1);
    double* dotpart = ws.dotpart;
    double* normpart = dotpart + dp;
    double* Q = ws.Q;
    double* w = ws.w;
    double* base = ws.small;
    double* hvec = base;                             // coefficients of one Gram-Schmidt pass
    double* hacc[2] = {base + COL, base + 2 * COL};  // Hessenberg columns, double-buffered
    double* ycoef = base + 3 * COL;                  // [m]
    double* scal = ycoef + COL;                      // scalars
    double* hcol_host[2] = {ws.host, ws.host + COL};
    double* y_host = ws.host + 2 * COL;
    auto norm_host = [&](const double* v) {
      check(launch_norm(v, N, normpart, scal, s), "norm");
      check(hipMemcpyAsync(y_host, scal, sizeof(double), hipMemcpyDeviceToHost, s), "norm");
      check(hipStreamSynchronize(s), "norm");
      return y_host[0];
    };
    // One Arnoldi step j: w = A q_j, two classical Gram-Schmidt passes against
    // q_0..q_j (Hessenberg column in hacc[j % 2]), q_{j+1} = w / ||w||, and the
    // column in host memory: written by the normalisation kernel into pinned
    // memory (event col_ev[j % 2]), or copied into ordinary host memory
    // (allocation-free solve). The normalisation also writes q_{j+1} in
    // cluster order into the product's input buffer, so step j+1's product
    // skips its gather; step 0 gathers (the residual's product uses that
    // buffer in between).
    auto enqueue_step = [&](int j) {
      double* col = hacc[j % 2];
      matvec_impl(h, prec, 1, Q + (size_t)j * N, N, w, N, s, piped, j > 0);
      for (int pass = 0; pass < 2; pass++)
        check(launch_cgs_pass(Q, N, N, j + 1, w, dotpart, hvec, col, pass == 0,
                              pass == 1 ? normpart : nullptr, s),
              "project");
      check(launch_scale_norm(w, N, normpart, col + j + 1, Q + (size_t)(j + 1) * N,
                              h->d_order.as<int32_t>(), h->d_xp.as<double>(), col, j + 1,
                              piped ? hcol_host[j % 2] : nullptr, s),
            "scale");
      if (piped) {
        check(hipEventRecord(ws.ev[j % 2], s), "hessenberg");
      } else {
        check(hipMemcpyAsync(hcol_host[j % 2], col, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, s),
              "hessenberg");
        check(hipStreamSynchronize(s), "hessenberg");
      }
    };
    check(launch_fill(x, N, 0.0, s), "fill");
    const double bn = norm_host(b);
    int used = 0, launched = 0, restarts = 0;
    double rel = 0.0;
    hmat_status status = HMAT_ENOCONV;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), yv(m);
    if (bn == 0.0) {
      status = HMAT_OK;
      rel = 0.0;
    } else {
      // x0 = 0: the first residual is b (b - 0, bit for bit), so neither a
      // product nor its norm is needed (scal[0] still holds ||b||)
      bool x_zero = true;
      for (;;) {
        if (x_zero)
          check(launch_fill(w, N, 0.0, s), "fill");
        else
          matvec_impl(h, prec, 1, x, N, w, N, s, piped);
        check(launch_residual(b, N, w, s), "residual");
        const double beta = x_zero ? bn : norm_host(w);
        x_zero = false;
        rel = beta / bn;
        if (beta <= tol * bn) {
          status = HMAT_OK;
          break;
        }
        if (launched >= maxit) break;
        check(launch_scale(w, N, scal, Q, s), "scale");  // scal[0] = ||r|| from norm_host
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        // Pipelined Arnoldi: step j+1 is enqueued before the host waits for
        // column j (it needs only device data), so the host's Givens update
        // overlaps the device's next product. A step enqueued past convergence
        // is discarded (a whole product); so when the residual estimate,
        // shrinking at twice its last rate, would meet the tolerance after
        // column j, step j+1 waits until column j has been checked (a held-back
        // step costs one host round trip, far less than a discarded one).
        enqueue_step(0);
        launched++;
        int j = 0, queued = 1;  // steps 0 .. queued - 1 of this cycle are enqueued
        double res = beta, res_prev = 0.0;  // residual estimates after j and j - 1 steps
        for (;;) {
          bool near = false;
          if (res_prev > 0.0) near = res * std::min(1.0, 0.5 * res / res_prev) <= tol * bn;
          if (!near && queued == j + 1 && j + 1 < m && launched < maxit) {
            enqueue_step(j + 1);
            launched++;
            queued++;
          }
          if (piped) check(hipEventSynchronize(ws.ev[j % 2]), "hessenberg");
          const double* col = hcol_host[j % 2];
          for (int i = 0; i <= j + 1; i++) H[(size_t)i * m + j] = col[i];
          const double hn = col[j + 1];
          for (int i = 0; i < j; i++) {
            const double a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
            H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
          }
          const double a = H[(size_t)j * m + j], c2 = H[(size_t)(j + 1) * m + j];
          const double den = std::sqrt(a * a + c2 * c2);
          cs[j] = den == 0.0 ? 1.0 : a / den;
          sn[j] = den == 0.0 ? 0.0 : c2 / den;
          H[(size_t)j * m + j] = cs[j] * a + sn[j] * c2;
          H[(size_t)(j + 1) * m + j] = 0.0;
          g[j + 1] = -sn[j] * g[j];
          g[j] = cs[j] * g[j];
          j++;
          used++;
          res_prev = res;
          res = std::fabs(g[j]);
          if (res <= tol * bn || hn == 0.0) break;
          if (queued == j) {  // step j was held back, or no step is left
            if (j >= m || launched >= maxit) break;
            enqueue_step(j);
            launched++;
            queued++;
          }
        }
        for (int i = j - 1; i >= 0; i--) {
          double sum = g[i];
          for (int q = i + 1; q < j; q++) sum -= H[(size_t)i * m + q] * yv[q];
          yv[i] = sum / H[(size_t)i * m + i];
        }
        // the pinned buffer is free again once the stream passes this copy
        check(hipStreamSynchronize(s), "update");
        std::memcpy(y_host, yv.data(), sizeof(double) * j);
        check(hipMemcpyAsync(ycoef, y_host, sizeof(double) * j, hipMemcpyHostToDevice, s), "update");
        if (!piped) check(hipStreamSynchronize(s), "update");  // y_host is ordinary host memory
        check(launch_add_comb(Q, N, N, j, ycoef, x, s), "update");
        restarts++;
      }
    }
  check(hipStreamSynchronize(s), "solve");
  *used_out = used;
  *restarts_out = restarts;
  *rel_out = rel;
  return status;
}

// Precision of the stored entries a call uses: FP64 unless only FP32 is stored.
inline int stored_prec(const hmat* h) { return h->fp32_only ? 1 : 0; }

hmat_status check_solve_args(hmat_t h, const double* b, const double* x, double tol,
                             int32_t restart, int32_t maxit) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (!b || !x) return fail(HMAT_EINVAL, "b or x is NULL");
  if (b == x) return fail(HMAT_EINVAL, "b and x alias");
  if (!(tol > 0.0)) return fail(HMAT_EINVAL, "tol must be > 0");
  if (restart < 1 || restart > 1024) return fail(HMAT_EINVAL, "restart must lie in [1, 1024]");
  if (maxit < 1) return fail(HMAT_EINVAL, "maxit must be >= 1");
  return HMAT_OK;
}

// Adaptive matrix-vector multiplication (Algorithm 2, Sec. 3) on the device:
// resumable ACA (k_aca with saved state, paused at a step count), the
// rank-two look-ahead contributions d_b = (A^_k - A_k)_b x_s per admissible
// block, and the marking (amvm.hip). A_0: dense blocks exact, admissible
// blocks of rank 0; the look-ahead adds two ACA steps per block; rows are
// visited in decreasing |(b^_k - b_k)_i| (ties: lower row first), blocks of a
// row in canonical order; a block joins P_k when its entry in that row
// reaches (1 - theta)(c_sp M N)^(-1/2) gamma_k; marking stops after the
// first row at which ||sum_{b not in P_k} d_b|| <= (1 - theta) gamma_k. Stop
// when gamma_k <= tol ||b^_k|| (relative tolerance) or after max_rounds.
hmat_status amvm_impl(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                      const double* x, double* y, double theta, double tol, int32_t max_rounds,
                      int32_t kmax, hipStream_t s, int32_t* ranks_out, hmat_amvm_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  StreamScope scope(s);
  init_pool();
  std::unique_ptr<hmat> hp(new (std::nothrow) hmat());
  if (!hp) return fail(HMAT_ENOMEM, "host allocation failed");
  hmat* h = hp.get();
  h->last_stream = s;
  constexpr int LOOK = 2;  // look-ahead ACA steps
  try {
    check(hipGetDevice(&h->device), "hipGetDevice");
    DevBuf near_stage;
    std::vector<int64_t> near_off;
    EventPair evn;
    setup_dense(h, {BodyIn{mesh, E, nu, 0.5}}, eta, leaf, s, t0, near_stage, near_off, evn);
    const Plan& P = h->plan;
    const int64_t N = h->N;
    const size_t nf = h->far_blocks.size();
    // x in cluster order
    DevBuf xp;
    xp.alloc(sizeof(double) * std::max<int64_t>(N, 1), "amvm vectors");
    check(launch_gather(1, x, N, h->d_order.as<int32_t>(), N, xp.as<double>(), N, s), "gather");
    // b_0: dense blocks
    std::vector<double> b(N, 0.0);
    {
      std::vector<DenseMvTask> dt;
      int64_t o = 0;
      for (size_t q = 0; q < h->near_blocks.size(); q++) {
        const int32_t bb = h->near_blocks[q];
        const int32_t m = (int32_t)block_m(h, bb), n = (int32_t)block_n(h, bb);
        dt.push_back(DenseMvTask{near_off[q], o, m, n, 3 * P.cl[P.blk[bb].s].off, 0});
        o += m;
      }
      DevBuf d_t, d_out;
      upload(d_t, dt, s, "amvm dense");
      d_out.alloc(sizeof(double) * std::max<int64_t>(o, 1), "amvm dense");
      check(launch_dense_mv(d_t.as<DenseMvTask>(), (int)dt.size(), near_stage.as<double>(), xp.as<double>(),
                            d_out.as<double>(), s), "amvm dense");
      std::vector<double> out(std::max<int64_t>(o, 1));
      check(hipMemcpyAsync(out.data(), d_out.p, sizeof(double) * o, hipMemcpyDeviceToHost, s), "amvm dense");
      check(hipStreamSynchronize(s), "amvm dense");
      for (size_t q = 0; q < h->near_blocks.size(); q++) {
        const int32_t bb = h->near_blocks[q];
        const int64_t R0 = 3 * (int64_t)P.cl[P.blk[bb].t].off, m = block_m(h, bb);
        for (int64_t r = 0; r < m; r++) b[R0 + r] += out[dt[q].out + r];
      }
    }
    // resumable ACA state of every admissible block
    std::vector<int32_t> kcap(nf), r_use(nf, 0), k_avail(nf, 0), done(nf, 0);
    std::vector<int64_t> poff(nf), zoff(nf), doff(nf), R0(nf), M(nf), Nn(nf);
    int64_t ptot = 0, ztot = 0, vtot = 0, dtot = 0;
    for (size_t f = 0; f < nf; f++) {
      const int32_t bb = h->far_blocks[f];
      M[f] = block_m(h, bb);
      Nn[f] = block_n(h, bb);
      R0[f] = 3 * (int64_t)P.cl[P.blk[bb].t].off;
      kcap[f] = (int32_t)std::min<int64_t>(std::min(M[f], Nn[f]), kmax);
      poff[f] = ptot;
      ptot += (M[f] + Nn[f]) * kcap[f];
      zoff[f] = ztot;
      ztot += (M[f] + 31) / 32;
      vtot += 2 * (int64_t)kcap[f];
      doff[f] = dtot;
      dtot += M[f];
    }
    DevBuf panels, pivs, states, zbits, d_back, d_ratio, d_d;
    panels.alloc(sizeof(double) * std::max<int64_t>(ptot, 1), "amvm panels");
    pivs.alloc(sizeof(int32_t) * std::max<int64_t>(vtot, 1), "amvm panels");
    states.alloc(sizeof(AcaState) * std::max<size_t>(nf, 1), "amvm state");
    zbits.alloc(sizeof(uint32_t) * std::max<int64_t>(ztot, 1), "amvm state");
    check(hipMemsetAsync(states.p, 0, states.bytes, s), "amvm state");
    check(hipMemsetAsync(zbits.p, 0, zbits.bytes, s), "amvm state");
    // what a round reads back, in one piece: the round's scalars, the order
    // of the candidate blocks, and the ACA ranks and stop codes
    const size_t nf1 = std::max<size_t>(nf, 1);
    const size_t back_bytes = sizeof(AmvmCtl) + 3 * sizeof(int32_t) * nf1;
    d_back.alloc(back_bytes, "amvm state");
    AmvmCtl* const dv_ctl = d_back.as<AmvmCtl>();
    int32_t* const dv_sf = reinterpret_cast<int32_t*>(dv_ctl + 1);
    int32_t* const dv_rank = dv_sf + nf1;
    int32_t* const dv_stop = dv_rank + nf1;
    d_ratio.alloc(sizeof(double) * nf1, "amvm state");
    d_d.alloc(sizeof(double) * std::max<int64_t>(dtot, 1), "amvm deltas");
    std::vector<AcaTask> base(nf);
    {
      int64_t vo = 0;
      for (size_t f = 0; f < nf; f++) {
        const BlockRec& B = P.blk[h->far_blocks[f]];
        AcaTask& t = base[f];
        t = AcaTask{};
        t.t_off = P.cl[B.t].off;
        t.t_len = P.cl[B.t].len;
        t.s_off = P.cl[B.s].off;
        t.s_len = P.cl[B.s].len;
        t.panel = panels.as<double>() + poff[f];
        t.piv = pivs.as<int32_t>() + vo;
        vo += 2 * (int64_t)kcap[f];
        t.kcap = kcap[f];
        t.blk = (int32_t)f;
        t.eps = 0.0;  // no accuracy test: steps are steered by the estimator
        t.cycle = 1;  // rows cycle through the components (coplanar clusters decouple them)
        t.st = states.as<AcaState>() + f;
        t.zbits = zbits.as<uint32_t>() + zoff[f];
      }
    }
    size_t shmem[2] = {0, 0};  // 256-thread blocks, one-wave blocks
    for (size_t f = 0; f < nf; f++) {
      const bool small = std::max(base[f].t_len, base[f].s_len) <= AMVM_SMALL_TRI;
      shmem[small ? 1 : 0] =
          std::max(shmem[small ? 1 : 0], aca_shmem(kcap[f], M[f], Nn[f], small ? 1 : ACA_WIDE_NWV));
    }
    if (std::max(shmem[0], shmem[1]) > 160 * 1024)
      throw HipError{HMAT_ENOTSUP, "ACA panel row exceeds LDS capacity"};
    // Leaf clusters: the rows of a leaf all lie in the same admissible blocks
    // (those whose row cluster contains the leaf), listed in canonical order.
    std::vector<AmvmLeaf> leaves;
    for (const Cluster& c : P.cl)
      if (c.son0 < 0) leaves.push_back(AmvmLeaf{3 * (int64_t)c.off, 0, 3 * c.len, 0});
    std::sort(leaves.begin(), leaves.end(), [](const AmvmLeaf& u, const AmvmLeaf& v) { return u.r0 < v.r0; });
    const int nl = (int)leaves.size();
    // leaves inside a block's row cluster: a contiguous range of `leaves`
    const auto leaf_range = [&](size_t f) {
      const auto lo = std::lower_bound(leaves.begin(), leaves.end(), R0[f],
                                       [](const AmvmLeaf& u, int64_t r) { return u.r0 < r; });
      const auto hi = std::lower_bound(lo, leaves.end(), R0[f] + M[f],
                                       [](const AmvmLeaf& u, int64_t r) { return u.r0 < r; });
      return std::make_pair(lo - leaves.begin(), hi - leaves.begin());
    };
    for (size_t f = 0; f < nf; f++) {
      const auto lr = leaf_range(f);
      for (auto l = lr.first; l < lr.second; l++) leaves[l].nb++;
    }
    int64_t ltot = 0;
    int nbmax = 0;
    for (AmvmLeaf& L : leaves) {
      L.b0 = ltot;
      ltot += L.nb;
      nbmax = std::max(nbmax, L.nb);
    }
    std::vector<int32_t> lblk(std::max<int64_t>(ltot, 1));
    {
      std::vector<int64_t> fill(nl);
      for (int l = 0; l < nl; l++) fill[l] = leaves[l].b0;
      for (size_t f = 0; f < nf; f++) {
        const auto lr = leaf_range(f);
        for (auto l = lr.first; l < lr.second; l++) lblk[fill[l]++] = (int32_t)f;
      }
    }
    if (amvm_leaf_shmem(nbmax) > 64 * 1024)
      throw HipError{HMAT_ENOTSUP, "adaptive multiplication: too many admissible blocks over one leaf cluster"};
    std::vector<int64_t> dbase(nf);
    std::vector<int32_t> mrow(nf);
    for (size_t f = 0; f < nf; f++) {
      dbase[f] = doff[f] - R0[f];
      mrow[f] = (int32_t)M[f];
    }
    DevBuf d_leaves, d_lblk, d_lsorted, d_lcount, d_has, d_dbase, d_doff, d_r0, d_mrow, d_dsq, d_restv, d_b, d_e,
        d_rkey, d_rval, d_rrank, d_part, d_bkey, d_pos, d_ds, d_sort;
    upload(d_leaves, leaves, s, "amvm leaves");
    upload(d_lblk, lblk, s, "amvm leaves");
    upload(d_dbase, dbase, s, "amvm blocks");
    upload(d_doff, doff, s, "amvm blocks");
    upload(d_r0, R0, s, "amvm blocks");
    upload(d_mrow, mrow, s, "amvm blocks");
    upload(d_b, b, s, "amvm vectors");
    const auto nz = [](int64_t v) { return (size_t)std::max<int64_t>(v, 1); };
    d_lsorted.alloc(sizeof(int32_t) * nz(ltot), "amvm leaves");
    d_lcount.alloc(sizeof(int32_t) * nz(nl), "amvm leaves");
    d_has.alloc(nz(nf), "amvm blocks");
    d_dsq.alloc(sizeof(double) * nz(dtot), "amvm deltas");
    d_restv.alloc(sizeof(double) * nz(dtot), "amvm deltas");
    d_e.alloc(sizeof(double) * nz(N), "amvm vectors");
    d_rkey.alloc(sizeof(uint64_t) * 2 * nz(N), "amvm sort");
    d_rval.alloc(sizeof(int32_t) * 2 * nz(N), "amvm sort");
    d_rrank.alloc(sizeof(int32_t) * nz(N), "amvm sort");
    d_part.alloc(sizeof(double) * 2 * nz(nl), "amvm sort");
    d_bkey.alloc(sizeof(uint64_t) * 2 * nz(nf), "amvm sort");
    d_pos.alloc(sizeof(int32_t) * nz(nf), "amvm sort");
    d_ds.alloc(sizeof(double) * nz(nf), "amvm sort");
    const size_t sort_bytes = amvm_sort_bytes(N, (int)nf);
    d_sort.alloc(sort_bytes, "amvm sort");
    AmvmDev A{};
    A.leaves = d_leaves.as<AmvmLeaf>();
    A.n_leaves = nl;
    A.nbmax = nbmax;
    A.nf = (int)nf;
    A.n = N;
    A.lblk = d_lblk.as<int32_t>();
    A.has_d = d_has.as<char>();
    A.dbase = d_dbase.as<int64_t>();
    A.doff = d_doff.as<int64_t>();
    A.r0 = d_r0.as<int64_t>();
    A.mrow = d_mrow.as<int32_t>();
    A.d = d_d.as<double>();
    A.b = d_b.as<double>();
    A.e = d_e.as<double>();
    A.part = d_part.as<double>();
    A.dsq = d_dsq.as<double>();
    A.restv = d_restv.as<double>();
    A.ds = d_ds.as<double>();
    A.rkey = d_rkey.as<uint64_t>();
    A.bkey = d_bkey.as<uint64_t>();
    A.rval = d_rval.as<int32_t>();
    A.rank = d_rrank.as<int32_t>();
    A.sf = dv_sf;
    A.pos = d_pos.as<int32_t>();
    A.lsorted = d_lsorted.as<int32_t>();
    A.lcount = d_lcount.as<int32_t>();
    A.ctl = dv_ctl;
    A.sort_tmp = d_sort.p;
    A.sort_bytes = sort_bytes;
    // per-block templates of the round's tasks, on the device
    std::vector<DeltaTask> tmpl(nf);
    for (size_t f = 0; f < nf; f++) {
      const double* pan = panels.as<double>() + poff[f];
      tmpl[f] = DeltaTask{pan, pan + M[f] * kcap[f], doff[f], (int32_t)M[f], (int32_t)Nn[f], 0, 0,
                          3 * P.cl[P.blk[h->far_blocks[f]].s].off, 0};
    }
    DevBuf d_base, d_tmpl, d_aca_list, d_dl_list, d_pf_list, d_tasks, d_pf_tasks, d_rank_pf, d_stop_pf, d_ratio_pf;
    upload(d_base, base, s, "amvm ACA");
    upload(d_tmpl, tmpl, s, "amvm deltas");
    d_aca_list.alloc(sizeof(int2) * nz(nf), "amvm ACA");
    d_pf_list.alloc(sizeof(int2) * nz(nf), "amvm ACA");
    d_dl_list.alloc(sizeof(int4) * nz(nf), "amvm deltas");
    d_tasks.alloc(sizeof(AcaTask) * nz(nf), "amvm ACA");
    d_pf_tasks.alloc(sizeof(AcaTask) * nz(nf), "amvm ACA");
    d_rank_pf.alloc(sizeof(int32_t) * nz(nf), "amvm ACA");
    d_stop_pf.alloc(sizeof(int32_t) * nz(nf), "amvm ACA");
    d_ratio_pf.alloc(sizeof(double) * nz(nf), "amvm ACA");
    check(hipMemsetAsync(d_has.p, 0, d_has.bytes, s), "amvm deltas");
    check(hipMemsetAsync(d_lcount.p, 0, d_lcount.bytes, s), "amvm leaves");
    // pinned host buffers: the round's lists (ACA: block, pause; deltas:
    // block, first column, last column, its source), what a round reads back
    // (scalars, order of the candidate blocks, ACA ranks and stop codes), and
    // the run-ahead launch's list and results
    struct Pinned {
      void* p = nullptr;
      ~Pinned() {
        if (p) (void)hipHostFree(p);
      }
    } up, back, pf_up, pf_back;
    check(hipHostMalloc(&up.p, (sizeof(int2) + sizeof(int4)) * nz(nf)), "amvm host buffer");
    check(hipHostMalloc(&back.p, back_bytes), "amvm host buffer");
    check(hipHostMalloc(&pf_up.p, sizeof(int2) * nz(nf)), "amvm host buffer");
    check(hipHostMalloc(&pf_back.p, 2 * sizeof(int32_t) * nz(nf)), "amvm host buffer");
    int2* const aca_list = (int2*)up.p;
    int4* const dl_list = (int4*)(aca_list + nz(nf));
    AmvmCtl* const ctl = (AmvmCtl*)back.p;
    int32_t* const sf = (int32_t*)(ctl + 1);
    int32_t* const rk = sf + nz(nf);
    int32_t* const sp = rk + nz(nf);
    int2* const pf_list = (int2*)pf_up.p;
    int32_t* const rk_pf = (int32_t*)pf_back.p;
    int32_t* const sp_pf = rk_pf + nz(nf);
    // The one-wave ACA launch runs beside the wide one on a second stream.
    // The largest blocks, whose two steps would outlast the rest of a round,
    // run ahead on a third: each round takes them to two windows past their
    // used rank (r_use + 4), so the window a round uses was computed during
    // the round before. The crosses are the same; only when they are computed
    // differs (a block's last run-ahead window may stay unused).
    struct Side {
      hipStream_t s2 = nullptr, s3 = nullptr;
      hipEvent_t fork = nullptr, join = nullptr, pf_done = nullptr;
      ~Side() {
        if (s3) (void)hipStreamSynchronize(s3);
        if (s2) (void)hipStreamSynchronize(s2);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (pf_done) (void)hipEventDestroy(pf_done);
        if (s2) (void)hipStreamDestroy(s2);
        if (s3) (void)hipStreamDestroy(s3);
      }
    } side;
    check(hipStreamCreateWithFlags(&side.s2, hipStreamNonBlocking), "amvm stream");
    check(hipStreamCreateWithFlags(&side.s3, hipStreamNonBlocking), "amvm stream");
    check(hipEventCreateWithFlags(&side.fork, hipEventDisableTiming), "amvm stream");
    check(hipEventCreateWithFlags(&side.join, hipEventDisableTiming), "amvm stream");
    check(hipEventCreateWithFlags(&side.pf_done, hipEventDisableTiming), "amvm stream");
    const double den = std::sqrt((double)P.csp * (double)N * (double)N);
    std::vector<char> adv(nf, 1);  // blocks marked in the last round (all at first)
    std::vector<char> big(nf), ahead(nf);
    for (size_t f = 0; f < nf; f++) {
      big[f] = std::max(base[f].t_len, base[f].s_len) > AMVM_SMALL_TRI;
      ahead[f] = big[f] && M[f] + Nn[f] >= AMVM_AHEAD_ROWS;
    }
    int n_pf = 0;
    bool pf_pending = false;
    const auto collect_ahead = [&]() {  // results of the last run-ahead launch
      if (!pf_pending) return;
      check(hipEventSynchronize(side.pf_done), "amvm stream");
      for (int q = 0; q < n_pf; q++) {
        const int32_t f = pf_list[q].x;
        if (sp_pf[f] == 5) throw HipError{HMAT_EINVAL, "non-finite matrix entries (overlapping or duplicate triangles?)"};
        k_avail[f] = rk_pf[f];
        done[f] = sp_pf[f] != 6;
      }
      pf_pending = false;
    };
    int rounds = 0;
    int64_t marked_total = 0;
    double gamma = 0.0;
    for (;;) {
      collect_ahead();
      // (a) resume ACA up to r_use + LOOK on the marked blocks that need it
      // (wide launch first in the list), the run-ahead blocks up to
      // r_use + 2 LOOK, and (b) recompute d_b for the marked blocks: the
      // windows of the others have not moved
      int na = 0, nd = 0;
      for (int pass = 0; pass < 2; pass++)
        for (size_t f = 0; f < nf; f++) {
          if (!adv[f] || done[f] || ahead[f] || big[f] != (pass == 0)) continue;
          const int32_t target = std::min(r_use[f] + LOOK, kcap[f]);
          if (k_avail[f] < target) aca_list[na++] = int2{(int)f, target};
        }
      int n_big = 0;
      while (n_big < na && big[aca_list[n_big].x]) n_big++;
      n_pf = 0;
      for (size_t f = 0; f < nf; f++) {
        if (!ahead[f] || done[f]) continue;
        const int32_t target = std::min(r_use[f] + 2 * LOOK, kcap[f]);
        if (k_avail[f] < target) pf_list[n_pf++] = int2{(int)f, target};
      }
      const bool first = rounds == 0 && !pf_pending;  // the first window of a run-ahead block is computed now
      for (size_t f = 0; f < nf; f++) {
        if (!adv[f]) continue;
        if (ahead[f] && !first)  // its window is known: computed during the last round
          dl_list[nd++] = int4{(int)f, r_use[f], std::min(r_use[f] + LOOK, k_avail[f]), 2};
        else
          dl_list[nd++] = int4{(int)f, r_use[f], 0, ahead[f] ? 1 : 0};
      }
      if (n_pf > 0) {
        check(hipMemcpyAsync(d_pf_list.p, pf_list, sizeof(int2) * n_pf, hipMemcpyHostToDevice, side.s3), "amvm ACA");
        check(launch_amvm_aca_tasks(d_base.as<AcaTask>(), d_pf_list.as<int2>(), n_pf, d_pf_tasks.as<AcaTask>(),
                                    side.s3), "amvm ACA");
        check(launch_aca(h->G, d_pf_tasks.as<AcaTask>(), n_pf, n_pf, shmem[0], shmem[1], true, false,
                         d_rank_pf.as<int32_t>(), d_stop_pf.as<int32_t>(), d_ratio_pf.as<double>(), side.s3),
              "amvm ACA");
        check(hipMemcpyAsync(rk_pf, d_rank_pf.p, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, side.s3), "amvm ACA");
        check(hipMemcpyAsync(sp_pf, d_stop_pf.p, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, side.s3), "amvm ACA");
        check(hipEventRecord(side.pf_done, side.s3), "amvm stream");
        pf_pending = true;
      }
      if (na > 0) {
        check(hipMemcpyAsync(d_aca_list.p, aca_list, sizeof(int2) * na, hipMemcpyHostToDevice, s), "amvm ACA");
        check(launch_amvm_aca_tasks(d_base.as<AcaTask>(), d_aca_list.as<int2>(), na, d_tasks.as<AcaTask>(), s),
              "amvm ACA");
        check(hipEventRecord(side.fork, s), "amvm stream");
        check(hipStreamWaitEvent(side.s2, side.fork, 0), "amvm stream");
        check(launch_aca(h->G, d_tasks.as<AcaTask>(), n_big, n_big, shmem[0], shmem[1], true, false,
                         dv_rank, dv_stop, d_ratio.as<double>(), s), "amvm ACA");
        check(launch_aca(h->G, d_tasks.as<AcaTask>() + n_big, na - n_big, 0, shmem[0], shmem[1], true, false,
                         dv_rank, dv_stop, d_ratio.as<double>(), side.s2), "amvm ACA");
        check(hipEventRecord(side.join, side.s2), "amvm stream");
        check(hipStreamWaitEvent(s, side.join, 0), "amvm stream");
      }
      if (first && n_pf > 0) check(hipStreamWaitEvent(s, side.pf_done, 0), "amvm stream");
      if (nd > 0) {
        check(hipMemcpyAsync(d_dl_list.p, dl_list, sizeof(int4) * nd, hipMemcpyHostToDevice, s), "amvm deltas");
        check(launch_lowrank_delta(d_tmpl.as<DeltaTask>(), d_dl_list.as<int4>(), nd, dv_rank,
                                   d_rank_pf.as<int32_t>(), LOOK, xp.as<double>(), d_d.as<double>(), d_has.as<char>(),
                                   s), "amvm deltas");
      }
      // (c) the estimator and a candidate P_k, on the device
      check(launch_amvm_estimate(A, theta, den, s), "amvm estimator");
      check(launch_amvm_stop(A, theta, 0, s), "amvm marking");
      check(hipMemcpyAsync(back.p, d_back.p, back_bytes, hipMemcpyDeviceToHost, s), "amvm marking");
      check(hipStreamSynchronize(s), "amvm marking");
      for (int q = 0; q < na; q++) {
        const int32_t f = aca_list[q].x;
        if (sp[f] == 5) throw HipError{HMAT_EINVAL, "non-finite matrix entries (overlapping or duplicate triangles?)"};
        k_avail[f] = rk[f];
        done[f] = sp[f] != 6;
      }
      if (first) collect_ahead();  // the run-ahead blocks' first windows were waited for
      std::fill(adv.begin(), adv.end(), 0);
      // no block with a window (all exhausted) gives gamma = 0 and stops here
      gamma = std::sqrt(ctl->g2);
      if (gamma <= tol * std::sqrt(ctl->bh2) || rounds >= max_rounds) break;
      // (d) the first candidate whose exact rest norm reaches the goal
      const double goal = (1.0 - theta) * gamma;
      while (ctl->p_cand < ctl->ncand && !(std::sqrt(ctl->exact2) <= goal)) {
        check(launch_amvm_stop(A, theta, ctl->p_cand, s), "amvm marking");
        check(hipMemcpyAsync(ctl, dv_ctl, sizeof(AmvmCtl), hipMemcpyDeviceToHost, s), "amvm marking");
        check(hipStreamSynchronize(s), "amvm marking");
      }
      const int32_t pk = ctl->p_cand;
      if (pk == 0) break;
      // (e) A_{k+1} = A^_k on the marked blocks
      check(launch_amvm_update(A, pk, s), "amvm update");
      for (int32_t j = 0; j < pk; j++) {
        const int32_t f = sf[j];
        r_use[f] = std::min(r_use[f] + LOOK, k_avail[f]);
        adv[f] = 1;
      }
      marked_total += pk;
      rounds++;
    }
    collect_ahead();
    // result in the caller's order
    check(launch_amvm_out(d_b.as<double>(), h->d_order.as<int32_t>(), N, y, s), "amvm result");
    check(hipStreamSynchronize(s), "amvm result");
    if (ranks_out) {
      for (size_t q = 0; q < P.blk.size(); q++) ranks_out[q] = -1;
      for (size_t f = 0; f < nf; f++) ranks_out[h->far_blocks[f]] = r_use[f];
    }
    if (info) {
      int64_t steps = 0;
      int32_t exhausted = 0;
      for (size_t f = 0; f < nf; f++) {
        steps += k_avail[f];
        exhausted += done[f] ? 1 : 0;
      }
      info->rounds = rounds;
      info->aca_steps = steps;
      info->marked_total = marked_total;
      info->exhausted = exhausted;
      info->gamma = gamma;
      info->time_ms = ms_since(t0);
    }
    check(hipStreamSynchronize(s), "amvm");
    return HMAT_OK;
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.st, e.msg);
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(s);
    return fail(HMAT_ENOMEM, "host allocation failed");
  }
}

}  // namespace

void hm::set_thread_aca_budget(int64_t bytes) { g_aca_budget = bytes > 0 ? bytes : 0; }

void hm::serving_pool(bool begin) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pool_servers += begin ? 1 : -1;
  apply_pool_threshold();
}

extern "C" {

const char* hmat_last_error(void) { return g_err.c_str(); }

hmat_status hmat_build(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                       double eps, void* hip_stream, hmat_t* out) {
  if (!out) return fail(HMAT_EINVAL, "out is NULL");
  *out = nullptr;
  std::string err;
  hmat_status st = validate_params(E, nu, eta, leaf, eps, err);
  if (st != HMAT_OK) return fail(st, err);
  st = validate_mesh(mesh, err);
  if (st != HMAT_OK) return fail(st, err);
  g_err.clear();
  return build_impl({BodyIn{mesh, E, nu, eps}}, eta, leaf, (hipStream_t)hip_stream, out);
}

hmat_status hmat_build_ex(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                          double eps, const hmat_opts* opts, void* hip_stream, hmat_t* out) {
  if (!out) return fail(HMAT_EINVAL, "out is NULL");
  *out = nullptr;
  BuildOpts o;
  std::string err;
  if (parse_opts(opts, eps, o, err) != HMAT_OK) return fail(HMAT_EINVAL, err);
  hmat_status st = validate_params(E, nu, eta, leaf, eps, err);
  if (st != HMAT_OK) return fail(st, err);
  st = validate_mesh(mesh, err);
  if (st != HMAT_OK) return fail(st, err);
  g_err.clear();
  return build_impl({BodyIn{mesh, E, nu, eps}}, eta, leaf, (hipStream_t)hip_stream, out, o);
}

hmat_status hmat_tune_aca(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf, double eps,
                          const hmat_opts* opts, int32_t reps, void* hip_stream, hmat_aca_tune_info* info) {
  if (!info) return fail(HMAT_EINVAL, "info is NULL");
  if (reps < 1) return fail(HMAT_EINVAL, "reps must be >= 1");
  BuildOpts base;
  std::string err;
  if (opts) {
    hmat_opts o = *opts;
    o.aca_small_tri = 0;
    o.aca_wide = 0;
    if (parse_opts(&o, eps, base, err) != HMAT_OK) return fail(HMAT_EINVAL, err);
  }
  hmat_status st = validate_params(E, nu, eta, leaf, eps, err);
  if (st != HMAT_OK) return fail(st, err);
  st = validate_mesh(mesh, err);
  if (st != HMAT_OK) return fail(st, err);
  g_err.clear();
  *info = hmat_aca_tune_info{};
  int n = 0;
  for (int32_t small : {32, 64, 128})
    for (int32_t wide : {0, 1}) {
      BuildOpts o = base;
      o.small_tri = small;
      o.wide = wide == 1;
      double best = INFINITY;
      for (int r = 0; r < reps; r++) {
        hmat* h = nullptr;
        st = build_impl({BodyIn{mesh, E, nu, eps}}, eta, leaf, (hipStream_t)hip_stream, &h, o);
        if (st != HMAT_OK) return st;
        best = std::min(best, h->st.t_aca_kernel_ms);
        hmat_free(h);
      }
      info->small_tri[n] = small;
      info->wide[n] = wide;
      info->aca_ms[n] = best;
      if (n == 0 || best < info->best_ms) {
        info->best = n;
        info->best_ms = best;
      }
      n++;
    }
  info->n_candidates = n;
  return HMAT_OK;
}

hmat_status hmat_build_batch(int32_t n_bodies, const hmat_mesh* meshes, const double* E,
                             const double* nu, const double* eps, double eta, int32_t leaf,
                             void* hip_stream, hmat_t* out) {
  if (!out) return fail(HMAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_bodies < 1) return fail(HMAT_EINVAL, "n_bodies must be >= 1");
  if (!meshes || !E || !nu || !eps) return fail(HMAT_EINVAL, "meshes, E, nu or eps is NULL");
  std::vector<BodyIn> in;
  int64_t nt = 0, nv = 0;
  for (int32_t b = 0; b < n_bodies; b++) {
    std::string err;
    hmat_status st = validate_params(E[b], nu[b], eta, leaf, eps[b], err);
    if (st == HMAT_OK) st = validate_mesh(&meshes[b], err);
    if (st != HMAT_OK) return fail(st, "body " + std::to_string(b) + ": " + err);
    nt += meshes[b].n_triangles;
    nv += meshes[b].n_vertices;
    in.push_back(BodyIn{&meshes[b], E[b], nu[b], eps[b]});
  }
  if (nt > INT32_MAX / 3 || nv > INT32_MAX) return fail(HMAT_EINVAL, "batch too large (triangles or vertices beyond 32-bit indexing)");
  g_err.clear();
  return build_impl(in, eta, leaf, (hipStream_t)hip_stream, out);
}

hmat_status hmat_amvm(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                      const double* x, double* y, double theta, double tol, int32_t max_rounds,
                      int32_t kmax, void* hip_stream, int32_t* ranks, hmat_amvm_info* info) {
  std::string err;
  hmat_status st = validate_params(E, nu, eta, leaf, 0.5, err);
  if (st == HMAT_OK) st = validate_mesh(mesh, err);
  if (st != HMAT_OK) return fail(st, err);
  if (!x || !y) return fail(HMAT_EINVAL, "x or y is NULL");
  if (!(theta > 0.0 && theta < 1.0)) return fail(HMAT_EINVAL, "theta must lie in (0, 1)");
  if (!(tol > 0.0)) return fail(HMAT_EINVAL, "tol must be > 0");
  if (max_rounds < 0) return fail(HMAT_EINVAL, "max_rounds must be >= 0");
  if (kmax < 2 || kmax > 4096) return fail(HMAT_EINVAL, "kmax must lie in [2, 4096]");
  if (x == y) return fail(HMAT_EINVAL, "x and y alias");
  g_err.clear();
  return amvm_impl(mesh, E, nu, eta, leaf, x, y, theta, tol, max_rounds, kmax,
                   (hipStream_t)hip_stream, ranks, info);
}

hmat_status hmat_matvec_graph(hmat_t h, int32_t precision, int32_t nrhs, const double* x,
                              int64_t ldx, double* y, int64_t ldy, void* hip_stream) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (precision != 0 && precision != 1) return fail(HMAT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (precision == 1 && !h->far32.p && !h->stream32.p)
    return fail(HMAT_EINVAL, "no FP32 copy: call hmat_set_precision(h, 1, ...) first");
  if (precision == 0 && h->fp32_only) return fail(HMAT_ENOTSUP, "the handle stores FP32 entries only");
  if (!x || !y) return fail(HMAT_EINVAL, "x or y is NULL");
  if (nrhs < 1 || nrhs > 64) return fail(HMAT_EINVAL, "nrhs must lie in [1, 64]");
  if (ldx < h->N || ldy < h->N) return fail(HMAT_EINVAL, "ldx and ldy must be >= n_dof");
  const char* xa = (const char*)x;
  const char* xb = (const char*)(x + (nrhs - 1) * ldx + h->N);
  const char* ya = (const char*)y;
  const char* yb = (const char*)(y + (nrhs - 1) * ldy + h->N);
  if (xa < yb && ya < xb) return fail(HMAT_EINVAL, "x and y overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  try {
    if (!h->graph_stream) {
      check(hipStreamCreateWithFlags(&h->graph_stream, hipStreamNonBlocking), "graph stream");
      check(hipEventCreateWithFlags(&h->graph_done, hipEventDisableTiming), "graph stream");
    }
    const hmat::GraphKey key{precision, nrhs, x, ldx, y, ldy};
    hipGraphExec_t exec = nullptr;
    for (auto& g : h->graphs)
      if (g.first == key) exec = g.second;
    if (!exec) {
      // capture the product's launches (no allocation, no memset inside)
      const bool prof = h->prof;
      h->prof = false;
      hipGraph_t graph = nullptr;
      check(hipStreamBeginCapture(h->graph_stream, hipStreamCaptureModeThreadLocal), "graph capture");
      try {
        matvec_impl(h, precision, nrhs, x, ldx, y, ldy, h->graph_stream);
      } catch (...) {
        (void)hipStreamEndCapture(h->graph_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        h->prof = prof;
        throw;
      }
      h->prof = prof;
      check(hipStreamEndCapture(h->graph_stream, &graph), "graph capture");
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      check(e, "graph instantiate");
      if (h->graphs.size() >= 256) {  // bounded cache: drop the oldest
        if (h->graph_live) (void)hipEventSynchronize(h->graph_done);
        (void)hipGraphExecDestroy(h->graphs.front().second);
        h->graphs.erase(h->graphs.begin());
      }
      h->graphs.push_back({key, exec});
    }
    // replayed on the caller's stream; the event marks the latest replay so
    // that dropping the graphs can wait for it
    check(hipGraphLaunch(exec, s), "graph launch");
    check(hipEventRecord(h->graph_done, s), "graph launch");
    h->graph_live = true;
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

hmat_status hmat_tune(hmat_t h, int32_t nrhs, int32_t reps, void* hip_stream, hmat_tune_info* info) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (nrhs < 1 || nrhs > MV_MAX_NR) return fail(HMAT_EINVAL, "nrhs must lie in [1, 16]");
  if (reps < 1 || reps > 1000) return fail(HMAT_EINVAL, "reps must lie in [1, 1000]");
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  // candidates: (chunk KB, columns per batch of the single-vector kernels)
  std::vector<std::pair<int, int>> cand;
  if (nrhs == 1) {
    for (int kb : {8, 16, 32, 64})
      for (int u : {8, 16}) cand.push_back({kb, u});
  } else {
    for (int kb : {64, 128, 256, 512}) cand.push_back({kb, h->mv_unroll});
  }
  const int l = nrhs > 1 ? 1 : 0;
  try {
    DevBuf dx, dy;
    dx.alloc(sizeof(double) * h->N * nrhs, "tune vectors");
    dy.alloc(sizeof(double) * h->N * nrhs, "tune vectors");
    check(launch_fill(dx.as<double>(), h->N * nrhs, 1.0, s), "tune vectors");
    EventPair ev;
    std::vector<double> ms(cand.size(), 0.0);
    size_t best = 0;
    for (size_t c = 0; c < cand.size(); c++) {
      set_chunk_list(h, l, (int64_t)cand[c].first * 1024, s);
      h->mv_unroll = cand[c].second;
      matvec_impl(h, stored_prec(h), nrhs, dx.as<double>(), h->N, dy.as<double>(), h->N, s);  // warm-up
      check(hipEventRecord(ev.a, s), "tune");
      for (int r = 0; r < reps; r++)
        matvec_impl(h, stored_prec(h), nrhs, dx.as<double>(), h->N, dy.as<double>(), h->N, s);
      check(hipEventRecord(ev.b, s), "tune");
      check(hipEventSynchronize(ev.b), "tune");
      ms[c] = ev.ms() / reps;
      if (ms[c] < ms[best]) best = c;
    }
    if (l == 0) {
      h->mv_chunk_bytes = (int64_t)cand[best].first * 1024;
      h->mv_unroll = cand[best].second;
    } else {
      h->mv_chunk_bytes_multi = (int64_t)cand[best].first * 1024;
    }
    set_chunk_list(h, l, (int64_t)cand[best].first * 1024, s);
    check(hipStreamSynchronize(s), "tune");
    if (info) {
      *info = hmat_tune_info{};
      info->nrhs = nrhs;
      info->n_candidates = (int32_t)std::min<size_t>(cand.size(), 8);
      for (size_t c = 0; c < cand.size() && c < 8; c++) {
        info->chunk_kb[c] = cand[c].first;
        info->unroll[c] = cand[c].second;
        info->ms[c] = ms[c];
      }
      info->best = (int32_t)best;
      info->best_ms = ms[best];
    }
    fill_stats(h);
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

hmat_status hmat_bodies(hmat_t h, int32_t* n_bodies, int64_t* dof_off) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (n_bodies) *n_bodies = (int32_t)h->bodies.size();
  if (dof_off) {
    for (size_t b = 0; b < h->bodies.size(); b++) dof_off[b] = 3 * (int64_t)h->bodies[b].tri_off;
    dof_off[h->bodies.size()] = h->N;
  }
  return HMAT_OK;
}

hmat_status hmat_matvec(hmat_t h, int32_t nrhs, const double* x, int64_t ldx, double* y,
                        int64_t ldy, void* hip_stream) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (!x || !y) return fail(HMAT_EINVAL, "x or y is NULL");
  if (nrhs < 1 || nrhs > 64) return fail(HMAT_EINVAL, "nrhs must lie in [1, 64]");
  if (ldx < h->N || ldy < h->N) return fail(HMAT_EINVAL, "ldx and ldy must be >= n_dof");
  const char* xa = (const char*)x;
  const char* xb = (const char*)(x + (nrhs - 1) * ldx + h->N);
  const char* ya = (const char*)y;
  const char* yb = (const char*)(y + (nrhs - 1) * ldy + h->N);
  if (xa < yb && ya < xb) return fail(HMAT_EINVAL, "x and y overlap");
  StreamScope scope((hipStream_t)hip_stream);
  h->last_stream = (hipStream_t)hip_stream;
  try {
    matvec_impl(h, stored_prec(h), nrhs, x, ldx, y, ldy, (hipStream_t)hip_stream);
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

hmat_status hmat_solve(hmat_t h, const double* b, double* x, double tol, int32_t restart,
                       int32_t maxit, void* hip_stream, hmat_solve_info* info) {
  hmat_status st = check_solve_args(h, b, x, tol, restart, maxit);
  if (st != HMAT_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  auto t0 = std::chrono::steady_clock::now();
  try {
    int used = 0, restarts = 0;
    double rel = 0.0;
    const GmresWs ws = ensure_gmres_ws(h, restart);
    st = gmres_impl(h, stored_prec(h), ws, b, x, tol, restart, maxit, s, &used, &restarts, &rel);
    if (info) {
      info->iterations = used;
      info->restarts = restarts;
      info->relres = rel;
      info->time_ms = ms_since(t0);
      info->refinements = 0;
    }
    if (st != HMAT_OK) return fail(st, "GMRES reached maxit before tol");
    return HMAT_OK;
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.st, e.msg);
  }
}

hmat_status hmat_solve_noalloc(hmat_t h, const double* b, double* x, double tol, int32_t restart,
                               int32_t maxit, void* hip_stream, hmat_solve_info* info) {
  hmat_status st = check_solve_args(h, b, x, tol, restart, maxit);
  if (st != HMAT_OK) return st;
  size_t off[4];
  const size_t need = gmres_ws_doubles(h->N, restart, off);
  if (need > NOALLOC_DOUBLES)
    return fail(HMAT_EINVAL, "hmat_solve_noalloc: n_dof x (restart + 1) exceeds the fixed workspace (" +
                                 std::to_string(need * 8) + " bytes needed, " +
                                 std::to_string(NOALLOC_DOUBLES * 8) + " available)");
  hipStream_t s = (hipStream_t)hip_stream;
  h->last_stream = s;
  auto t0 = std::chrono::steady_clock::now();
  // one call at a time per process: every call on a device uses its array
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  try {
    double* base = nullptr;
    check(noalloc_workspace(&base), "fixed workspace");
    std::array<double, 3 * GM_COL> host{};
    GmresWs ws;
    ws.Q = base + off[0];
    ws.w = base + off[1];
    ws.dotpart = base + off[2];
    ws.small = base + off[3];
    ws.host = host.data();
    int used = 0, restarts = 0;
    double rel = 0.0;
    st = gmres_impl(h, stored_prec(h), ws, b, x, tol, restart, maxit, s, &used, &restarts, &rel);
    if (info) {
      info->iterations = used;
      info->restarts = restarts;
      info->relres = rel;
      info->time_ms = ms_since(t0);
      info->refinements = 0;
    }
    if (st != HMAT_OK) return fail(st, "GMRES reached maxit before tol");
    return HMAT_OK;
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.st, e.msg);
  }
}

hmat_status hmat_solve_ir(hmat_t h, const double* b, double* x, double tol, int32_t restart,
                          int32_t maxit, int32_t inner_precision, double inner_tol,
                          void* hip_stream, hmat_solve_info* info) {
  hmat_status st = check_solve_args(h, b, x, tol, restart, maxit);
  if (st != HMAT_OK) return st;
  if (inner_precision != 0 && inner_precision != 1) return fail(HMAT_EINVAL, "inner_precision must be 0 or 1");
  if (inner_precision == 1 && !h->far32.p && !h->stream32.p)
    return fail(HMAT_EINVAL, "no FP32 copy: call hmat_set_precision(h, 1, ...) first");
  if (inner_precision == 0 && h->fp32_only) return fail(HMAT_ENOTSUP, "the handle stores FP32 entries only");
  if (!(inner_tol > 0.0 && inner_tol < 1.0)) return fail(HMAT_EINVAL, "inner_tol must lie in (0, 1)");
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  auto t0 = std::chrono::steady_clock::now();
  const int64_t N = h->N;
  try {
    check(hipStreamSynchronize(s), "solve");
    if (h->d_ir.bytes < sizeof(double) * 2 * N) h->d_ir.alloc(sizeof(double) * 2 * N, "refinement work");
    double* r = h->d_ir.as<double>();
    double* d = r + N;
    const GmresWs ws = ensure_gmres_ws(h, restart);
    auto norm_host = [&](const double* v) {
      check(launch_norm(v, N, h->d_dotpart.as<double>(), h->d_small.as<double>(), s), "norm");
      check(hipMemcpyAsync(h->h_pinned, h->d_small.p, sizeof(double), hipMemcpyDeviceToHost, s), "norm");
      check(hipStreamSynchronize(s), "norm");
      return h->h_pinned[0];
    };
    check(launch_fill(x, N, 0.0, s), "fill");
    const double bn = norm_host(b);
    int used = 0, restarts = 0, outer = 0;
    double rel = 0.0;
    st = HMAT_ENOCONV;
    if (bn == 0.0) {
      st = HMAT_OK;
    } else {
      // x_{k+1} = x_k + d_k with A_p d_k = b - A x_k solved by GMRES to a
      // relative residual max(inner_tol, tol ||b|| / (2 ||r_k||)); the
      // residual r_k = b - A x_k uses the FP64 matrix.
      // x0 = 0: the first residual is b (b - 0, bit for bit), so neither a
      // product nor its norm is needed
      bool x_zero = true;
      for (;;) {
        if (x_zero)
          check(launch_fill(r, N, 0.0, s), "fill");
        else
          matvec_impl(h, stored_prec(h), 1, x, N, r, N, s);
        check(launch_residual(b, N, r, s), "residual");
        const double rn = x_zero ? bn : norm_host(r);
        x_zero = false;
        rel = rn / bn;
        if (rn <= tol * bn) {
          st = HMAT_OK;
          break;
        }
        if (used >= maxit || outer >= 64) break;
        const double itol = std::max(inner_tol, 0.5 * tol * bn / rn);
        int u = 0, rs = 0;
        double irel = 0.0;
        (void)gmres_impl(h, inner_precision, ws, r, d, itol, restart, maxit - used, s, &u, &rs, &irel);
        used += u;
        restarts += rs;
        outer++;
        check(launch_axpy(1.0, d, N, x, s), "update");
      }
    }
    check(hipStreamSynchronize(s), "solve");
    if (info) {
      info->iterations = used;
      info->restarts = restarts;
      info->relres = rel;
      info->time_ms = ms_since(t0);
      info->refinements = outer;
    }
    if (st != HMAT_OK) return fail(st, "refinement reached maxit before tol");
    return HMAT_OK;
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.st, e.msg);
  }
}

hmat_status hmat_set_precision(hmat_t h, int32_t precision, void* hip_stream) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (precision != 0 && precision != 1) return fail(HMAT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (h->fp32_only) {
    if (precision == 1) return HMAT_OK;  // already so
    return fail(HMAT_ENOTSUP, "the handle stores FP32 entries only");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  try {
    check(hipStreamSynchronize(s), "set precision");
    drop_graphs(h);
    h->far32.release();
    h->stream32.release();
    if (precision == 1) {
      const int64_t nf = (int64_t)(h->far_arena.bytes / sizeof(double));
      const int64_t ns = (int64_t)(h->stream.bytes / sizeof(double));
      h->far32.alloc(sizeof(float) * std::max<int64_t>(nf, 2), "FP32 copy");
      h->stream32.alloc(sizeof(float) * std::max<int64_t>(ns, 2), "FP32 copy");
      check(launch_to_f32(h->far_arena.as<double>(), h->far32.as<float>(), nf, s), "FP32 copy");
      check(launch_to_f32(h->stream.as<double>(), h->stream32.as<float>(), ns, s), "FP32 copy");
      check(hipStreamSynchronize(s), "FP32 copy");
    }
    fill_stats(h);
  } catch (const HipError& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

hmat_status hmat_matvec_ex(hmat_t h, int32_t precision, int32_t nrhs, const double* x, int64_t ldx,
                           double* y, int64_t ldy, void* hip_stream) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (precision != 0 && precision != 1) return fail(HMAT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (precision == 1 && !h->far32.p && !h->stream32.p)
    return fail(HMAT_EINVAL, "no FP32 copy: call hmat_set_precision(h, 1, ...) first");
  if (precision == 0 && h->fp32_only) return fail(HMAT_ENOTSUP, "the handle stores FP32 entries only");
  if (!x || !y) return fail(HMAT_EINVAL, "x or y is NULL");
  if (nrhs < 1 || nrhs > 64) return fail(HMAT_EINVAL, "nrhs must lie in [1, 64]");
  if (ldx < h->N || ldy < h->N) return fail(HMAT_EINVAL, "ldx and ldy must be >= n_dof");
  const char* xa = (const char*)x;
  const char* xb = (const char*)(x + (nrhs - 1) * ldx + h->N);
  const char* ya = (const char*)y;
  const char* yb = (const char*)(y + (nrhs - 1) * ldy + h->N);
  if (xa < yb && ya < xb) return fail(HMAT_EINVAL, "x and y overlap");
  StreamScope scope((hipStream_t)hip_stream);
  h->last_stream = (hipStream_t)hip_stream;
  try {
    matvec_impl(h, precision, nrhs, x, ldx, y, ldy, (hipStream_t)hip_stream);
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

hmat_status hmat_info(hmat_t h, hmat_stats* st) {
  if (!h || !st) return fail(HMAT_EINVAL, "handle or stats is NULL");
  fill_stats(h);
  *st = h->st;
  return HMAT_OK;
}

hmat_status hmat_release_memory(void* hip_stream) {
  const hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  const int dev = current_device();
  if (dev < 0) return fail(HMAT_EDEVICE, "no HIP device");
  drop_idle_panels(dev, s);
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HMAT_EDEVICE, std::string("release memory: ") + hipGetErrorString(e));
  }
  mem_trim(dev, s);  // cached blocks, then the pool
  return HMAT_OK;
}

hmat_status hmat_set_mem_budget(int64_t bytes) {
  if (bytes < 0) return fail(HMAT_EINVAL, "budget must be >= 0 (0: none)");
  g_budget.store(bytes);
  return HMAT_OK;
}

hmat_status hmat_mem_held(int64_t* held, int64_t* peak) {
  if (!held) return fail(HMAT_EINVAL, "held is NULL");
  const int dev = current_device();
  if (dev < 0) return fail(HMAT_EDEVICE, "no HIP device");
  *held = g_held[dev].load();
  const int64_t pk = g_peak[dev].exchange(0);
  if (peak) *peak = pk;
  return HMAT_OK;
}

hmat_status hmat_free(hmat_t h) {
  if (!h) return HMAT_OK;
  const hipStream_t s = h->last_stream;
  StreamScope scope(s);
  (void)hipStreamSynchronize(s);
  delete h;
  (void)hipStreamSynchronize(s);
  return HMAT_OK;
}

hmat_status hmat_plan(const hmat_mesh* mesh, double eta, int32_t leaf, int32_t* order,
                      int32_t* n_blocks, int32_t* blocks) {
  std::string err;
  hmat_status st = validate_params(1.0, 0.25, eta, leaf, 0.5, err);
  if (st != HMAT_OK) return fail(st, err);
  st = validate_mesh(mesh, err);
  if (st != HMAT_OK) return fail(st, err);
  if (!n_blocks) return fail(HMAT_EINVAL, "n_blocks is NULL");
  try {
    Plan P;
    make_plan(mesh, eta, leaf, P);
    if (order) std::memcpy(order, P.order.data(), sizeof(int32_t) * P.nt);
    const int32_t capacity = *n_blocks;
    *n_blocks = (int32_t)P.blk.size();
    if (blocks) {
      if (capacity < (int32_t)P.blk.size()) return fail(HMAT_EINVAL, "blocks capacity too small");
      for (size_t b = 0; b < P.blk.size(); b++) {
        const BlockRec& B = P.blk[b];
        blocks[5 * b + 0] = P.cl[B.t].off;
        blocks[5 * b + 1] = P.cl[B.t].len;
        blocks[5 * b + 2] = P.cl[B.s].off;
        blocks[5 * b + 3] = P.cl[B.s].len;
        blocks[5 * b + 4] = B.far;
      }
    }
  } catch (const std::bad_alloc&) {
    return fail(HMAT_ENOMEM, "host allocation failed");
  }
  return HMAT_OK;
}

hmat_status hmat_block(hmat_t h, int32_t b, int32_t* info, double* A, double* B, int32_t* prow,
                       int32_t* pcol) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (b < 0 || b >= (int32_t)h->plan.blk.size()) return fail(HMAT_EINVAL, "block index out of range");
  const BlockRec& R = h->plan.blk[b];
  const int64_t m = block_m(h, b), n = block_n(h, b);
  const int32_t idx = h->kind_index[b];
  const int32_t k = R.far ? h->rank[idx] : 0;
  if (info) {
    info[0] = h->plan.cl[R.t].off;
    info[1] = h->plan.cl[R.t].len;
    info[2] = h->plan.cl[R.s].off;
    info[3] = h->plan.cl[R.s].len;
    info[4] = R.far;
    info[5] = k;
    info[6] = R.far ? h->stop[idx] : 0;
    info[7] = 0;
  }
  StreamScope scope(h->last_stream);
  try {
    if (R.far) {
      if (A) copy_stream_out(h, b, m, k, A, h->last_stream);
      if (B) copy_v_out(h, idx, n, k, B);
      if (h->piv_ptr[idx] && k) {
        if (prow) check(hipMemcpy(prow, h->piv_ptr[idx], sizeof(int32_t) * k, hipMemcpyDeviceToHost), "pivots");
        if (pcol)
          check(hipMemcpy(pcol, h->piv_ptr[idx] + h->piv_cap[idx], sizeof(int32_t) * k, hipMemcpyDeviceToHost), "pivots");
      }
    } else if (A) {
      copy_stream_out(h, b, m, n, A, h->last_stream);
    }
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HMAT_ENOMEM, "host allocation failed");
  }
  return HMAT_OK;
}

hmat_status hmat_entries(hmat_t h, int64_t n, const int64_t* rows, const int64_t* cols,
                         double* out, void* hip_stream) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  if (n < 0 || (n > 0 && (!rows || !cols || !out))) return fail(HMAT_EINVAL, "bad arrays");
  std::vector<int64_t> r(n), c(n);
  for (int64_t k = 0; k < n; k++) {
    if (rows[k] < 0 || rows[k] >= h->N || cols[k] < 0 || cols[k] >= h->N)
      return fail(HMAT_EINVAL, "entry index out of range");
    r[k] = 3 * (int64_t)h->inv_order[rows[k] / 3] + rows[k] % 3;
    c[k] = 3 * (int64_t)h->inv_order[cols[k] / 3] + cols[k] % 3;
  }
  if (n == 0) return HMAT_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  try {
    DevBuf dr, dc, dout;
    upload(dr, r, s, "entries");
    upload(dc, c, s, "entries");
    dout.alloc(sizeof(double) * n, "entries");
    check(launch_entries(h->G, n, dr.as<int64_t>(), dc.as<int64_t>(), dout.as<double>(), s), "entries");
    check(hipMemcpyAsync(out, dout.p, sizeof(double) * n, hipMemcpyDeviceToHost, s), "entries");
    check(hipStreamSynchronize(s), "entries");
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

hmat_status hmat_set_factors(hmat_t h, const int32_t* ranks, const double* U, const double* V,
                             void* hip_stream) {
  if (!h || !ranks) return fail(HMAT_EINVAL, "handle or ranks is NULL");
  if (h->fp32_only) return fail(HMAT_ENOTSUP, "the handle stores FP32 entries only");
  hipStream_t s = (hipStream_t)hip_stream;
  StreamScope scope(s);
  h->last_stream = s;
  const size_t nf = h->far_blocks.size();
  int64_t total = 0, usz = 0;
  for (size_t f = 0; f < nf; f++) {
    const int32_t b = h->far_blocks[f], k = ranks[b];
    if (k < 0 || k > std::min(block_m(h, b), block_n(h, b))) return fail(HMAT_EINVAL, "rank out of range");
    total += k;
    usz += block_m(h, b) * k;
  }
  if (total > 0 && (!U || !V)) return fail(HMAT_EINVAL, "U or V is NULL");
  try {
    check(hipStreamSynchronize(s), "set factors");
    // dense blocks back out of the current stream into a plain staging arena
    std::vector<int64_t> near_off;
    int64_t noff = 0;
    for (int32_t b : h->near_blocks) {
      near_off.push_back(noff);
      noff += block_m(h, b) * block_n(h, b);
    }
    DevBuf near_stage, u_stage;
    near_stage.alloc(sizeof(double) * std::max<int64_t>(noff, 1), "set factors");
    {
      auto tasks = stream_tasks(
          h, [&](int32_t b) { return !h->plan.blk[b].far; },
          [&](int32_t b) { return near_stage.as<double>() + near_off[h->kind_index[b]]; });
      DevBuf d_t;
      upload(d_t, tasks, s, "set factors");
      check(launch_from_stream(d_t.as<StreamTask>(), (int)tasks.size(), h->stream.as<double>(), s), "set factors");
      check(hipStreamSynchronize(s), "set factors");
    }
    for (size_t f = 0; f < nf; f++) {
      h->rank[f] = ranks[h->far_blocks[f]];
      h->stop[f] = 0;
      h->ratio[f] = 0.0;
      h->piv_ptr[f] = nullptr;
    }
    // V into the panel layout (host packing), U staged plain column-major
    const int64_t fo = far_layout(h);
    std::vector<double> host(std::max<int64_t>(fo, PANEL_ALIGN), 0.0);
    u_stage.alloc(sizeof(double) * std::max<int64_t>(usz, 1), "set factors");
    std::vector<const double*> u_ptr(nf, nullptr);
    int64_t uo = 0, vo = 0;
    for (size_t f = 0; f < nf; f++) {
      const int32_t b = h->far_blocks[f], k = h->rank[f];
      const int64_t m = block_m(h, b), n = block_n(h, b);
      const PanelShape sv = h->far_vshape[f];
      for (int32_t c = 0; c < k; c++)
        std::memcpy(host.data() + h->far_voff[f] + (int64_t)c * sv.ld + sv.fp, V + vo + c * n, sizeof(double) * n);
      u_ptr[f] = u_stage.as<double>() + uo;
      uo += m * k;
      vo += n * k;
    }
    if (uo > 0) check(hipMemcpyAsync(u_stage.p, U, sizeof(double) * uo, hipMemcpyHostToDevice, s), "set factors");
    h->far_arena.alloc(sizeof(double) * host.size(), "low-rank arena");
    check(hipMemcpyAsync(h->far_arena.p, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, s), "set factors");
    check(hipStreamSynchronize(s), "set factors");
    build_product_plan(h, s);
    fill_stream(h, near_stage.as<double>(), near_off, u_ptr, s);
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HMAT_ENOMEM, "host allocation failed");
  }
  return HMAT_OK;
}

hmat_status hmat_profile(hmat_t h, int32_t enable, double* phase_ms, int64_t* calls) {
  if (!h) return fail(HMAT_EINVAL, "handle is NULL");
  try {
    prof_collect(h);
    if (phase_ms)
      for (int k = 0; k < 4; k++) phase_ms[k] = h->prof_ms[k];
    if (calls) *calls = h->prof_calls;
    if (enable) {
      for (double& t : h->prof_ms) t = 0.0;
      h->prof_calls = 0;
    }
    h->prof = enable != 0;
  } catch (const HipError& e) {
    return fail(e.st, e.msg);
  }
  return HMAT_OK;
}

}  // extern "C"
