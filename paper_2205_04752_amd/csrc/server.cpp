// Request server: continuous admission of H-matrix requests (build + products
// or a solve) under a device-memory budget, with the admitted requests'
// work overlapping on the device.
//
// Each of `slots` worker threads owns a HIP stream (default priority) and
// runs one admitted request at a time through the library's C ABI: build,
// then its products or its solve, then free. A worker takes the oldest
// pending request once its memory estimate fits beside what the running
// requests hold; after the build the reservation is corrected to the bytes
// the handle actually holds. Requests are independent, and each one's device
// work is deterministic, so a result does not depend on what else runs.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hmat_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  // inputs (host copies)
  std::vector<double> V;
  std::vector<int32_t> T;
  hmat_request q{};
  std::vector<double> in;  // nvec x N (products) or N (solve)
  // outputs
  std::vector<double> out;
  hmat_result res{};
  std::string err;
  int64_t reserved = 0;
  bool done = false;
  std::atomic<bool> cancel{false};  // set by hmat_server_cancel; checked between phases
};

// Device bytes a request is assumed to need before it is built: the stored
// matrix at 25% of dense FP64 (a bound above what the admissibility and
// accuracy settings of this library produce at these sizes; 9-11% measured
// at 61k DOF, eps 1e-5 .. 1e-6), FP32 entries if asked for (copies beside the
// FP64 ones, or the conversion peak of an FP32-only build), the ACA panels
// (the first pass's and the later passes', each capped by the worker's ACA
// budget), and vectors.
int64_t estimate_bytes(const Request& r, int64_t aca_cap) {
  const double N = (double)r.T.size();  // 3 DOF per triangle
  const double stored = 0.25 * N * N;
  const double mat = 8.0 * stored * (r.q.precision == 1 ? 1.5 : 1.0);
  const double vec = 8.0 * N * (60.0 + 2.0 * std::max(1, r.q.nvec));
  return (int64_t)(mat + vec) + 2 * aca_cap;
}

}  // namespace

struct hmat_server {
  int device = 0;
  int32_t slots = 1;
  int64_t budget = 0;
  int64_t aca_cap = 0;
  double eta = 2.0;
  int32_t leaf = 32;
  Clock::time_point t0 = Clock::now();
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::map<int64_t, std::shared_ptr<Request>> all;  // submitted, not collected
  int64_t next_id = 1;
  int64_t in_use = 0;
  int32_t running = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
  void run_worker();
  void execute(Request& r, hipStream_t s);
};

namespace {

thread_local std::string g_srv_err;

hmat_status srv_fail(hmat_status st, const std::string& m) {
  g_srv_err = m;
  return st;
}

// Request vectors, stream-ordered on the worker's stream (no device-wide
// synchronisation on allocation or release).
struct DevVec {
  double* p = nullptr;
  hipStream_t s = nullptr;
  bool alloc(size_t bytes, hipStream_t st) {
    s = st;
    return hipMallocAsync((void**)&p, bytes, st) == hipSuccess;
  }
  ~DevVec() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

}  // namespace

void hmat_server::execute(Request& r, hipStream_t s) {
  const int32_t nt = (int32_t)(r.T.size() / 3);
  const int64_t N = 3 * (int64_t)nt;
  hmat_mesh mesh{(int32_t)(r.V.size() / 3), nt, r.V.data(), r.T.data()};
  hmat_t h = nullptr;
  auto fail_req = [&](hmat_status st) {
    r.res.status = st;
    r.err = hmat_last_error();
    if (h) hmat_free(h);
  };
  auto cancelled = [&]() {
    if (!r.cancel.load()) return false;
    r.res.status = HMAT_ECANCELED;
    r.err = "request cancelled";
    if (h) hmat_free(h);
    return true;
  };
  if (cancelled()) return;
  // reduced-precision products need only the FP32 entries; a solve keeps the
  // FP64 operator for the refinement residual
  const bool f32_only = r.q.precision == 1 && r.q.kind != HMAT_REQ_SOLVE;
  hmat_status st;
  if (f32_only) {
    hmat_opts o{};
    o.precision = 1;
    o.aca_stop_factor = 1.0;
    st = hmat_build_ex(&mesh, r.q.E, r.q.nu, eta, leaf, r.q.eps, &o, s, &h);
  } else {
    st = hmat_build(&mesh, r.q.E, r.q.nu, eta, leaf, r.q.eps, s, &h);
  }
  if (st != HMAT_OK) return fail_req(st);
  if (cancelled()) return;
  hmat_stats hs{};
  hmat_info(h, &hs);
  r.res.build_ms = hs.t_build_ms;
  if (r.q.precision == 1 && !f32_only) {
    st = hmat_set_precision(h, 1, s);
    if (st != HMAT_OK) return fail_req(st);
    hmat_info(h, &hs);
  }
  {
    // correct the reservation to what the handle holds (plus the vectors)
    std::lock_guard<std::mutex> lk(mu);
    const int64_t actual = hs.device_bytes + 8 * N * (60 + 2 * (int64_t)std::max(1, r.q.nvec));
    in_use += actual - r.reserved;
    r.reserved = actual;
    r.res.device_bytes = hs.device_bytes;
  }
  cv_work.notify_all();
  if (cancelled()) return;
  const int nv = r.q.kind == HMAT_REQ_SOLVE ? 1 : r.q.nvec;
  DevVec dx, dy;
  if (!dx.alloc(sizeof(double) * N * nv, s) || !dy.alloc(sizeof(double) * N * nv, s)) {
    (void)hipGetLastError();
    g_srv_err = "request vectors: out of device memory";
    r.res.status = HMAT_ENOMEM;
    r.err = g_srv_err;
    hmat_free(h);
    return;
  }
  if (hipMemcpyAsync(dx.p, r.in.data(), sizeof(double) * N * nv, hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipGetLastError();
    r.res.status = HMAT_EDEVICE;
    r.err = "request vectors: copy failed";
    hmat_free(h);
    return;
  }
  if (r.q.kind == HMAT_REQ_SOLVE) {
    hmat_solve_info si{};
    if (r.q.precision == 1)
      st = hmat_solve_ir(h, dx.p, dy.p, r.q.tol, r.q.restart, 100000, 1, 1e-6, s, &si);
    else
      st = hmat_solve(h, dx.p, dy.p, r.q.tol, r.q.restart, 100000, s, &si);
    r.res.iterations = si.iterations;
    r.res.refinements = si.refinements;
    r.res.relres = si.relres;
  } else {
    // all of the request's vectors in one call (matrix-core kernels for 2..16 per pass)
    st = hmat_matvec_ex(h, r.q.precision, nv, dx.p, N, dy.p, N, s);
  }
  if (st != HMAT_OK) return fail_req(st);
  r.out.assign((size_t)N * nv, 0.0);
  if (hipMemcpyAsync(r.out.data(), dy.p, sizeof(double) * N * nv, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    r.res.status = HMAT_EDEVICE;
    r.err = "request result: copy failed";
    hmat_free(h);
    return;
  }
  r.res.status = HMAT_OK;
  hmat_free(h);
}

void hmat_server::run_worker() {
  (void)hipSetDevice(device);
  hm::set_thread_aca_budget(aca_cap);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    s = nullptr;
  }
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(mu);
      // the oldest request is admitted when it fits (always when nothing runs);
      // after hmat_server_destroy the workers drain the queue, then exit
      cv_work.wait(lk, [&] {
        if (pending.empty()) return stop;
        const int64_t est = estimate_bytes(*pending.front(), aca_cap);
        return in_use == 0 || in_use + est <= budget;
      });
      if (pending.empty()) break;
      r = pending.front();
      pending.pop_front();
      r->reserved = estimate_bytes(*r, aca_cap);
      in_use += r->reserved;
      running++;
      r->res.t_admit_ms = now_ms();
    }
    execute(*r, s);
    {
      std::lock_guard<std::mutex> lk(mu);
      running--;
      in_use -= r->reserved;
      r->reserved = 0;
      r->res.t_done_ms = now_ms();
      r->done = true;
      r->V.clear();
      r->V.shrink_to_fit();
      r->T.clear();
      r->T.shrink_to_fit();
      r->in.clear();
      r->in.shrink_to_fit();
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
  if (s) (void)hipStreamDestroy(s);
}

extern "C" {

hmat_status hmat_server_create(int32_t slots, int64_t hbm_budget, double eta, int32_t leaf,
                               hmat_server_t* out) {
  if (!out) return srv_fail(HMAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (slots < 1 || slots > 64) return srv_fail(HMAT_EINVAL, "slots must lie in [1, 64]");
  if (hbm_budget < 0) return srv_fail(HMAT_EINVAL, "hbm_budget must be >= 0");
  if (!(eta > 0.0) || leaf < 1) return srv_fail(HMAT_EINVAL, "eta must be > 0 and leaf >= 1");
  hmat_server* S = new (std::nothrow) hmat_server();
  if (!S) return srv_fail(HMAT_ENOMEM, "host allocation failed");
  if (hipGetDevice(&S->device) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return srv_fail(HMAT_EDEVICE, "no HIP device");
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    fr = 0;
  }
  S->budget = hbm_budget > 0 ? hbm_budget : (int64_t)(fr * 0.8);
  S->slots = slots;
  S->aca_cap = std::max<int64_t>((int64_t)256 << 20, std::min<int64_t>((int64_t)2 << 30, S->budget / (4 * slots)));
  S->eta = eta;
  S->leaf = leaf;
  hm::serving_pool(true);
  try {
    for (int i = 0; i < slots; i++) S->workers.emplace_back([S] { S->run_worker(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
    hm::serving_pool(false);
    return srv_fail(HMAT_ENOMEM, "cannot start worker threads");
  }
  *out = S;
  return HMAT_OK;
}

hmat_status hmat_server_submit(hmat_server_t S, const hmat_mesh* mesh, const hmat_request* req,
                               const double* in, int64_t* id) {
  if (!S) return srv_fail(HMAT_EINVAL, "server is NULL");
  if (!req || !in || !id) return srv_fail(HMAT_EINVAL, "req, in or id is NULL");
  std::string err;
  hmat_status st = hm::validate_mesh(mesh, err);
  if (st == HMAT_OK) st = hm::validate_params(req->E, req->nu, S->eta, S->leaf, req->eps, err);
  if (st != HMAT_OK) return srv_fail(st, err);
  if (req->kind != HMAT_REQ_MATVEC && req->kind != HMAT_REQ_SOLVE) return srv_fail(HMAT_EINVAL, "kind must be HMAT_REQ_MATVEC or HMAT_REQ_SOLVE");
  if (req->precision != 0 && req->precision != 1) return srv_fail(HMAT_EINVAL, "precision must be 0 or 1");
  if (req->kind == HMAT_REQ_MATVEC && (req->nvec < 1 || req->nvec > 64)) return srv_fail(HMAT_EINVAL, "nvec must lie in [1, 64]");
  if (req->kind == HMAT_REQ_SOLVE && (!(req->tol > 0.0) || req->restart < 1 || req->restart > 1024))
    return srv_fail(HMAT_EINVAL, "solve needs tol > 0 and restart in [1, 1024]");
  auto r = std::make_shared<Request>();
  const int64_t nv = mesh->n_vertices, nt = mesh->n_triangles, N = 3 * nt;
  const int64_t nin = req->kind == HMAT_REQ_SOLVE ? N : N * req->nvec;
  try {
    r->V.assign(mesh->vertices, mesh->vertices + 3 * nv);
    r->T.assign(mesh->triangles, mesh->triangles + 3 * nt);
    r->in.assign(in, in + nin);
  } catch (const std::bad_alloc&) {
    return srv_fail(HMAT_ENOMEM, "host allocation failed");
  }
  r->q = *req;
  if (r->q.kind == HMAT_REQ_SOLVE) r->q.nvec = 1;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->id = S->next_id++;
    r->res.t_submit_ms = S->now_ms();
    S->all[r->id] = r;
    S->pending.push_back(r);
  }
  S->cv_work.notify_all();
  *id = r->id;
  return HMAT_OK;
}

hmat_status hmat_server_wait(hmat_server_t S, int64_t id, double* out, hmat_result* res) {
  if (!S) return srv_fail(HMAT_EINVAL, "server is NULL");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end()) return srv_fail(HMAT_EINVAL, "unknown request id (or already collected)");
    r = it->second;
    S->all.erase(it);  // collected by this wait: another wait on id finds nothing
    S->cv_done.wait(lk, [&] { return r->done; });
  }
  if (res) *res = r->res;
  if (r->res.status != HMAT_OK) return srv_fail((hmat_status)r->res.status, r->err);
  if (out) std::memcpy(out, r->out.data(), sizeof(double) * r->out.size());
  return HMAT_OK;
}

hmat_status hmat_server_cancel(hmat_server_t S, int64_t id) {
  if (!S) return srv_fail(HMAT_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end()) return srv_fail(HMAT_EINVAL, "unknown request id (or already collected)");
    const std::shared_ptr<Request>& r = it->second;
    if (r->done) return HMAT_OK;
    r->cancel.store(true);
    auto q = std::find(S->pending.begin(), S->pending.end(), r);
    if (q != S->pending.end()) {  // still queued: finish it here, never admitted
      S->pending.erase(q);
      r->res.status = HMAT_ECANCELED;
      r->err = "request cancelled";
      r->res.t_done_ms = S->now_ms();
      r->done = true;
    }
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
  return HMAT_OK;
}

hmat_status hmat_server_status(hmat_server_t S, int64_t* in_use, int32_t* queued, int32_t* running) {
  if (!S) return srv_fail(HMAT_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  if (in_use) *in_use = S->in_use;
  if (queued) *queued = (int32_t)S->pending.size();
  if (running) *running = S->running;
  return HMAT_OK;
}

hmat_status hmat_server_destroy(hmat_server_t S) {
  if (!S) return HMAT_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  delete S;
  hm::serving_pool(false);
  return HMAT_OK;
}

const char* hmat_server_last_error(void) { return g_srv_err.c_str(); }

}  // extern "C"
