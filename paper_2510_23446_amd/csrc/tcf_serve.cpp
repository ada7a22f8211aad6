// Serving loop of libtcf: admission by device footprint, one worker thread
// and HIP stream per running request, results kept on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/tcf.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int id = 0;
  tcf_problem* h = nullptr;
  size_t footprint = 0;
  int state = TCF_REQ_QUEUED;
  int status = TCF_OK;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<std::vector<double>> fields;
  tcf_stats stats{};
  std::vector<double> step_ms;
  std::string err;
};

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct tcf_server {
  size_t max_bytes = 0;
  int max_slots = 1;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int> queue;
  std::vector<std::unique_ptr<Request>> reqs;
  size_t used = 0, peak = 0;
  int running = 0;
  bool stopping = false;
  double t_first_admit = -1, t_last_done = -1;
  std::thread dispatcher;
  // worker threads of admitted requests not yet joined; finished ones are
  // joined at the next admission, so at most about 2 max_slots stay here
  std::vector<std::pair<Request*, std::thread>> workers;

  void run_request(Request* r);
  void dispatch_loop();
  void reap_finished(std::unique_lock<std::mutex>& lk);
};

void tcf_server::run_request(Request* r) {
  // The error text is built locally and moved into the request together with
  // the state change, under the lock that tcf_server_error reads it with.
  std::string err;
  std::vector<std::vector<double>> fields;
  std::vector<double> step_ms;
  tcf_stats stats{};
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  const hipError_t se = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  int rc = se == hipSuccess ? TCF_OK : TCF_EHIP;
  if (rc != TCF_OK) {
    st = nullptr;
    err = std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(se);
  }
  if (rc == TCF_OK) rc = tcf_setup(r->h, st);
  if (rc == TCF_OK) {
    rc = tcf_step(r->h, 1 << 30, st);
    if (rc == TCF_ENOCONV) rc = TCF_OK;  // flagged in the stats, results kept
  }
  if (rc == TCF_OK) {
    // no exception may leave this thread: any failure fails the request
    try {
      rc = tcf_get_stats(r->h, &stats);
      const int n = stats.steps_done;
      if (rc == TCF_OK) {
        step_ms.resize(n);
        rc = tcf_get_step_log(r->h, n, nullptr, nullptr, step_ms.data());
      }
      int64_t cnt[8] = {0};
      size_t len = 8;
      if (rc == TCF_OK) rc = tcf_get_topology(r->h, TCF_TOPO_COUNTS, cnt, &len);
      if (rc == TCF_OK && (len < 1 || cnt[0] <= 0)) rc = TCF_EINVAL;
      // number of excitations: fetch until the library refuses the index
      for (int k = 0; rc == TCF_OK; ++k) {
        std::vector<double> f((size_t)cnt[0]);
        if (tcf_get_field(r->h, k, f.data(), f.size(), 0, st) != TCF_OK) break;
        fields.push_back(std::move(f));
      }
      if (rc != TCF_OK) err = std::string("reading the results: ") + tcf_last_error(r->h);
    } catch (const std::exception& ex) {
      rc = TCF_ENOMEM;
      fields.clear();
      err = std::string("while fetching the results: ") + ex.what();
    }
  }
  if (rc != TCF_OK && err.empty()) {
    try {
      err = std::string("status ") + std::to_string(rc) + ": " + tcf_last_error(r->h);
    } catch (const std::exception&) {
    }
  }
  tcf_destroy(r->h);  // gives the request's device memory back on its stream
  r->h = nullptr;
  if (st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  std::lock_guard<std::mutex> lk(mu);
  r->stats = stats;
  r->step_ms = std::move(step_ms);
  r->fields = std::move(fields);
  r->err = std::move(err);
  r->status = rc;
  r->state = rc == TCF_OK ? TCF_REQ_DONE : TCF_REQ_FAILED;
  r->t_done = now_ms();
  t_last_done = r->t_done;
  used -= r->footprint;
  --running;
  cv.notify_all();
}

// Joins the threads of finished requests, outside the lock.  A worker marks
// its request DONE or FAILED as its last action under the lock and takes the
// lock no more, so each join here waits only for the thread's own exit.
void tcf_server::reap_finished(std::unique_lock<std::mutex>& lk) {
  std::vector<std::thread> done;
  for (size_t i = 0; i < workers.size();) {
    const int st = workers[i].first->state;
    if (st == TCF_REQ_DONE || st == TCF_REQ_FAILED) {
      done.push_back(std::move(workers[i].second));
      if (i + 1 != workers.size()) workers[i] = std::move(workers.back());
      workers.pop_back();
    } else {
      ++i;
    }
  }
  if (done.empty()) return;
  lk.unlock();
  for (auto& t : done) t.join();
  lk.lock();
}

void tcf_server::dispatch_loop() {
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv.wait(lk, [&] {
      if (stopping && queue.empty()) return true;
      if (queue.empty()) return false;
      const Request* r = reqs[queue.front()].get();
      return running < max_slots && (running == 0 || used + r->footprint <= max_bytes);
    });
    if (queue.empty()) {
      if (stopping) break;
      continue;
    }
    reap_finished(lk);
    Request* r = reqs[queue.front()].get();
    queue.pop_front();
    r->state = TCF_REQ_RUNNING;
    r->t_admit = now_ms();
    if (t_first_admit < 0) t_first_admit = r->t_admit;
    used += r->footprint;
    peak = std::max(peak, used);
    ++running;
    // room first, so that a started thread is always stored (a joinable
    // std::thread destroyed unjoined ends the process); if no thread can be
    // started, the request fails here and gives its slot back
    try {
      workers.reserve(workers.size() + 1);
      workers.emplace_back(r, std::thread([this, r] { run_request(r); }));
    } catch (const std::exception&) {
      used -= r->footprint;
      --running;
      r->status = TCF_ENOMEM;
      r->state = TCF_REQ_FAILED;
      r->err = "could not start a worker thread for the request";
      r->t_done = now_ms();
      tcf_destroy(r->h);
      r->h = nullptr;
      cv.notify_all();
    }
  }
}

extern "C" {

int tcf_server_create(size_t max_bytes, int32_t max_slots, tcf_server** out) {
  if (!out || max_slots < 1 || max_bytes == 0) return TCF_EINVAL;
  auto* s = new (std::nothrow) tcf_server();
  if (!s) return TCF_ENOMEM;
  s->max_bytes = max_bytes;
  s->max_slots = max_slots;
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  try {
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
  } catch (const std::exception&) {
    delete s;
    return TCF_ENOMEM;
  }
  *out = s;
  return TCF_OK;
}

int tcf_server_submit(tcf_server* srv, const tcf_problem_desc* desc, const tcf_options* opts,
                      int32_t* req_id) {
  if (!srv || !desc || !req_id) return TCF_EINVAL;
  tcf_problem* h = nullptr;
  int rc = tcf_create(desc, opts, nullptr, &h);
  if (rc != TCF_OK) return rc;
  size_t b64 = 0, b32 = 0;
  tcf_footprint(h, &b64, &b32);
  const int prec = opts ? opts->precision : TCF_FP64;
  const size_t footprint = prec == TCF_FP64 ? b64 : b32;
  const bool fits = footprint <= srv->max_bytes;
  std::lock_guard<std::mutex> lk(srv->mu);
  // everything that can throw comes first, before the request is visible:
  // the record, room in the request list and the queue entry
  std::unique_ptr<Request> r;
  try {
    r = std::make_unique<Request>();
    if (!fits) r->err = "request footprint exceeds the server memory budget";
    srv->reqs.reserve(srv->reqs.size() + 1);
    if (fits) srv->queue.push_back((int)srv->reqs.size());
  } catch (const std::bad_alloc&) {
    tcf_destroy(h);
    return TCF_ENOMEM;
  }
  r->h = h;
  r->footprint = footprint;
  r->t_submit = now_ms();
  r->id = (int)srv->reqs.size();
  *req_id = r->id;
  if (!fits) {
    r->state = TCF_REQ_FAILED;
    r->status = TCF_ENOMEM;
    tcf_destroy(r->h);
    r->h = nullptr;
  }
  srv->reqs.push_back(std::move(r));  // room reserved above
  if (!fits) return TCF_ENOMEM;
  srv->cv.notify_all();
  return TCF_OK;
}

int tcf_server_poll(tcf_server* srv, int32_t id, int32_t* state) {
  if (!srv || !state) return TCF_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (id < 0 || id >= (int)srv->reqs.size()) return TCF_EINVAL;
  *state = srv->reqs[id]->state;
  return TCF_OK;
}

int tcf_server_wait(tcf_server* srv, int32_t id) {
  if (!srv) return TCF_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (id < 0 || id >= (int)srv->reqs.size()) return TCF_EINVAL;
  Request* r = srv->reqs[id].get();
  srv->cv.wait(lk, [&] { return r->state == TCF_REQ_DONE || r->state == TCF_REQ_FAILED; });
  return r->status;
}

int tcf_server_fetch(tcf_server* srv, int32_t id, int32_t k, double* out, size_t len,
                     tcf_stats* stats) {
  if (!srv) return TCF_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (id < 0 || id >= (int)srv->reqs.size()) return TCF_EINVAL;
  Request* r = srv->reqs[id].get();
  if (r->state != TCF_REQ_DONE) return r->state == TCF_REQ_FAILED ? r->status : TCF_ESTATE;
  if (stats) *stats = r->stats;
  if (out) {
    if (k < 0 || k >= (int)r->fields.size()) return TCF_EINVAL;
    if (len < r->fields[k].size()) return TCF_EINVAL;
    std::memcpy(out, r->fields[k].data(), r->fields[k].size() * sizeof(double));
  }
  return TCF_OK;
}

int tcf_server_stats(tcf_server* srv, tcf_server_report* st) {
  if (!srv || !st) return TCF_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  std::memset(st, 0, sizeof(*st));
  std::vector<double> steps, waits;
  for (auto& r : srv->reqs) {
    ++st->submitted;
    if (r->state != TCF_REQ_QUEUED && r->t_admit > 0) {
      ++st->admitted;
      waits.push_back(r->t_admit - r->t_submit);
    }
    if (r->state == TCF_REQ_DONE) {
      ++st->completed;
      steps.insert(steps.end(), r->step_ms.begin(), r->step_ms.end());
      st->steps += (int64_t)r->step_ms.size();
    }
    if (r->state == TCF_REQ_FAILED) ++st->failed;
    if (r->state == TCF_REQ_RUNNING) ++st->running;
    if (r->state == TCF_REQ_QUEUED) ++st->queued;
  }
  st->p50_step_ms = percentile(steps, 0.50);
  st->p99_step_ms = percentile(steps, 0.99);
  st->p50_queue_ms = percentile(waits, 0.50);
  st->p99_queue_ms = percentile(waits, 0.99);
  st->busy_ms = (srv->t_first_admit >= 0 && srv->t_last_done >= 0)
                    ? srv->t_last_done - srv->t_first_admit
                    : 0.0;
  st->peak_bytes = srv->peak;
  return TCF_OK;
}

const char* tcf_server_error(tcf_server* srv, int32_t id) {
  if (!srv) return "";
  std::lock_guard<std::mutex> lk(srv->mu);
  if (id < 0 || id >= (int)srv->reqs.size()) return "";
  return srv->reqs[id]->err.c_str();
}

void tcf_server_destroy(tcf_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    srv->cv.notify_all();
  }
  if (srv->dispatcher.joinable()) srv->dispatcher.join();
  for (auto& w : srv->workers)
    if (w.second.joinable()) w.second.join();
  for (auto& r : srv->reqs)
    if (r->h) tcf_destroy(r->h);
  delete srv;
}

}  // extern "C"
