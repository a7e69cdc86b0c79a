// Served form: a worker thread that admits independent 3D solves under a device-memory
// budget and a slot limit and advances every running solve one gas step per round through
// the batch interface, and transfer threads, some that set solves up (handle, state
// upload) and some that take them down (result read back to host memory, handle freed),
// while the worker keeps the device busy with the others. The server is a client of
// the public C interface (include/rhd.h) and owns no kernels; every solve still takes the
// step of Sec. 3.1 (gas CFL step of Eq. algorithm:gastimestep, subcycle count of
// Eq. algorithm:radtimestep at the request's reduced speed of light).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rhd.h"

namespace {

using Clock = std::chrono::steady_clock;

thread_local char g_server_error[256] = "";

struct Request {
  long long id = 0;
  rhd_params p{};
  long long cells = 0;
  long long footprint = 0;
  int steps = 0;
  double chat = 0.0;
  int kappa_scalar = 0;
  bool mixed = false;
  // inputs until admission; rho..Fr then hold the result
  std::vector<double> rho, mom, E, Er, Fr, kP, kF, j;
  bool have_E = false;
  // life cycle (guarded by the server mutex)
  int status = RHD_REQ_QUEUED;
  int error = RHD_OK;
  int steps_done = 0;
  long long zone_updates = 0;
  double t_submit = 0.0, t_start = -1.0, t_done = -1.0;
  bool cancel = false;
  rhd_diag diag{};
  // owned by the worker thread while running
  rhd_t* h = nullptr;
};

using ReqPtr = std::shared_ptr<Request>;

}  // namespace

struct rhd_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ReqPtr> queue;             // submission order
  std::map<long long, ReqPtr> all;      // every request not yet forgotten
  long long next_id = 1;
  long long budget = 0, used = 0;
  int max_slots = 1, rows = 8, zchunk = 8;
  int persistent = 0;  // the persistent launch is switched off (see rhd_batch_set_persistent)
  int device = 0;
  bool stop = false;
  Clock::time_point t0;
  rhd_server_stats stats{};
  // the last failure's message: written by API calls (with or without mu held) and by
  // the worker, so it has a lock of its own
  std::mutex err_mu;
  char err[256] = "";
  // work for the transfer threads (guarded by mu): queue 0 sets requests up, queue 1
  // reads results back or frees requests; and the requests set up, waiting to join a
  // batch
  struct Job {
    ReqPtr r;
    int kind = 0;       // JOB_PREPARE, JOB_COLLECT or JOB_DISCARD
    int status = 0;     // JOB_DISCARD: the final status; JOB_COLLECT: 0 or the failure code
    int error = 0;
    std::string why;    // message of a failure
  };
  std::deque<Job> jobs[2];
  std::vector<ReqPtr> ready;
  bool xstop = false;  // the transfer threads drain their jobs and end
  std::condition_variable cv_xfer[2];
  // worker-only state: one batch per precision (0 FP64, 1 mixed) and its members in
  // batch order
  rhd_batch_t* batch[2] = {nullptr, nullptr};
  std::vector<ReqPtr> members[2];
  // transfer threads per queue: host-device copies from pageable memory are staged by the
  // runtime through the CPU, so several threads in parallel move more bytes per second
  static constexpr int XFER_THREADS = 6;
  std::thread worker, xfer[2 * XFER_THREADS];

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int sfail(rhd_server* s, int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (s) {
    std::lock_guard<std::mutex> lk(s->err_mu);
    std::snprintf(s->err, sizeof(s->err), "%s", buf);
  } else {
    std::snprintf(g_server_error, sizeof(g_server_error), "%s", buf);
  }
  return code;
}

void fill_info(const Request& r, rhd_request_info* info) {
  if (!info) return;
  info->status = r.status;
  info->error = r.error;
  info->steps_done = r.steps_done;
  info->zone_updates = r.zone_updates;
  info->t_submit = r.t_submit;
  info->t_start = r.t_start;
  info->t_done = r.t_done;
}

bool finished(int status) {
  return status == RHD_REQ_DONE || status == RHD_REQ_FAILED || status == RHD_REQ_CANCELLED;
}

void drop_inputs(Request& r) {
  std::vector<double>().swap(r.kP);
  std::vector<double>().swap(r.kF);
  std::vector<double>().swap(r.j);
}

void drop_all(Request& r) {
  drop_inputs(r);
  std::vector<double>().swap(r.rho);
  std::vector<double>().swap(r.mom);
  std::vector<double>().swap(r.E);
  std::vector<double>().swap(r.Er);
  std::vector<double>().swap(r.Fr);
}

enum { JOB_PREPARE = 0, JOB_COLLECT = 1, JOB_DISCARD = 2 };

// Called with the lock held: the request leaves the running set with a final status,
// and its budget and slot go to the next ones.
void retire(rhd_server* s, Request& r, int status, int error) {
  r.status = status;
  r.error = error;
  r.t_done = s->now();
  s->used -= r.footprint;
  s->stats.bytes_in_use = s->used;
  s->stats.running -= 1;
  if (status == RHD_REQ_DONE) s->stats.completed += 1;
  else if (status == RHD_REQ_FAILED) s->stats.failed += 1;
  else s->stats.cancelled += 1;
  if (status == RHD_REQ_CANCELLED) drop_all(r);
  s->cv_done.notify_all();
  s->cv_work.notify_one();
}

// Called with the lock held: hand a job to its transfer thread.
void post(rhd_server* s, rhd_server::Job job) {
  const int q = job.kind == JOB_PREPARE ? 0 : 1;
  s->jobs[q].push_back(std::move(job));
  s->cv_xfer[q].notify_one();
}

// Called with the lock held: the oldest queued request fits the budget and a slot.
bool can_admit(const rhd_server* s) {
  return !s->queue.empty() && s->stats.running < s->max_slots &&
         s->used + s->queue.front()->footprint <= s->budget;
}

// Transfer thread: create the handle and upload the state of an admitted request (the
// handle's own stream; no batch involved). Returns an RHD_* code.
int prepare_request(Request& r, char* msg) {
  rhd_t* h = nullptr;
  int rc = rhd_create(&r.p, nullptr, &h);
  if (rc) {
    std::snprintf(msg, 256, "rhd_create: %s", rhd_last_error(nullptr));
    return rc;
  }
  rc = rhd_set_state(h, r.rho.data(), r.mom.data(), r.have_E ? r.E.data() : nullptr,
                     r.Er.data(), r.Fr.data(), r.kP.data(), r.kF.data(), r.kappa_scalar);
  if (!rc && !r.j.empty()) rc = rhd_set_emission(h, r.j.data());
  if (rc) {
    std::snprintf(msg, 256, "%s", rhd_last_error(h));
    rhd_destroy(h);
    return rc;
  }
  r.h = h;
  drop_inputs(r);
  return RHD_OK;
}

// Transfer thread: copy the final state and diagnostics of a request out of its handle
// (which has left its batch) and free the handle. fail is the code of a failure already
// known (the state is still copied, as computed); returns the request's final code.
int collect_request(Request& r, int fail) {
  int rc = rhd_get_state(r.h, r.rho.data(), r.mom.data(), r.have_E ? r.E.data() : nullptr,
                         r.Er.data(), r.Fr.data());
  rhd_diag d{};
  const int rd = rhd_get_diagnostics(r.h, &d);
  if (rd == RHD_OK) r.diag = d;
  if (!rc) rc = rd;
  if (!rc && r.diag.nonfinite > 0) rc = RHD_ENONFINITE;
  rhd_destroy(r.h);
  r.h = nullptr;
  return fail ? fail : rc;
}

// A transfer thread of queue q: 0 takes the set-up jobs, 1 the read-back and free jobs.
void xfer_main(rhd_server* s, int q) {
  (void)hipSetDevice(s->device);
  for (;;) {
    rhd_server::Job job;
    bool cleanup;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_xfer[q].wait(lk, [&] { return s->xstop || !s->jobs[q].empty(); });
      if (s->jobs[q].empty()) break;
      job = std::move(s->jobs[q].front());
      s->jobs[q].pop_front();
      cleanup = s->stop;
    }
    Request& r = *job.r;
    if (job.kind == JOB_PREPARE) {
      bool skip;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        skip = cleanup || r.cancel;
      }
      char msg[256] = "";
      const int rc = skip ? RHD_OK : prepare_request(r, msg);
      std::lock_guard<std::mutex> lk(s->mu);
      if (skip) {
        retire(s, r, RHD_REQ_CANCELLED, RHD_OK);
      } else if (rc) {
        sfail(s, rc, "request %lld: %s", r.id, msg);
        retire(s, r, RHD_REQ_FAILED, rc);
      } else {
        s->ready.push_back(job.r);
        s->cv_work.notify_one();
      }
    } else if (job.kind == JOB_COLLECT) {
      const int rc = collect_request(r, job.status);
      std::lock_guard<std::mutex> lk(s->mu);
      if (rc) {
        if (!job.why.empty()) sfail(s, rc, "request %lld: %s", r.id, job.why.c_str());
        else sfail(s, rc, "request %lld: final state: code %d", r.id, rc);
        retire(s, r, RHD_REQ_FAILED, rc);
      } else {
        retire(s, r, RHD_REQ_DONE, RHD_OK);
      }
    } else {
      if (r.h) rhd_destroy(r.h);
      r.h = nullptr;
      std::lock_guard<std::mutex> lk(s->mu);
      if (job.status == RHD_REQ_FAILED) sfail(s, job.error, "request %lld: %s", r.id, job.why.c_str());
      retire(s, r, job.status, job.error);
    }
  }
}

// Worker: take a member out of its batch (no lock held); the handle stays alive.
void leave_batch(rhd_server* s, const ReqPtr& r, int prec) {
  auto& m = s->members[prec];
  for (size_t i = 0; i < m.size(); ++i)
    if (m[i] == r) {
      (void)rhd_batch_remove(s->batch[prec], r->h);
      m.erase(m.begin() + long(i));
      return;
    }
}

void worker_main(rhd_server* s) {
  (void)hipSetDevice(s->device);
  std::vector<int> nsub;
  for (;;) {
    std::vector<ReqPtr> enrol, cancelled;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        return s->stop || !s->ready.empty() || !s->members[0].empty() ||
               !s->members[1].empty() || can_admit(s);
      });
      if (s->stop) break;
      for (int prec = 0; prec < 2; ++prec)
        for (auto& r : s->members[prec])
          if (r->cancel) cancelled.push_back(r);
      // admission in submission order: stop at the first request that does not fit; an
      // admitted request holds its budget and slot from here until it is retired
      while (can_admit(s)) {
        ReqPtr r = s->queue.front();
        s->queue.pop_front();
        s->used += r->footprint;
        s->stats.running += 1;
        r->status = RHD_REQ_RUNNING;
        r->t_start = s->now();
        rhd_server::Job job;
        job.r = r;
        job.kind = JOB_PREPARE;
        post(s, std::move(job));
      }
      s->stats.queued = int(s->queue.size());
      s->stats.peak_running = std::max(s->stats.peak_running, s->stats.running);
      s->stats.bytes_in_use = s->used;
      s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->used);
      // requests the transfer thread has set up join their batch below; one cancelled
      // meanwhile is freed instead
      for (auto& r : s->ready) {
        if (r->cancel) {
          rhd_server::Job job;
          job.r = r;
          job.kind = JOB_DISCARD;
          job.status = RHD_REQ_CANCELLED;
          post(s, std::move(job));
        } else {
          enrol.push_back(r);
        }
      }
      s->ready.clear();
    }
    for (auto& r : cancelled) {
      leave_batch(s, r, r->mixed ? 1 : 0);
      std::lock_guard<std::mutex> lk(s->mu);
      rhd_server::Job job;
      job.r = r;
      job.kind = JOB_DISCARD;
      job.status = RHD_REQ_CANCELLED;
      post(s, std::move(job));
    }
    for (auto& r : enrol) {
      const int prec = r->mixed ? 1 : 0;
      int rc = RHD_OK;
      std::string why;
      if (!s->batch[prec]) {
        rc = rhd_batch_create(nullptr, s->max_slots, s->rows, s->zchunk, &s->batch[prec]);
        if (rc) why = std::string("rhd_batch_create: ") + rhd_batch_last_error(nullptr);
        else if (s->persistent) (void)rhd_batch_set_persistent(s->batch[prec], 1);
      }
      if (!rc) {
        rc = rhd_batch_add(s->batch[prec], r->h, r->chat);
        if (rc) why = std::string("rhd_batch_add: ") + rhd_batch_last_error(s->batch[prec]);
      }
      std::lock_guard<std::mutex> lk(s->mu);
      if (rc) {
        rhd_server::Job job;
        job.r = r;
        job.kind = JOB_DISCARD;
        job.status = RHD_REQ_FAILED;
        job.error = rc;
        job.why = why;
        post(s, std::move(job));
      } else {
        // a request cancelled while it joined leaves at the top of the next round
        s->members[prec].push_back(r);
      }
    }
    // one round: every running request takes one gas step
    for (int prec = 0; prec < 2; ++prec) {
      auto& m = s->members[prec];
      while (!m.empty()) {
        bool skip = false;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          for (auto& r : m) skip = skip || r->cancel;
        }
        if (skip) break;  // a request was cancelled meanwhile: handle it first
        nsub.assign(m.size(), 0);
        const int rc = rhd_batch_step(s->batch[prec], nsub.data(), nullptr);
        if (rc == RHD_OK) {
          std::lock_guard<std::mutex> lk(s->mu);
          for (size_t i = 0; i < m.size(); ++i) {
            m[i]->steps_done += 1;
            m[i]->zone_updates += m[i]->cells * nsub[i];
            s->stats.zone_updates += m[i]->cells * nsub[i];
          }
          s->stats.rounds += 1;
          break;
        }
        // a member that cannot step is named by -1: it fails alone, the others retry
        int bad = -1;
        for (size_t i = 0; i < m.size(); ++i)
          if (nsub[i] == -1) bad = int(i);
        const std::string why = rhd_batch_last_error(s->batch[prec]);
        std::vector<ReqPtr> gone;
        if (bad >= 0) gone.push_back(m[size_t(bad)]);
        else gone.assign(m.begin(), m.end());  // a device failure: the whole batch fails
        for (auto& r : gone) leave_batch(s, r, prec);
        std::lock_guard<std::mutex> lk(s->mu);
        if (bad < 0) sfail(s, rc, "batch step: %s", why.c_str());
        for (auto& r : gone) {
          // the state is still copied out, as computed
          rhd_server::Job job;
          job.r = r;
          job.kind = JOB_COLLECT;
          job.status = rc;
          job.why = why;
          post(s, std::move(job));
        }
      }
    }
    // requests that took all their steps leave their batch and go to the transfer
    // thread, which copies their results out; one cancelled during its last round counts
    // as cancelled
    for (int prec = 0; prec < 2; ++prec) {
      std::vector<ReqPtr> done;
      std::vector<bool> dropped;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& r : s->members[prec])
          if (r->steps_done >= r->steps) {
            done.push_back(r);
            dropped.push_back(r->cancel);
          }
      }
      for (size_t k = 0; k < done.size(); ++k) {
        leave_batch(s, done[k], prec);
        std::lock_guard<std::mutex> lk(s->mu);
        rhd_server::Job job;
        job.r = done[k];
        job.kind = dropped[k] ? JOB_DISCARD : JOB_COLLECT;
        job.status = dropped[k] ? RHD_REQ_CANCELLED : 0;
        post(s, std::move(job));
      }
    }
  }
  // stopping: free every member's handle and every batch
  for (int prec = 0; prec < 2; ++prec) {
    for (auto& r : s->members[prec]) {
      if (r->h) rhd_destroy(r->h);
      r->h = nullptr;
    }
    s->members[prec].clear();
    rhd_batch_destroy(s->batch[prec]);
    s->batch[prec] = nullptr;
  }
}

}  // namespace

extern "C" {

int rhd_server_create(long long budget_bytes, int max_slots, int tile_rows, int zchunk,
                      rhd_server_t** out) {
  if (!out) return sfail(nullptr, RHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (budget_bytes <= 0) return sfail(nullptr, RHD_EINVAL, "budget_bytes must be > 0");
  if (max_slots < 1) return sfail(nullptr, RHD_EINVAL, "max_slots must be >= 1");
  if (!(tile_rows == 4 || tile_rows == 8 || tile_rows == 16))
    return sfail(nullptr, RHD_EINVAL, "tile_rows must be 4, 8 or 16");
  if (zchunk < 1) return sfail(nullptr, RHD_EINVAL, "zchunk must be >= 1");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return sfail(nullptr, RHD_EDEVICE, "hipGetDevice failed");
  auto* s = new (std::nothrow) rhd_server;
  if (!s) return sfail(nullptr, RHD_ENOMEM, "out of host memory");
  s->budget = budget_bytes;
  s->max_slots = max_slots;
  s->rows = tile_rows;
  s->zchunk = zchunk;
  s->device = dev;
  s->t0 = Clock::now();
  auto stop_transfers = [](rhd_server* sv) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->xstop = true;
      sv->cv_xfer[0].notify_all();
      sv->cv_xfer[1].notify_all();
    }
    for (auto& t : sv->xfer)
      if (t.joinable()) t.join();
  };
  try {
    for (int t = 0; t < 2 * rhd_server::XFER_THREADS; ++t)
      s->xfer[t] = std::thread(xfer_main, s, t % 2);
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    stop_transfers(s);
    delete s;
    return sfail(nullptr, RHD_EDEVICE, "cannot start the server's threads");
  }
  *out = s;
  return RHD_OK;
}

int rhd_server_set_persistent(rhd_server_t* s, int on) {
  if (!s) return sfail(nullptr, RHD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->next_id != 1) return sfail(s, RHD_ESTATE, "the launch mode is set before the first submission");
  if (on)
    return sfail(s, RHD_EINVAL, "the persistent launch is switched off: it did not finish on the GPU");
  s->persistent = 0;
  return RHD_OK;
}

int rhd_server_submit(rhd_server_t* s, const rhd_params* p, const double* rho,
                      const double* mom, const double* E, const double* Er, const double* Fr,
                      const double* kappaP, const double* kappaF, int kappa_scalar,
                      const double* j, int steps, double chat, long long* id) {
  if (!s) return sfail(nullptr, RHD_EINVAL, "server is NULL");
  if (!p || !id) return sfail(s, RHD_EINVAL, "p or id is NULL");
  const long long fp = rhd_footprint_bytes(p);
  if (fp < 0) return sfail(s, RHD_EINVAL, "invalid parameters");
  if (!(p->nx > 1 && p->ny > 1 && p->nz > 1)) return sfail(s, RHD_EINVAL, "the grid must be 3D");
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] == RHD_BC_FIXED) return sfail(s, RHD_EINVAL, "fixed faces cannot be served");
  if (steps < 1) return sfail(s, RHD_EINVAL, "steps must be >= 1");
  if (!(chat > 0.0)) return sfail(s, RHD_EINVAL, "chat must be > 0");
  if (!rho || !mom || !Er || !Fr || !kappaP || !kappaF)
    return sfail(s, RHD_EINVAL, "rho, mom, Er, Fr, kappaP and kappaF must be non-NULL");
  const bool iso = (p->flags & RHD_ISOTHERMAL) != 0;
  if (!E && !iso) return sfail(s, RHD_EINVAL, "E must be non-NULL for an ideal gas");
  if (fp > s->budget) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.rejected += 1;
    return sfail(s, RHD_ENOMEM, "request needs %lld bytes, the budget is %lld", fp, s->budget);
  }
  auto r = std::make_shared<Request>();
  const size_t N = size_t(p->nx) * size_t(p->ny) * size_t(p->nz);
  r->p = *p;
  r->cells = (long long)N;
  r->footprint = fp;
  r->steps = steps;
  r->chat = chat;
  r->kappa_scalar = kappa_scalar ? 1 : 0;
  r->mixed = (p->flags & RHD_PRECISION_MIXED) != 0;
  const size_t nk = kappa_scalar ? 1 : N;
  try {
    r->rho.assign(rho, rho + N);
    r->mom.assign(mom, mom + 3 * N);
    r->have_E = E != nullptr;
    if (E) r->E.assign(E, E + N);
    r->Er.assign(Er, Er + N);
    r->Fr.assign(Fr, Fr + 3 * N);
    r->kP.assign(kappaP, kappaP + nk);
    r->kF.assign(kappaF, kappaF + nk);
    if (j) r->j.assign(j, j + N);
  } catch (...) {
    return sfail(s, RHD_ENOMEM, "out of host memory for the request's copy");
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->t_submit = s->now();
  s->queue.push_back(r);
  s->all[r->id] = r;
  s->stats.submitted += 1;
  s->stats.queued = int(s->queue.size());
  *id = r->id;
  s->cv_work.notify_one();
  return RHD_OK;
}

int rhd_server_poll(rhd_server_t* s, long long id, rhd_request_info* info) {
  if (!s) return sfail(nullptr, RHD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return sfail(s, RHD_EINVAL, "unknown request %lld", id);
  fill_info(*it->second, info);
  return RHD_OK;
}

int rhd_server_wait(rhd_server_t* s, long long id, double timeout_s, rhd_request_info* info) {
  if (!s) return sfail(nullptr, RHD_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return sfail(s, RHD_EINVAL, "unknown request %lld", id);
  ReqPtr r = it->second;
  auto ready = [&] { return finished(r->status); };
  if (timeout_s < 0.0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    fill_info(*r, info);
    return sfail(s, RHD_ETIMEOUT, "request %lld not finished after %g s", id, timeout_s);
  }
  fill_info(*r, info);
  return RHD_OK;
}

int rhd_server_fetch(rhd_server_t* s, long long id, double* rho, double* mom, double* E,
                     double* Er, double* Fr, rhd_diag* diag) {
  if (!s) return sfail(nullptr, RHD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return sfail(s, RHD_EINVAL, "unknown request %lld", id);
  Request& r = *it->second;
  if (r.status != RHD_REQ_DONE && r.status != RHD_REQ_FAILED)
    return sfail(s, RHD_ESTATE, "request %lld has no result (status %d)", id, r.status);
  const size_t N = size_t(r.cells);
  auto put = [](double* dst, const std::vector<double>& src) {
    if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(double));
  };
  put(rho, r.rho);
  put(mom, r.mom);
  if (E) {
    if (r.have_E) put(E, r.E);
    else std::fill(E, E + N, 0.0);
  }
  put(Er, r.Er);
  put(Fr, r.Fr);
  if (diag) *diag = r.diag;
  const int code = r.status == RHD_REQ_DONE ? RHD_OK : r.error;
  s->all.erase(it);
  if (code) sfail(s, code, "request %lld failed with code %d", id, code);
  return code;
}

int rhd_server_cancel(rhd_server_t* s, long long id) {
  if (!s) return sfail(nullptr, RHD_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return sfail(s, RHD_EINVAL, "unknown request %lld", id);
  ReqPtr r = it->second;
  if (finished(r->status)) {
    s->all.erase(it);
    return RHD_OK;
  }
  if (r->status == RHD_REQ_QUEUED) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
    r->status = RHD_REQ_CANCELLED;
    r->t_done = s->now();
    drop_all(*r);
    s->stats.cancelled += 1;
    s->stats.queued = int(s->queue.size());
    s->cv_done.notify_all();
    return RHD_OK;
  }
  r->cancel = true;
  s->cv_work.notify_one();
  return RHD_OK;
}

int rhd_server_get_stats(rhd_server_t* s, rhd_server_stats* out) {
  if (!s || !out) return sfail(s, RHD_EINVAL, "server or out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued = int(s->queue.size());
  return RHD_OK;
}

void rhd_server_destroy(rhd_server_t* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  // the worker has freed its members; the transfer threads free what they still hold
  // (jobs queued after stop skip their uploads) and end
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->xstop = true;
    s->cv_xfer[0].notify_all();
    s->cv_xfer[1].notify_all();
  }
  for (auto& t : s->xfer)
    if (t.joinable()) t.join();
  for (auto& r : s->ready)
    if (r->h) {
      rhd_destroy(r->h);
      r->h = nullptr;
    }
  s->ready.clear();
  delete s;
}

const char* rhd_server_last_error(const rhd_server_t* s) {
  if (!s) return g_server_error;
  // a copy for the calling thread, taken under the message's lock
  thread_local char copy[256];
  auto* m = const_cast<rhd_server_t*>(s);
  std::lock_guard<std::mutex> lk(m->err_mu);
  std::snprintf(copy, sizeof(copy), "%s", m->err);
  return copy;
}

}  // extern "C"
