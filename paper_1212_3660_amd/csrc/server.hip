// Solve server: continuous admission of shifted-system requests.
//
// A request is a 2-D field, a set of shifts and a block of right-hand sides.
// All device memory of a request (operator faces and multigrid hierarchy,
// Krylov workspace, right-hand sides, output) comes from one contiguous
// region of the server's device arena: the caller's buffer, or one
// allocation the server makes when it is created.  Worker threads (one per
// slot, each with its own non-blocking HIP stream) take the oldest pending
// request for which a region of its footprint is free (first fit), set the
// problem up, solve it, copy its output to the host and release the region;
// requests that arrive while others run are admitted as soon as a slot and a
// region free up, and their kernels overlap on the device with those of the
// running requests.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

using shk::c128;

namespace {

struct Job {
  long long ticket;
  int nx, ny;
  std::vector<double> K;
  double Ss, h;
  std::vector<shk_c128> sigma;
  int n_rhs;
  std::vector<shk_c128> b;
  shk_params prm;
  std::vector<shk_c128> taus;
  std::vector<long long> rows;
  size_t need = 0;
  size_t region = 0;   // arena offset while running
  // results (written by the worker under the server mutex)
  shk_result res{};
  std::vector<shk_c128> x;
  std::vector<shk_status> st;
  bool keep_x = true;
};

}  // namespace

struct shk_server {
  size_t budget;
  int slots;
  char* arena = nullptr;
  bool own_arena = false;
  std::map<size_t, size_t> free_;   // free regions of the arena: offset -> length
  int running = 0;
  bool stop = false;
  long long next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> pending;
  std::map<long long, std::unique_ptr<Job>> jobs;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;
  int device = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  // First free region of at least len bytes (256-byte granules); false if none.
  bool reserve(size_t len, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const size_t rest = it->second - len;
      const size_t at = it->first + len;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  // Returns a region, merging it with free neighbours.
  void release(size_t off, size_t len) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
};

static size_t granule(size_t b) { return (b + 255) & ~size_t(255); }

// Device bytes of a request: problem arrays, workspace, right-hand sides and
// the device copy of its output, each rounded to the region's alignment.
static size_t footprint(const Job& j) {
  shk_problem tmp{};
  tmp.kind = shk::Kind::FV2D;
  tmp.nx = j.nx;
  tmp.ny = j.ny;
  tmp.nz = 1;
  tmp.n = (long long)j.nx * j.ny;
  shk::problem_plan_levels(&tmp);   // the workspace holds multigrid buffers per level
  const int nf = (int)j.sigma.size();
  const size_t ws = shk::workspace_bytes(&tmp, &j.prm, nf, j.n_rhs, false);
  const size_t xb = sizeof(c128) * shk::output_elems(&j.prm, tmp.n, nf, j.n_rhs, nullptr);
  const size_t bb = sizeof(c128) * (size_t)tmp.n * j.n_rhs;
  return granule(granule(shk::problem_bytes(&tmp)) + granule(ws) + granule(xb) + granule(bb) + (1u << 20));
}

// Runs one request on stream st inside its arena region.  Only this thread
// touches the request's inputs while it runs; the outputs go to res_out /
// x_out / st_out, which the caller publishes under the server mutex.
static void run_job(shk_server* s, Job* j, hipStream_t st, shk_result& res_out, std::vector<shk_c128>& x_out,
                    std::vector<shk_status>& st_out) {
  res_out.t_start = s->now();
  shk::Bump bump{s->arena + j->region, 0, j->need};
  shk_problem* p = new shk_problem();
  p->kind = shk::Kind::FV2D;
  p->nx = j->nx;
  p->ny = j->ny;
  p->nz = 1;
  p->bump = &bump;
  int rc = shk::problem_setup_fv(p, j->K.data(), j->Ss, j->h, st);
  const long long n = (long long)j->nx * j->ny;
  const int nf = (int)j->sigma.size();
  st_out.assign((size_t)nf * j->n_rhs, shk_status{});
  if (rc == SHK_OK) {
    const size_t wsb = shk::workspace_bytes(p, &j->prm, nf, j->n_rhs, false);
    const size_t xe = shk::output_elems(&j->prm, n, nf, j->n_rhs, nullptr);
    void* ws = bump.take(wsb);
    void* xd = bump.take(sizeof(c128) * xe);
    void* bd = bump.take(sizeof(c128) * (size_t)n * j->n_rhs);
    if (!ws || !xd || !bd) {
      rc = shk::fail(SHK_ERR_OOM, "server request region too small");
    } else {
      (void)hipMemcpyAsync(bd, j->b.data(), sizeof(c128) * (size_t)n * j->n_rhs, hipMemcpyHostToDevice, st);
      rc = shk::solve_all(p, &j->prm, nf, reinterpret_cast<const c128*>(j->sigma.data()), j->n_rhs,
                          reinterpret_cast<const c128*>(bd), reinterpret_cast<c128*>(xd), st_out.data(), ws, wsb,
                          st, SHK_PTR_DEVICE);
      if (rc == SHK_OK && j->keep_x) {
        x_out.resize(xe);
        (void)hipMemcpyAsync(x_out.data(), xd, sizeof(c128) * xe, hipMemcpyDeviceToHost, st);
      }
    }
  }
  shk::problem_free(p, st);
  delete p;
  (void)hipStreamSynchronize(st);
  res_out.error = rc;
  int nconv = 0;
  double worst = 0.0;
  for (const shk_status& x : st_out) {
    nconv += (x.status == SHK_CONVERGED || x.status == SHK_BREAKDOWN_EXACT);
    worst = std::max(worst, x.true_relres);
  }
  res_out.n_converged = nconv;
  res_out.max_true_relres = worst;
  res_out.t_done = s->now();
}

static void worker(shk_server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    Job* pick = nullptr;
    s->cv_work.wait(lk, [&] {
      if (s->stop) return true;
      // the oldest pending request that a free region can hold
      for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
        size_t off = 0;
        if (s->reserve((*it)->need, &off)) {
          pick = *it;
          pick->region = off;
          s->pending.erase(it);
          return true;
        }
      }
      return false;
    });
    if (!pick) {
      if (s->stop) break;
      continue;
    }
    s->running += 1;
    shk_result res = pick->res;   // t_arrival, set at submit under the mutex
    lk.unlock();
    std::vector<shk_c128> x;
    std::vector<shk_status> stv;
    run_job(s, pick, st, res, x, stv);
    lk.lock();
    // publish: shk_server_poll reads these under the mutex only
    res.done = 1;
    pick->res = res;
    pick->x.swap(x);
    pick->st.swap(stv);
    std::vector<double>().swap(pick->K);      // the request's inputs are no longer needed
    std::vector<shk_c128>().swap(pick->b);
    s->release(pick->region, pick->need);
    s->running -= 1;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  lk.unlock();
  (void)hipStreamDestroy(st);
}

extern "C" {

int shk_server_create(size_t mem_budget_bytes, int max_slots, void* device_arena, shk_server** out) {
  if (!out || max_slots < 1 || max_slots > 16 || mem_budget_bytes < (1u << 20))
    return shk::fail(SHK_ERR_INVALID_ARG, "server arguments (1 <= max_slots <= 16, budget >= 1 MiB)");
  shk_server* s = new shk_server();
  s->budget = mem_budget_bytes & ~size_t(255);
  s->slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return shk::fail(SHK_ERR_HIP, "no HIP device");
  }
  if (device_arena) {
    if (reinterpret_cast<uintptr_t>(device_arena) & 255) {
      delete s;
      return shk::fail(SHK_ERR_INVALID_ARG, "the device arena must be 256-byte aligned");
    }
    s->arena = static_cast<char*>(device_arena);
  } else {
    void* a = nullptr;
    if (hipMalloc(&a, s->budget) != hipSuccess) {
      delete s;
      return shk::fail(SHK_ERR_OOM, "server arena allocation");
    }
    s->arena = static_cast<char*>(a);
    s->own_arena = true;
  }
  s->free_[0] = s->budget;
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return SHK_OK;
}

int shk_server_submit(shk_server* s, const shk_request* req, long long* ticket) {
  if (!s || !req || !ticket || !req->cell_K || !req->sigma || !req->b || req->nx < 1 || req->ny < 1 ||
      req->n_shifts < 1 || req->n_rhs < 1 || req->params.n_tau < 1 || !req->params.tau_seq)
    return shk::fail(SHK_ERR_INVALID_ARG, "request arguments");
  const shk_params& pr = req->params;
  const long long n = (long long)req->nx * req->ny;
  if (pr.output == SHK_OUT_ROWS) {
    if (pr.n_out_rows < 1 || !pr.out_rows) return shk::fail(SHK_ERR_INVALID_ARG, "SHK_OUT_ROWS needs out_rows");
    for (int q = 0; q < pr.n_out_rows; ++q)
      if (pr.out_rows[q] < 0 || pr.out_rows[q] >= n) return shk::fail(SHK_ERR_INVALID_ARG, "out_rows outside [0, n)");
  }
  auto j = std::make_unique<Job>();
  j->nx = req->nx;
  j->ny = req->ny;
  j->K.assign(req->cell_K, req->cell_K + n);
  j->Ss = req->Ss;
  j->h = req->h;
  j->sigma.assign(req->sigma, req->sigma + req->n_shifts);
  j->n_rhs = req->n_rhs;
  j->b.assign(req->b, req->b + n * req->n_rhs);
  j->prm = pr;
  j->taus.assign(pr.tau_seq, pr.tau_seq + pr.n_tau);
  j->prm.tau_seq = j->taus.data();
  if (pr.output == SHK_OUT_ROWS) {
    j->rows.assign(pr.out_rows, pr.out_rows + pr.n_out_rows);
    j->prm.out_rows = j->rows.data();
  } else {
    j->prm.out_rows = nullptr;
  }
  j->keep_x = req->keep_solution != 0;
  j->need = footprint(*j);
  std::lock_guard<std::mutex> g(s->mu);
  if (j->need > s->budget) return shk::fail(SHK_ERR_REJECTED, "request exceeds the memory budget");
  j->ticket = s->next_ticket++;
  j->res.t_arrival = s->now();
  *ticket = j->ticket;
  s->pending.push_back(j.get());
  s->jobs[j->ticket] = std::move(j);
  s->cv_work.notify_all();
  return SHK_OK;
}

int shk_server_poll(shk_server* s, long long ticket, shk_result* res, shk_c128* x, shk_status* st) {
  if (!s || !res) return shk::fail(SHK_ERR_INVALID_ARG, "poll arguments");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return shk::fail(SHK_ERR_INVALID_ARG, "unknown ticket");
  Job* j = it->second.get();
  if (!j->res.done) return SHK_ERR_NOT_READY;
  *res = j->res;
  if (x && !j->x.empty()) std::copy(j->x.begin(), j->x.end(), x);
  if (st) std::copy(j->st.begin(), j->st.end(), st);
  return SHK_OK;
}

int shk_server_drain(shk_server* s) {
  if (!s) return shk::fail(SHK_ERR_INVALID_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->running == 0; });
  return SHK_OK;
}

double shk_server_clock(shk_server* s) { return s ? s->now() : 0.0; }

int shk_server_destroy(shk_server* s) {
  if (!s) return SHK_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    // requests never started are dropped
    s->pending.clear();
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  if (s->own_arena) (void)hipFree(s->arena);
  delete s;
  return SHK_OK;
}

}  // extern "C"
