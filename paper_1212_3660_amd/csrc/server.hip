// Solve server: continuous admission of shifted-system requests.
//
// A request is a 2-D field, a set of shifts and a block of right-hand sides.
// Worker threads (one per slot, each with its own non-blocking HIP stream)
// take the oldest pending request whose device footprint (operator faces,
// Krylov workspace and solution) fits the unused part of the memory budget,
// set the problem up, solve it, and release the memory; requests that arrive
// while others run are admitted as soon as a slot and memory free up, and
// their kernels overlap on the device with those of the running requests.
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
  size_t need = 0;
  // results
  shk_result res{};
  std::vector<shk_c128> x;
  std::vector<shk_status> st;
  bool keep_x = true;
};

}  // namespace

struct shk_server {
  size_t budget;
  int slots;
  size_t used = 0;
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
};

static size_t footprint(const Job& j) {
  shk_problem tmp{};
  tmp.kind = shk::Kind::FV2D;
  tmp.nx = j.nx;
  tmp.ny = j.ny;
  tmp.nz = 1;
  tmp.n = (long long)j.nx * j.ny;
  const size_t ws = shk::workspace_bytes(&tmp, &j.prm, (int)j.sigma.size(), j.n_rhs, false);
  const size_t xb = sizeof(c128) * (size_t)tmp.n * j.sigma.size() * j.n_rhs;
  return ws + xb + shk::problem_bytes(&tmp) + (64u << 20);
}

// Runs one request on stream st.  Only this thread touches the request's
// inputs while it runs; the outputs go to x_out / st_out / res_out, which the
// caller publishes under the server mutex.
static void run_job(shk_server* s, Job* j, hipStream_t st, shk_result& res_out, std::vector<shk_c128>& x_out,
                    std::vector<shk_status>& st_out) {
  res_out.t_start = s->now();
  shk_problem* p = new shk_problem();
  p->kind = shk::Kind::FV2D;
  p->nx = j->nx;
  p->ny = j->ny;
  p->nz = 1;
  int rc = shk::problem_setup_fv(p, j->K.data(), j->Ss, j->h, st);
  const long long n = (long long)j->nx * j->ny;
  const int nf = (int)j->sigma.size();
  void* ws = nullptr;
  void* xd = nullptr;
  void* bd = nullptr;
  st_out.assign((size_t)nf * j->n_rhs, shk_status{});
  if (rc == SHK_OK) {
    const size_t wsb = shk::workspace_bytes(p, &j->prm, nf, j->n_rhs, false);
    const size_t xb = sizeof(c128) * (size_t)n * nf * j->n_rhs;
    if (hipMallocAsync(&ws, wsb, st) != hipSuccess || hipMallocAsync(&xd, xb, st) != hipSuccess ||
        hipMallocAsync(&bd, sizeof(c128) * (size_t)n * j->n_rhs, st) != hipSuccess) {
      rc = shk::fail(SHK_ERR_OOM, "server request allocation");
    } else {
      (void)hipMemcpyAsync(bd, j->b.data(), sizeof(c128) * (size_t)n * j->n_rhs, hipMemcpyHostToDevice, st);
      rc = shk::solve_all(p, &j->prm, nf, reinterpret_cast<const c128*>(j->sigma.data()), j->n_rhs,
                          reinterpret_cast<const c128*>(bd), reinterpret_cast<c128*>(xd), st_out.data(), ws, wsb,
                          st, SHK_PTR_DEVICE);
      if (rc == SHK_OK && j->keep_x) {
        x_out.resize((size_t)n * nf * j->n_rhs);
        (void)hipMemcpyAsync(x_out.data(), xd, xb, hipMemcpyDeviceToHost, st);
      }
    }
  }
  if (ws) (void)hipFreeAsync(ws, st);
  if (xd) (void)hipFreeAsync(xd, st);
  if (bd) (void)hipFreeAsync(bd, st);
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
      for (Job* j : s->pending)
        if (s->used + j->need <= s->budget) return true;
      return false;
    });
    if (s->stop && s->pending.empty()) break;
    for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
      if (s->used + (*it)->need <= s->budget) {
        pick = *it;
        s->pending.erase(it);
        break;
      }
    }
    if (!pick) continue;
    s->used += pick->need;
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
    s->used -= pick->need;
    s->running -= 1;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  lk.unlock();
  (void)hipStreamDestroy(st);
}

extern "C" {

int shk_server_create(size_t mem_budget_bytes, int max_slots, shk_server** out) {
  if (!out || max_slots < 1 || max_slots > 16 || mem_budget_bytes == 0)
    return shk::fail(SHK_ERR_INVALID_ARG, "server arguments (1 <= max_slots <= 16)");
  shk_server* s = new shk_server();
  s->budget = mem_budget_bytes;
  s->slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return shk::fail(SHK_ERR_HIP, "no HIP device");
  }
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return SHK_OK;
}

int shk_server_submit(shk_server* s, const shk_request* req, long long* ticket) {
  if (!s || !req || !ticket || !req->cell_K || !req->sigma || !req->b || req->nx < 1 || req->ny < 1 ||
      req->n_shifts < 1 || req->n_rhs < 1 || req->params.n_tau < 1 || !req->params.tau_seq)
    return shk::fail(SHK_ERR_INVALID_ARG, "request arguments");
  auto j = std::make_unique<Job>();
  const long long n = (long long)req->nx * req->ny;
  j->nx = req->nx;
  j->ny = req->ny;
  j->K.assign(req->cell_K, req->cell_K + n);
  j->Ss = req->Ss;
  j->h = req->h;
  j->sigma.assign(req->sigma, req->sigma + req->n_shifts);
  j->n_rhs = req->n_rhs;
  j->b.assign(req->b, req->b + n * req->n_rhs);
  j->prm = req->params;
  j->taus.assign(req->params.tau_seq, req->params.tau_seq + req->params.n_tau);
  j->prm.tau_seq = j->taus.data();
  j->keep_x = req->keep_solution != 0;
  j->need = footprint(*j);
  std::lock_guard<std::mutex> g(s->mu);
  if (j->need > s->budget) return shk::fail(SHK_ERR_REJECTED, "request exceeds the memory budget");
  j->ticket = s->next_ticket++;
  j->res.t_arrival = s->now();
  *ticket = j->ticket;
  s->pending.push_back(j.get());
  s->jobs[j->ticket] = std::move(j);
  s->cv_work.notify_one();
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
  delete s;
  return SHK_OK;
}

}  // extern "C"
