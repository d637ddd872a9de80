// Stress of the serving loop's host logic (server.cpp) with the fake engine:
// several client threads submit requests of four size classes (so several
// lanes run at once), cancel some while queued or running, wait with and
// without time-outs and poll, while another thread reads the counters; the
// server is destroyed with requests still queued.  Checks that every
// request ends DONE or CANCELED, that finished requests carry their outputs
// (T_final = T0 + nsteps) and cancelled ones none, and that the counters
// add up.  Built with the host compiler under ThreadSanitizer or
// AddressSanitizer by tests/test_server_host.py.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <memory>
#include <random>
#include <thread>
#include <vector>

#include "server.hpp"

using namespace femheat;

namespace {

struct Job {
  uint64_t ticket = 0;
  int n = 0;
  int32_t nsteps = 0;
  std::vector<double> k, rc, T0, T_final;
  std::vector<int32_t> iters;
  fem_out out{};
  bool cancel_sent = false;
};

std::atomic<int> failures{0};

void fail(const char* what, uint64_t t) {
  std::fprintf(stderr, "stress: %s (ticket %llu)\n", what, (unsigned long long)t);
  failures++;
}

void client(fem_server* srv, int id, int njobs, std::vector<std::unique_ptr<Job>>* keep) {
  std::mt19937 rng(1234u + (unsigned)id);
  const int sizes[4] = {3, 6, 10, 14};
  std::vector<Job*> mine;
  for (int j = 0; j < njobs; ++j) {
    auto job = std::make_unique<Job>();
    job->n = sizes[rng() % 4];
    job->nsteps = 1 + (int32_t)(rng() % 12);
    const size_t E = (size_t)job->n * job->n * job->n, N = (size_t)(job->n + 1) * (job->n + 1) * (job->n + 1);
    job->k.assign(E, 1.0);
    job->rc.assign(E, 1.0);
    job->T0.resize(N);
    for (size_t i = 0; i < N; ++i) job->T0[i] = (double)((i * 7 + (size_t)j) % 13);
    job->T_final.assign(N, NAN);
    job->iters.assign((size_t)job->nsteps, -1);
    job->out.T_final = job->T_final.data();
    job->out.iters = job->iters.data();
    fem_request q{};
    q.grid = fem_grid{job->n, job->n, job->n, 1.0 / job->n, 1.0 / job->n, 1.0 / job->n};
    q.k_e = job->k.data();
    q.rhoc_e = job->rc.data();
    q.T0 = job->T0.data();
    q.dt = 1e-3;
    q.theta = 1.0;
    q.rtol = 1e-8;
    q.nsteps = job->nsteps;
    q.out = &job->out;
    std::string err;
    if (server_submit(srv, q, &job->ticket, &err) != FEM_OK) {
      fail("submit failed", 0);
      continue;
    }
    const unsigned c = rng() % 10;
    if (c < 2) {  // cancel at once (mostly queued)
      server_cancel(srv, job->ticket);
      job->cancel_sent = true;
    } else if (c < 3) {  // cancel a little later (often running or admitting)
      std::this_thread::sleep_for(std::chrono::microseconds(rng() % 400));
      server_cancel(srv, job->ticket);
      job->cancel_sent = true;
    }
    if (rng() % 4 == 0) {
      fem_status st{};
      server_wait(srv, job->ticket, 1e-4, &st);  // usually times out
    }
    mine.push_back(job.get());
    keep->push_back(std::move(job));
  }
  for (Job* job : mine) {
    fem_status st{};
    const int rc = server_wait(srv, job->ticket, 60.0, &st);
    if (st.state == FEM_REQ_DONE) {
      if (rc != FEM_OK || st.status != FEM_OK) fail("finished with an error", job->ticket);
      for (size_t i = 0; i < job->T0.size(); ++i)
        if (job->T_final[i] != job->T0[i] + job->nsteps) {
          fail("wrong or missing output", job->ticket);
          break;
        }
      if (job->out.total_iters != job->nsteps) fail("total_iters not written back", job->ticket);
      if (st.steps_done != job->nsteps) fail("steps_done", job->ticket);
    } else if (st.state == FEM_REQ_CANCELED) {
      if (!job->cancel_sent) fail("cancelled without a cancel", job->ticket);
      for (double v : job->T_final)
        if (!std::isnan(v)) {
          fail("a cancelled request wrote outputs", job->ticket);
          break;
        }
    } else {
      fail("not terminal after the wait", job->ticket);
    }
  }
}

}  // namespace

int main() {
  fem_server_opts o{};
  o.hbm_budget_bytes = 8 * 4000 * 6;  // a few mid-size requests at once: admission blocks often
  o.max_slots = 6;
  o.opts = fem_opts{};  // device 0, no allocator: the server makes its pool
  fem_server* srv = nullptr;
  std::string err;
  if (server_create(o, &srv, &err) != FEM_OK) {
    std::fprintf(stderr, "create: %s\n", err.c_str());
    return 2;
  }
  std::atomic<bool> stop{false};
  std::thread watcher([&] {
    while (!stop) {
      fem_server_info info{};
      server_info(srv, &info);
      if (info.bytes_in_use > info.budget_bytes) fail("budget exceeded", 0);
      if (info.running > o.max_slots) fail("slots exceeded", 0);
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  const int nclients = 4, njobs = 40;
  std::vector<std::vector<std::unique_ptr<Job>>> jobs(nclients);
  std::vector<std::thread> th;
  for (int c = 0; c < nclients; ++c) th.emplace_back(client, srv, c, njobs, &jobs[c]);
  for (auto& t : th) t.join();
  stop = true;
  watcher.join();
  fem_server_info info{};
  server_info(srv, &info);
  if (info.submitted != nclients * njobs) fail("submitted count", 0);
  if (info.completed + info.canceled + info.failed != info.submitted) fail("counters do not add up", 0);
  if (info.failed != 0) fail("failed requests", 0);
  if (info.queued != 0 || info.running != 0 || info.bytes_in_use != 0) fail("server not idle at the end", 0);
  // destroy with work outstanding: queued requests are cancelled, running ones stop
  std::vector<std::unique_ptr<Job>> tail;
  for (int j = 0; j < 12; ++j) {
    auto job = std::make_unique<Job>();
    job->n = 10;
    job->nsteps = 50;
    const size_t E = 1000, N = 1331;
    job->k.assign(E, 1.0);
    job->rc.assign(E, 1.0);
    job->T0.assign(N, 0.0);
    job->T_final.assign(N, NAN);
    job->out.T_final = job->T_final.data();
    fem_request q{};
    q.grid = fem_grid{10, 10, 10, 0.1, 0.1, 0.1};
    q.k_e = job->k.data();
    q.rhoc_e = job->rc.data();
    q.T0 = job->T0.data();
    q.dt = 1e-3;
    q.theta = 1.0;
    q.rtol = 1e-8;
    q.nsteps = job->nsteps;
    q.out = &job->out;
    if (server_submit(srv, q, &job->ticket, &err) != FEM_OK) fail("tail submit", 0);
    tail.push_back(std::move(job));
  }
  server_destroy(srv);
  std::printf("stress: %lld submitted, %lld completed, %lld cancelled, %d failures\n", (long long)info.submitted,
              (long long)info.completed, (long long)info.canceled, failures.load());
  return failures.load() == 0 ? 0 : 1;
}
