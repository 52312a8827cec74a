// Serving loop: k-th eigenvalue queries against matrices resident in HBM, with
// continuous batching.  Each resident matrix has a worker thread (and the
// matrix's own stream, so that matrices overlap on the device).  Every tick a
// worker admits queued queries up to the matrix's slot count, puts the next
// midpoint of every in-flight bracket into ONE h2_inertia call (Algorithm 1 of
// Sec. 2, all queries of the matrix merged, inertia reuse of Sec. 4.2 through
// the matrix's record cache), narrows every bracket with every new record and
// completes the queries whose bracket is narrower than their tolerance.
// Latency is taken from submission to completion.
//
// Admission by memory: the server owns one device-memory budget for the
// factorization workspace of all its matrices.  Each matrix's workspace per
// shift is measured when it is added (one factorization), and a worker holds
// budget for as many shifts as it has admitted queries: it grows its share at
// each tick while the budget allows, queues the rest, and gives its share
// (and its workspace) back when it has nothing in flight.
#include <algorithm>
#include <atomic>
#include <climits>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/h2eig.h"
#include "records.hpp"

namespace h2 {
void set_last_error(const std::string& msg);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Query {
  int32_t mat = 0;
  int64_t k = 0;
  double tol = 0.0;
  double lo = 0.0, hi = 0.0;
  Clock::time_point t_submit, t_done;
  double split = 0.0;   // the shift of the current step
  int nudge = 0;        // split moved by nudge/64 of the width after a singular pivot
  int state = 0;        // 0 queued, 1 in flight, 2 done, 3 failed
  h2_status status = H2_OK;
  double lambda = 0.0;
};

struct Resident {
  h2_matrix A = nullptr;
  int64_t n = 0;
  int32_t slots = 1;        // most queries in flight
  double a0 = 0.0, b0 = 0.0;
  int64_t per_shift = 0;    // workspace bytes of one shift (measured at admission of the matrix, +10%)
  int64_t held = 0;         // budget held: per_shift times the shifts it can factor together now
  std::deque<int64_t> queue;
  std::vector<int64_t> active;
  std::vector<h2::Record> records;   // (mu, nu), sorted by mu, runs of equal nu compacted
  std::thread worker;
};

}  // namespace

struct h2_server_s {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int32_t max_slots = 0;
  int64_t budget = 0, used = 0;   // device bytes for workspace, shared by all matrices
  int waiting = 0;                // workers blocked until the budget has room
  std::vector<std::unique_ptr<Resident>> mats;
  std::map<int64_t, Query> q;
  int64_t next_ticket = 1;
  int64_t submitted = 0, served = 0, failed = 0;
  std::vector<double> lat_ms;
};

namespace {

h2_status fail(h2_status s, const char* msg) {
  h2::set_last_error(msg);
  return s;
}

// the starting bracket of a query for lambda_k from the matrix's records
void seed_bracket(const Resident& R, Query& x) { h2::record_bracket(R.records, x.k, R.a0, R.b0, &x.lo, &x.hi); }

// narrow [lo, hi] of every in-flight query of the matrix by the record (mu, nu)
void narrow(h2_server S, Resident& R, double mu, int64_t nu) {
  for (int64_t t : R.active) {
    Query& x = S->q[t];
    if (!(mu > x.lo && mu < x.hi)) continue;
    if (nu >= x.k) x.hi = mu;
    else x.lo = mu;
  }
}

void fail_query(h2_server S, Query& x, h2_status r) {
  x.state = 3;
  x.status = r;
  x.t_done = Clock::now();
  S->failed += 1;
}

// complete the in-flight queries whose bracket is below their tolerance
void complete(h2_server S, Resident& R) {
  std::vector<int64_t> keep;
  for (int64_t t : R.active) {
    Query& x = S->q[t];
    const double mid = 0.5 * (x.lo + x.hi);
    // done below the tolerance, or once the bracket has no double inside it
    if (x.hi - x.lo < x.tol || !(mid > x.lo && mid < x.hi)) {
      x.lambda = mid;
      x.state = 2;
      x.t_done = Clock::now();
      S->served += 1;
      S->lat_ms.push_back(std::chrono::duration<double, std::milli>(x.t_done - x.t_submit).count());
    } else {
      keep.push_back(t);
    }
  }
  if (keep.size() != R.active.size()) S->cv_done.notify_all();
  R.active.swap(keep);
}

void worker_loop(h2_server S, Resident* R) {
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    // wake for work: queries in flight, or queued ones and budget for one
    // shift (already held, or free)
    auto runnable = [&] {
      return S->stop || !R->active.empty() ||
             (!R->queue.empty() && (R->held >= R->per_shift || S->budget - S->used >= R->per_shift));
    };
    if (!runnable()) {
      ++S->waiting;
      S->cv_work.wait(lk, runnable);
      --S->waiting;
    }
    if (S->stop) break;
    // admission by memory: grow the held share toward the wanted shifts
    {
      const int64_t want = std::min<int64_t>(R->slots, (int64_t)(R->active.size() + R->queue.size()));
      if (want * R->per_shift > R->held) {
        const int64_t room = S->budget - S->used + R->held;
        const int64_t can = std::min<int64_t>(want, room / std::max<int64_t>(1, R->per_shift));
        if (can * R->per_shift > R->held) {
          S->used += can * R->per_shift - R->held;
          R->held = can * R->per_shift;
        }
      }
    }
    const int64_t cap_shifts = R->held / std::max<int64_t>(1, R->per_shift);
    while ((int64_t)R->active.size() < std::min<int64_t>(R->slots, cap_shifts) && !R->queue.empty()) {
      const int64_t t = R->queue.front();
      R->queue.pop_front();
      Query& x = S->q[t];
      x.state = 1;
      seed_bracket(*R, x);
      R->active.push_back(t);
    }
    complete(S, *R);
    std::vector<double> mus;
    for (int64_t t : R->active) {
      Query& x = S->q[t];
      x.split = x.lo + (x.hi - x.lo) * (0.5 + x.nudge / 64.0);
      mus.push_back(x.split);
    }
    if (mus.empty()) {
      // nothing in flight: give the workspace and the budget share back
      if (R->held > 0) {
        S->used -= R->held;
        R->held = 0;
        lk.unlock();
        (void)h2_release_workspace(R->A);
        lk.lock();
        S->cv_work.notify_all();
      }
      continue;
    }
    std::sort(mus.begin(), mus.end());
    mus.erase(std::unique(mus.begin(), mus.end()), mus.end());
    std::vector<int64_t> nus(mus.size());
    std::vector<int32_t> sts(mus.size());
    const int32_t batch = (int32_t)std::max<int64_t>(1, cap_shifts);
    lk.unlock();
    (void)h2_set_max_shifts(R->A, batch);
    const h2_status r = h2_inertia(R->A, mus.data(), (int64_t)mus.size(), nus.data(), sts.data());
    lk.lock();
    if (r != H2_OK && r != H2_ENUMERIC) {   // the in-flight queries fail with the call's status
      for (int64_t t : R->active) fail_query(S, S->q[t], r);
      R->active.clear();
      S->cv_done.notify_all();
      continue;
    }
    // a shift that met an exactly singular pivot gives no count: its queries
    // split elsewhere inside their brackets next time
    std::vector<int64_t> keep;
    for (int64_t t : R->active) {
      Query& x = S->q[t];
      const size_t j = std::lower_bound(mus.begin(), mus.end(), x.split) - mus.begin();
      if (sts[j] == H2_OK) {
        x.nudge = 0;
      } else if (++x.nudge > 8) {
        fail_query(S, x, H2_ENUMERIC);
        S->cv_done.notify_all();
        continue;
      }
      keep.push_back(t);
    }
    R->active.swap(keep);
    for (size_t j = 0; j < mus.size(); ++j) {
      if (sts[j] != H2_OK) continue;
      h2::record_insert(R->records, mus[j], nus[j]);
      narrow(S, *R, mus[j], nus[j]);
    }
    h2::record_compact(R->records);
    complete(S, *R);
    // nothing in flight: give the share back when the queue is empty, or
    // when another matrix waits for budget (then step aside briefly so that
    // it can take the share before this worker competes again)
    if (R->active.empty() && R->held > 0 && (R->queue.empty() || S->waiting > 0)) {
      const bool yield = !R->queue.empty();
      S->used -= R->held;
      R->held = 0;
      lk.unlock();
      (void)h2_release_workspace(R->A);
      S->cv_work.notify_all();
      if (yield) std::this_thread::sleep_for(std::chrono::milliseconds(2));
      lk.lock();
    }
  }
  // stopping: the share goes back and the matrix's workspace is freed, so that
  // a later server (or the caller) finds the memory free
  if (R->held > 0) {
    S->used -= R->held;
    R->held = 0;
  }
  lk.unlock();
  (void)h2_release_workspace(R->A);
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

h2_status h2s_create(int64_t budget_bytes, int32_t max_slots, h2_server* out) {
  if (!out) return fail(H2_EINVAL, "out is NULL");
  if (max_slots < 0 || budget_bytes < 0) return fail(H2_EINVAL, "max_slots and budget_bytes must be >= 0");
  int64_t budget = budget_bytes;
  if (budget == 0) {
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) {
      (void)hipGetLastError();
      return fail(H2_EDEVICE, "hipMemGetInfo failed");
    }
    budget = (int64_t)(0.85 * (double)freeb);
  }
  *out = new h2_server_s();
  (*out)->max_slots = max_slots;
  (*out)->budget = budget;
  return H2_OK;
}

h2_status h2s_add(h2_server S, h2_matrix A, int32_t slots, int32_t* id) {
  if (!S || !A || !id) return fail(H2_EINVAL, "NULL argument");
  if (slots < 0) return fail(H2_EINVAL, "slots must be >= 0");
  auto R = std::make_unique<Resident>();
  R->A = A;
  double ab[2];
  h2_status r = h2_interval(A, ab);
  if (r != H2_OK) return r;
  h2_stats_t st;
  r = h2_stats(A, &st);
  if (r != H2_OK) return r;
  R->n = st.n;
  R->a0 = ab[0];
  R->b0 = ab[1];
  R->slots = slots > 0 ? slots : (S->max_slots > 0 ? S->max_slots : 64);
  // workspace of one shift: one factorization at the middle of the starting
  // interval (its count seeds the records), then the workspace is released
  r = h2_set_max_shifts(A, 1);
  if (r != H2_OK) return r;
  const double mu = 0.5 * (R->a0 + R->b0);
  int64_t nu = 0;
  int32_t stv = 0;
  r = h2_inertia(A, &mu, 1, &nu, &stv);
  if (r != H2_OK && r != H2_ENUMERIC) return r;
  if (stv == H2_OK) R->records.push_back({mu, nu});
  r = h2_stats(A, &st);
  if (r != H2_OK) return r;
  R->per_shift = std::max<int64_t>(1, st.last_work_bytes + st.last_work_bytes / 10);
  (void)h2_release_workspace(A);
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return fail(H2_EINVAL, "server is shutting down");
  if (R->per_shift > S->budget) return fail(H2_ENOMEM, "one shift of this matrix needs more than the server's budget");
  *id = (int32_t)S->mats.size();
  S->mats.push_back(std::move(R));
  Resident* p = S->mats.back().get();
  p->worker = std::thread(worker_loop, S, p);
  return H2_OK;
}

h2_status h2s_submit(h2_server S, int32_t id, int64_t k, double tol, int64_t* ticket) {
  if (!S || !ticket) return fail(H2_EINVAL, "NULL argument");
  if (!(tol > 0.0)) return fail(H2_EINVAL, "tol must be > 0");
  std::lock_guard<std::mutex> g(S->mu);
  if (id < 0 || id >= (int32_t)S->mats.size()) return fail(H2_EINVAL, "unknown matrix id");
  if (k < 1 || k > S->mats[id]->n) return fail(H2_EINVAL, "k out of range [1, n]");
  Query x;
  x.mat = id;
  x.k = k;
  x.tol = tol;
  x.t_submit = Clock::now();
  const int64_t t = S->next_ticket++;
  S->q[t] = x;
  S->mats[id]->queue.push_back(t);
  S->submitted += 1;
  S->cv_work.notify_all();
  *ticket = t;
  return H2_OK;
}

h2_status h2s_poll(h2_server S, int64_t ticket, double* lambda, int32_t* done) {
  if (!S || !done) return fail(H2_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->q.find(ticket);
  if (it == S->q.end()) return fail(H2_EINVAL, "unknown ticket");
  *done = it->second.state >= 2 ? 1 : 0;
  if (it->second.state == 3) {
    const h2_status st = it->second.status;
    S->q.erase(it);
    return fail(st, "the query's factorization failed");
  }
  if (*done) {
    if (lambda) *lambda = it->second.lambda;
    S->q.erase(it);   // a finished ticket is read once
  }
  return H2_OK;
}

h2_status h2s_wait(h2_server S, int64_t ticket, double* lambda) {
  if (!S) return fail(H2_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->q.find(ticket);
  if (it == S->q.end()) return fail(H2_EINVAL, "unknown ticket");
  // looked up again at every wake: another h2s_poll or h2s_wait on the same
  // ticket may have read, and so forgotten, it meanwhile
  S->cv_done.wait(lk, [&] {
    it = S->q.find(ticket);
    return it == S->q.end() || it->second.state >= 2 || S->stop;
  });
  if (it == S->q.end()) return fail(H2_EINVAL, "ticket read by another call");
  if (it->second.state == 3) {
    const h2_status st = it->second.status;
    S->q.erase(it);
    return fail(st, "the query's factorization failed");
  }
  if (it->second.state != 2) return fail(H2_EINVAL, "server stopped");
  if (lambda) *lambda = it->second.lambda;
  S->q.erase(it);   // a finished ticket is read once
  return H2_OK;
}

h2_status h2s_stats(h2_server S, double* p50_ms, double* p99_ms, int64_t* served, int64_t* submitted) {
  if (!S) return fail(H2_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  if (p50_ms) *p50_ms = percentile(S->lat_ms, 0.50);
  if (p99_ms) *p99_ms = percentile(S->lat_ms, 0.99);
  if (served) *served = S->served;
  if (submitted) *submitted = S->submitted;
  return H2_OK;
}

h2_status h2s_latency(h2_server S, double* p50_ms, double* p99_ms, int64_t* unfinished, int64_t* budget_bytes,
                      int64_t* used_bytes) {
  if (!S) return fail(H2_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  std::vector<double> v = S->lat_ms;
  int64_t open = 0;
  const auto now = Clock::now();
  for (const auto& kv : S->q)
    if (kv.second.state < 2) {
      v.push_back(std::chrono::duration<double, std::milli>(now - kv.second.t_submit).count());
      ++open;
    }
  if (p50_ms) *p50_ms = percentile(v, 0.50);
  if (p99_ms) *p99_ms = percentile(v, 0.99);
  if (unfinished) *unfinished = open;
  if (budget_bytes) *budget_bytes = S->budget;
  if (used_bytes) *used_bytes = S->used;
  return H2_OK;
}

void h2s_destroy(h2_server S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  for (auto& R : S->mats)
    if (R->worker.joinable()) R->worker.join();
  delete S;
}

}  // extern "C"
