// Serving loop: k-th eigenvalue queries against matrices resident in HBM, with
// continuous batching.  Each resident matrix has a worker thread (and the
// matrix's own stream, so that matrices overlap on the device).  Every tick a
// worker admits queued queries up to the matrix's slot count, puts the next
// midpoint of every in-flight bracket into ONE h2_inertia call (Algorithm 1 of
// Sec. 2, all queries of the matrix merged, inertia reuse of Sec. 4.2 through
// the matrix's record cache), narrows every bracket with every new record and
// completes the queries whose bracket is narrower than their tolerance.
// Latency is taken from submission to completion.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/h2eig.h"

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
  int32_t slots = 1;
  double a0 = 0.0, b0 = 0.0;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;
  std::vector<std::pair<double, int64_t>> records;
  std::thread worker;
};

}  // namespace

struct h2_server_s {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int32_t max_slots = 0;
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
    S->cv_work.wait(lk, [&] { return S->stop || !R->queue.empty() || !R->active.empty(); });
    if (S->stop) break;
    // admission: one bracket per slot
    while ((int32_t)R->active.size() < R->slots && !R->queue.empty()) {
      const int64_t t = R->queue.front();
      R->queue.pop_front();
      Query& x = S->q[t];
      x.state = 1;
      x.lo = R->a0;
      x.hi = R->b0;
      for (auto& rec : R->records)
        if (rec.first > x.lo && rec.first < x.hi) {
          if (rec.second >= x.k) x.hi = rec.first;
          else x.lo = rec.first;
        }
      R->active.push_back(t);
    }
    complete(S, *R);
    std::vector<double> mus;
    for (int64_t t : R->active) {
      Query& x = S->q[t];
      x.split = x.lo + (x.hi - x.lo) * (0.5 + x.nudge / 64.0);
      mus.push_back(x.split);
    }
    if (mus.empty()) continue;
    std::sort(mus.begin(), mus.end());
    mus.erase(std::unique(mus.begin(), mus.end()), mus.end());
    std::vector<int64_t> nus(mus.size());
    std::vector<int32_t> sts(mus.size());
    lk.unlock();
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
      R->records.push_back({mus[j], nus[j]});
      narrow(S, *R, mus[j], nus[j]);
    }
    complete(S, *R);
  }
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

h2_status h2s_create(int32_t max_slots, h2_server* out) {
  if (!out) return fail(H2_EINVAL, "out is NULL");
  if (max_slots < 0) return fail(H2_EINVAL, "max_slots must be >= 0");
  *out = new h2_server_s();
  (*out)->max_slots = max_slots;
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
  int32_t cap = 1;
  r = h2_capacity(A, &cap);
  if (r != H2_OK) return r;
  h2_stats_t st;
  r = h2_stats(A, &st);
  if (r != H2_OK) return r;
  R->n = st.n;
  R->a0 = ab[0];
  R->b0 = ab[1];
  R->slots = slots > 0 ? slots : std::max(1, S->max_slots > 0 ? std::min(S->max_slots, cap) : cap);
  // reserve the workspace of `slots` shifts: the first step of every query,
  // a multisection of the starting interval
  r = h2_set_max_shifts(A, R->slots);
  if (r != H2_OK) return r;
  std::vector<double> mus(R->slots);
  std::vector<int64_t> nus(R->slots);
  std::vector<int32_t> sts(R->slots);
  for (int j = 0; j < R->slots; ++j) mus[j] = R->a0 + (R->b0 - R->a0) * (j + 1) / (R->slots + 1);
  r = h2_inertia(A, mus.data(), R->slots, nus.data(), sts.data());
  if (r != H2_OK && r != H2_ENUMERIC) return r;
  for (int j = 0; j < R->slots; ++j)
    if (sts[j] == H2_OK) R->records.push_back({mus[j], nus[j]});
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return fail(H2_EINVAL, "server is shutting down");
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
  if (it->second.state == 3) return fail(it->second.status, "the query's factorization failed");
  if (*done && lambda) *lambda = it->second.lambda;
  return H2_OK;
}

h2_status h2s_wait(h2_server S, int64_t ticket, double* lambda) {
  if (!S) return fail(H2_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->q.find(ticket);
  if (it == S->q.end()) return fail(H2_EINVAL, "unknown ticket");
  S->cv_done.wait(lk, [&] { return it->second.state >= 2 || S->stop; });
  if (it->second.state == 3) return fail(it->second.status, "the query's factorization failed");
  if (it->second.state != 2) return fail(H2_EINVAL, "server stopped");
  if (lambda) *lambda = it->second.lambda;
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
