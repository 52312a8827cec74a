// Host check of the inertia-record cache (paper_2311_08618_amd/csrc/records.hpp),
// built with g++ by tests/test_host_tools.py.  For random record sequences it
// checks that the compacted list is sorted with distinct shifts and holds only
// inserted records.  With counts that grow with the shift (exact inertia) it
// keeps at most two records per distinct count, drops only records inside a
// run of equal counts, and gives every k the same bracket as the full list
// (searched by brute force over the unsorted pairs); with counts that do not
// (rounding near an eigenvalue) every bracket still ends at records whose counts
// are < k and >= k.  Prints "ok" and exits 0, else names the failing case and
// exits 1.
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "../paper_2311_08618_amd/csrc/records.hpp"

using h2::Record;

static void brute_bracket(const std::vector<Record>& all, int64_t k, double a0, double b0, double* lo, double* hi) {
  double L = a0, H = b0;
  for (const Record& r : all)
    if (r.second < k && r.first > L && r.first < b0) L = r.first;
  for (const Record& r : all)
    if (r.second >= k && r.first > L && r.first < H) H = r.first;
  *lo = L;
  *hi = H;
}

// each end of [lo, hi] is its end of (a0, b0) or a record with a count < k
// (lo) or >= k (hi), and lo < hi
static bool valid_ends(const std::vector<Record>& all, int64_t k, double a0, double b0, double lo, double hi) {
  bool okl = lo == a0, okh = hi == b0;
  for (const Record& r : all) {
    if (r.first == lo && r.second < k) okl = true;
    if (r.first == hi && r.second >= k) okh = true;
  }
  return okl && okh && lo < hi;
}

int main() {
  std::mt19937_64 g(12345);
  for (int trial = 0; trial < 4000; ++trial) {
    const bool monotone = trial % 2 == 0;
    const int n = 1 + (int)(g() % 40);             // eigenvalues of the imagined matrix
    const int steps = 1 + (int)(g() % 12);         // factorization batches
    std::vector<Record> v, all;
    std::set<double> seen;
    std::uniform_real_distribution<double> U(0.0, 1.0);
    // shifts on a coarse grid, so that equal shifts recur; one shift always
    // gives the same count
    int64_t count_at[64];
    for (int i = 0; i < 64; ++i)
      count_at[i] = monotone ? (int64_t)(i * n / 64) : (int64_t)(g() % (uint64_t)(n + 1));
    for (int s = 0; s < steps; ++s) {
      const int batch = 1 + (int)(g() % 6);
      for (int b = 0; b < batch; ++b) {
        const int i = (int)(g() % 64);
        const double mu = (double)i / 64.0;
        const int64_t nu = count_at[i];
        if (!seen.count(mu)) {
          seen.insert(mu);
          all.push_back({mu, nu});
        }
        h2::record_insert(v, mu, nu);
      }
      h2::record_compact(v);
      // sorted, distinct shifts; every kept record is one of the inserted ones
      for (size_t i = 1; i < v.size(); ++i)
        if (!(v[i - 1].first < v[i].first)) {
          std::printf("trial %d: not sorted at %zu\n", trial, i);
          return 1;
        }
      for (const Record& r : v) {
        bool found = false;
        for (const Record& q : all) found = found || (q == r);
        if (!found) {
          std::printf("trial %d: record (%g, %lld) was never inserted\n", trial, r.first, (long long)r.second);
          return 1;
        }
      }
      // no record inside a run of equal counts; at most two per count
      for (size_t i = 1; i + 1 < v.size(); ++i)
        if (v[i - 1].second == v[i].second && v[i + 1].second == v[i].second) {
          std::printf("trial %d: record %zu inside a run\n", trial, i);
          return 1;
        }
      if (monotone) {
        std::set<int64_t> counts;
        for (const Record& r : v) counts.insert(r.second);
        if (v.size() > 2 * counts.size()) {
          std::printf("trial %d: %zu records for %zu counts\n", trial, v.size(), counts.size());
          return 1;
        }
      }
      // the same bracket for every k, from inside and around the interval
      const double a0 = -0.25 + 0.25 * U(g), b0 = 1.0 + 0.25 * U(g);
      for (int64_t k = 0; k <= n + 1; ++k) {
        double l1, h1, l2, h2v;
        brute_bracket(all, k, a0, b0, &l1, &h1);
        h2::record_bracket(v, k, a0, b0, &l2, &h2v);
        if (monotone ? (l1 != l2 || h1 != h2v) : !valid_ends(all, k, a0, b0, l2, h2v)) {
          std::printf("trial %d k %lld: full [%g, %g] compacted [%g, %g]\n", trial, (long long)k, l1, h1, l2, h2v);
          return 1;
        }
      }
      if (!monotone) continue;
      for (const Record& q : all)
        if (!h2::record_has(v, q.first)) {
          // a dropped record lies inside a run: both neighbours in the list share its count
          size_t i = 0;
          while (i < v.size() && v[i].first < q.first) ++i;
          if (i == 0 || i == v.size() || v[i - 1].second != q.second || v[i].second != q.second) {
            std::printf("trial %d: record (%g, %lld) dropped outside a run\n", trial, q.first, (long long)q.second);
            return 1;
          }
        }
    }
  }
  std::printf("ok\n");
  return 0;
}
