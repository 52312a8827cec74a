// Inertia records of one matrix: pairs (mu, nu(mu)) with nu(mu) = #{lambda < mu}
// from earlier factorizations, kept sorted by mu.  They seed and narrow the
// brackets of later k-th eigenvalue queries (inertia reuse, Sec. 4.2).
//
// A bracket for lambda_k ends at the largest recorded mu with nu < k and at the
// smallest recorded mu above that with nu >= k.  Of a run of records with equal
// counts (adjacent in mu order) only the first and the last can be such an end,
// so the records inside a run are dropped: at most two records per distinct
// count remain, however many shifts were factored.  This holds whether or not
// the counts grow with mu.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace h2 {

using Record = std::pair<double, int64_t>;   // (mu, nu(mu))

// insert (mu, nu) in mu order; a record at an equal mu is kept as it was
inline void record_insert(std::vector<Record>& v, double mu, int64_t nu) {
  auto it = std::lower_bound(v.begin(), v.end(), mu, [](const Record& r, double m) { return r.first < m; });
  if (it != v.end() && it->first == mu) return;
  v.insert(it, {mu, nu});
}

// drop every record whose neighbours on both sides have its count
inline void record_compact(std::vector<Record>& v) {
  if (v.size() < 3) return;
  size_t w = 1;
  int64_t prev = v[0].second;   // count of the record left of v[j] before compaction
  for (size_t j = 1; j + 1 < v.size(); ++j) {
    const int64_t c = v[j].second;
    const bool inside = prev == c && v[j + 1].second == c;
    prev = c;
    if (!inside) v[w++] = v[j];
  }
  v[w++] = v.back();
  v.resize(w);
}

// is there a record at exactly mu?
inline bool record_has(const std::vector<Record>& v, double mu) {
  auto it = std::lower_bound(v.begin(), v.end(), mu, [](const Record& r, double m) { return r.first < m; });
  return it != v.end() && it->first == mu;
}

// the bracket [lo, hi] of lambda_k inside (a0, b0) from the records alone: lo
// the largest recorded mu in (a0, b0) with nu < k (else a0), hi the smallest
// recorded mu in (lo, b0) with nu >= k (else b0)
inline void record_bracket(const std::vector<Record>& v, int64_t k, double a0, double b0, double* lo, double* hi) {
  double L = a0, H = b0;
  for (const Record& r : v)
    if (r.second < k && r.first > L && r.first < b0) L = r.first;
  for (const Record& r : v)
    if (r.second >= k && r.first > L && r.first < H) H = r.first;
  *lo = L;
  *hi = H;
}

}  // namespace h2
