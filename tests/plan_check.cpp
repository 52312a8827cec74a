// Host check of the library's static schedule (h2::build_plan in
// paper_2311_08618_amd/csrc/plan.cpp), linked against libh2eig.so and run by
// tests/test_host_tools.py without a GPU.
//
// Reads "n dim leaf eta" and then n*dim coordinates (row-major) from stdin,
// builds the cluster tree and the schedule (whose block structure does not
// depend on the ranks, so every construction rank is set to 1), and prints per
// level l: "near l i ..." (the near-pair CSR row of cluster i), "carried l i
// ..." (the partners j > i whose fill-in block is carried into level l), and
// "class l c ..." (the clusters of colour class c).
#include <cstdio>
#include <vector>

#include "../paper_2311_08618_amd/csrc/plan.hpp"

int main() {
  long long n = 0;
  int dim = 0, leaf = 0;
  double eta = 0.0;
  if (std::scanf("%lld %d %d %lf", &n, &dim, &leaf, &eta) != 4 || n < 1 || dim < 1 || dim > 3) return 2;
  std::vector<double> X((size_t)n * dim);
  for (auto& x : X)
    if (std::scanf("%lf", &x) != 1) return 2;
  h2::Tree T;
  h2::build_tree(T, X.data(), n, dim, leaf, eta);
  h2::Basis B;
  B.r.assign(T.L + 1, {});
  for (int l = 0; l <= T.L; ++l) B.r[l].assign(T.nclusters(l), 1);
  const std::vector<h2::LevelPlan> P = h2::build_plan(T, B);
  std::printf("L %d\n", T.L);
  for (int l = 0; l <= T.L; ++l) {
    const h2::LevelPlan& lp = P[l];
    for (int i = 0; i < lp.N; ++i) {
      std::printf("near %d %d", l, i);
      for (int p = lp.near_ptr[i]; p < lp.near_ptr[i + 1]; ++p) std::printf(" %d", lp.near_idx[p]);
      std::printf("\ncarried %d %d", l, i);
      for (int p = lp.f_ptr[i]; p < lp.f_ptr[i + 1]; ++p) std::printf(" %d", lp.f_idx[p]);
      std::printf("\n");
    }
    for (size_t c = 0; c < lp.colours.size(); ++c) {
      std::printf("class %d %d", l, (int)c);
      for (int i : lp.colours[c].clusters) std::printf(" %d", i);
      std::printf("\n");
    }
  }
  return 0;
}
