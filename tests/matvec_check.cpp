// Host check of the library's H^2 matrix-vector product (h2::h2_matvec_host in
// paper_2311_08618_amd/csrc/host.cpp, the diagnostic behind h2_matvec), linked
// against libh2eig.so and run by tests/test_host_tools.py without a GPU.
//
// Reads "n dim leaf eta kind diag p0 p1", the n*dim coordinates (row-major),
// then for every level l = 1..L and cluster i: "m r", the m x m matrix Q
// (column-major; the leaf basis at l = L, the transfer matrix above, skeleton
// columns last), the number of couplings and, for each, "j r_j" and the r_i x r_j
// coupling (column-major); then x (n values, original order).  Builds the
// library's cluster tree, fills the bases with what it read, and prints y = A~ x.
#include <cstdio>
#include <vector>

#include "../paper_2311_08618_amd/csrc/host.hpp"

static bool rd(double& v) { return std::scanf("%lf", &v) == 1; }
static bool rd(int& v) { return std::scanf("%d", &v) == 1; }

int main() {
  long long n = 0;
  int dim = 0, leaf = 0;
  double eta = 0.0;
  h2::KernelSpec k{};
  if (std::scanf("%lld %d %d %lf %d %lf %lf %lf", &n, &dim, &leaf, &eta, &k.kind, &k.diag, &k.p0, &k.p1) != 8 ||
      n < 1 || dim < 1 || dim > 3)
    return 2;
  std::vector<double> X((size_t)n * dim);
  for (auto& x : X)
    if (!rd(x)) return 2;
  h2::Tree T;
  h2::build_tree(T, X.data(), n, dim, leaf, eta);
  const int L = T.L;
  h2::Basis B;
  B.m.assign(L + 1, {});
  B.r.assign(L + 1, {});
  B.Q.assign(L + 1, {});
  B.C.assign(L + 1, {});
  for (int l = 0; l <= L; ++l) {
    const int N = T.nclusters(l);
    B.m[l].assign(N, 0);
    B.r[l].assign(N, 0);
    B.Q[l].assign(N, {});
    B.C[l].assign(N, {});
  }
  for (int l = 1; l <= L; ++l)
    for (int i = 0; i < T.nclusters(l); ++i) {
      int m = 0, r = 0, nc = 0;
      if (!rd(m) || !rd(r) || m < 0 || r < 0 || r > m) return 2;
      B.m[l][i] = m;
      B.r[l][i] = r;
      B.Q[l][i].resize((size_t)m * m);
      for (auto& v : B.Q[l][i])
        if (!rd(v)) return 2;
      if (!rd(nc) || nc < 0) return 2;
      for (int c = 0; c < nc; ++c) {
        int j = 0, rj = 0;
        if (!rd(j) || !rd(rj) || j < 0 || j >= T.nclusters(l)) return 2;
        std::vector<double> C((size_t)r * rj);
        for (auto& v : C)
          if (!rd(v)) return 2;
        B.C[l][i].push_back({j, std::move(C)});
      }
    }
  // the coupling's column count must be the partner's rank
  for (int l = 1; l <= L; ++l)
    for (int i = 0; i < T.nclusters(l); ++i)
      for (const auto& jc : B.C[l][i])
        if (jc.second.size() != (size_t)B.r[l][i] * B.r[l][jc.first]) return 2;
  std::vector<double> x((size_t)n), y((size_t)n);
  for (auto& v : x)
    if (!rd(v)) return 2;
  h2::h2_matvec_host(T, k, B, x.data(), y.data());
  for (double v : y) std::printf("%.17g\n", v);
  return 0;
}
