// Host check of the library's cluster tree, block tree and colouring
// (h2::build_tree), its norm estimate (h2::estimate_norm) and its kernel
// entries (h2::kernel_block), all host code of paper_2311_08618_amd/csrc/host.cpp,
// linked against libh2eig.so and run by tests/test_host_tools.py without a GPU.
//
// Reads "n dim leaf eta kind diag p0 p1" and then n*dim coordinates
// (row-major) from stdin and prints the tree: "L <depth>", then per level l and
// cluster i the lines "idx l i ...", "near l i ...", "far l i ...", then
// "colour l ..." per level and "perm ..."; then "norm <normA>" and, for the
// first min(n, 24) points in original order, "kblock i <A(i, 0..)>".  The test
// compares every line with the oracle.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "../paper_2311_08618_amd/csrc/host.hpp"

static void put(const char* tag, int l, int i, const std::vector<int64_t>& v) {
  std::printf("%s %d %d", tag, l, i);
  for (int64_t x : v) std::printf(" %lld", (long long)x);
  std::printf("\n");
}

static void put(const char* tag, int l, int i, const std::vector<int>& v) {
  std::printf("%s %d %d", tag, l, i);
  for (int x : v) std::printf(" %d", x);
  std::printf("\n");
}

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
    if (std::scanf("%lf", &x) != 1) return 2;
  h2::Tree T;
  h2::build_tree(T, X.data(), n, dim, leaf, eta);
  std::printf("L %d\n", T.L);
  for (int l = 0; l <= T.L; ++l) {
    for (int i = 0; i < T.nclusters(l); ++i) {
      put("idx", l, i, T.idx[l][i]);
      put("near", l, i, T.near[l][i]);
      put("far", l, i, T.far[l][i]);
    }
    put("colour", l, -1, T.colour[l]);
  }
  put("perm", -1, -1, T.perm);
  std::printf("norm %.17g\n", h2::estimate_norm(T, k));
  const int m = (int)std::min<long long>(n, 24);
  std::vector<int64_t> ids(m);
  for (int i = 0; i < m; ++i) ids[i] = i;
  std::vector<double> blk((size_t)m * m);
  h2::kernel_block(T, k, ids.data(), m, ids.data(), m, blk.data(), m);
  for (int i = 0; i < m; ++i) {
    std::printf("kblock %d", i);
    for (int j = 0; j < m; ++j) std::printf(" %.17g", blk[i + (size_t)j * m]);
    std::printf("\n");
  }
  return 0;
}
