// Host-side structures of the H^2 matrix: cluster tree, block tree, colouring,
// nested orthonormal bases, transfer matrices and couplings.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <functional>
#include <string>
#include <thread>
#include <vector>

namespace h2 {

struct KernelSpec {
  int kind;
  double diag, p0, p1;
};

// Off-diagonal kernel value at distance r.
double kernel_f(const KernelSpec& k, double r);

struct Tree {
  int64_t n = 0;
  int dim = 0, L = 0, leaf = 0;
  double eta = 1.0;
  std::vector<double> X;                                  // n*dim row-major
  std::vector<std::vector<std::vector<int64_t>>> idx;     // [l][i] original indices (split order)
  std::vector<std::vector<double>> centre, radius;        // [l][i*3], [l][i]
  std::vector<std::vector<std::vector<int>>> near, far;   // [l][i] sorted
  std::vector<std::vector<int>> colour;                   // [l][i]
  std::vector<int> ncolour;                               // [l]
  std::vector<int64_t> perm;                              // leaf order -> original
  std::vector<std::vector<int64_t>> start;                // [l][i] offset of cluster in leaf order
  std::vector<std::vector<int64_t>> size;                 // [l][i]

  int nclusters(int l) const { return 1 << l; }
  bool admissible(int l, int i, int j) const;
  bool is_near(int l, int i, int j) const;
};

void build_tree(Tree& T, const double* pts, int64_t n, int dim, int leaf, double eta);

struct Basis {
  // per level, per cluster
  std::vector<std::vector<int>> m;                        // dimension at the start of the level (build)
  std::vector<std::vector<int>> r;                        // skeleton rank
  std::vector<std::vector<std::vector<int64_t>>> skel;    // skeleton points (original indices)
  std::vector<std::vector<std::vector<double>>> Tf;       // r x r triangular factor (col-major)
  std::vector<std::vector<std::vector<double>>> Q;        // leaf: m x m basis [U^R | U^S];
                                                          // parent: transfer matrix E, same order
  // couplings of admissible pairs at each level: map (i,j) -> r_i x r_j col-major
  std::vector<std::vector<std::vector<std::pair<int, std::vector<double>>>>> C;  // [l][i] list (j, C)
};

struct BuildParams {
  KernelSpec kern;
  double eps = 1e-8;
  int nthreads = 0;
};

// The nested bases (far-field IDs on the GPU, on stream st) and the couplings.
void build_basis(const Tree& T, const BuildParams& P, double tau, Basis& B, hipStream_t st);
double estimate_norm(const Tree& T, const KernelSpec& k);

// small dense helpers (column-major)
void kernel_block(const Tree& T, const KernelSpec& k, const int64_t* rows, int nr,
                  const int64_t* cols, int nc, double* out, int ldo);

int default_threads();

// y = A~ x with the built H^2 matrix, on the host (a diagnostic of the
// construction; x, y in original point order).
void h2_matvec_host(const Tree& T, const KernelSpec& kern, const Basis& B, const double* x, double* y);

// Dynamic parallel loop over [0, n) on nthreads std::threads.
inline void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t)>& fn) {
  if (nthreads <= 1 || n <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  int nt = (int)std::min<int64_t>(nthreads, n);
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= n) break;
        fn(i);
      }
    });
  for (auto& x : th) x.join();
}

}  // namespace h2
