// Host construction of the H^2 matrix (Sec. 3.1 of the paper): cluster tree,
// strong-admissibility block tree, colouring of the near graph, nested
// orthonormal shared bases and transfer matrices by an interpolative
// decomposition of each cluster's whole far field (the rank-revealing step
// runs on the GPU, construct.hip), and couplings.
//
// Readings (the paper leaves these open):
//  * split every cluster at the median of its longest bounding-box axis
//    (lowest axis on ties, stable order), down to the depth L at which every
//    cluster holds at most `leaf` points; children of p are 2p and 2p+1;
//  * admissible iff i != j, |c_i - c_j| > 0 and eta*|c_i - c_j| >= rho_i + rho_j
//    (bounding-box centres and half diagonals);
//  * greedy colouring of each level's near graph in ascending index;
//  * far field of cluster i at level l = every point of every cluster in the
//    interaction list of i or of one of its ancestors;
//  * rank-revealing step: column-pivoted QR of the far-field block's
//    transpose, pivots by largest remaining norm, stop when the Frobenius norm
//    of the remaining block is <= tau_i = tau * sqrt(|cluster i| / n),
//    tau = eps*normA (so the interpolation error of the block row is at most
//    tau_i, the criterion of Sec. 3.1, and the block rows of one level err by
//    at most tau together);
//  * orthonormal completion ordered [redundant | skeleton]; couplings
//    C_ij = T_i A(s_i, s_j) T_j^T.
#include "host.hpp"

#include "construct.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <numeric>

namespace h2 {

int default_threads() {
  unsigned hc = std::thread::hardware_concurrency();
  int n = hc ? (int)hc : 4;
  return std::min(n, 16);
}

double kernel_f(const KernelSpec& k, double r) {
  switch (k.kind) {
    case 0: return 1.0 / r;
    case 1: return std::exp(-r) / r;
    case 2: return std::exp(-r * r / k.p0) / (r + k.p1);
    case 3: return 1.0 / (r + k.p0);
    case 4: return (std::fabs(r - k.p0) < 1e-9 * k.p0) ? -1.0 : 0.0;
    default: return 0.0;
  }
}

static inline double dist(const Tree& T, int64_t a, int64_t b) {
  double s = 0.0;
  for (int d = 0; d < T.dim; ++d) {
    double x = T.X[a * T.dim + d] - T.X[b * T.dim + d];
    s += x * x;
  }
  return std::sqrt(s);
}

void kernel_block(const Tree& T, const KernelSpec& k, const int64_t* rows, int nr,
                  const int64_t* cols, int nc, double* out, int ldo) {
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i < nr; ++i)
      out[i + (int64_t)j * ldo] = rows[i] == cols[j] ? k.diag : kernel_f(k, dist(T, rows[i], cols[j]));
}

bool Tree::admissible(int l, int i, int j) const {
  if (i == j) return false;
  double s = 0.0;
  for (int d = 0; d < dim; ++d) {
    double x = centre[l][i * dim + d] - centre[l][j * dim + d];
    s += x * x;
  }
  double dd = std::sqrt(s);
  return dd > 0.0 && eta * dd >= radius[l][i] + radius[l][j];
}

bool Tree::is_near(int l, int i, int j) const {
  const auto& v = near[l][i];
  return std::binary_search(v.begin(), v.end(), j);
}

void build_tree(Tree& T, const double* pts, int64_t n, int dim, int leaf, double eta) {
  T.n = n;
  T.dim = dim;
  T.leaf = leaf;
  T.eta = eta;
  T.X.assign(pts, pts + n * dim);
  int L = 0;
  while (((n + (1LL << L) - 1) >> L) > leaf) ++L;
  T.L = L;
  T.idx.assign(L + 1, {});
  T.idx[0].push_back(std::vector<int64_t>(n));
  std::iota(T.idx[0][0].begin(), T.idx[0][0].end(), 0);
  for (int l = 1; l <= L; ++l) {
    auto& prev = T.idx[l - 1];
    auto& cur = T.idx[l];
    cur.resize(prev.size() * 2);
    for (size_t p = 0; p < prev.size(); ++p) {
      std::vector<int64_t> a = prev[p];
      int ax = 0;
      double best = -1.0;
      for (int d = 0; d < dim; ++d) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t v : a) {
          lo = std::min(lo, T.X[v * dim + d]);
          hi = std::max(hi, T.X[v * dim + d]);
        }
        double e = a.empty() ? 0.0 : hi - lo;
        if (e > best) { best = e; ax = d; }
      }
      std::stable_sort(a.begin(), a.end(), [&](int64_t u, int64_t v) {
        return T.X[u * dim + ax] < T.X[v * dim + ax];
      });
      size_t half = a.size() / 2;
      cur[2 * p].assign(a.begin(), a.begin() + half);
      cur[2 * p + 1].assign(a.begin() + half, a.end());
    }
  }
  T.centre.assign(L + 1, {});
  T.radius.assign(L + 1, {});
  for (int l = 0; l <= L; ++l) {
    int N = 1 << l;
    T.centre[l].assign((size_t)N * dim, 0.0);
    T.radius[l].assign(N, 0.0);
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int d = 0; d < dim; ++d) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t v : T.idx[l][i]) {
          lo = std::min(lo, T.X[v * dim + d]);
          hi = std::max(hi, T.X[v * dim + d]);
        }
        if (T.idx[l][i].empty()) lo = hi = 0.0;
        T.centre[l][i * dim + d] = 0.5 * (lo + hi);
        s += (hi - lo) * (hi - lo);
      }
      T.radius[l][i] = 0.5 * std::sqrt(s);
    }
  }
  T.near.assign(L + 1, {});
  T.far.assign(L + 1, {});
  T.near[0] = {{0}};
  T.far[0] = {{}};
  for (int l = 1; l <= L; ++l) {
    int N = 1 << l;
    T.near[l].assign(N, {});
    T.far[l].assign(N, {});
    for (int p = 0; p < (N >> 1); ++p)
      for (int q : T.near[l - 1][p])
        for (int c = 2 * p; c <= 2 * p + 1; ++c)
          for (int d = 2 * q; d <= 2 * q + 1; ++d) {
            if (T.admissible(l, c, d)) T.far[l][c].push_back(d);
            else T.near[l][c].push_back(d);
          }
    for (int i = 0; i < N; ++i) {
      std::sort(T.near[l][i].begin(), T.near[l][i].end());
      std::sort(T.far[l][i].begin(), T.far[l][i].end());
    }
  }
  T.colour.assign(L + 1, {});
  T.ncolour.assign(L + 1, 0);
  for (int l = 0; l <= L; ++l) {
    int N = 1 << l;
    T.colour[l].assign(N, -1);
    int nc = 0;
    for (int i = 0; i < N; ++i) {
      std::vector<char> used(T.near[l][i].size() + 2, 0);
      for (int j : T.near[l][i])
        if (j < i && T.colour[l][j] < (int)used.size()) used[T.colour[l][j]] = 1;
      int c = 0;
      while (used[c]) ++c;
      T.colour[l][i] = c;
      nc = std::max(nc, c + 1);
    }
    T.ncolour[l] = nc;
  }
  T.perm.clear();
  for (auto& v : T.idx[L]) T.perm.insert(T.perm.end(), v.begin(), v.end());
  T.start.assign(L + 1, {});
  T.size.assign(L + 1, {});
  T.start[L].assign(1 << L, 0);
  T.size[L].assign(1 << L, 0);
  int64_t off = 0;
  for (int i = 0; i < (1 << L); ++i) {
    T.start[L][i] = off;
    T.size[L][i] = (int64_t)T.idx[L][i].size();
    off += T.size[L][i];
  }
  for (int l = L - 1; l >= 0; --l) {
    int N = 1 << l;
    T.start[l].assign(N, 0);
    T.size[l].assign(N, 0);
    for (int i = 0; i < N; ++i) {
      T.start[l][i] = T.start[l + 1][2 * i];
      T.size[l][i] = T.size[l + 1][2 * i] + T.size[l + 1][2 * i + 1];
    }
  }
}

// ---------------------------------------------------------------- dense helpers
// Householder QR of Y (m x r, col-major), completed to a square orthonormal Q
// (m x m) ordered [redundant | skeleton]; T = upper r x r factor with
// Y = Q[:, m-r:] T.
static void complete_basis(const double* Y, int m, int r, std::vector<double>& Q, std::vector<double>& T) {
  Q.assign((size_t)m * m, 0.0);
  T.assign((size_t)r * r, 0.0);
  if (r == 0) {
    for (int i = 0; i < m; ++i) Q[i + (size_t)i * m] = 1.0;
    return;
  }
  std::vector<double> A(Y, Y + (size_t)m * r);
  std::vector<double> V((size_t)m * r, 0.0), beta(r, 0.0);
  for (int k = 0; k < r; ++k) {
    double* x = A.data() + (size_t)k * m;
    double xn = 0.0;
    for (int i = k; i < m; ++i) xn += x[i] * x[i];
    xn = std::sqrt(xn);
    double alpha = -std::copysign(xn, x[k] != 0.0 ? x[k] : 1.0);
    double* v = V.data() + (size_t)k * m;
    for (int i = k; i < m; ++i) v[i] = x[i];
    v[k] -= alpha;
    double vn = 0.0;
    for (int i = k; i < m; ++i) vn += v[i] * v[i];
    beta[k] = vn > 0.0 ? 2.0 / vn : 0.0;
    for (int j = k; j < r; ++j) {
      double* c = A.data() + (size_t)j * m;
      double s = 0.0;
      for (int i = k; i < m; ++i) s += v[i] * c[i];
      s *= beta[k];
      for (int i = k; i < m; ++i) c[i] -= v[i] * s;
    }
  }
  for (int j = 0; j < r; ++j)
    for (int i = 0; i <= j; ++i) T[i + (size_t)j * r] = A[i + (size_t)j * m];
  // Qfull = H_0 H_1 ... H_{r-1} applied to the identity; column c of Qfull
  std::vector<double> q(m);
  for (int c = 0; c < m; ++c) {
    std::fill(q.begin(), q.end(), 0.0);
    q[c] = 1.0;
    for (int k = r - 1; k >= 0; --k) {
      const double* v = V.data() + (size_t)k * m;
      double s = 0.0;
      for (int i = k; i < m; ++i) s += v[i] * q[i];
      s *= beta[k];
      for (int i = k; i < m; ++i) q[i] -= v[i] * s;
    }
    // Qfull column c goes to position: c < r -> m - r + c (skeleton), else c - r
    int dst = c < r ? m - r + c : c - r;
    std::copy(q.begin(), q.end(), Q.begin() + (size_t)dst * m);
  }
}

static std::vector<int64_t> cluster_points(const Tree& T, int l, int i) {
  std::vector<int64_t> v(T.perm.begin() + T.start[l][i], T.perm.begin() + T.start[l][i] + T.size[l][i]);
  return v;
}

// Far field of cluster i at level l as ranges of point positions in tree order:
// the clusters of the interaction lists of i and of its ancestors, sorted, with
// touching ranges merged.
static std::vector<std::pair<int64_t, int64_t>> far_ranges(const Tree& T, int l, int i) {
  std::vector<std::pair<int64_t, int64_t>> r;
  int a = i;
  for (int lv = l; lv >= 1; --lv) {
    for (int q : T.far[lv][a]) r.push_back({T.start[lv][q], T.start[lv][q] + T.size[lv][q]});
    a >>= 1;
  }
  std::sort(r.begin(), r.end());
  std::vector<std::pair<int64_t, int64_t>> out;
  for (auto& x : r) {
    if (!out.empty() && x.first <= out.back().second) out.back().second = std::max(out.back().second, x.second);
    else out.push_back(x);
  }
  return out;
}

double estimate_norm(const Tree& T, const KernelSpec& k) {
  int64_t n = T.n;
  int64_t s = std::max<int64_t>(1, n / 16384);
  int64_t nrows = (n + s - 1) / s;
  std::vector<double> rs(nrows, 0.0);
  parallel_for(nrows, default_threads(), [&](int64_t t) {
    int64_t i = t * s;
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j) acc += (i == j) ? k.diag : kernel_f(k, dist(T, i, j));
    rs[t] = acc;
  });
  double tot = 0.0;
  for (double v : rs) tot += v;
  return std::max(tot / (double)nrows, std::fabs(k.diag));
}

void build_basis(const Tree& T, const BuildParams& P, double tau, Basis& B, hipStream_t st) {
  int L = T.L;
  int nth = P.nthreads > 0 ? P.nthreads : default_threads();
  B.m.assign(L + 1, {});
  B.r.assign(L + 1, {});
  B.skel.assign(L + 1, {});
  B.Tf.assign(L + 1, {});
  B.Q.assign(L + 1, {});
  B.C.assign(L + 1, {});
  FarIdPoints FP;
  far_points_upload(FP, T.X.data(), T.perm.data(), T.n, T.dim, st);
  struct Guard {
    FarIdPoints& p;
    ~Guard() { far_points_free(p); }
  } guard{FP};
  for (int l = L; l >= 0; --l) {
    int N = 1 << l;
    B.m[l].assign(N, 0);
    B.r[l].assign(N, 0);
    B.skel[l].assign(N, {});
    B.Tf[l].assign(N, {});
    B.Q[l].assign(N, {});
    // rows of every cluster: its points at the leaf level, its children's
    // skeleton points above
    std::vector<std::vector<int64_t>> rows_of(N);
    FarIdLevel lev;
    lev.N = N;
    lev.m.assign(N, 0);
    lev.tau2.assign(N, 0.0);
    lev.fptr.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) {
      auto& rows = rows_of[i];
      if (l == L) rows = T.idx[L][i];
      else {
        rows = B.skel[l + 1][2 * i];
        rows.insert(rows.end(), B.skel[l + 1][2 * i + 1].begin(), B.skel[l + 1][2 * i + 1].end());
      }
      lev.m[i] = (int)rows.size();
      lev.tau2[i] = tau * tau * (double)T.size[l][i] / (double)T.n;
      for (int64_t v : rows) {
        lev.rx.push_back(T.X[v * T.dim]);
        lev.ry.push_back(T.dim > 1 ? T.X[v * T.dim + 1] : 0.0);
        lev.rz.push_back(T.dim > 2 ? T.X[v * T.dim + 2] : 0.0);
      }
      for (auto& fr : far_ranges(T, l, i)) {
        lev.fr0.push_back(fr.first);
        lev.fr1.push_back(fr.second);
      }
      lev.fptr[i + 1] = (int64_t)lev.fr0.size();
    }
    FarIdResult ids;
    far_field_ids(FP, P.kern.kind, P.kern.p0, P.kern.p1, lev, ids, st);
    if (const char* pe = std::getenv("H2EIG_PROGRESS"); pe && pe[0] == '1')
      std::fprintf(stderr, "[h2eig] build: far-field interpolative decompositions of level %d done\n", l);
    parallel_for(N, nth, [&](int64_t ii) {
      int i = (int)ii;
      const std::vector<int64_t>& rows = rows_of[i];
      int m = (int)rows.size();
      int r = ids.r[i];
      const std::vector<int>& piv = ids.piv[i];
      const std::vector<double>& Lf = ids.Lf[i];   // m x r: L(j, a) = R(a, j)
      std::vector<double> X((size_t)m * r, 0.0);   // m x r interpolation matrix, X[piv] = I
      if (r > 0) {
        // R11(a, b) = L(piv[b], a) (upper triangular); for a row j not chosen,
        // X(j, :) solves R11 z = R(:, j)
        std::vector<char> chosen(m, 0);
        for (int b = 0; b < r; ++b) {
          chosen[piv[b]] = 1;
          X[piv[b] + (size_t)b * m] = 1.0;
        }
        std::vector<double> z(r);
        for (int j = 0; j < m; ++j) {
          if (chosen[j]) continue;
          for (int a = r - 1; a >= 0; --a) {
            double s = Lf[j + (size_t)a * m];
            for (int b = a + 1; b < r; ++b) s -= Lf[piv[b] + (size_t)a * m] * z[b];
            z[a] = s / Lf[piv[a] + (size_t)a * m];
          }
          for (int a = 0; a < r; ++a) X[j + (size_t)a * m] = z[a];
        }
      }
      std::vector<double> Y;
      if (l < L && r > 0) {
        int r1 = B.r[l + 1][2 * i], r2 = B.r[l + 1][2 * i + 1];
        const auto& T1 = B.Tf[l + 1][2 * i];
        const auto& T2 = B.Tf[l + 1][2 * i + 1];
        Y.assign((size_t)m * r, 0.0);
        for (int c = 0; c < r; ++c) {
          for (int a = 0; a < r1; ++a) {
            double s = 0.0;
            for (int b = 0; b < r1; ++b) s += T1[a + (size_t)b * r1] * X[b + (size_t)c * m];
            Y[a + (size_t)c * m] = s;
          }
          for (int a = 0; a < r2; ++a) {
            double s = 0.0;
            for (int b = 0; b < r2; ++b) s += T2[a + (size_t)b * r2] * X[r1 + b + (size_t)c * m];
            Y[r1 + a + (size_t)c * m] = s;
          }
        }
      } else {
        Y = X;
      }
      std::vector<double> Q, Tm;
      complete_basis(Y.data(), m, r, Q, Tm);
      B.m[l][i] = m;
      B.r[l][i] = r;
      std::vector<int64_t> sk(r);
      for (int a = 0; a < r; ++a) sk[a] = rows[piv[a]];
      B.skel[l][i] = sk;
      B.Tf[l][i] = Tm;
      B.Q[l][i] = Q;
    });
  }
  // couplings
  for (int l = 1; l <= L; ++l) {
    int N = 1 << l;
    B.C[l].assign(N, {});
    parallel_for(N, nth, [&](int64_t ii) {
      int i = (int)ii;
      int ri = B.r[l][i];
      for (int j : T.far[l][i]) {
        int rj = B.r[l][j];
        std::vector<double> A((size_t)ri * rj), W((size_t)ri * rj), C((size_t)ri * rj, 0.0);
        if (ri && rj) {
          kernel_block(T, P.kern, B.skel[l][i].data(), ri, B.skel[l][j].data(), rj, A.data(), ri);
          const auto& Ti = B.Tf[l][i];
          const auto& Tj = B.Tf[l][j];
          // W = Ti * A
          for (int c = 0; c < rj; ++c)
            for (int a = 0; a < ri; ++a) {
              double s = 0.0;
              for (int b = a; b < ri; ++b) s += Ti[a + (size_t)b * ri] * A[b + (size_t)c * ri];
              W[a + (size_t)c * ri] = s;
            }
          // C = W * Tj^T
          for (int c = 0; c < rj; ++c)
            for (int a = 0; a < ri; ++a) {
              double s = 0.0;
              for (int b = c; b < rj; ++b) s += W[a + (size_t)b * ri] * Tj[c + (size_t)b * rj];
              C[a + (size_t)c * ri] = s;
            }
        }
        B.C[l][i].push_back({j, std::move(C)});
      }
    });
  }
}

}  // namespace h2

namespace h2 {

// y = A~ x for the built H^2 matrix (original point order).  Near blocks of the
// leaf level are kernel blocks, evaluated on the fly; every admissible pair
// (i, j) of level l contributes U_i C_ij U_j^T x(tau_j), with the nested bases
// applied by an upward pass (x^_i = U_i^T x) and a downward pass (Sec. 3.1,
// Eq. notation-example).
void h2_matvec_host(const Tree& T, const KernelSpec& kern, const Basis& B, const double* x, double* y) {
  const int L = T.L;
  const int nth = default_threads();
  const int64_t n = T.n;
  std::vector<double> xp(n), yp(n, 0.0);   // leaf order
  for (int64_t p = 0; p < n; ++p) xp[p] = x[T.perm[p]];
  // upward pass: xs[l][i] = skeleton coordinates of x on cluster i
  std::vector<std::vector<std::vector<double>>> xs(L + 1), ys(L + 1);
  for (int l = L; l >= 1; --l) {
    const int N = 1 << l;
    xs[l].assign(N, {});
    ys[l].assign(N, {});
    parallel_for(N, nth, [&](int64_t ii) {
      const int i = (int)ii;
      const int m = B.m[l][i], r = B.r[l][i];
      const std::vector<double>& Q = B.Q[l][i];
      std::vector<double> in(m);
      if (l == L) {
        for (int a = 0; a < m; ++a) in[a] = xp[T.start[L][i] + a];
      } else {
        const auto& a1 = xs[l + 1][2 * i];
        const auto& a2 = xs[l + 1][2 * i + 1];
        std::copy(a1.begin(), a1.end(), in.begin());
        std::copy(a2.begin(), a2.end(), in.begin() + a1.size());
      }
      std::vector<double> out(r, 0.0);
      for (int c = 0; c < r; ++c) {
        const double* q = Q.data() + (size_t)(m - r + c) * m;
        double s = 0.0;
        for (int a = 0; a < m; ++a) s += q[a] * in[a];
        out[c] = s;
      }
      xs[l][i] = std::move(out);
      ys[l][i].assign(r, 0.0);
    });
  }
  // couplings
  for (int l = 1; l <= L; ++l) {
    const int N = 1 << l;
    parallel_for(N, nth, [&](int64_t ii) {
      const int i = (int)ii;
      const int ri = B.r[l][i];
      for (const auto& jc : B.C[l][i]) {
        const int j = jc.first, rj = B.r[l][j];
        const std::vector<double>& C = jc.second;
        for (int b = 0; b < rj; ++b) {
          const double v = xs[l][j][b];
          for (int a = 0; a < ri; ++a) ys[l][i][a] += C[a + (size_t)b * ri] * v;
        }
      }
    });
  }
  // downward pass
  for (int l = 1; l <= L; ++l) {
    const int N = 1 << l;
    parallel_for(N, nth, [&](int64_t ii) {
      const int i = (int)ii;
      const int m = B.m[l][i], r = B.r[l][i];
      const std::vector<double>& Q = B.Q[l][i];
      std::vector<double> out(m, 0.0);
      for (int c = 0; c < r; ++c) {
        const double* q = Q.data() + (size_t)(m - r + c) * m;
        const double v = ys[l][i][c];
        for (int a = 0; a < m; ++a) out[a] += q[a] * v;
      }
      if (l == L) {
        for (int a = 0; a < m; ++a) yp[T.start[L][i] + a] += out[a];
      } else {
        auto& c1 = ys[l + 1][2 * i];
        auto& c2 = ys[l + 1][2 * i + 1];
        for (size_t a = 0; a < c1.size(); ++a) c1[a] += out[a];
        for (size_t a = 0; a < c2.size(); ++a) c2[a] += out[c1.size() + a];
      }
    });
  }
  // near field (leaf level, exact kernel blocks)
  const int N = 1 << L;
  parallel_for(N, nth, [&](int64_t ii) {
    const int i = (int)ii;
    const int64_t si = T.start[L][i], mi = T.size[L][i];
    for (int j : T.near[L][i]) {
      const int64_t sj = T.start[L][j], mj = T.size[L][j];
      for (int64_t a = 0; a < mi; ++a) {
        const int64_t pa = T.perm[si + a];
        double s = 0.0;
        for (int64_t b = 0; b < mj; ++b) {
          const int64_t pb = T.perm[sj + b];
          s += (pa == pb ? kern.diag : kernel_f(kern, dist(T, pa, pb))) * xp[sj + b];
        }
        yp[si + a] += s;
      }
    }
  });
  for (int64_t p = 0; p < n; ++p) y[T.perm[p]] = yp[p];
}

}  // namespace h2
