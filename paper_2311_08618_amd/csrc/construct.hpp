// Far-field interpolative decompositions of one level of the cluster tree, on
// the GPU (Sec. 3.1, Eqs. shared-bases and transfer-matrices).
//
// For every cluster i of the level, M_i = A(rows_i, F_i) is the block of the
// kernel matrix between the cluster's rows (its points at the leaf level, its
// children's skeleton points above) and every point of its far field F_i (the
// interaction lists of i and of all its ancestors).  The rank-revealing step
// of the shared basis is a column-pivoted QR of M_i^T.  It is computed here as
// the pivoted Cholesky factorization of the Gram matrix G_i = M_i M_i^T: the
// diagonal of each Schur complement of G_i is the squared norm of the
// corresponding remaining column of M_i^T, so the pivot sequence, the R factor
// (R = L^T) and the remaining Frobenius norm are those of the QR.  Both the
// Gram matrix and the Cholesky steps run in double-double arithmetic (about
// 32 significant digits), so squaring the singular values loses nothing that
// an FP64 QR of M_i^T would keep: the stopping test
//     sum of the remaining diagonal  <=  tau^2
// resolves remaining norms down to about 1e-16 * ||M_i||.  The budget tau_i of
// cluster i is tau * sqrt(|cluster i| / n): the block rows of one level
// partition the rows of A, so their residuals then add up to at most tau in
// the 2-norm at every n.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace h2 {

struct FarIdLevel {
  int N = 0;                          // clusters of the level
  std::vector<int> m;                 // rows of each cluster
  std::vector<double> tau2;           // squared truncation budget of each cluster
  std::vector<double> rx, ry, rz;     // row point coordinates, clusters concatenated
  std::vector<int64_t> fptr;          // N+1 offsets into the far ranges
  std::vector<int64_t> fr0, fr1;      // far ranges [fr0, fr1) of point positions in tree order
};

struct FarIdResult {
  std::vector<int> r;                       // rank of each cluster
  std::vector<std::vector<int>> piv;        // pivot rows (positions in rows_i), r of them
  std::vector<std::vector<double>> Lf;      // m x r column-major: L(j, a) = R(a, j) rounded to FP64
};

// Points of the whole matrix in tree order, resident on the device for the
// duration of a build.
struct FarIdPoints {
  double *px = nullptr, *py = nullptr, *pz = nullptr;
  int64_t n = 0;
};

// Throws std::runtime_error on a HIP failure and std::invalid_argument on a
// non-finite kernel value.
void far_points_upload(FarIdPoints& P, const double* X, const int64_t* perm, int64_t n, int dim, hipStream_t st);
void far_points_free(FarIdPoints& P);
void far_field_ids(const FarIdPoints& P, int kind, double p0, double p1, const FarIdLevel& lev, FarIdResult& out,
                   hipStream_t st);

// y = A x for the exact kernel matrix of the n points X (row-major n x dim,
// A_ii = diag), on the GPU; x and y are host arrays.  O(n^2) work: a check of
// the construction error at sizes where no dense matrix fits.
void kernel_matvec_gpu(const double* X, int64_t n, int dim, int kind, double diag, double p0, double p1,
                       const double* x, double* y, hipStream_t st);

// Exact-kernel matvec on device arrays (X row-major n x dim, x and y of n).
void launch_kernel_matvec(const double* dX, int64_t n, int dim, int kind, double diag, double p0, double p1,
                          const double* dx, double* dy, hipStream_t st);

// The same product with the points, x and y staged through a static device
// scratch array instead of allocated memory (no hipMalloc or hipFree); n is at
// most kernel_matvec_noalloc_max_n(dim).  Calls that overlap on one GPU race.
int64_t kernel_matvec_noalloc_max_n(int dim);
void kernel_matvec_noalloc(const double* X, int64_t n, int dim, int kind, double diag, double p0, double p1,
                           const double* x, double* y, int device, hipStream_t st);

}  // namespace h2
