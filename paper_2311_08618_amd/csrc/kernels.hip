// HIP kernels (gfx950 / CDNA4) of the generalized H^2-LDL inertia path.
//
// Every kernel works on a batch of shifts (blockIdx.z = shift) and on a list
// of static descriptors (blockIdx.y = item); block sizes are resolved per
// shift on the device from the size tables, because the redundant/skeleton
// split of each cluster depends on the shift.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>

#include "desc.hpp"
#include "kernels.hpp"

namespace h2 {

__device__ inline double* addr(const BufTab& bt, int buf, int blk, int s, int row, int col) {
  return bt.p[buf] + (int64_t)s * bt.ss[buf] + (int64_t)blk * bt.bs[buf] + row + (int64_t)col * bt.ld[buf];
}

__device__ inline void ref_origin(const Ref& r, const SizeTab& z, int s, int* row, int* col) {
  *row = dev_eval(r.r0, z, s) + dev_eval(r.r1, z, s);
  *col = dev_eval(r.c0, z, s) + dev_eval(r.c1, z, s);
}

// ------------------------------------------------------------------ fill
__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_int(int* p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------- GEMM (FP64 MFMA)
// C[M x N] = beta*C + alpha * sum_t op(A_t) diag(w_t) op(B_t), 64x64 tiles,
// 256 threads = 4 waves in 2x2, each wave 32x32 = 2x2 MFMA 16x16x4 f64 tiles.
// op(A): TA ? A^T (A stored K x M) : A (M x K);  op(B): TB ? B^T (B stored N x K) : B (K x N).
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // output tile
constexpr int GK = 16;   // k step

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(const GItem* __restrict__ items, const GTerm* __restrict__ terms,
                                              BufTab bt, SizeTab sz, int tiles_n) {
  const int s = blockIdx.z;
  const GItem it = items[blockIdx.y];
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  const int m0 = (blockIdx.x / tiles_n) * GT, n0 = (blockIdx.x % tiles_n) * GT;
  if (m0 >= M || n0 >= N) return;
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  v4d acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int tt = 0; tt < it.nt; ++tt) {
    const GTerm tm = terms[it.t0 + tt];
    const int K = dev_eval(tm.K, sz, s);
    if (K <= 0) continue;
    int ar, ac, br, bc;
    ref_origin(tm.a, sz, s, &ar, &ac);
    ref_origin(tm.b, sz, s, &br, &bc);
    const double* A = addr(bt, tm.a.buf, tm.a.blk, s, ar, ac);
    const double* B = addr(bt, tm.b.buf, tm.b.blk, s, br, bc);
    const int lda = bt.ld[tm.a.buf], ldb = bt.ld[tm.b.buf];
    const double* w = tm.wbuf >= 0 ? addr(bt, tm.wbuf, 0, s, 0, 0) + (int64_t)tm.wblk * bt.bs[tm.wbuf] : nullptr;
    for (int k0 = 0; k0 < K; k0 += GK) {
      // A tile: GT (m) x GK (k)
      for (int e = tid; e < GT * GK; e += 256) {
        int mm, kk;
        if (TA) { kk = e % GK; mm = e / GK; } else { mm = e % GT; kk = e / GT; }
        int gm = m0 + mm, gk = k0 + kk;
        double v = 0.0;
        if (gm < M && gk < K) {
          v = TA ? A[gk + (int64_t)gm * lda] : A[gm + (int64_t)gk * lda];
          if (w) v *= w[gk];
        }
        As[kk][mm] = v;
      }
      // B tile: GK (k) x GT (n)
      for (int e = tid; e < GT * GK; e += 256) {
        int nn, kk;
        if (TB) { nn = e % GT; kk = e / GT; } else { kk = e % GK; nn = e / GK; }
        int gn = n0 + nn, gk = k0 + kk;
        double v = 0.0;
        if (gn < N && gk < K) v = TB ? B[gn + (int64_t)gk * ldb] : B[gk + (int64_t)gn * ldb];
        Bs[kk][nn] = v;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        const int kr = kk + (lane >> 4);
        double a0 = As[kr][wm * 32 + (lane & 15)];
        double a1 = As[kr][wm * 32 + 16 + (lane & 15)];
        double b0 = Bs[kr][wn * 32 + (lane & 15)];
        double b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  int cr, cc;
  ref_origin(it.c, sz, s, &cr, &cc);
  double* C = addr(bt, it.c.buf, it.c.blk, s, cr, cc);
  const int ldc = bt.ld[it.c.buf];
  double* C2 = nullptr;
  int ldc2 = 0;
  if (it.c2.buf >= 0) {
    int r2, c2;
    ref_origin(it.c2, sz, s, &r2, &c2);
    C2 = addr(bt, it.c2.buf, it.c2.blk, s, r2, c2);
    ldc2 = bt.ld[it.c2.buf];
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        int r = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;   // D[i][j]: lane j + 16*(i%4), reg i/4
        int c = n0 + wn * 32 + j * 16 + (lane & 15);
        if (r < M && c < N) {
          double x = it.alpha * acc[i][j][v];
          double* p = C + r + (int64_t)c * ldc;
          *p = it.beta != 0.0 ? it.beta * *p + x : x;
          if (C2) {
            double* q = C2 + c + (int64_t)r * ldc2;
            *q = it.beta != 0.0 ? it.beta * *q + x : x;
          }
        }
      }
}

// --------------------------------------------------------------- matrix sums
__global__ void k_matsum(const SumItem* __restrict__ items, const int* __restrict__ src, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const SumItem it = items[blockIdx.y];
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  double* C = addr(bt, it.cbuf, it.cblk, s, 0, 0);
  const int ldc = bt.ld[it.cbuf];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)M * N; e += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(e % M), c = (int)(e / M);
    double acc = 0.0;
    for (int t = 0; t < it.nt; ++t) {
      int b = src[2 * (it.t0 + t)], k = src[2 * (it.t0 + t) + 1];
      acc += addr(bt, b, k, s, r, c)[0];
    }
    C[r + (int64_t)c * ldc] = acc;
  }
}

// -------------------------------------------------------- block reductions
__device__ inline void argmax_reduce(double* sv, int* si, int tid, int nthr) {
  // first maximum wins ties (smaller index)
  for (int off = nthr / 2; off > 0; off >>= 1) {
    if (tid < off) {
      double a = sv[tid], b = sv[tid + off];
      int ia = si[tid], ib = si[tid + off];
      if (b > a || (b == a && ib < ia)) { sv[tid] = b; si[tid] = ib; }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------- recompression
// Rank-revealing QR of the concatenated fill-in products of cluster i (Sec. 3.4),
// computed as pivoted Cholesky of their Gram G = X X^T (pivot = largest remaining
// squared row norm of X, first index on ties; stop when <= tau^2), then
// Householder QR of the kept columns, giving W = [Q_perp | Q_t] in place of G.
constexpr int RT_THREADS = 256;

__global__ __launch_bounds__(RT_THREADS) void k_recompress(const int* __restrict__ clusters, BufTab bt, SizeTab sz,
                                                           double tau2, int* __restrict__ status) {
  extern __shared__ double sh[];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int R = sz.R[s * N + i];
  const int tid = threadIdx.x;
  const int ld = bt.ld[B_G];
  double* G = addr(bt, B_G, i, s, 0, 0);
  double* V = addr(bt, B_V, i, s, 0, 0);
  const int cap = ld;
  double* d = sh;                       // remaining diagonal [cap]
  double* beta = sh + cap;              // Householder scalars [cap]
  double* red = sh + 2 * cap;           // reduction values [RT_THREADS]
  int* redi = (int*)(sh + 2 * cap + RT_THREADS);
  int* piv = redi + RT_THREADS;         // pivot order [cap]
  char* used = (char*)(piv + cap);      // [cap]
  if (R <= 0) {
    if (tid == 0) sz.t[s * N + i] = 0;
    return;
  }
  for (int a = tid; a < R; a += RT_THREADS) {
    d[a] = G[a + (int64_t)a * ld];
    used[a] = 0;
  }
  __syncthreads();
  int t = 0;
  for (;;) {
    if (t >= R) break;
    double bv = -1.0;
    int bi = R;
    for (int a = tid; a < R; a += RT_THREADS)
      if (!used[a] && (d[a] > bv || (d[a] == bv && a < bi))) { bv = d[a]; bi = a; }
    red[tid] = bv;
    redi[tid] = bi;
    __syncthreads();
    argmax_reduce(red, redi, tid, RT_THREADS);
    const double dmax = red[0];
    const int p = redi[0];
    __syncthreads();
    if (!(dmax > tau2)) break;
    const double inv = 1.0 / sqrt(dmax);
    // column t of L in original coordinates
    for (int a = tid; a < R; a += RT_THREADS) {
      double v = 0.0;
      if (!used[a] && a != p) {
        v = G[a + (int64_t)p * ld];
        for (int l = 0; l < t; ++l) v -= V[a + (int64_t)l * ld] * V[p + (int64_t)l * ld];
        v *= inv;
      } else if (a == p) {
        v = sqrt(dmax);
      }
      V[a + (int64_t)t * ld] = v;
    }
    __syncthreads();
    for (int a = tid; a < R; a += RT_THREADS) {
      if (!used[a] && a != p) {
        double v = V[a + (int64_t)t * ld];
        d[a] -= v * v;
      }
    }
    if (tid == 0) { used[p] = 1; piv[t] = p; }
    __syncthreads();
    ++t;
  }
  if (tid == 0) {
    sz.t[s * N + i] = t;
    sz.R[s * N + i] = R - t;
  }
  if (t == 0) return;
  // Householder QR of V[:, 0:t] (R x t) in place
  for (int k = 0; k < t; ++k) {
    double part = 0.0;
    for (int a = k + tid; a < R; a += RT_THREADS) {
      double x = V[a + (int64_t)k * ld];
      part += x * x;
    }
    red[tid] = part;
    __syncthreads();
    for (int off = RT_THREADS / 2; off > 0; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    const double xn = sqrt(red[0]);
    const double x0 = V[k + (int64_t)k * ld];
    __syncthreads();
    const double alpha = -copysign(xn, x0 != 0.0 ? x0 : 1.0);
    // v = x - alpha e_k ; ||v||^2 = xn^2 - 2 alpha x0 + alpha^2
    const double v0 = x0 - alpha;
    const double vn = xn * xn - x0 * x0 + v0 * v0;
    const double bk = vn > 0.0 ? 2.0 / vn : 0.0;
    if (tid == 0) {
      V[k + (int64_t)k * ld] = v0;
      beta[k] = bk;
    }
    __syncthreads();
    // apply to columns k+1..t-1: each thread group handles one column
    for (int j = k + 1; j < t; ++j) {
      double pj = 0.0;
      for (int a = k + tid; a < R; a += RT_THREADS) pj += V[a + (int64_t)k * ld] * V[a + (int64_t)j * ld];
      red[tid] = pj;
      __syncthreads();
      for (int off = RT_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
      }
      const double f = red[0] * bk;
      __syncthreads();
      for (int a = k + tid; a < R; a += RT_THREADS) V[a + (int64_t)j * ld] -= V[a + (int64_t)k * ld] * f;
      __syncthreads();
    }
  }
  // W = Q with columns reordered [Q(:, t:R) | Q(:, 0:t)]: start from the permuted
  // identity, then apply H_{t-1}, ..., H_0 from the left.
  for (int64_t e = tid; e < (int64_t)R * R; e += RT_THREADS) {
    int a = (int)(e % R), c = (int)(e / R);
    int src = c < R - t ? c + t : c - (R - t);   // column of Q stored at position c
    G[a + (int64_t)c * ld] = (a == src) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = t - 1; k >= 0; --k) {
    const double bk = beta[k];
    for (int c = tid; c < R; c += RT_THREADS) {
      double pj = 0.0;
      for (int a = k; a < R; ++a) pj += V[a + (int64_t)k * ld] * G[a + (int64_t)c * ld];
      pj *= bk;
      for (int a = k; a < R; ++a) G[a + (int64_t)c * ld] -= V[a + (int64_t)k * ld] * pj;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- rotation
// side 0: rows [0, RT) of the block <- W^T rows ; side 1: cols [0, RT) <- cols W.
static inline int strip_for(int cap) { return std::max(1, std::min(16, 65536 / (cap * 8))); }

__global__ __launch_bounds__(256) void k_rotate(const RotItem* __restrict__ items, BufTab bt, SizeTab sz, int STRIP) {
  extern __shared__ double sh[];
  const int s = blockIdx.z;
  const RotItem it = items[blockIdx.y];
  const int N = sz.N;
  const int t = sz.t[s * N + it.cluster];
  if (t == 0) return;
  const int RT = sz.R[s * N + it.cluster] + t;
  const int other = dev_eval(it.other, sz, s);
  const int o0 = blockIdx.x * STRIP;
  if (o0 >= other) return;
  const int no = min(STRIP, other - o0);
  const double* W = addr(bt, B_G, it.cluster, s, 0, 0);
  const int ldw = bt.ld[B_G];
  double* X = addr(bt, it.buf, it.blk, s, 0, 0);
  const int ldx = bt.ld[it.buf];
  const int tid = threadIdx.x;
  // load strip: RT x no (side 0: rows 0..RT, cols o0..; side 1: cols 0..RT, rows o0..)
  for (int e = tid; e < RT * no; e += 256) {
    int a = e % RT, o = e / RT;
    sh[a + o * RT] = it.side == 0 ? X[a + (int64_t)(o0 + o) * ldx] : X[(o0 + o) + (int64_t)a * ldx];
  }
  __syncthreads();
  for (int e = tid; e < RT * no; e += 256) {
    int a = e % RT, o = e / RT;
    const double* wc = W + (int64_t)a * ldw;   // column a of W
    const double* xs = sh + o * RT;
    double acc = 0.0;
    for (int b = 0; b < RT; ++b) acc += wc[b] * xs[b];
    if (it.side == 0) X[a + (int64_t)(o0 + o) * ldx] = acc;
    else X[(o0 + o) + (int64_t)a * ldx] = acc;
  }
}

// ------------------------------------------------------- pivot-block LDL^T
// Bunch-Kaufman (partial pivoting, alpha = (1+sqrt(17))/8) on the redundant
// block P = S_ii^{RR} (Eq. blr2-diag-ldl), in place, full storage.  With
// P[perm, perm] = L D L^T and D = J Lambda J^T (2x2 blocks diagonalised by a
// Jacobi rotation), the elimination operator K = Pi L^{-T} J |Lambda|^{-1/2} and
// the signs sgn(Lambda) let every later step use the scaled generators
// Y~ = B K (Eq. blr2-diag-elimination) and S -= Y~ diag(sgn) Y~^T
// (Eq. blr2-diag-schur).  The number of negative entries of Lambda is added to
// nu (Sylvester's law of inertia).
constexpr int LDL_THREADS = 256;

__global__ __launch_bounds__(LDL_THREADS) void k_ldl(const int* __restrict__ clusters, const int* __restrict__ diag_blk,
                                                     BufTab bt, SizeTab sz, unsigned long long* __restrict__ nu,
                                                     int* __restrict__ status) {
  extern __shared__ double sh[];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int R = sz.R[s * N + i];
  const int tid = threadIdx.x;
  if (R <= 0) return;
  const int ld = bt.ld[B_S];
  double* A = addr(bt, B_S, diag_blk[i], s, 0, 0);
  double* K = addr(bt, B_G, i, s, 0, 0);
  double* Li = addr(bt, B_V, i, s, 0, 0);
  double* sg = addr(bt, B_SIGN, 0, s, 0, 0) + (int64_t)i * bt.bs[B_SIGN];
  const int cap = ld;
  double* l1 = sh;                 // [cap]
  double* l2 = sh + cap;           // [cap]
  double* c1 = sh + 2 * cap;       // [cap]
  double* c2 = sh + 3 * cap;       // [cap]
  double* red = sh + 4 * cap;      // [LDL_THREADS]
  int* redi = (int*)(red + LDL_THREADS);
  int* perm = redi + LDL_THREADS;  // [cap]
  int* psz = perm + cap;           // [cap] 1, 2 (first of a 2x2), 0 (second)
  __shared__ int s_bad;
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  for (int a = tid; a < R; a += LDL_THREADS) perm[a] = a;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  int k = 0;
  while (k < R) {
    // column max below the diagonal
    double bv = -1.0;
    int bi = R;
    for (int a = k + 1 + tid; a < R; a += LDL_THREADS) {
      double v = fabs(A[a + (int64_t)k * ld]);
      if (v > bv) { bv = v; bi = a; }
    }
    red[tid] = bv;
    redi[tid] = bi;
    __syncthreads();
    argmax_reduce(red, redi, tid, LDL_THREADS);
    const double colmax = red[0] < 0.0 ? 0.0 : red[0];
    const int imax = redi[0];
    __syncthreads();
    const double absakk = fabs(A[k + (int64_t)k * ld]);
    int kind = 1, kp = k;
    if (fmax(absakk, colmax) == 0.0 || !(absakk == absakk)) {
      kind = 1; kp = k;
      if (tid == 0) s_bad = 1;
    } else if (absakk >= alpha * colmax) {
      kind = 1; kp = k;
    } else {
      double rv = 0.0;
      for (int j = k + tid; j < R; j += LDL_THREADS)
        if (j != imax) rv = fmax(rv, fabs(A[imax + (int64_t)j * ld]));
      red[tid] = rv;
      __syncthreads();
      for (int off = LDL_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
        __syncthreads();
      }
      const double rowmax = red[0];
      __syncthreads();
      if (absakk >= alpha * colmax * (colmax / rowmax)) {
        kind = 1; kp = k;
      } else if (fabs(A[imax + (int64_t)imax * ld]) >= alpha * rowmax) {
        kind = 1; kp = imax;
      } else {
        kind = 2; kp = imax;
      }
    }
    const int kk = (kind == 2) ? k + 1 : k;   // position receiving the pivot row
    __syncthreads();                          // every thread has read the pivot data
    if (kp != kk) {
      // symmetric swap kk <-> kp: full rows then full columns
      for (int j = tid; j < R; j += LDL_THREADS) {
        double x = A[kk + (int64_t)j * ld];
        A[kk + (int64_t)j * ld] = A[kp + (int64_t)j * ld];
        A[kp + (int64_t)j * ld] = x;
      }
      __syncthreads();
      for (int a = tid; a < R; a += LDL_THREADS) {
        double x = A[a + (int64_t)kk * ld];
        A[a + (int64_t)kk * ld] = A[a + (int64_t)kp * ld];
        A[a + (int64_t)kp * ld] = x;
      }
      if (tid == 0) {
        int x = perm[kk];
        perm[kk] = perm[kp];
        perm[kp] = x;
      }
      __syncthreads();
    }
    if (kind == 1) {
      const double dk = A[k + (int64_t)k * ld];
      const double inv = dk != 0.0 ? 1.0 / dk : 0.0;
      for (int a = k + 1 + tid; a < R; a += LDL_THREADS) {
        c1[a] = A[a + (int64_t)k * ld];
        l1[a] = c1[a] * inv;
      }
      if (tid == 0) psz[k] = 1;
      __syncthreads();
      const int nt = R - k - 1;
      for (int64_t e = tid; e < (int64_t)nt * nt; e += LDL_THREADS) {
        int a = k + 1 + (int)(e % nt), b = k + 1 + (int)(e / nt);
        A[a + (int64_t)b * ld] -= l1[a] * c1[b];
      }
      __syncthreads();
      for (int a = k + 1 + tid; a < R; a += LDL_THREADS) A[a + (int64_t)k * ld] = l1[a];
      __syncthreads();
      k += 1;
    } else {
      const double a11 = A[k + (int64_t)k * ld], a21 = A[k + 1 + (int64_t)k * ld], a22 = A[k + 1 + (int64_t)(k + 1) * ld];
      const double det = a11 * a22 - a21 * a21;
      if (tid == 0 && !(det != 0.0 && det == det)) s_bad = 1;
      const double idet = det != 0.0 ? 1.0 / det : 0.0;
      for (int a = k + 2 + tid; a < R; a += LDL_THREADS) {
        double x1 = A[a + (int64_t)k * ld], x2 = A[a + (int64_t)(k + 1) * ld];
        c1[a] = x1;
        c2[a] = x2;
        l1[a] = (x1 * a22 - x2 * a21) * idet;
        l2[a] = (x2 * a11 - x1 * a21) * idet;
      }
      if (tid == 0) { psz[k] = 2; psz[k + 1] = 0; }
      __syncthreads();
      const int nt = R - k - 2;
      for (int64_t e = tid; e < (int64_t)nt * nt; e += LDL_THREADS) {
        int a = k + 2 + (int)(e % nt), b = k + 2 + (int)(e / nt);
        A[a + (int64_t)b * ld] -= l1[a] * c1[b] + l2[a] * c2[b];
      }
      __syncthreads();
      for (int a = k + 2 + tid; a < R; a += LDL_THREADS) {
        A[a + (int64_t)k * ld] = l1[a];
        A[a + (int64_t)(k + 1) * ld] = l2[a];
      }
      __syncthreads();
      k += 2;
    }
  }
  // unit lower inverse: column j of L^{-1} by forward substitution (L_{k+1,k} = 0
  // inside a 2x2 pivot block, where A holds D's off-diagonal entry)
  for (int j = tid; j < R; j += LDL_THREADS) {
    for (int a = 0; a < j; ++a) Li[a + (int64_t)j * ld] = 0.0;
    Li[j + (int64_t)j * ld] = 1.0;
    for (int a = j + 1; a < R; ++a) {
      double acc = 0.0;
      for (int b = j; b < a; ++b) {
        double lab = (psz[b] == 2 && a == b + 1) ? 0.0 : A[a + (int64_t)b * ld];
        acc -= lab * Li[b + (int64_t)j * ld];
      }
      Li[a + (int64_t)j * ld] = acc;
    }
  }
  __syncthreads();
  // K[perm[a], b] = (L^{-T} J |Lambda|^{-1/2})[a, b],  (L^{-T})[a, b] = Li[b, a]
  int neg = 0;
  for (int b = tid; b < R; b += LDL_THREADS) {
    if (psz[b] == 0) continue;
    if (psz[b] == 1) {
      const double dk = A[b + (int64_t)b * ld];
      const double sc = (dk != 0.0 && dk == dk) ? 1.0 / sqrt(fabs(dk)) : 0.0;
      sg[b] = dk < 0.0 ? -1.0 : 1.0;
      neg += dk < 0.0 ? 1 : 0;
      for (int a = 0; a < R; ++a) K[perm[a] + (int64_t)b * ld] = Li[b + (int64_t)a * ld] * sc;
    } else {
      const double a11 = A[b + (int64_t)b * ld], a21 = A[b + 1 + (int64_t)b * ld], a22 = A[b + 1 + (int64_t)(b + 1) * ld];
      double cs = 1.0, sn = 0.0;
      if (a21 != 0.0) {
        double tau = (a22 - a11) / (2.0 * a21);
        double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        cs = 1.0 / sqrt(1.0 + tt * tt);
        sn = tt * cs;
      }
      // J = [[cs, sn], [-sn, cs]], J^T D J = diag(lam1, lam2)
      const double lam1 = cs * cs * a11 - 2.0 * cs * sn * a21 + sn * sn * a22;
      const double lam2 = sn * sn * a11 + 2.0 * cs * sn * a21 + cs * cs * a22;
      const double s1 = (lam1 != 0.0 && lam1 == lam1) ? 1.0 / sqrt(fabs(lam1)) : 0.0;
      const double s2 = (lam2 != 0.0 && lam2 == lam2) ? 1.0 / sqrt(fabs(lam2)) : 0.0;
      sg[b] = lam1 < 0.0 ? -1.0 : 1.0;
      sg[b + 1] = lam2 < 0.0 ? -1.0 : 1.0;
      neg += (lam1 < 0.0 ? 1 : 0) + (lam2 < 0.0 ? 1 : 0);
      for (int a = 0; a < R; ++a) {
        double x1 = Li[b + (int64_t)a * ld], x2 = Li[b + 1 + (int64_t)a * ld];
        K[perm[a] + (int64_t)b * ld] = (x1 * cs - x2 * sn) * s1;
        K[perm[a] + (int64_t)(b + 1) * ld] = (x1 * sn + x2 * cs) * s2;
      }
    }
  }
  red[tid] = (double)neg;
  __syncthreads();
  for (int off = LDL_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    atomicAdd(nu + s, (unsigned long long)(red[0] + 0.5));
    if (s_bad) atomicOr(status + s, 1);
  }
}

// ------------------------------------------------------------ elimination
// rows [row0, row0+nrows) x cols [0, R_i) of block (k, i) <- rows * K_i
__global__ __launch_bounds__(256) void k_trsm(const TrsmItem* __restrict__ items, BufTab bt, SizeTab sz, int STRIP) {
  extern __shared__ double sh[];
  const int s = blockIdx.z;
  const TrsmItem it = items[blockIdx.y];
  const int Ri = sz.R[s * sz.N + it.cluster];
  const int row0 = dev_eval(it.row0, sz, s), nrows = dev_eval(it.nrows, sz, s);
  const int r0 = blockIdx.x * STRIP;
  if (Ri <= 0 || r0 >= nrows) return;
  const int nr = min(STRIP, nrows - r0);
  const int ld = bt.ld[B_S];
  double* X = addr(bt, B_S, it.blk, s, row0 + r0, 0);
  const double* K = addr(bt, B_G, it.cluster, s, 0, 0);
  const int ldk = bt.ld[B_G];
  const int tid = threadIdx.x;
  for (int e = tid; e < Ri * nr; e += 256) {
    int r = e % nr, a = e / nr;
    sh[a + r * Ri] = X[r + (int64_t)a * ld];
  }
  __syncthreads();
  for (int e = tid; e < Ri * nr; e += 256) {
    int r = e % nr, b = e / nr;
    const double* kc = K + (int64_t)b * ldk;
    const double* xr = sh + r * Ri;
    double acc = 0.0;
    for (int a = 0; a < Ri; ++a) acc += xr[a] * kc[a];
    X[r + (int64_t)b * ld] = acc;
  }
}

// ------------------------------------------------------------------- merge
__global__ void k_merge_sizes(SizeTab sz, int Np) {
  const int s = blockIdx.y;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < Np; p += gridDim.x * blockDim.x) {
    const int N = sz.N;
    int c1 = 2 * p, c2 = 2 * p + 1;
    int s1 = sz.m[s * N + c1] - sz.R[s * N + c1];
    int s2 = sz.m[s * N + c2] - sz.R[s * N + c2];
    int mp = s1 + s2;
    sz.pm[s * Np + p] = mp;
    sz.pR[s * Np + p] = mp - sz.pr0[p];
  }
}

// P_p (m_p x m_p): parent coordinates [new c1 | new c2 | E^T (old c1, old c2)]
__global__ void k_pmat(BufTab bt, SizeTab sz, const int* __restrict__ edim) {
  const int s = blockIdx.z, p = blockIdx.y;
  const int N = sz.N;
  const int c1 = 2 * p, c2 = 2 * p + 1;
  const int t1 = sz.t[s * N + c1], t2 = sz.t[s * N + c2];
  const int s1 = sz.m[s * N + c1] - sz.R[s * N + c1];
  const int r01 = sz.r0[c1];
  const int mp = sz.pm[s * sz.Np + p];
  const int ed = edim[p];
  double* P = addr(bt, B_PMAT, p, s, 0, 0);
  const int ld = bt.ld[B_PMAT];
  const double* E = addr(bt, B_EMAT, p, 0, 0, 0);
  const int lde = bt.ld[B_EMAT];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)mp * mp; e += (int64_t)gridDim.x * blockDim.x) {
    int row = (int)(e % mp), col = (int)(e / mp);
    double v = 0.0;
    if (col < t1) v = (row == col) ? 1.0 : 0.0;
    else if (col < t1 + t2) v = (row == s1 + (col - t1)) ? 1.0 : 0.0;
    else {
      int o = -1;
      if (row >= t1 && row < s1) o = row - t1;
      else if (row >= s1 + t2) o = r01 + (row - s1 - t2);
      int b = col - t1 - t2;
      if (o >= 0 && o < ed && b < ed) v = E[o + (int64_t)b * lde];
    }
    P[row + (int64_t)col * ld] = v;
  }
}

__global__ void k_gather(const GatherItem* __restrict__ items, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const GatherItem g = items[blockIdx.y];
  const int N = sz.N;
  const int p = g.p, q = g.q;
  const int sp1 = sz.m[s * N + 2 * p] - sz.R[s * N + 2 * p];
  const int sq1 = sz.m[s * N + 2 * q] - sz.R[s * N + 2 * q];
  const int mp = sz.pm[s * sz.Np + p], mq = sz.pm[s * sz.Np + q];
  double* H = addr(bt, B_HAT, g.out_blk, s, 0, 0);
  const int ldh = bt.ld[B_HAT];
  const int ldc = bt.ld[B_CPL];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)mp * mq; e += (int64_t)gridDim.x * blockDim.x) {
    int row = (int)(e % mp), col = (int)(e / mp);
    int a = row < sp1 ? 0 : 1, b = col < sq1 ? 0 : 1;
    int c = 2 * p + a, d = 2 * q + b;
    int rr = row - (a ? sp1 : 0), cc = col - (b ? sq1 : 0);
    int slot = 2 * a + b;
    int Rc = sz.R[s * N + c], Rd = sz.R[s * N + d];
    double v = 0.0;
    if (g.src_kind[slot] == 1) v = addr(bt, B_S, g.src_blk[slot], s, Rc + rr, Rd + cc)[0];
    else if (g.src_kind[slot] == 2) v = addr(bt, B_F, g.src_blk[slot], s, Rc + rr, Rd + cc)[0];
    if (g.cpl_blk[slot] >= 0) {
      int tc = sz.t[s * N + c], td = sz.t[s * N + d];
      if (rr >= tc && cc >= td) v += bt.p[B_CPL][(int64_t)g.cpl_blk[slot] * bt.bs[B_CPL] + (rr - tc) + (int64_t)(cc - td) * ldc];
    }
    H[row + (int64_t)col * ldh] = v;
  }
}

__global__ void k_next_sizes(SizeTab sz) {
  // after the merge: current <- parent (the size table of the next level)
  const int s = blockIdx.y;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < sz.Np; p += gridDim.x * blockDim.x) {
    sz.m[s * sz.Np + p] = sz.pm[s * sz.Np + p];
    sz.R[s * sz.Np + p] = sz.pR[s * sz.Np + p];
    sz.t[s * sz.Np + p] = 0;
  }
}

// ----------------------------------------------------------- leaf start
// S[shift][blk] = Bres[blk]; diagonal blocks get -sigma on the diagonal.
__global__ void k_leaf_init(BufTab bt, int nblk, const int* __restrict__ blk_diag_m, const double* __restrict__ sigma) {
  const int s = blockIdx.z;
  const int b = blockIdx.y;
  const int64_t n = bt.bs[B_S];
  const int ld = bt.ld[B_S];
  double* dst = addr(bt, B_S, b, s, 0, 0);
  const double* src = bt.p[B_BRES] + (int64_t)b * bt.bs[B_BRES];
  const int md = blk_diag_m[b];
  const double sig = sigma[s];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double v = src[e];
    int r = (int)(e % ld), c = (int)(e / ld);
    if (md > 0 && r == c && r < md) v -= sig;
    dst[e] = v;
  }
}

__global__ void k_sizes_init(SizeTab sz, const int* __restrict__ m0) {
  const int s = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < sz.N; i += gridDim.x * blockDim.x) {
    sz.m[s * sz.N + i] = m0[i];
    sz.R[s * sz.N + i] = m0[i] - sz.r0[i];
    sz.t[s * sz.N + i] = 0;
  }
}

// ------------------------------------------------------ kernel evaluation
__device__ inline double kf(int kind, double p0, double p1, double r) {
  switch (kind) {
    case 0: return 1.0 / r;
    case 1: return exp(-r) / r;
    case 2: return exp(-r * r / p0) / (r + p1);
    case 3: return 1.0 / (r + p0);
    case 4: return (fabs(r - p0) < 1e-9 * p0) ? -1.0 : 0.0;
  }
  return 0.0;
}

// near block (i, j) of the leaf level: A(tau_i, tau_j) in leaf order
__global__ void k_kernel_blocks(double* out, int64_t bstride, int ld, const int* __restrict__ bi, const int* __restrict__ bj,
                                const int64_t* __restrict__ start, const int* __restrict__ msz, const double* __restrict__ X,
                                int dim, int kind, double diag, double p0, double p1, int* __restrict__ bad) {
  const int b = blockIdx.y;
  const int i = bi[b], j = bj[b];
  const int mi = msz[i], mj = msz[j];
  const int64_t si = start[i], sj = start[j];
  double* o = out + (int64_t)b * bstride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)ld * ld; e += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(e % ld), c = (int)(e / ld);
    double v = 0.0;
    if (r < mi && c < mj) {
      int64_t a = si + r, bb = sj + c;
      if (a == bb) v = diag;
      else {
        double acc = 0.0;
        for (int d = 0; d < dim; ++d) {
          double x = X[a * dim + d] - X[bb * dim + d];
          acc += x * x;
        }
        v = kf(kind, p0, p1, sqrt(acc));
        if (!isfinite(v)) atomicOr(bad, 1);
      }
    }
    o[e] = v;
  }
}

// =================================================================== launchers
static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = (unsigned)std::min<int64_t>(cdiv(n, 256), 65535 * 4);
  hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, st, p, n, v);
}

void launch_fill_int(int* p, int64_t n, int v, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = (unsigned)std::min<int64_t>(cdiv(n, 256), 65535);
  hipLaunchKernelGGL(k_fill_int, dim3(g), dim3(256), 0, st, p, n, v);
}

void launch_gemm(int kind, const GItem* items, int nitems, const GTerm* terms, const BufTab& bt, const SizeTab& sz,
                 int mcap, int ncap, int nshift, hipStream_t st) {
  if (nitems <= 0) return;
  int tm = (int)cdiv(mcap, GT), tn = (int)cdiv(ncap, GT);
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    int ni = std::min(65535, nitems - i0);
    dim3 grid(tm * tn, ni, nshift);
    switch (kind) {
      case GEMM_NN: hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn); break;
      case GEMM_NT: hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn); break;
      case GEMM_TN: hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn); break;
      default: hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn); break;
    }
  }
}

void launch_matsum(const SumItem* items, int nitems, const int* src, const BufTab& bt, const SizeTab& sz, int cap,
                   int nshift, hipStream_t st) {
  if (nitems <= 0) return;
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    int ni = std::min(65535, nitems - i0);
    dim3 grid(std::max(1u, cdiv((int64_t)cap * cap, 256 * 4)), ni, nshift);
    hipLaunchKernelGGL(k_matsum, grid, dim3(256), 0, st, items + i0, src, bt, sz);
  }
}

void launch_recompress(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, double tau2, int* status,
                       int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  size_t shmem = (size_t)2 * cap * sizeof(double) + RT_THREADS * sizeof(double) + RT_THREADS * sizeof(int) +
                 (size_t)cap * sizeof(int) + cap + 16;
  hipLaunchKernelGGL(k_recompress, dim3(1, n, nshift), dim3(RT_THREADS), shmem, st, clusters, bt, sz, tau2, status);
}

void launch_rotate(const RotItem* items, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  const int strip = strip_for(cap);
  size_t shmem = (size_t)cap * strip * sizeof(double);
  for (int i0 = 0; i0 < n; i0 += 65535) {
    int ni = std::min(65535, n - i0);
    hipLaunchKernelGGL(k_rotate, dim3(cdiv(cap, strip), ni, nshift), dim3(256), shmem, st, items + i0, bt, sz, strip);
  }
}

void launch_ldl(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz,
                unsigned long long* nu, int* status, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  size_t shmem = (size_t)4 * cap * sizeof(double) + LDL_THREADS * (sizeof(double) + sizeof(int)) + (size_t)2 * cap * sizeof(int);
  hipLaunchKernelGGL(k_ldl, dim3(1, n, nshift), dim3(LDL_THREADS), shmem, st, clusters, diag_blk, bt, sz, nu, status);
}

void launch_trsm(const TrsmItem* items, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  const int strip = strip_for(cap);
  size_t shmem = (size_t)cap * strip * sizeof(double);
  for (int i0 = 0; i0 < n; i0 += 65535) {
    int ni = std::min(65535, n - i0);
    hipLaunchKernelGGL(k_trsm, dim3(cdiv(cap, strip), ni, nshift), dim3(256), shmem, st, items + i0, bt, sz, strip);
  }
}

void launch_merge_sizes(const SizeTab& sz, int Np, int nshift, hipStream_t st) {
  hipLaunchKernelGGL(k_merge_sizes, dim3(cdiv(Np, 256), nshift), dim3(256), 0, st, sz, Np);
}

void launch_pmat(const BufTab& bt, const SizeTab& sz, const int* edim, int Np, int pcap, int nshift, hipStream_t st) {
  hipLaunchKernelGGL(k_pmat, dim3(std::max(1u, cdiv((int64_t)pcap * pcap, 256 * 8)), Np, nshift), dim3(256), 0, st, bt, sz, edim);
}

void launch_gather(const GatherItem* items, int n, const BufTab& bt, const SizeTab& sz, int pcap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  for (int i0 = 0; i0 < n; i0 += 65535) {
    int ni = std::min(65535, n - i0);
    hipLaunchKernelGGL(k_gather, dim3(std::max(1u, cdiv((int64_t)pcap * pcap, 256 * 8)), ni, nshift), dim3(256), 0, st,
                       items + i0, bt, sz);
  }
}

void launch_next_sizes(const SizeTab& sz, int nshift, hipStream_t st) {
  hipLaunchKernelGGL(k_next_sizes, dim3(cdiv(sz.Np, 256), nshift), dim3(256), 0, st, sz);
}

void launch_leaf_init(const BufTab& bt, int nblk, const int* blk_diag_m, const double* sigma, int cap, int nshift, hipStream_t st) {
  for (int b0 = 0; b0 < nblk; b0 += 65535) {
    int nb = std::min(65535, nblk - b0);
    BufTab t = bt;
    t.p[B_S] = bt.p[B_S] + (int64_t)b0 * bt.bs[B_S];
    t.p[B_BRES] = bt.p[B_BRES] + (int64_t)b0 * bt.bs[B_BRES];
    hipLaunchKernelGGL(k_leaf_init, dim3(std::max(1u, cdiv((int64_t)cap * cap, 256 * 8)), nb, nshift), dim3(256), 0, st, t,
                       nb, blk_diag_m + b0, sigma);
  }
}

void launch_sizes_init(const SizeTab& sz, const int* m0, int nshift, hipStream_t st) {
  hipLaunchKernelGGL(k_sizes_init, dim3(cdiv(sz.N, 256), nshift), dim3(256), 0, st, sz, m0);
}

void launch_kernel_blocks(double* out, int64_t bstride, int ld, const int* bi, const int* bj, int nblk, const int64_t* start,
                          const int* msz, const double* X, int dim, int kind, double diag, double p0, double p1, int* bad,
                          hipStream_t st) {
  for (int b0 = 0; b0 < nblk; b0 += 65535) {
    int nb = std::min(65535, nblk - b0);
    hipLaunchKernelGGL(k_kernel_blocks, dim3(std::max(1u, cdiv((int64_t)ld * ld, 256 * 8)), nb), dim3(256), 0, st,
                       out + (int64_t)b0 * bstride, bstride, ld, bi + b0, bj + b0, start, msz, X, dim, kind, diag, p0, p1, bad);
  }
}

}  // namespace h2
