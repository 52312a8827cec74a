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
                                              BufTab bt, SizeTab sz, int tiles_n, int slot_base) {
  const int s = blockIdx.z;
  const GItem it = items[blockIdx.y];
  if (it.guard != -1 && dev_eval(it.guard, sz, s) == 0) return;
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  const int m0 = (blockIdx.x / tiles_n) * GT, n0 = (blockIdx.x % tiles_n) * GT;
  if (m0 >= M || n0 >= N) return;
  if (bt.fc && blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long kk = 0;
    for (int tt = 0; tt < it.nt; ++tt) kk += (unsigned long long)max(0, dev_eval(terms[it.t0 + tt].K, sz, s));
    atomicAdd(bt.fc, 2ull * (unsigned long long)M * (unsigned long long)N * kk);
  }
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
  double* C = addr(bt, it.c.buf, it.c.blk >= 0 ? it.c.blk : (int)blockIdx.y + slot_base, s, cr, cc);
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

// -------------------------------------------------------- scratch copy-back
__global__ void k_copyback(const CopyItem* __restrict__ items, BufTab bt, SizeTab sz, int slot_base) {
  const int s = blockIdx.z;
  const CopyItem it = items[blockIdx.y];
  if (it.guard != -1 && dev_eval(it.guard, sz, s) == 0) return;
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  int r0, c0;
  ref_origin(it.x, sz, s, &r0, &c0);
  double* X = addr(bt, it.x.buf, it.x.blk, s, r0, c0);
  const int ldx = bt.ld[it.x.buf];
  const double* Sc = addr(bt, B_RS, (int)blockIdx.y + slot_base, s, 0, 0);
  const int lds = bt.ld[B_RS];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)M * N; e += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(e % M), b = (int)(e / M);
    X[a + (int64_t)b * ldx] = Sc[a + (int64_t)b * lds];
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
// Rank-revealing QR of the concatenated fill-in products of cluster i (Sec. 3.4):
//  * pivoted Cholesky of their Gram G = X X^T (pivot = largest remaining squared
//    row norm of X, first index on ties; stop when <= tau^2).  Its t columns L
//    (original row order) span the kept directions: they are the first t columns
//    of P R^T of the column-pivoted QR of X^T.  Blocked: a panel of PC_NB pivots
//    per step (k_pchol_panel), then G -= L_p L_p^T on the matrix cores;
//  * Householder QR of L with reflector k acting on rows 0..R-1-k, so that
//    W = H_0 ... H_{t-1} maps the kept directions onto the last t redundant
//    coordinates.  Blocked: a panel of HB columns (k_hqr_panel, which also forms
//    T_p and Y_p T_p^T), then the trailing columns receive
//    V <- V - (Y_p T_p^T)(Y_p^T V) on the matrix cores;
//  * W = prod_p (I - Y_p T_p Y_p^T), accumulated panel by panel with GEMMs.
// Per-cluster panel state: a0 = panel start, a1 = panel width; the scratch
// B_Z holds the remaining diagonal (column 0) during the Cholesky and the
// columns Y_p T_p^T during the QR.
constexpr int RT_THREADS = 256;
constexpr int PC_NB = 32;
constexpr int HB = 32;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum over RT_THREADS threads (4 waves); red has >= 4 slots
__device__ inline double block_sum(double v, double* red, int tid) {
  v = wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return r;
}

__global__ void k_pchol_init(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int R = sz.R[s * N + i];
  const int ld = bt.ld[B_G];
  const double* G = addr(bt, B_G, i, s, 0, 0);
  double* d = addr(bt, B_Z, i, s, 0, 0);
  for (int a = threadIdx.x; a < R; a += blockDim.x) d[a] = G[a + (int64_t)a * ld];
  if (threadIdx.x == 0) {
    sz.t[s * N + i] = 0;
    sz.a0[s * N + i] = 0;
    sz.a1[s * N + i] = R > 0 ? 1 : 0;   // a1 = 1 while the Cholesky runs
  }
}

// One panel of at most PC_NB pivots.  G holds the Gram updated by all previous
// panels; columns of this panel are formed from G and the panel's own columns.
__global__ __launch_bounds__(RT_THREADS) void k_pchol_panel(const int* __restrict__ clusters, BufTab bt, SizeTab sz,
                                                            double tau2, int* __restrict__ more) {
  extern __shared__ double sh[];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int tid = threadIdx.x;
  if (sz.a1[s * N + i] == 0) {                // finished: no new columns for the update
    if (tid == 0) sz.a0[s * N + i] = sz.t[s * N + i];
    return;
  }
  const int R = sz.R[s * N + i];
  const int ld = bt.ld[B_G];
  const double* G = addr(bt, B_G, i, s, 0, 0);
  double* V = addr(bt, B_V, i, s, 0, 0);
  double* dg = addr(bt, B_Z, i, s, 0, 0);
  double* d = sh;                             // [cap]
  double* red = sh + ld;                      // [RT_THREADS]
  int* redi = (int*)(red + RT_THREADS);       // [RT_THREADS]
  __shared__ int s_stop;
  for (int a = tid; a < R; a += RT_THREADS) d[a] = dg[a];
  if (tid == 0) s_stop = 0;
  __syncthreads();
  const int t0 = sz.t[s * N + i];
  int t = t0;
  for (int j = 0; j < PC_NB && t < R; ++j) {
    double bv = -INFINITY;
    int bi = R;
    for (int a = tid; a < R; a += RT_THREADS)
      if (d[a] > bv || (d[a] == bv && a < bi)) { bv = d[a]; bi = a; }
    red[tid] = bv;
    redi[tid] = bi;
    __syncthreads();
    argmax_reduce(red, redi, tid, RT_THREADS);
    const double dmax = red[0];
    const int p = redi[0];
    __syncthreads();
    if (!(dmax > tau2)) {
      if (tid == 0) s_stop = 1;
      break;
    }
    const double sq = sqrt(dmax), inv = 1.0 / sq;
    for (int a = tid; a < R; a += RT_THREADS) {
      double v = 0.0;
      if (a == p) v = sq;
      else if (d[a] != -INFINITY) {
        v = G[a + (int64_t)p * ld];
        for (int l = t0; l < t; ++l) v -= V[a + (int64_t)l * ld] * V[p + (int64_t)l * ld];
        v *= inv;
        d[a] -= v * v;
      }
      V[a + (int64_t)t * ld] = v;
    }
    __syncthreads();
    if (tid == 0) d[p] = -INFINITY;
    __syncthreads();
    ++t;
  }
  for (int a = tid; a < R; a += RT_THREADS) dg[a] = d[a];
  if (tid == 0) {
    sz.t[s * N + i] = t;
    sz.a0[s * N + i] = t0;
    const bool go = !s_stop && t < R;
    sz.a1[s * N + i] = go ? 1 : 0;
    if (go) atomicAdd(more, 1);
  }
}

__global__ void k_pchol_finish(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  if (threadIdx.x == 0) {
    const int R = sz.R[s * N + i], t = sz.t[s * N + i];
    sz.R[s * N + i] = R - t;
    if (bt.fc) atomicAdd(bt.fc, (unsigned long long)R * (unsigned long long)t * (unsigned long long)(t > 0 ? t - 1 : 0));
  }
}

// Panel `it` of the Householder QR: columns k0 = it*HB .. k0+nb-1 of V (RT x t).
__global__ __launch_bounds__(RT_THREADS) void k_hqr_panel(const int* __restrict__ clusters, BufTab bt, SizeTab sz, int it,
                                                          int* __restrict__ more) {
  extern __shared__ double sh[];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int t = sz.t[s * N + i];
  const int k0 = it * HB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (k0 >= t) {
    if (tid == 0) { sz.a0[s * N + i] = k0; sz.a1[s * N + i] = 0; }
    return;
  }
  const int nb = min(HB, t - k0);
  const int RT = sz.R[s * N + i] + t;
  if (bt.fc && tid == 0) {   // Householder QR flops of this panel's columns
    double f = 0.0;
    for (int k = k0; k < k0 + nb; ++k) f += 4.0 * (double)(RT - k) * (double)(t - k);
    atomicAdd(bt.fc, (unsigned long long)f);
  }
  const int ld = bt.ld[B_V];
  double* V = addr(bt, B_V, i, s, 0, 0);
  double* Yt = addr(bt, B_Z, i, s, 0, 0);
  double* red = sh;                 // [8]
  double* wd = sh + 8;              // [HB]
  double* Tp = sh + 8 + HB;         // [HB * HB]
  double* bp = Tp + HB * HB;        // [HB]
  for (int kk = 0; kk < nb; ++kk) {
    const int k = k0 + kk;
    const int p = RT - 1 - k;
    double part = 0.0;
    for (int a = tid; a <= p; a += RT_THREADS) {
      double x = V[a + (int64_t)k * ld];
      part += x * x;
    }
    const double xn2 = block_sum(part, red, tid);
    const double x0 = V[p + (int64_t)k * ld];
    const double xn = sqrt(xn2);
    const double alpha = -copysign(xn, x0 != 0.0 ? x0 : 1.0);
    const double v0 = x0 - alpha;
    const double vn = xn2 - x0 * x0 + v0 * v0;
    const double bk = vn > 0.0 ? 2.0 / vn : 0.0;
    __syncthreads();
    if (tid == 0) {
      V[p + (int64_t)k * ld] = v0;
      bp[kk] = bk;
    }
    __syncthreads();
    for (int j = k + 1 + wave; j < k0 + nb; j += RT_THREADS / 64) {
      double q = 0.0;
      for (int a = lane; a <= p; a += 64) q += V[a + (int64_t)k * ld] * V[a + (int64_t)j * ld];
      q = wave_sum(q);
      if (lane == 0) wd[j - k0] = q * bk;
    }
    __syncthreads();
    const int nj = k0 + nb - k - 1, nr = p + 1;
    for (int64_t e = tid; e < (int64_t)nj * nr; e += RT_THREADS) {
      int a = (int)(e % nr), j = k + 1 + (int)(e / nr);
      V[a + (int64_t)j * ld] -= V[a + (int64_t)k * ld] * wd[j - k0];
    }
    __syncthreads();
  }
  // reflectors of the panel: zero below their anchors (those rows hold R entries)
  for (int64_t e = tid; e < (int64_t)nb * RT; e += RT_THREADS) {
    int a = (int)(e % RT), kk = (int)(e / RT);
    if (a > RT - 1 - (k0 + kk)) V[a + (int64_t)(k0 + kk) * ld] = 0.0;
  }
  for (int e = tid; e < HB * HB; e += RT_THREADS) Tp[e] = 0.0;
  __syncthreads();
  // T_p: T_kk = beta_k, T[0:kk, kk] = -beta_kk T[0:kk, 0:kk] (Y_p^T y_kk)
  for (int kk = 0; kk < nb; ++kk) {
    const int p = RT - 1 - (k0 + kk);
    for (int j = wave; j < kk; j += RT_THREADS / 64) {
      double q = 0.0;
      for (int a = lane; a <= p; a += 64) q += V[a + (int64_t)(k0 + j) * ld] * V[a + (int64_t)(k0 + kk) * ld];
      q = wave_sum(q);
      if (lane == 0) wd[j] = q;
    }
    __syncthreads();
    if (tid < kk) {
      double v = 0.0;
      for (int b2 = tid; b2 < kk; ++b2) v += Tp[tid + b2 * HB] * wd[b2];
      Tp[tid + kk * HB] = -bp[kk] * v;
    } else if (tid == kk) {
      Tp[kk + kk * HB] = bp[kk];
    }
    __syncthreads();
  }
  // Yt = Y_p T_p^T  (RT x nb) into B_Z columns k0 .. k0+nb-1
  for (int64_t e = tid; e < (int64_t)nb * RT; e += RT_THREADS) {
    int a = (int)(e % RT), c = (int)(e / RT);
    double v = 0.0;
    for (int b2 = c; b2 < nb; ++b2) v += V[a + (int64_t)(k0 + b2) * ld] * Tp[c + b2 * HB];   // T^T[b2][c] = T[c][b2]
    Yt[a + (int64_t)(k0 + c) * ld] = v;
  }
  if (tid == 0) {
    sz.a0[s * N + i] = k0;
    sz.a1[s * N + i] = nb;
    if (k0 + nb < t) atomicAdd(more, 1);
  }
}

// panel state of step `it` for the accumulation of W (a0 = it*HB, a1 = panel width)
__global__ void k_set_panel(const int* __restrict__ clusters, SizeTab sz, int it) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  if (threadIdx.x == 0) {
    const int t = sz.t[s * N + i], k0 = it * HB;
    sz.a0[s * N + i] = k0;
    sz.a1[s * N + i] = k0 < t ? min(HB, t - k0) : 0;
  }
}

// W = I on the first RT x RT entries of B_W (clusters with t > 0)
__global__ void k_eye(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int t = sz.t[s * sz.N + i];
  if (t == 0) return;
  const int RT = sz.R[s * sz.N + i] + t;
  double* W = addr(bt, B_W, i, s, 0, 0);
  const int ld = bt.ld[B_W];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)RT * RT; e += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(e % RT), c = (int)(e / RT);
    W[a + (int64_t)c * ld] = a == c ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------- pivot-block LDL^T
// Bunch-Kaufman (partial pivoting, alpha = (1+sqrt(17))/8) on the redundant
// block P = S_ii^{RR} (Eq. blr2-diag-ldl), in place, full storage, blocked: a
// panel of up to LDL_NB columns is factored lazily by one workgroup
// (k_ldl_panel: columns are brought up to date from the panel's L and
// W = L D columns only when needed), then the trailing matrix receives
// A -= L_p W_p^T on the matrix cores.  With P[perm, perm] = L D L^T and
// D = J Lambda J^T (2x2 blocks diagonalised by a Jacobi rotation), k_ldl_finish
// forms the elimination operator K = Pi L^{-T} J |Lambda|^{-1/2} and the signs
// sgn(Lambda): every later step uses the scaled generators Y~ = B K
// (Eq. blr2-diag-elimination) and S -= Y~ diag(sgn) Y~^T (Eq. blr2-diag-schur).
// The number of negative entries of Lambda is added to nu (Sylvester's law).
// State: a0 = panel start, a1 = panel width, perm and pivot sizes in B_Z
// columns 0 and 1, the panel's W columns in B_W.
constexpr int LDL_THREADS = 512;
constexpr int LDL_NB = 32;

__device__ inline double block_max512(double v, double* red, int tid) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < LDL_THREADS / 64; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// argmax of |x[a]| over a in [lo, R), first index on ties; returns value, index in *idx
__device__ inline double block_argmax512(const double* x, int lo, int R, double* red, int* redi, int tid, int* idx) {
  double bv = -1.0;
  int bi = R;
  for (int a = lo + tid; a < R; a += LDL_THREADS) {
    double v = fabs(x[a]);
    if (v > bv) { bv = v; bi = a; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(bv, off, 64);
    int oi = __shfl_xor(bi, off, 64);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if ((tid & 63) == 0) { red[tid >> 6] = bv; redi[tid >> 6] = bi; }
  __syncthreads();
  double r = red[0];
  int ri = redi[0];
  for (int w = 1; w < LDL_THREADS / 64; ++w)
    if (red[w] > r || (red[w] == r && redi[w] < ri)) { r = red[w]; ri = redi[w]; }
  __syncthreads();
  *idx = ri;
  return r;
}

__global__ void k_ldl_init(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int R = sz.R[s * N + i];
  double* pz = addr(bt, B_Z, i, s, 0, 0);
  const int ld = bt.ld[B_Z];
  for (int a = threadIdx.x; a < R; a += blockDim.x) {
    pz[a] = (double)a;              // perm
    pz[a + ld] = 0.0;               // pivot size
  }
  if (threadIdx.x == 0) {
    sz.a0[s * N + i] = 0;
    sz.a1[s * N + i] = 0;
  }
}

__global__ __launch_bounds__(LDL_THREADS) void k_ldl_panel(const int* __restrict__ clusters,
                                                           const int* __restrict__ diag_blk, BufTab bt, SizeTab sz,
                                                           int* __restrict__ status, int* __restrict__ more) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int R = sz.R[s * N + i];
  const int tid = threadIdx.x;
  const int kstart = sz.a0[s * N + i] + sz.a1[s * N + i];
  if (kstart >= R) {
    if (tid == 0) { sz.a0[s * N + i] = kstart; sz.a1[s * N + i] = 0; }
    return;
  }
  const int ld = bt.ld[B_S];
  double* A = addr(bt, B_S, diag_blk[i], s, 0, 0);
  double* Wp = addr(bt, B_W, i, s, 0, 0);     // panel W = L D columns, LDL_NB + 2 columns
  double* pz = addr(bt, B_Z, i, s, 0, 0);     // perm (col 0), pivot sizes (col 1)
  const int cap = ld;
  __shared__ double red[16];
  __shared__ int redi[16];
  __shared__ int s_bad;
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  const int NB = min(LDL_NB, cap - 2);
  if (tid == 0) s_bad = 0;
  __syncthreads();
  const int k0 = kstart;
  int k = k0, jw = 0;
  while (jw < NB && k < R) {
    double* w = Wp + (int64_t)jw * ld;
    double* u = Wp + (int64_t)(jw + 1) * ld;
    for (int a = k + tid; a < R; a += LDL_THREADS) {
      double v = A[a + (int64_t)k * ld];
      for (int c = 0; c < jw; ++c) v -= A[a + (int64_t)(k0 + c) * ld] * Wp[k + (int64_t)c * ld];
      w[a] = v;
    }
    __syncthreads();
    int imax = R;
    const double colmax0 = block_argmax512(w, k + 1, R, red, redi, tid, &imax);
    const double colmax = colmax0 < 0.0 ? 0.0 : colmax0;
    const double absakk = fabs(w[k]);
    int kind = 1, kp = k;
    bool use_u = false;
    if (fmax(absakk, colmax) == 0.0 || !(absakk == absakk)) {
      if (tid == 0) s_bad = 1;
    } else if (absakk < alpha * colmax) {
      for (int a = k + tid; a < R; a += LDL_THREADS) {
        double v = A[a + (int64_t)imax * ld];
        for (int c = 0; c < jw; ++c) v -= A[a + (int64_t)(k0 + c) * ld] * Wp[imax + (int64_t)c * ld];
        u[a] = v;
      }
      __syncthreads();
      double rv = 0.0;
      for (int a = k + tid; a < R; a += LDL_THREADS)
        if (a != imax) rv = fmax(rv, fabs(u[a]));
      const double rowmax = block_max512(rv, red, tid);
      if (absakk >= alpha * colmax * (colmax / rowmax)) {
        kind = 1; kp = k;
      } else if (fabs(u[imax]) >= alpha * rowmax) {
        kind = 1; kp = imax; use_u = true;
      } else {
        kind = 2; kp = imax;
      }
    }
    const int kk = (kind == 2) ? k + 1 : k;
    __syncthreads();
    if (use_u) {
      for (int a = k + tid; a < R; a += LDL_THREADS) w[a] = u[a];
      __syncthreads();
    }
    if (kp != kk) {
      for (int j = tid; j < R; j += LDL_THREADS) {
        double x = A[kk + (int64_t)j * ld];
        A[kk + (int64_t)j * ld] = A[kp + (int64_t)j * ld];
        A[kp + (int64_t)j * ld] = x;
      }
      for (int c = tid; c < jw + 2; c += LDL_THREADS) {
        double x = Wp[kk + (int64_t)c * ld];
        Wp[kk + (int64_t)c * ld] = Wp[kp + (int64_t)c * ld];
        Wp[kp + (int64_t)c * ld] = x;
      }
      __syncthreads();
      for (int a = tid; a < R; a += LDL_THREADS) {
        double x = A[a + (int64_t)kk * ld];
        A[a + (int64_t)kk * ld] = A[a + (int64_t)kp * ld];
        A[a + (int64_t)kp * ld] = x;
      }
      if (tid == 0) {
        double x = pz[kk];
        pz[kk] = pz[kp];
        pz[kp] = x;
      }
      __syncthreads();
    }
    if (kind == 1) {
      const double dk = w[k];
      const double inv = dk != 0.0 ? 1.0 / dk : 0.0;
      for (int a = k + 1 + tid; a < R; a += LDL_THREADS) A[a + (int64_t)k * ld] = w[a] * inv;
      if (tid == 0) {
        A[k + (int64_t)k * ld] = dk;
        pz[k + ld] = 1.0;
      }
      __syncthreads();
      k += 1;
      jw += 1;
    } else {
      const double a11 = w[k], a21 = w[k + 1], a22 = u[k + 1];
      const double det = a11 * a22 - a21 * a21;
      if (tid == 0 && !(det != 0.0 && det == det)) s_bad = 1;
      const double idet = det != 0.0 ? 1.0 / det : 0.0;
      for (int a = k + 2 + tid; a < R; a += LDL_THREADS) {
        double x1 = w[a], x2 = u[a];
        A[a + (int64_t)k * ld] = (x1 * a22 - x2 * a21) * idet;
        A[a + (int64_t)(k + 1) * ld] = (x2 * a11 - x1 * a21) * idet;
      }
      if (tid == 0) {
        A[k + (int64_t)k * ld] = a11;
        A[k + 1 + (int64_t)k * ld] = a21;
        A[k + 1 + (int64_t)(k + 1) * ld] = a22;
        pz[k + ld] = 2.0;
        pz[k + 1 + ld] = 0.0;
      }
      __syncthreads();
      k += 2;
      jw += 2;
    }
  }
  if (tid == 0) {
    sz.a0[s * N + i] = k0;
    sz.a1[s * N + i] = jw;
    if (s_bad) atomicOr(status + s, 1);
    if (k < R) atomicAdd(more, 1);
  }
}

// After the panels: pivot coefficients and inertia.  For every pivot column b,
// K^T row b = cf1[b] * X[c1, :] + cf2[b] * X[c2, :] with X = L^{-1} and (c1, c2)
// the columns of its 1x1 / 2x2 block; coefficients go to B_Z columns 2 and 3,
// signs to B_SIGN; D's off-diagonal entries are cleared so that the strictly
// lower part of A is exactly L.
__global__ __launch_bounds__(LDL_THREADS) void k_ldl_prep(const int* __restrict__ clusters,
                                                          const int* __restrict__ diag_blk, BufTab bt, SizeTab sz,
                                                          unsigned long long* __restrict__ nu) {
  __shared__ double red[16];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int R = sz.R[s * N + i];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (R <= 0) return;
  const int ld = bt.ld[B_S];
  double* A = addr(bt, B_S, diag_blk[i], s, 0, 0);
  double* pz = addr(bt, B_Z, i, s, 0, 0);
  const int ldz = bt.ld[B_Z];
  double* sg = addr(bt, B_SIGN, 0, s, 0, 0) + (int64_t)i * bt.bs[B_SIGN];
  int neg = 0;
  for (int b = tid; b < R; b += LDL_THREADS) {
    const int ps = (int)pz[b + ldz];
    if (ps == 1) {
      const double dk = A[b + (int64_t)b * ld];
      pz[b + 2 * ldz] = (dk != 0.0 && dk == dk) ? 1.0 / sqrt(fabs(dk)) : 0.0;
      pz[b + 3 * ldz] = 0.0;
      sg[b] = dk < 0.0 ? -1.0 : 1.0;
      neg += dk < 0.0 ? 1 : 0;
    } else if (ps == 2) {
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
      pz[b + 2 * ldz] = cs * s1;          // column b   = cs*s1*col(b) - sn*s1*col(b+1)
      pz[b + 3 * ldz] = -sn * s1;
      pz[b + 1 + 2 * ldz] = sn * s2;      // column b+1 = sn*s2*col(b) + cs*s2*col(b+1)
      pz[b + 1 + 3 * ldz] = cs * s2;
      sg[b] = lam1 < 0.0 ? -1.0 : 1.0;
      sg[b + 1] = lam2 < 0.0 ? -1.0 : 1.0;
      neg += (lam1 < 0.0 ? 1 : 0) + (lam2 < 0.0 ? 1 : 0);
    }
  }
  __syncthreads();
  for (int b = tid; b < R; b += LDL_THREADS)
    if ((int)pz[b + ldz] == 2) A[b + 1 + (int64_t)b * ld] = 0.0;
  double nv = (double)neg;
  for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off, 64);
  if (lane == 0) red[wave] = nv;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w2 = 0; w2 < LDL_THREADS / 64; ++w2) tot += red[w2];
    atomicAdd(nu + s, (unsigned long long)(tot + 0.5));
    if (bt.fc) atomicAdd(bt.fc, (unsigned long long)(2.0 / 3.0 * (double)R * R * R));
  }
}

// X = L^{-1} on the diagonal blocks of width INV_NB (unit lower L = strictly
// lower part of A); block ib = blockIdx.x.  X lives in B_V (zeroed beforehand).
constexpr int INV_NB = 128;

__global__ void k_diag_inv(const int* __restrict__ clusters, const int* __restrict__ diag_blk, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int R = sz.R[s * sz.N + i];
  const int r0 = blockIdx.x * INV_NB;
  if (r0 >= R) return;
  const int nb = min(INV_NB, R - r0);
  const int ld = bt.ld[B_S];
  const double* A = addr(bt, B_S, diag_blk[i], s, 0, 0);
  double* X = addr(bt, B_V, i, s, 0, 0);
  const int ldx = bt.ld[B_V];
  for (int c = threadIdx.x; c < nb; c += blockDim.x) {
    const int gc = r0 + c;
    X[gc + (int64_t)gc * ldx] = 1.0;
    for (int a = c + 1; a < nb; ++a) {
      const int ga = r0 + a;
      double v = 0.0;
      for (int b2 = c; b2 < a; ++b2) v -= A[ga + (int64_t)(r0 + b2) * ld] * X[r0 + b2 + (int64_t)gc * ldx];
      X[ga + (int64_t)gc * ldx] = v;
    }
  }
}

// panel state for block row ib of the inversion: a0 = ib*INV_NB, a1 = its height (0 beyond R)
__global__ void k_set_block(const int* __restrict__ clusters, SizeTab sz, int ib) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  if (threadIdx.x == 0) {
    const int R = sz.R[s * N + i], a0 = ib * INV_NB;
    sz.a0[s * N + i] = a0;
    sz.a1[s * N + i] = a0 < R ? min(INV_NB, R - a0) : 0;
  }
}

// K^T[b, perm[a]] = cf1[b] X[c1(b), a] + cf2[b] X[c2(b), a]  (K = Pi L^{-T} J |Lambda|^{-1/2})
__global__ void k_kform(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int R = sz.R[s * sz.N + i];
  const int ld = bt.ld[B_V];
  const double* X = addr(bt, B_V, i, s, 0, 0);
  const double* pz = addr(bt, B_Z, i, s, 0, 0);
  const int ldz = bt.ld[B_Z];
  double* KT = addr(bt, B_G, i, s, 0, 0);
  const int ldk = bt.ld[B_G];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)R * R; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e % R), a = (int)(e / R);
    const int ps = (int)pz[b + ldz];
    int c1i, c2i;
    if (ps == 0) { c1i = b - 1; c2i = b; }
    else if (ps == 2) { c1i = b; c2i = b + 1; }
    else { c1i = b; c2i = -1; }
    double v = X[c1i + (int64_t)a * ld] * pz[b + 2 * ldz];
    if (c2i >= 0) v += X[c2i + (int64_t)a * ld] * pz[b + 3 * ldz];
    KT[b + (int64_t)((int)pz[a]) * ldk] = v;
  }
}

__global__ void k_zero_clusters(const int* __restrict__ clusters, BufTab bt, int buf) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  double* p = addr(bt, buf, i, s, 0, 0);
  const int64_t n = bt.bs[buf];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = 0.0;
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

// Children skeleton coordinate of parent-order position x for parent p:
// [new c1 (t1) | new c2 (t2) | old c1 (r01) | old c2]; returns the child (0/1)
// and its local skeleton index (new directions first, then old coordinates).
__device__ inline int merge_pos(int x, int t1, int t2, int r01, int* loc) {
  const int tn = t1 + t2;
  if (x < t1) { *loc = x; return 0; }
  if (x < tn) { *loc = x - t1; return 1; }
  if (x < tn + r01) { *loc = t1 + (x - tn); return 0; }
  *loc = t2 + (x - tn - r01);
  return 1;
}

__global__ void k_gather(const GatherItem* __restrict__ items, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const GatherItem g = items[blockIdx.y];
  const int N = sz.N;
  const int p = g.p, q = g.q;
  const int tp1 = sz.t[s * N + 2 * p], tp2 = sz.t[s * N + 2 * p + 1];
  const int tq1 = sz.t[s * N + 2 * q], tq2 = sz.t[s * N + 2 * q + 1];
  const int rp1 = sz.r0[2 * p], rq1 = sz.r0[2 * q];
  const int tnp = tp1 + tp2, tnq = tq1 + tq2;
  const int mp = sz.pm[s * sz.Np + p], mq = sz.pm[s * sz.Np + q];
  double* H = addr(bt, B_HAT, g.out_blk, s, 0, 0);
  const int ldh = bt.ld[B_HAT];
  double* O = addr(bt, g.dst_buf, g.dst_blk, s, 0, 0);
  const int ldo = bt.ld[g.dst_buf];
  const int ldc = bt.ld[B_CPL];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)mp * mq; e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % mp), col = (int)(e / mp);
    int rr, cc;
    const int a = merge_pos(row, tp1, tp2, rp1, &rr);
    const int b = merge_pos(col, tq1, tq2, rq1, &cc);
    const int c = 2 * p + a, d = 2 * q + b;
    const int slot = 2 * a + b;
    const int Rc = sz.R[s * N + c], Rd = sz.R[s * N + d];
    double v = 0.0;
    if (g.src_kind[slot] == 1) v = addr(bt, B_S, g.src_blk[slot], s, Rc + rr, Rd + cc)[0];
    else if (g.src_kind[slot] == 2) v = addr(bt, B_F, g.src_blk[slot], s, Rc + rr, Rd + cc)[0];
    if (g.cpl_blk[slot] >= 0) {
      const int tc = sz.t[s * N + c], td = sz.t[s * N + d];
      if (rr >= tc && cc >= td) v += bt.p[B_CPL][(int64_t)g.cpl_blk[slot] * bt.bs[B_CPL] + (rr - tc) + (int64_t)(cc - td) * ldc];
    }
    if (row < tnp && col < tnq) O[row + (int64_t)col * ldo] = v;
    else H[row + (int64_t)col * ldh] = v;
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
      case GEMM_NN: hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn, i0); break;
      case GEMM_NT: hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn, i0); break;
      case GEMM_TN: hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn, i0); break;
      default: hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, items + i0, terms, bt, sz, tn, i0); break;
    }
  }
}

void launch_copyback(const CopyItem* items, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  for (int i0 = 0; i0 < n; i0 += 65535) {
    int ni = std::min(65535, n - i0);
    hipLaunchKernelGGL(k_copyback, dim3(std::max(1u, cdiv((int64_t)cap * cap, 256 * 8)), ni, nshift), dim3(256), 0, st,
                       items + i0, bt, sz, i0);
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

void launch_pchol_init(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pchol_init, dim3(1, n, nshift), dim3(256), 0, st, clusters, bt, sz);
}

void launch_pchol_panel(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, double tau2, int* more, int cap,
                        int nshift, hipStream_t st) {
  if (n <= 0) return;
  size_t shmem = (size_t)cap * sizeof(double) + RT_THREADS * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(k_pchol_panel, dim3(1, n, nshift), dim3(RT_THREADS), shmem, st, clusters, bt, sz, tau2, more);
}

void launch_pchol_finish(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pchol_finish, dim3(1, n, nshift), dim3(64), 0, st, clusters, bt, sz);
}

void launch_hqr_panel(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int it, int* more, int nshift,
                      hipStream_t st) {
  if (n <= 0) return;
  size_t shmem = (size_t)(8 + HB + HB * HB + HB) * sizeof(double);
  hipLaunchKernelGGL(k_hqr_panel, dim3(1, n, nshift), dim3(RT_THREADS), shmem, st, clusters, bt, sz, it, more);
}

void launch_set_panel(const int* clusters, int n, const SizeTab& sz, int it, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_set_panel, dim3(1, n, nshift), dim3(64), 0, st, clusters, sz, it);
}

void launch_eye(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_eye, dim3(std::max(1u, cdiv((int64_t)cap * cap, 256 * 8)), n, nshift), dim3(256), 0, st, clusters,
                     bt, sz);
}

void launch_ldl_init(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ldl_init, dim3(1, n, nshift), dim3(256), 0, st, clusters, bt, sz);
}

void launch_ldl_panel(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz, int* status,
                      int* more, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ldl_panel, dim3(1, n, nshift), dim3(LDL_THREADS), 0, st, clusters, diag_blk, bt, sz, status, more);
}

void launch_ldl_prep(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz,
                     unsigned long long* nu, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ldl_prep, dim3(1, n, nshift), dim3(LDL_THREADS), 0, st, clusters, diag_blk, bt, sz, nu);
}

void launch_diag_inv(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz, int cap,
                     int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_diag_inv, dim3(cdiv(cap, INV_NB), n, nshift), dim3(128), 0, st, clusters, diag_blk, bt, sz);
}

void launch_set_block(const int* clusters, int n, const SizeTab& sz, int ib, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_set_block, dim3(1, n, nshift), dim3(64), 0, st, clusters, sz, ib);
}

void launch_kform(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_kform, dim3(std::max(1u, cdiv((int64_t)cap * cap, 256 * 4)), n, nshift), dim3(256), 0, st, clusters,
                     bt, sz);
}

void launch_zero_clusters(const int* clusters, int n, const BufTab& bt, int buf, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_clusters, dim3(std::max(1u, cdiv((int64_t)cap * cap, 256 * 8)), n, nshift), dim3(256), 0, st,
                     clusters, bt, buf);
}

int inv_block() { return INV_NB; }

void launch_merge_sizes(const SizeTab& sz, int Np, int nshift, hipStream_t st) {
  hipLaunchKernelGGL(k_merge_sizes, dim3(cdiv(Np, 256), nshift), dim3(256), 0, st, sz, Np);
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
