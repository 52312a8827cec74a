// HIP kernels (gfx950 / CDNA4) of the generalized H^2-LDL inertia path.
//
// Every kernel works on a batch of shifts (blockIdx.z = shift) and on a list
// of static descriptors (blockIdx.y = item); block sizes are resolved per
// shift on the device from the size tables, because the redundant/skeleton
// split of each cluster depends on the shift.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <type_traits>

#include "desc.hpp"
#include "kernels.hpp"

namespace h2 {

// leading dimension of block blk of buffer buf
__device__ inline int ldof(const BufTab& bt, int buf, int blk) { return bt.bld[buf] ? bt.bld[buf][blk] : bt.ld[buf]; }

__device__ inline double* addr(const BufTab& bt, int buf, int blk, int s, int row, int col) {
  const int64_t off = bt.boff[buf] ? bt.boff[buf][blk] : (int64_t)blk * bt.bs[buf];
  return bt.p[buf] + (int64_t)s * bt.ss[buf] + off + row + (int64_t)col * ldof(bt, buf, blk);
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
// K runs in steps of GK through two LDS buffers: the next step's tiles are
// fetched into registers while the current step is multiplied (one barrier
// per step).
// op(A): TA ? A^T (A stored K x M) : A (M x K);  op(B): TB ? B^T (B stored N x K) : B (K x N).
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // output tile of k_gemm (k_gemm128: 128)
constexpr int GK = 16;   // k step

// Per shift, the exclusive prefix sum of the output tiles of every item of a
// list (0 for an item whose guard or sizes are 0): the GEMM below then runs on a
// fixed grid over the real tiles only.
__global__ __launch_bounds__(1024) void k_tile_scan(const GItem* __restrict__ items, int nitems, SizeTab sz,
                                                    int* __restrict__ prefix, int T) {
  __shared__ int wsum[16];
  __shared__ int carry;
  const int s = blockIdx.x;
  int* pre = prefix + (int64_t)s * (nitems + 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nitems; base += 1024) {
    const int i = base + tid;
    int v = 0;
    if (i < nitems) {
      const GItem it = items[i];
      const bool skip = it.guard != -1 && dev_eval(it.guard, sz, s) == 0;
      const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
      v = (skip || M <= 0 || N <= 0) ? 0 : ((M + T - 1) / T) * ((N + T - 1) / T);
    }
    int x = v;   // inclusive scan within the wave
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (tid < 16) {
      int w = wsum[tid];
      for (int d = 1; d < 16; d <<= 1) {
        const int y = __shfl_up(w, d, 64);
        if (tid >= d) w += y;
      }
      wsum[tid] = w;   // inclusive over waves
    }
    __syncthreads();
    const int before = carry + (wave > 0 ? wsum[wave - 1] : 0);
    if (i < nitems) pre[i] = before + x - v;
    __syncthreads();
    if (tid == 0) carry += wsum[15];
    __syncthreads();
  }
  if (tid == 0) pre[nitems] = carry;
}

// The GEMM proper: a fixed grid strides over the tiles counted by k_tile_scan;
// workgroups on one XCD (blockIdx.x % 8) take consecutive tiles, so that tiles
// sharing panels of A or B meet in the same L2.  Operands and results are FP64
// in memory; F32 converts the operands to FP32 on their way into LDS and
// multiplies them on FP32 MFMA with FP32 accumulation (the early bisection
// steps), else everything is FP64.  Output tiles are T x T (64 or 128), WM x WN
// waves (64 x 64: 2 x 2 waves of 32 x 32; 128 x 128: 2 x 4 waves of 64 x 32),
// each wave computing its part as FWM x FWN MFMA blocks of 16 x 16.  Per-K
// weights (the signs of the scaled pivots in the Schur and fill-in products)
// travel through LDS beside the operand tiles and scale the A fragments there:
// applied to the values in flight from global memory they would make every
// slab wait for its loads before the products of the previous slab.
template <bool TA, bool TB, bool F32, int T, int WM, int WN>
__device__ __forceinline__ void gemm_body(const GItem* __restrict__ items, int nitems, const GTerm* __restrict__ terms,
                                          const BufTab& bt, const SizeTab& sz, const int* __restrict__ prefix,
                                          int slot_base) {
  using CT = typename std::conditional<F32, float, double>::type;
  using VT = typename std::conditional<F32, v4f, v4d>::type;
  const int s = blockIdx.z;
  const int* pre = prefix + (int64_t)s * (nitems + 1);
  const int total = pre[nitems];
  const int G = gridDim.x;
  const int lw = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);   // G is a multiple of 8
  constexpr int NT = 64 * WM * WN;  // threads
  constexpr int HM = T / WM;        // rows of a wave's part of the tile
  constexpr int HN = T / WN;        // columns of a wave's part of the tile
  constexpr int FWM = HM / 16;      // MFMA blocks per wave, rows
  constexpr int FWN = HN / 16;      // MFMA blocks per wave, columns
  constexpr int NE = T * GK / NT;   // elements of each operand tile a thread stages
  static_assert(NE * NT == T * GK, "operand tile must split evenly over the threads");
  __shared__ CT ABs[2][2][GK][T + 1];   // [A or B][LDS buffer][k][m or n], one array: the epilogue reuses all of it
  __shared__ CT Ws[2][GK];              // per-K weights of the current term (1 when it has none), per LDS buffer
  CT(&As)[2][GK][T + 1] = ABs[0];
  CT(&Bs)[2][GK][T + 1] = ABs[1];
  for (int tile = lw; tile < total; tile += G) {
  int lo = 0, hi = nitems - 1;   // the item: the last i with pre[i] <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  const int idx = lo;
  const GItem it = items[idx];
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  const int tn = (N + T - 1) / T;
  const int local = tile - pre[idx];
  int mi, ni;
  if (bt.group_m <= 1) {
    mi = local / tn;
    ni = local % tn;
  } else {   // concurrent tiles share group_m row panels and a few column panels
    const int tm = (M + T - 1) / T, gsz = bt.group_m * tn;
    const int g = local / gsz, first = g * bt.group_m, rows = min(tm - first, bt.group_m), r = local - g * gsz;
    mi = first + r % rows;
    ni = r / rows;
  }
  const int m0 = mi * T, n0 = ni * T;
  if (bt.fc && local == 0 && threadIdx.x == 0) {
    unsigned long long kk = 0, kw = 0;
    for (int tt = 0; tt < it.nt; ++tt) {
      const unsigned long long k = (unsigned long long)max(0, dev_eval(terms[it.t0 + tt].K, sz, s));
      kk += k;
      if (terms[it.t0 + tt].wbuf >= 0) kw += k;
    }
    atomicAdd(bt.fc, 2ull * (unsigned long long)M * (unsigned long long)N * kk);
    if (bt.fck) atomicAdd(bt.fck, 2ull * (unsigned long long)M * (unsigned long long)N * kk);
    // the bytes the product must move at least: each operand once, the
    // weights, C written (and read when accumulated), the twin likewise
    if (bt.fbk && kk > 0) {
      const unsigned long long mn = (unsigned long long)M * (unsigned long long)N;
      const unsigned long long outs = (it.beta != 0.0 ? 2ull : 1ull) * (it.c2.buf >= 0 ? 2ull : 1ull);
      atomicAdd(bt.fbk, 8ull * ((unsigned long long)(M + N) * kk + kw + outs * mn));
    }
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  VT acc[FWM][FWN];
  for (int i = 0; i < FWM; ++i)
    for (int j = 0; j < FWN; ++j) acc[i][j] = VT{0, 0, 0, 0};

  for (int tt = 0; tt < it.nt; ++tt) {
    const GTerm tm = terms[it.t0 + tt];
    const int K = dev_eval(tm.K, sz, s);
    if (K <= 0) continue;
    int ar, ac, br, bc;
    ref_origin(tm.a, sz, s, &ar, &ac);
    ref_origin(tm.b, sz, s, &br, &bc);
    const double* A = addr(bt, tm.a.buf, tm.a.blk, s, ar, ac);
    const double* B = addr(bt, tm.b.buf, tm.b.blk, s, br, bc);
    const int lda = ldof(bt, tm.a.buf, tm.a.blk), ldb = ldof(bt, tm.b.buf, tm.b.blk);
    const double* w = tm.wbuf >= 0 ? addr(bt, tm.wbuf, 0, s, 0, 0) + (int64_t)tm.wblk * bt.bs[tm.wbuf] : nullptr;
    const int nk = (K + GK - 1) / GK;
    // this thread's NE elements of each tile: A as (mm, kk), B as (kk, nn); the
    // first GK threads also carry the slab's weights.  Loaded values are only
    // moved into LDS after the products of the current slab, so no arithmetic
    // may depend on them here (it would wait for the loads in flight).
    double ra[NE], rb[NE];
    double rw = 1.0;
    auto gload = [&](int kt) {
      const int k0 = kt * GK;
#pragma unroll
      for (int r = 0; r < NE; ++r) {
        const int e = tid + NT * r;
        int mm, kk;
        if (TA) { kk = e % GK; mm = e / GK; } else { mm = e % T; kk = e / T; }
        const int gm = m0 + mm, gk = k0 + kk;
        double v = 0.0;
        if (gm < M && gk < K) v = TA ? A[gk + (int64_t)gm * lda] : A[gm + (int64_t)gk * lda];
        ra[r] = v;
        int nn, kb;
        if (TB) { nn = e % T; kb = e / T; } else { kb = e % GK; nn = e / GK; }
        const int gn = n0 + nn, gkb = k0 + kb;
        rb[r] = (gn < N && gkb < K) ? (TB ? B[gn + (int64_t)gkb * ldb] : B[gkb + (int64_t)gn * ldb]) : 0.0;
      }
      if (w && tid < GK) rw = k0 + tid < K ? w[k0 + tid] : 0.0;
    };
    auto sstore = [&](int buf) {
#pragma unroll
      for (int r = 0; r < NE; ++r) {
        const int e = tid + NT * r;
        int mm, kk;
        if (TA) { kk = e % GK; mm = e / GK; } else { mm = e % T; kk = e / T; }
        As[buf][kk][mm] = (CT)ra[r];
        int nn, kb;
        if (TB) { nn = e % T; kb = e / T; } else { kb = e % GK; nn = e / GK; }
        Bs[buf][kb][nn] = (CT)rb[r];
      }
      if (tid < GK) Ws[buf][tid] = (CT)rw;
    };
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) gload(kt + 1);   // next tiles in flight during the products
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        const int kr = kk + (lane >> 4);
        CT a[FWM], b[FWN];
#pragma unroll
        for (int f = 0; f < FWM; ++f) a[f] = As[cur][kr][wm * HM + f * 16 + (lane & 15)];
        if (w) {   // uniform: the term's weights
          const CT wk = Ws[cur][kr];
#pragma unroll
          for (int f = 0; f < FWM; ++f) a[f] *= wk;
        }
#pragma unroll
        for (int f = 0; f < FWN; ++f) b[f] = Bs[cur][kr][wn * HN + f * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < FWM; ++i)
#pragma unroll
          for (int j = 0; j < FWN; ++j) {
            if constexpr (F32) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            else acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
          }
      }
      if (kt + 1 < nk) sstore(cur ^ 1);
      __syncthreads();
    }
  }
  int cr, cc;
  ref_origin(it.c, sz, s, &cr, &cc);
  const int cblk = it.c.blk >= 0 ? it.c.blk : idx + slot_base;
  double* C = addr(bt, it.c.buf, cblk, s, 0, 0);
  const int ldc = ldof(bt, it.c.buf, cblk);
  double* C2 = nullptr;
  int ldc2 = 0;
  const bool seg = it.c2.buf == SEG_OUT;
  int rs = M, cs = N, r2o = 0, c2o = 0;
  if (seg) {
    rs = dev_eval(it.rsplit, sz, s);
    cs = dev_eval(it.csplit, sz, s);
    ref_origin(it.c2, sz, s, &r2o, &c2o);
  } else if (it.c2.buf >= 0) {
    int r2, c2;
    ref_origin(it.c2, sz, s, &r2, &c2);
    C2 = addr(bt, it.c2.buf, it.c2.blk, s, r2, c2);
    ldc2 = ldof(bt, it.c2.buf, it.c2.blk);
  }
  {
    // Epilogue through LDS (the operand buffers, free after the last K step):
    // the tile goes to LDS column chunk by column chunk, then every wave reads
    // back whole columns (C, column-major) or whole row segments (the
    // transposed twin C2), so that global reads and writes are contiguous; each
    // thread loads all the old values it updates before it stores any.
    constexpr int CW = F32 ? 32 : 64;                // columns per chunk: the chunk fills the operand buffers
    constexpr int LDT = T + 1;                       // LDS column stride (doubles)
    constexpr int PER = T * CW / NT;                 // elements per thread per chunk
    static_assert(CW * LDT * sizeof(double) <= sizeof(ABs), "chunk must fit in the operand buffers");
    static_assert(PER * NT == T * CW && PER % 8 == 0, "chunk must split evenly over the threads");
    static_assert(NT % T == 0 && NT % CW == 0, "thread mapping of the epilogue");
    double* Ls = reinterpret_cast<double*>(&ABs[0][0][0][0]);
    const double alpha = it.alpha, beta = it.beta;
    for (int cb = 0; cb < T; cb += CW) {
      if (n0 + cb >= N) break;
      // registers -> LDS (local row r, local column c - cb)
      for (int i = 0; i < FWM; ++i)
        for (int j = 0; j < FWN; ++j) {
          const int cl = wn * HN + j * 16 + (lane & 15) - cb;
          if (cl < 0 || cl >= CW) continue;
          for (int v = 0; v < 4; ++v) {
            const int rl = wm * HM + i * 16 + (F32 ? 4 * (lane >> 4) + v : (lane >> 4) + 4 * v);
            Ls[rl + cl * LDT] = alpha * (double)acc[i][j][v];
          }
        }
      __syncthreads();
      // C: consecutive threads take consecutive rows of a column
      {
        // the row is fixed per thread (NT is a multiple of T); the column steps by NT / T
        const int rl = tid % T, r = m0 + rl;
        const int dr = r < rs ? cr + r : r2o + (r - rs);
        constexpr int CSTEP = NT / T;
  #pragma unroll
        for (int h = 0; h < PER; h += 8) {
          double old[8];
  #pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int cl = tid / T + (h + u) * CSTEP, c = n0 + cb + cl;
            old[u] = 0.0;
            if (beta != 0.0 && r < M && c < N) {
              const int dcol = c < cs ? cc + c : c2o + (c - cs);
              old[u] = C[dr + (int64_t)dcol * ldc];
            }
          }
  #pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int cl = tid / T + (h + u) * CSTEP, c = n0 + cb + cl;
            if (r < M && c < N) {
              const int dcol = c < cs ? cc + c : c2o + (c - cs);
              C[dr + (int64_t)dcol * ldc] = beta * old[u] + Ls[rl + cl * LDT];
            }
          }
        }
      }
      // C2 = the tile transposed: consecutive threads take consecutive columns of a row
      if (C2) {
        // the column is fixed per thread (NT is a multiple of CW); the row steps by NT / CW
        const int cl = tid % CW, c = n0 + cb + cl;
        constexpr int RSTEP = NT / CW;
  #pragma unroll
        for (int h = 0; h < PER; h += 8) {
          double old[8];
  #pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int rl = tid / CW + (h + u) * RSTEP, r = m0 + rl;
            old[u] = (beta != 0.0 && r < M && c < N) ? C2[c + (int64_t)r * ldc2] : 0.0;
          }
  #pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int rl = tid / CW + (h + u) * RSTEP, r = m0 + rl;
            if (r < M && c < N) C2[c + (int64_t)r * ldc2] = beta * old[u] + Ls[rl + cl * LDT];
          }
        }
      }
      __syncthreads();
    }
  }
  }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 4) void k_gemm(const GItem* __restrict__ items, int nitems,
                                              const GTerm* __restrict__ terms, BufTab bt, SizeTab sz,
                                              const int* __restrict__ prefix, int slot_base) {
  gemm_body<TA, TB, false, 64, 2, 2>(items, nitems, terms, bt, sz, prefix, slot_base);
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 4) void k_gemm_f32(const GItem* __restrict__ items, int nitems,
                                                  const GTerm* __restrict__ terms, BufTab bt, SizeTab sz,
                                                  const int* __restrict__ prefix, int slot_base) {
  gemm_body<TA, TB, true, 64, 2, 2>(items, nitems, terms, bt, sz, prefix, slot_base);
}

// 128 x 128 output tiles on eight waves: twice the arithmetic per operand byte
// of the 64 x 64 tile, at one resident workgroup per CU, for large blocks
template <bool TA, bool TB>
__global__ __launch_bounds__(512) void k_gemm128(const GItem* __restrict__ items, int nitems,
                                                 const GTerm* __restrict__ terms, BufTab bt, SizeTab sz,
                                                 const int* __restrict__ prefix, int slot_base) {
  gemm_body<TA, TB, false, 128, 2, 4>(items, nitems, terms, bt, sz, prefix, slot_base);
}

template <bool TA, bool TB>
__global__ __launch_bounds__(512) void k_gemm128_f32(const GItem* __restrict__ items, int nitems,
                                                     const GTerm* __restrict__ terms, BufTab bt, SizeTab sz,
                                                     const int* __restrict__ prefix, int slot_base) {
  gemm_body<TA, TB, true, 128, 2, 4>(items, nitems, terms, bt, sz, prefix, slot_base);
}

// Transposed copy of a scratch slot, or of a source block, into a block:
// X[r0 + a][c0 + b] = SRC[b][a] (a < M, b < N), through 64x64 LDS tiles so
// that both sides are coalesced.
__global__ __launch_bounds__(256) void k_copyback_t(const CopyItem* __restrict__ items, BufTab bt, SizeTab sz,
                                                    int slot_base) {
  __shared__ double tile[64][65];
  const int s = blockIdx.z;
  const CopyItem it = items[blockIdx.y];
  if (it.guard != -1 && dev_eval(it.guard, sz, s) == 0) return;
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  if (M <= 0 || N <= 0) return;
  int r0, c0;
  ref_origin(it.x, sz, s, &r0, &c0);
  double* X = addr(bt, it.x.buf, it.x.blk, s, r0, c0);
  const int ldx = ldof(bt, it.x.buf, it.x.blk);
  const double* Sc;
  int lds;
  if (it.src.buf >= 0) {   // from a block
    int sr, sc;
    ref_origin(it.src, sz, s, &sr, &sc);
    Sc = addr(bt, it.src.buf, it.src.blk, s, sr, sc);
    lds = ldof(bt, it.src.buf, it.src.blk);
  } else {                 // from the item's scratch slot
    Sc = addr(bt, B_RS, (int)blockIdx.y + slot_base, s, 0, 0);
    lds = bt.ld[B_RS];
  }
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  for (int t = blockIdx.x; t < tm * tn; t += gridDim.x) {
    const int a0 = (t % tm) * 64, b0 = (t / tm) * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {   // source rows are the destination's columns
      const int j = e % 64, i = e / 64;
      if (a0 + i < M && b0 + j < N) tile[i][j] = Sc[(b0 + j) + (int64_t)(a0 + i) * lds];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int i = e % 64, j = e / 64;
      if (a0 + i < M && b0 + j < N) X[(a0 + i) + (int64_t)(b0 + j) * ldx] = tile[i][j];
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------- matrix sums
__global__ void k_matsum(const SumItem* __restrict__ items, const int* __restrict__ src, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const SumItem it = items[blockIdx.y];
  const int M = dev_eval(it.M, sz, s), N = dev_eval(it.N, sz, s);
  double* C = addr(bt, it.cbuf, it.cblk, s, 0, 0);
  const int ldc = ldof(bt, it.cbuf, it.cblk);
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
  const int ldx = ldof(bt, it.x.buf, it.x.blk);
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
constexpr int INV_NB = 64;    // block size of the blocked triangular inverses
constexpr int PC_NB = PCHOL_NB;
constexpr int HB = HQR_NB;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Butterfly reduce-scatter of 64 per-lane values over a wave: afterwards lane L
// holds the wave sum of v[L] in v[0] (63 exchanges instead of 64 x 6).
template <int OFF>
__device__ inline void rs_step(double (&v)[64], int lane) {
  const bool up = (lane & OFF) != 0;
#pragma unroll
  for (int m = 0; m < OFF; ++m) {
    const double keep = up ? v[m + OFF] : v[m];
    const double send = up ? v[m] : v[m + OFF];
    v[m] = keep + __shfl_xor(send, OFF, 64);
  }
}

__device__ inline void wave_reduce_scatter64(double (&v)[64], int lane) {
  rs_step<32>(v, lane);
  rs_step<16>(v, lane);
  rs_step<8>(v, lane);
  rs_step<4>(v, lane);
  rs_step<2>(v, lane);
  rs_step<1>(v, lane);
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
// panels; columns of this panel are formed from G and the panel's own columns:
// column t = (G[:, p] - V[:, t0:t] V[p, t0:t]^T) / sqrt(d_p), taken four rows
// x eight columns of independent loads at a time.
constexpr int PC_THREADS = 1024;

__global__ __launch_bounds__(PC_THREADS) void k_pchol_panel(const int* __restrict__ clusters, BufTab bt, SizeTab sz,
                                                            const double* __restrict__ tau2c, int* __restrict__ more) {
  extern __shared__ double sh[];
  __shared__ double vp[PC_NB];               // V[p, t0 + l], zero beyond the panel's columns
  __shared__ double redv[PC_THREADS / 64];
  __shared__ double reds[PC_THREADS / 64];
  __shared__ int redi[PC_THREADS / 64];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const double tau2 = tau2c[i];
  const int N = sz.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  for (int a = tid; a < R; a += PC_THREADS) d[a] = dg[a];
  if (tid < PC_NB) vp[tid] = 0.0;
  __syncthreads();
  const int t0 = sz.t[s * N + i];
  int t = t0;
  bool stop = false;
  for (int j = 0; j < PC_NB && t < R; ++j) {
    // pivot: largest remaining diagonal, first index on ties; stop once the
    // remaining diagonal (the squared Frobenius norm of the part of the
    // fill-in not yet spanned) sums to <= tau2
    double bv = -INFINITY, sum = 0.0;
    int bi = R;
    for (int a = tid; a < R; a += PC_THREADS) {
      const double v = d[a];
      if (v != -INFINITY) sum += v;
      if (v > bv) { bv = v; bi = a; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      sum += __shfl_xor(sum, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { redv[wave] = bv; redi[wave] = bi; reds[wave] = sum; }
    __syncthreads();
    double dmax = redv[0], rem = reds[0];
    int p = redi[0];
    for (int w2 = 1; w2 < PC_THREADS / 64; ++w2) {
      rem += reds[w2];
      if (redv[w2] > dmax || (redv[w2] == dmax && redi[w2] < p)) { dmax = redv[w2]; p = redi[w2]; }
    }
    if (!(rem > tau2) || !(dmax > 0.0)) {
      stop = true;
      break;
    }
    const int jw = t - t0;
    if (tid < jw) vp[tid] = V[p + (int64_t)(t0 + tid) * ld];
    __syncthreads();
    const double sq = sqrt(dmax), inv = 1.0 / sq;
    for (int ab = tid; ab < R; ab += 4 * PC_THREADS) {
      int ar[4];
      bool live[4];
      double acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ar[u] = ab + u * PC_THREADS;
        live[u] = ar[u] < R && ar[u] != p && d[ar[u]] != -INFINITY;
        acc[u] = live[u] ? G[ar[u] + (int64_t)p * ld] : 0.0;
      }
      for (int l0 = 0; l0 < jw; l0 += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int col = t0 + min(l0 + q, jw - 1);   // vp = 0 beyond jw
          const double c = vp[min(l0 + q, PC_NB - 1)] * (l0 + q < jw ? 1.0 : 0.0);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (ar[u] < R) acc[u] -= V[ar[u] + (int64_t)col * ld] * c;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = ar[u];
        if (a < R) {
          double v = 0.0;
          if (a == p) {
            v = sq;
            d[a] = -INFINITY;
          } else if (live[u]) {
            v = acc[u] * inv;
            d[a] -= v * v;
          }
          V[a + (int64_t)t * ld] = v;
        }
      }
    }
    __syncthreads();
    ++t;
  }
  for (int a = tid; a < R; a += PC_THREADS) dg[a] = d[a];
  if (tid == 0) {
    sz.t[s * N + i] = t;
    sz.a0[s * N + i] = t0;
    const bool go = !stop && t < R;
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
    sz.a0[s * N + i] = 0;   // panel state of the Householder QR that follows
    sz.a1[s * N + i] = 0;
    if (bt.fc) atomicAdd(bt.fc, (unsigned long long)R * (unsigned long long)t * (unsigned long long)(t > 0 ? t - 1 : 0));
  }
}

constexpr int HQ_THREADS = 512;
constexpr int HQ_LDS = 16384;   // doubles of LDS holding the panel (RT x width)

// Panel width by the number of rows, so that the panel fits in LDS.
__host__ __device__ inline int hqr_width(int RT) { return RT <= 2048 ? 8 : RT <= 4096 ? 4 : RT <= 8192 ? 2 : 1; }

// One Householder panel of HW columns held in LDS (Ys, column j at Ys + j*LR,
// rows 0..P0 = RT-1-k0: everything the panel's reflectors touch).  One pass
// over the rows per column: it applies the previous reflector and, on the
// updated values, accumulates the norm and the dot products defining the next
// reflector together with y_j . y_{k-1} (a column of T_p, the UT transform
// T_p^{-1} = striu(Y_p^T Y_p) + diag(1/beta)); one block reduction per column.
template <int HW>
__device__ void hqr_lds_panel(double* __restrict__ V, double* __restrict__ Yt, double* __restrict__ beta, int ld, int RT,
                              int k0, int nb, double* Ys, double (*red)[64], double* sums, double* wv, double* rowp,
                              double* Tp, double* bp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P0 = RT - 1 - k0, LR = P0 + 1;
  for (int e0 = 0; e0 < nb * LR; e0 += 8 * HQ_THREADS) {   // eight independent loads in flight per thread
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * HQ_THREADS + tid;
      const int j = e / LR, a = e - j * LR;
      x[u] = e < nb * LR ? V[a + (int64_t)(k0 + j) * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * HQ_THREADS + tid;
      if (e < nb * LR) Ys[e] = x[u];
    }
  }
  __syncthreads();
  double v0prev = 0.0;
  int pprev = -1;
  for (int kk = 0; kk <= nb; ++kk) {
    const int pcur = kk < nb ? P0 - kk : -1;
    const int plim = kk > 0 ? pprev : pcur;
    const double wk = kk < nb ? wv[kk] : 0.0;
    double acc[2 * HW];   // [0, HW): x . V_j    [HW, 2HW): y_j . y_{kk-1}
#pragma unroll
    for (int jj = 0; jj < 2 * HW; ++jj) acc[jj] = 0.0;
    for (int a = tid; a <= plim; a += HQ_THREADS) {
      double vals[HW];
#pragma unroll
      for (int jj = 0; jj < HW; ++jj) vals[jj] = jj < nb ? Ys[jj * LR + a] : 0.0;
      double ym = kk > 0 ? Ys[(kk - 1) * LR + a] : 0.0;
      if (a == pprev) ym = v0prev;
      const double xk = (kk < nb && a <= pcur) ? Ys[kk * LR + a] - ym * wk : 0.0;
      const bool anchor = a == pcur;
#pragma unroll
      for (int jj = 0; jj < HW; ++jj) {
        if (jj < nb) {
          const double v = vals[jj] - ym * wv[jj];   // wv[jj] = 0 outside (kk-1, nb)
          if (kk > 0) Ys[jj * LR + a] = v;
          acc[jj] += xk * v;
          acc[HW + jj] += ym * v;
          if (anchor) rowp[jj] = v;
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < 2 * HW; ++jj) {
      const double v = wave_sum(acc[jj]);
      if (lane == 0) red[wave][jj] = v;
    }
    __syncthreads();
    if (tid < 2 * HW) {
      double v = 0.0;
      for (int w2 = 0; w2 < HQ_THREADS / 64; ++w2) v += red[w2][tid];
      sums[tid] = v;
    }
    __syncthreads();
    if (kk > 0) {   // column kk-1 of T_p from g_m = y_m . y_{kk-1}
      const int c = kk - 1;
      if (tid < c) {
        double v = 0.0;
        for (int m = tid; m < c; ++m) v += Tp[tid + m * HB] * sums[HW + m];
        Tp[tid + c * HB] = -bp[c] * v;
      } else if (tid == c) {
        Tp[c + c * HB] = bp[c];
      }
    }
    double v0 = 0.0;
    if (kk < nb) {
      const double xn2 = sums[kk];
      const double x0 = rowp[kk];
      const double xn = sqrt(xn2);
      const double alpha = -copysign(xn, x0 != 0.0 ? x0 : 1.0);
      v0 = x0 - alpha;
      const double vn = xn2 - x0 * x0 + v0 * v0;
      const double bk = vn > 0.0 ? 2.0 / vn : 0.0;
      __syncthreads();   // every thread has read wv / rowp of this step
      if (tid < HW) wv[tid] = (tid > kk && tid < nb) ? bk * (sums[tid] - alpha * rowp[tid]) : 0.0;
      if (tid == 0) {
        Ys[kk * LR + pcur] = v0;
        bp[kk] = bk;
        beta[k0 + kk] = bk;
      }
    }
    v0prev = v0;
    pprev = pcur;
    __syncthreads();
  }
  // the reflectors back to V (zero below their anchors: those rows hold R
  // entries), and Yt = Y_p T_p^T (RT x nb) to B_Z columns k0 .. k0+nb-1
  for (int a = tid; a < RT; a += HQ_THREADS) {
    double y[HW];
#pragma unroll
    for (int jj = 0; jj < HW; ++jj) y[jj] = (jj < nb && a <= P0 - jj) ? Ys[jj * LR + a] : 0.0;
#pragma unroll
    for (int jj = 0; jj < HW; ++jj)
      if (jj < nb) V[a + (int64_t)(k0 + jj) * ld] = y[jj];
#pragma unroll
    for (int c = 0; c < HW; ++c) {
      if (c < nb) {
        double v = 0.0;
#pragma unroll
        for (int b2 = c; b2 < HW; ++b2) v += y[b2] * Tp[c + b2 * HB];   // T^T[b2][c] = T[c][b2]
        Yt[a + (int64_t)(k0 + c) * ld] = v;
      }
    }
  }
}

// Next Householder panel of every cluster of a colour class: columns
// k0 = a0 + a1 .. k0 + nb - 1 of V (RT x t), nb = hqr_width(RT) or what is left.
// Sets a0 = k0, a1 = nb for the trailing update (a1 = 0 when done); beta goes
// to B_SIGN (used to form W afterwards).
__global__ __launch_bounds__(HQ_THREADS) void k_hqr_panel(const int* __restrict__ clusters, BufTab bt, SizeTab sz, int it,
                                                          int* __restrict__ more) {
  __shared__ double Ys[HQ_LDS];
  __shared__ double red[HQ_THREADS / 64][64];
  __shared__ double sums[64];
  __shared__ double wv[HB];
  __shared__ double rowp[HB];
  __shared__ double Tp[HB * HB];
  __shared__ double bp[HB];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int t = sz.t[s * N + i];
  const int k0 = sz.a0[s * N + i] + sz.a1[s * N + i];
  const int tid = threadIdx.x;
  if (k0 >= t) {
    if (tid == 0) { sz.a0[s * N + i] = k0; sz.a1[s * N + i] = 0; }
    return;
  }
  const int RT = sz.R[s * N + i] + t;
  const int hw = hqr_width(RT);
  const int nb = min(hw, t - k0);
  if (bt.fc && tid == 0) {   // Householder QR flops of this panel's columns
    double f = 0.0;
    for (int k = k0; k < k0 + nb; ++k) f += 4.0 * (double)(RT - k) * (double)(t - k);
    atomicAdd(bt.fc, (unsigned long long)f);
  }
  const int ld = bt.ld[B_V];
  double* V = addr(bt, B_V, i, s, 0, 0);
  double* Yt = addr(bt, B_Z, i, s, 0, 0);
  double* beta = addr(bt, B_SIGN, 0, s, 0, 0) + (int64_t)i * bt.bs[B_SIGN];
  for (int e = tid; e < HB * HB; e += HQ_THREADS) Tp[e] = 0.0;
  if (tid < HB) { wv[tid] = 0.0; rowp[tid] = 0.0; bp[tid] = 0.0; }
  __syncthreads();
  if (RT <= HQ_LDS) {
    if (hw == 8) hqr_lds_panel<8>(V, Yt, beta, ld, RT, k0, nb, Ys, red, sums, wv, rowp, Tp, bp);
    else if (hw == 4) hqr_lds_panel<4>(V, Yt, beta, ld, RT, k0, nb, Ys, red, sums, wv, rowp, Tp, bp);
    else if (hw == 2) hqr_lds_panel<2>(V, Yt, beta, ld, RT, k0, nb, Ys, red, sums, wv, rowp, Tp, bp);
    else hqr_lds_panel<1>(V, Yt, beta, ld, RT, k0, nb, Ys, red, sums, wv, rowp, Tp, bp);
  }
  __syncthreads();
  if (tid == 0) {
    sz.a0[s * N + i] = k0;
    sz.a1[s * N + i] = nb;
    if (k0 + nb < t) atomicAdd(more, 1);
  }
}

// Trailing update after a Householder panel: V[:, a0+a1 : t] <- H_p^T V (H_p
// the panel's block reflector I - Y_p T_p Y_p^T), i.e. V -= Yt (Y_p^T V) with
// Yt = Y_p T_p^T in B_Z.  A workgroup owns HQA_CW trailing columns: one pass over
// the rows for Z = Y_p^T V (butterfly reduction), one pass for V -= Yt Z.  Rows
// below RT-1-a0 are outside the panel's reflectors and untouched.
constexpr int HQA_CW = 8;

__global__ __launch_bounds__(256) void k_hqr_apply(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  __shared__ double red[4][64];
  __shared__ double Zs[64];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  const int a1 = sz.a1[s * N + i];
  if (a1 == 0) return;
  const int t = sz.t[s * N + i], a0 = sz.a0[s * N + i];
  const int j0 = a0 + a1 + blockIdx.x * HQA_CW;
  if (j0 >= t) return;
  const int cw = min(HQA_CW, t - j0);
  const int RT = sz.R[s * N + i] + t;
  const int P = RT - 1 - a0;
  const int ld = bt.ld[B_V];
  double* V = addr(bt, B_V, i, s, 0, 0);
  const double* Yt = addr(bt, B_Z, i, s, 0, 0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc[64];   // acc[k*8 + j] = sum_a Y[a, a0+k] V[a, j0+j]
#pragma unroll
  for (int q = 0; q < 64; ++q) acc[q] = 0.0;
  for (int a = tid; a <= P; a += 256) {
    double y[8], v[8];
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) y[k2] = k2 < a1 ? V[a + (int64_t)(a0 + k2) * ld] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j < cw ? V[a + (int64_t)(j0 + j) * ld] : 0.0;
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[k2 * 8 + j] += y[k2] * v[j];
  }
  wave_reduce_scatter64(acc, lane);
  red[wave][lane] = acc[0];
  __syncthreads();
  if (tid < 64) Zs[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  __syncthreads();
  for (int a = tid; a <= P; a += 256) {
    double yt[8], v[8];
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) yt[k2] = k2 < a1 ? Yt[a + (int64_t)(a0 + k2) * ld] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j < cw ? V[a + (int64_t)(j0 + j) * ld] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      double d = 0.0;
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) d += yt[k2] * Zs[k2 * 8 + j];
      if (j < cw) V[a + (int64_t)(j0 + j) * ld] = v[j] - d;
    }
  }
  if (bt.fc && blockIdx.x == 0 && tid == 0) {
    const double ntr = (double)(t - a0 - a1);
    atomicAdd(bt.fc, (unsigned long long)(4.0 * (double)(P + 1) * (double)a1 * ntr));
  }
}

// ---- W = H_0 ... H_{t-1} = I - Y T Y^T by the UT transform: T^{-1} = S with
// S = striu(Y^T Y) + diag(1/beta).  S (t x t, from a GEMM) is in B_G; T is
// formed in B_Z by a blocked upper-triangular inverse (diagonal blocks here,
// block columns by GEMMs), then U = Y T and W = I - U Y^T on the matrix cores.
__global__ void k_ut_prep(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int t = sz.t[s * sz.N + i];
  double* S = addr(bt, B_G, i, s, 0, 0);
  double* T = addr(bt, B_Z, i, s, 0, 0);
  const int ld = bt.ld[B_G], ldt = bt.ld[B_Z];
  const double* beta = addr(bt, B_SIGN, 0, s, 0, 0) + (int64_t)i * bt.bs[B_SIGN];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)t * t; e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % t), b = (int)(e / t);
    if (a > b) S[a + (int64_t)b * ld] = 0.0;
    else if (a == b) S[a + (int64_t)b * ld] = beta[a] != 0.0 ? 1.0 / beta[a] : 1.0;   // beta = 0: H = I, y = 0
    T[a + (int64_t)b * ldt] = 0.0;
  }
}

__global__ __launch_bounds__(64) void k_ut_diag_inv(const int* __restrict__ clusters, BufTab bt, SizeTab sz) {
  __shared__ double Ss[INV_NB][INV_NB + 1];
  __shared__ double Ts[INV_NB][INV_NB + 1];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int t = sz.t[s * sz.N + i];
  const int r0 = blockIdx.x * INV_NB;
  if (r0 >= t) return;
  const int nb = min(INV_NB, t - r0);
  const double* S = addr(bt, B_G, i, s, r0, r0);
  double* T = addr(bt, B_Z, i, s, r0, r0);
  const int ld = bt.ld[B_G], ldt = bt.ld[B_Z];
  const int c = threadIdx.x;
  for (int b2 = 0; b2 < nb; ++b2)
    if (c < nb) { Ss[c][b2] = S[c + (int64_t)b2 * ld]; Ts[c][b2] = 0.0; }
  __syncthreads();
  if (c < nb) {   // column c of the upper inverse, by back substitution
    Ts[c][c] = 1.0 / Ss[c][c];
    for (int a = c - 1; a >= 0; --a) {
      double v = 0.0;
      for (int b2 = a + 1; b2 <= c; ++b2) v += Ss[a][b2] * Ts[b2][c];
      Ts[a][c] = -v / Ss[a][a];
    }
  }
  __syncthreads();
  for (int b2 = 0; b2 < nb; ++b2)
    if (c < nb) T[c + (int64_t)b2 * ldt] = Ts[c][b2];
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

// out[a] = A[a, col] - sum_{c < jw} A[a, k0 + c] wr[c] for a in [lo, R): a column
// brought up to date from the panel (wr = the pivot's row of W_p, in LDS), four
// rows x eight columns of independent loads at a time.
__device__ inline void ldl_lazy_col(const double* __restrict__ A, int ld, int col, int k0, int jw, int lo, int R,
                                    double* __restrict__ out, const double* wr, int tid) {
  for (int ab = lo + tid; ab < R; ab += 4 * LDL_THREADS) {
    int ar[4];
    double acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ar[u] = ab + u * LDL_THREADS;
      acc[u] = ar[u] < R ? A[ar[u] + (int64_t)col * ld] : 0.0;
    }
    for (int l0 = 0; l0 < jw; l0 += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int cidx = k0 + min(l0 + q, jw - 1);
        const double c = l0 + q < jw ? wr[min(l0 + q, LDL_NB - 1)] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (ar[u] < R) acc[u] -= A[ar[u] + (int64_t)cidx * ld] * c;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ar[u] < R) out[ar[u]] = acc[u];
  }
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
  const int ld = ldof(bt, B_S, diag_blk[i]);  // the pivot block
  const int ldw = bt.ld[B_W], ldz = bt.ld[B_Z];
  double* A = addr(bt, B_S, diag_blk[i], s, 0, 0);
  double* Wp = addr(bt, B_W, i, s, 0, 0);     // panel W = L D columns, LDL_NB + 2 columns
  double* pz = addr(bt, B_Z, i, s, 0, 0);     // perm (col 0), pivot sizes (col 1)
  const int cap = ldw;                        // the level's capacity: the panel width the host plans with
  __shared__ double red[16];
  __shared__ int redi[16];
  __shared__ int s_bad;
  __shared__ double wr[LDL_NB];
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  const int NB = min(LDL_NB, cap - 2);
  if (tid == 0) s_bad = 0;
  __syncthreads();
  const int k0 = kstart;
  int k = k0, jw = 0;
  while (jw < NB && k < R) {
    double* w = Wp + (int64_t)jw * ldw;
    double* u = Wp + (int64_t)(jw + 1) * ldw;
    if (tid < jw) wr[tid] = Wp[k + (int64_t)tid * ldw];
    __syncthreads();
    ldl_lazy_col(A, ld, k, k0, jw, k, R, w, wr, tid);
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
      if (tid < jw) wr[tid] = Wp[imax + (int64_t)tid * ldw];
      __syncthreads();
      ldl_lazy_col(A, ld, imax, k0, jw, k, R, u, wr, tid);
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
        double x = Wp[kk + (int64_t)c * ldw];
        Wp[kk + (int64_t)c * ldw] = Wp[kp + (int64_t)c * ldw];
        Wp[kp + (int64_t)c * ldw] = x;
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
        pz[k + ldz] = 1.0;
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
        pz[k + ldz] = 2.0;
        pz[k + 1 + ldz] = 0.0;
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
  const int ld = ldof(bt, B_S, diag_blk[i]);
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

__global__ __launch_bounds__(64) void k_diag_inv(const int* __restrict__ clusters, const int* __restrict__ diag_blk,
                                                 BufTab bt, SizeTab sz) {
  __shared__ double Ls[INV_NB][INV_NB + 1];
  __shared__ double Xs[INV_NB][INV_NB + 1];
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int R = sz.R[s * sz.N + i];
  const int r0 = blockIdx.x * INV_NB;
  if (r0 >= R) return;
  const int nb = min(INV_NB, R - r0);
  const int ld = ldof(bt, B_S, diag_blk[i]);
  const double* A = addr(bt, B_S, diag_blk[i], s, r0, r0);
  double* X = addr(bt, B_V, i, s, r0, r0);
  const int ldx = bt.ld[B_V];
  const int c = threadIdx.x;
  for (int b2 = 0; b2 < nb; ++b2)
    if (c < nb) { Ls[c][b2] = A[c + (int64_t)b2 * ld]; Xs[c][b2] = 0.0; }
  __syncthreads();
  if (c < nb) {   // column c of the unit lower inverse, by forward substitution
    Xs[c][c] = 1.0;
    for (int a = c + 1; a < nb; ++a) {
      double v = 0.0;
      for (int b2 = c; b2 < a; ++b2) v -= Ls[a][b2] * Xs[b2][c];
      Xs[a][c] = v;
    }
  }
  __syncthreads();
  for (int b2 = 0; b2 < nb; ++b2)
    if (c < nb) X[c + (int64_t)b2 * ldx] = Xs[c][b2];
}

// panel state for block ib of a blocked inverse: a0 = ib*INV_NB, a1 = its width (0 beyond R, or t)
__global__ void k_set_block(const int* __restrict__ clusters, SizeTab sz, int ib, int use_t) {
  const int s = blockIdx.z;
  const int i = clusters[blockIdx.y];
  const int N = sz.N;
  if (threadIdx.x == 0) {
    const int R = use_t ? sz.t[s * N + i] : sz.R[s * N + i], a0 = ib * INV_NB;
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
  const int mp = sz.pm[s * sz.Np + p], mq = sz.pm[s * sz.Np + q];
  double* H = addr(bt, B_HAT, g.out_blk, s, 0, 0);
  const int ldh = bt.ld[B_HAT];
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
    else if (g.src_kind[slot] == 3) v = addr(bt, B_F, g.src_blk[slot], s, Rd + cc, Rc + rr)[0];
    if (g.cpl_blk[slot] >= 0) {
      const int tc = sz.t[s * N + c], td = sz.t[s * N + d];
      if (rr >= tc && cc >= td) v += bt.p[B_CPL][(int64_t)g.cpl_blk[slot] * bt.bs[B_CPL] + (rr - tc) + (int64_t)(cc - td) * ldc];
    }
    H[row + (int64_t)col * ldh] = v;
  }
}

// The new-new part of a merged parent block is final once the fill-in is in:
// out[0:tn_p, 0:tn_q] = HAT[0:tn_p, 0:tn_q].
__global__ void k_merge_nn(const GatherItem* __restrict__ items, BufTab bt, SizeTab sz) {
  const int s = blockIdx.z;
  const GatherItem g = items[blockIdx.y];
  const int N = sz.N;
  const int tnp = sz.t[s * N + 2 * g.p] + sz.t[s * N + 2 * g.p + 1];
  const int tnq = sz.t[s * N + 2 * g.q] + sz.t[s * N + 2 * g.q + 1];
  const double* H = addr(bt, B_HAT, g.out_blk, s, 0, 0);
  const int ldh = bt.ld[B_HAT];
  double* O = addr(bt, g.dst_buf, g.dst_blk, s, 0, 0);
  const int ldo = ldof(bt, g.dst_buf, g.dst_blk);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)tnp * tnq; e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e % tnp), col = (int)(e / tnp);
    O[row + (int64_t)col * ldo] = H[row + (int64_t)col * ldh];
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

// Gershgorin radii: rad_i = sum_{j != i} |f(|x_i - x_j|)| over all n points
// (X row-major n x dim).  One row per thread; the column points stream through
// LDS in tiles of 256.
template <int KIND>
__global__ __launch_bounds__(256) void k_row_abs_sum(const double* __restrict__ X, int64_t n, int dim, double p0,
                                                     double p1, double* __restrict__ rad) {
  __shared__ double tx[256], ty[256], tz[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (i < n) {
    xi = X[i * dim];
    if (dim > 1) yi = X[i * dim + 1];
    if (dim > 2) zi = X[i * dim + 2];
  }
  double acc = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += 256) {
    __syncthreads();
    const int64_t j = j0 + threadIdx.x;
    tx[threadIdx.x] = j < n ? X[j * dim] : 0.0;
    ty[threadIdx.x] = (j < n && dim > 1) ? X[j * dim + 1] : 0.0;
    tz[threadIdx.x] = (j < n && dim > 2) ? X[j * dim + 2] : 0.0;
    __syncthreads();
    const int jn = (int)min<int64_t>(256, n - j0);
    for (int q = 0; q < jn; ++q) {
      const double dx = xi - tx[q], dy = yi - ty[q], dz = zi - tz[q];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double v = fabs(kf(KIND, p0, p1, r));
      acc += (j0 + q == i) ? 0.0 : v;
    }
  }
  if (i < n) rad[i] = acc;
}

void launch_row_abs_sum(const double* X, int64_t n, int dim, int kind, double p0, double p1, double* rad,
                        hipStream_t st) {
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_row_abs_sum<0>, g, b, 0, st, X, n, dim, p0, p1, rad); break;
    case 1: hipLaunchKernelGGL(k_row_abs_sum<1>, g, b, 0, st, X, n, dim, p0, p1, rad); break;
    case 2: hipLaunchKernelGGL(k_row_abs_sum<2>, g, b, 0, st, X, n, dim, p0, p1, rad); break;
    case 3: hipLaunchKernelGGL(k_row_abs_sum<3>, g, b, 0, st, X, n, dim, p0, p1, rad); break;
    default: hipLaunchKernelGGL(k_row_abs_sum<4>, g, b, 0, st, X, n, dim, p0, p1, rad); break;
  }
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

// GEMM launch parameters by operand layout, precision and capacity bucket
// (largest block dimension <= 256, 512, 1024, 2048, larger): workgroups per
// shift, tile order and tile size.  The defaults come from a sweep of square
// batches on gfx950 (grid 2048/4096/2048/1024/1024, row-by-row tile order,
// 64 x 64 tiles); the autotuner's table overrides them.  Process-wide; atomics
// because concurrent factorizations read it.
namespace {
constexpr int kDefaultGrid[GEMM_BUCKETS] = {2048, 4096, 2048, 1024, 1024};
std::atomic<int> g_tune_grid[4][2][GEMM_BUCKETS];    // 0 = default
std::atomic<int> g_tune_group[4][2][GEMM_BUCKETS];   // 0 = row by row
std::atomic<int> g_tune_tile[4][2][GEMM_BUCKETS];    // 0 = 64

template <bool TA, bool TB>
void launch_variant(int f32, int T, dim3 grid, const GItem* items, int nitems, const GTerm* terms, const BufTab& bt,
                    const SizeTab& sz, int* prefix, hipStream_t st) {
  if (T == 128) {
    if (f32) hipLaunchKernelGGL((k_gemm128_f32<TA, TB>), grid, dim3(512), 0, st, items, nitems, terms, bt, sz, prefix, 0);
    else hipLaunchKernelGGL((k_gemm128<TA, TB>), grid, dim3(512), 0, st, items, nitems, terms, bt, sz, prefix, 0);
  } else {
    if (f32) hipLaunchKernelGGL((k_gemm_f32<TA, TB>), grid, dim3(256), 0, st, items, nitems, terms, bt, sz, prefix, 0);
    else hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, st, items, nitems, terms, bt, sz, prefix, 0);
  }
}
}  // namespace

int gemm_bucket(int cap) { return cap <= 256 ? 0 : cap <= 512 ? 1 : cap <= 1024 ? 2 : cap <= 2048 ? 3 : 4; }

void set_gemm_tuning(int layout, int f32, int bucket, int grid, int group_m, int tile) {
  g_tune_grid[layout][f32][bucket].store(grid);
  g_tune_group[layout][f32][bucket].store(group_m);
  g_tune_tile[layout][f32][bucket].store(tile);
}

void get_gemm_tuning(int layout, int f32, int bucket, int* grid, int* group_m, int* tile) {
  const int g = g_tune_grid[layout][f32][bucket].load();
  *grid = g > 0 ? g : kDefaultGrid[bucket];
  *group_m = std::max(1, g_tune_group[layout][f32][bucket].load());
  *tile = g_tune_tile[layout][f32][bucket].load() == 128 ? 128 : 64;
}

void launch_gemm(int kind, const GItem* items, int nitems, const GTerm* terms, const BufTab& bt_in, const SizeTab& sz,
                 int mcap, int ncap, int nshift, int* prefix, hipStream_t st) {
  BufTab bt = bt_in;
  if (bt.grid <= 0)   // launch parameters from the tuning table
    get_gemm_tuning(kind, bt.f32 ? 1 : 0, gemm_bucket(std::max(mcap, ncap)), &bt.grid, &bt.group_m, &bt.tile);
  const int T = bt.tile == 128 ? 128 : 64;
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_tile_scan, dim3(nshift), dim3(1024), 0, st, items, nitems, sz, prefix, T);
  // a fixed grid, no larger than the tiles the capacities allow (multiple of 8)
  const int64_t upper = (int64_t)nitems * cdiv(mcap, T) * cdiv(ncap, T);
  const int G = (int)std::max<int64_t>(8, std::min<int64_t>(bt.grid, (upper + 7) / 8 * 8));
  const dim3 grid(G, 1, nshift);
  const int f32 = bt.f32 ? 1 : 0;
  switch (kind) {
    case GEMM_NN: launch_variant<false, false>(f32, T, grid, items, nitems, terms, bt, sz, prefix, st); break;
    case GEMM_NT: launch_variant<false, true>(f32, T, grid, items, nitems, terms, bt, sz, prefix, st); break;
    case GEMM_TN: launch_variant<true, false>(f32, T, grid, items, nitems, terms, bt, sz, prefix, st); break;
    default: launch_variant<true, true>(f32, T, grid, items, nitems, terms, bt, sz, prefix, st); break;
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

void launch_copyback_t(const CopyItem* items, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st) {
  if (n <= 0) return;
  for (int i0 = 0; i0 < n; i0 += 65535) {
    int ni = std::min(65535, n - i0);
    hipLaunchKernelGGL(k_copyback_t, dim3(16, ni, nshift), dim3(256), 0, st, items + i0, bt, sz, i0);
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

void launch_pchol_panel(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, const double* tau2c, int* more,
                        int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  size_t shmem = (size_t)cap * sizeof(double);
  hipLaunchKernelGGL(k_pchol_panel, dim3(1, n, nshift), dim3(PC_THREADS), shmem, st, clusters, bt, sz, tau2c, more);
}

void launch_pchol_finish(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pchol_finish, dim3(1, n, nshift), dim3(64), 0, st, clusters, bt, sz);
}

void launch_hqr_panel(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int it, int* more, int nshift,
                      hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_hqr_panel, dim3(1, n, nshift), dim3(HQ_THREADS), 0, st, clusters, bt, sz, it, more);
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
  hipLaunchKernelGGL(k_diag_inv, dim3(cdiv(cap, INV_NB), n, nshift), dim3(64), 0, st, clusters, diag_blk, bt, sz);
}

void launch_set_block(const int* clusters, int n, const SizeTab& sz, int ib, int use_t, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_set_block, dim3(1, n, nshift), dim3(64), 0, st, clusters, sz, ib, use_t);
}

void launch_ut_prep(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ut_prep, dim3(std::max(1u, cdiv((int64_t)cap * cap, 256 * 8)), n, nshift), dim3(256), 0, st,
                     clusters, bt, sz);
}

void launch_ut_diag_inv(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift,
                        hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ut_diag_inv, dim3(cdiv(cap, INV_NB), n, nshift), dim3(64), 0, st, clusters, bt, sz);
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

void launch_hqr_apply(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int tmax, int nshift, hipStream_t st) {
  if (n <= 0 || tmax <= 0) return;
  hipLaunchKernelGGL(k_hqr_apply, dim3(cdiv(tmax, HQA_CW), n, nshift), dim3(256), 0, st, clusters, bt, sz);
}
int hqr_max_rows() { return HQ_LDS; }
int ldl_panel_min(int cap) { return std::max(1, std::min(LDL_NB, cap - 2)); }

__global__ void k_colour_max(const int* __restrict__ clusters, int n, SizeTab sz, int* __restrict__ out) {
  const int s = blockIdx.y;
  int tm = 0, rm = 0, pm = 0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int i = clusters[c];
    const int t = sz.t[s * sz.N + i], R = sz.R[s * sz.N + i];
    tm = max(tm, t);
    rm = max(rm, R);
    const int hw = hqr_width(R + t);
    pm = max(pm, (t + hw - 1) / hw);
  }
  atomicMax(out, tm);
  atomicMax(out + 1, rm);
  atomicMax(out + 2, pm);
}

void launch_colour_max(const int* clusters, int n, const SizeTab& sz, int* out, int nshift, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_colour_max, dim3(1, nshift), dim3(256), 0, st, clusters, n, sz, out);
}

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

void launch_merge_nn(const GatherItem* items, int n, const BufTab& bt, const SizeTab& sz, int pcap, int nshift,
                     hipStream_t st) {
  if (n <= 0) return;
  for (int i0 = 0; i0 < n; i0 += 65535) {
    int ni = std::min(65535, n - i0);
    hipLaunchKernelGGL(k_merge_nn, dim3(std::max(1u, cdiv((int64_t)pcap * pcap, 256 * 8)), ni, nshift), dim3(256), 0, st,
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
