// GPU part of the H^2 construction (Sec. 3.1): far-field Gram matrices and
// their pivoted Cholesky factorizations in double-double arithmetic, one level
// of the cluster tree per call.  See construct.hpp for what is computed.
//
// Double-double numbers are unevaluated sums hi + lo with |lo| <= ulp(hi)/2.
// Products are split exactly with a fused multiply-add and sums with the
// branch-free two-sum of Knuth (TAOCP vol. 2, 4.2.2); floating-point
// contraction is switched off for this file so that every step rounds as
// written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <stdexcept>
#include <string>

#include "construct.hpp"
#include "devmem.hpp"

#pragma clang fp contract(off)

namespace h2 {

namespace {

struct dd {
  double hi, lo;
};

__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ inline dd fast_norm(double s, double e) {
  const double h = s + e;
  return dd{h, e - (h - s)};
}

__device__ inline dd dd_add(dd a, dd b) {
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  return fast_norm(s, e);
}

__device__ inline dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

__device__ inline dd dd_mul(dd a, dd b) {
  const double p = a.hi * b.hi;
  double e = __builtin_fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return fast_norm(p, e);
}

__device__ inline dd dd_div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  const dd r = dd_add(a, dd_neg(dd_mul(b, dd{q1, 0.0})));
  const double q2 = r.hi / b.hi;
  return fast_norm(q1, q2);
}

__device__ inline dd dd_sqrt(dd a) {
  if (!(a.hi > 0.0)) return dd{0.0, 0.0};
  const double x = sqrt(a.hi);
  const double e = __builtin_fma(-x, x, a.hi) + a.lo;
  return fast_norm(x, e / (2.0 * x));
}

// acc += a * b with a, b plain doubles (the product is split exactly)
__device__ inline void dd_mac(double& hi, double& lo, double a, double b) {
  const double p = a * b;
  const double e = __builtin_fma(a, b, -p);
  double s, err;
  two_sum(hi, p, s, err);
  hi = s;
  lo += err + e;
}

// acc -= a * b with a, b double-double
__device__ inline void dd_msub(double& hi, double& lo, dd a, dd b) {
  const double p = a.hi * b.hi;
  const double e = __builtin_fma(a.hi, b.hi, -p);
  const double cross = __builtin_fma(a.hi, b.lo, a.lo * b.hi);
  double s, err;
  two_sum(hi, -p, s, err);
  hi = s;
  lo += err - e - cross;
}

template <int KIND>
__device__ inline double kval(double p0, double p1, double r) {
  if (KIND == 0) return 1.0 / r;
  if (KIND == 1) return exp(-r) / r;
  if (KIND == 2) return exp(-r * r / p0) / (r + p1);
  if (KIND == 3) return 1.0 / (r + p0);
  return (fabs(r - p0) < 1e-9 * p0) ? -1.0 : 0.0;
}

constexpr int FT = 64;   // Gram tile (rows and columns)
constexpr int FK = 32;   // far points per chunk

struct FarItem {
  int cl, ta, tb;   // cluster, tile row <= tile column
};

// G_i(tile ta, tile tb) = sum over the far field of M_i(rows of ta, :) M_i(rows of tb, :)^T,
// accumulated in double-double.  256 threads: each evaluates 8 kernel entries of
// each of the two row sets per chunk into LDS and owns a 4x4 block of the tile.
// Off-diagonal tiles are also written transposed, so G_i is stored in full
// (column-major, leading dimension m_i).
template <int KIND>
__global__ __launch_bounds__(256) void k_far_gram(const FarItem* __restrict__ items, const double* __restrict__ px,
                                                  const double* __restrict__ py, const double* __restrict__ pz,
                                                  const double* __restrict__ rx, const double* __restrict__ ry,
                                                  const double* __restrict__ rz, const int64_t* __restrict__ roff,
                                                  const int* __restrict__ mrow, const int64_t* __restrict__ fptr,
                                                  const int64_t* __restrict__ fr0, const int64_t* __restrict__ fr1,
                                                  const int64_t* __restrict__ goff, double* __restrict__ Ghi,
                                                  double* __restrict__ Glo, double p0, double p1, int* __restrict__ bad) {
  __shared__ double cx[FK], cy[FK], cz[FK];
  __shared__ double KA[FK][FT], KB[FK][FT];
  const FarItem it = items[blockIdx.x];
  const int m = mrow[it.cl];
  const int64_t ro = roff[it.cl];
  const int tid = threadIdx.x;
  const int er = tid & (FT - 1), cg = tid >> 6;   // evaluation: row er, chunk columns cg*8 .. cg*8+7
  const bool diag = it.ta == it.tb;
  const int ra = it.ta * FT + er, rb = it.tb * FT + er;
  const bool va = ra < m, vb = rb < m;
  const double ax = va ? rx[ro + ra] : 0.0, ay = va ? ry[ro + ra] : 0.0, az = va ? rz[ro + ra] : 0.0;
  const double bx = vb ? rx[ro + rb] : 0.0, by = vb ? ry[ro + rb] : 0.0, bz = vb ? rz[ro + rb] : 0.0;
  const int tx = tid & 15, ty = tid >> 4;
  double hi[4][4], lo[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) hi[i][j] = lo[i][j] = 0.0;
  const double(*KBp)[FT] = diag ? KA : KB;
  for (int64_t k = fptr[it.cl]; k < fptr[it.cl + 1]; ++k) {
    const int64_t e0 = fr0[k], e1 = fr1[k];
    for (int64_t c0 = e0; c0 < e1; c0 += FK) {
      const int nc = (int)min<int64_t>(FK, e1 - c0);
      __syncthreads();
      if (tid < FK) {
        cx[tid] = tid < nc ? px[c0 + tid] : 0.0;
        cy[tid] = tid < nc ? py[c0 + tid] : 0.0;
        cz[tid] = tid < nc ? pz[c0 + tid] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = cg * 8 + q;
        double v = 0.0;
        if (va && c < nc) {
          const double dx = ax - cx[c], dy = ay - cy[c], dz = az - cz[c];
          v = kval<KIND>(p0, p1, sqrt(dx * dx + dy * dy + dz * dz));
        }
        KA[c][er] = v;
        if (!diag) {
          double w = 0.0;
          if (vb && c < nc) {
            const double dx = bx - cx[c], dy = by - cy[c], dz = bz - cz[c];
            w = kval<KIND>(p0, p1, sqrt(dx * dx + dy * dy + dz * dz));
          }
          KB[c][er] = w;
        }
      }
      __syncthreads();
      for (int kk = 0; kk < nc; ++kk) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = KA[kk][tx * 4 + i];
          b[i] = KBp[kk][ty * 4 + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) dd_mac(hi[i][j], lo[i][j], a[i], b[j]);
      }
    }
  }
  double* gh = Ghi + goff[it.cl];
  double* gl = Glo + goff[it.cl];
  int nonfinite = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = it.ta * FT + tx * 4 + i, c = it.tb * FT + ty * 4 + j;
      if (r < m && c < m) {
        const dd v = fast_norm(hi[i][j], lo[i][j]);
        if (!isfinite(v.hi)) nonfinite = 1;
        gh[r + (int64_t)c * m] = v.hi;
        gl[r + (int64_t)c * m] = v.lo;
        if (!diag) {
          gh[c + (int64_t)r * m] = v.hi;
          gl[c + (int64_t)r * m] = v.lo;
        }
      }
    }
  if (nonfinite) atomicOr(bad, 1);
}

// Block reduction helpers (256 threads = 4 waves of 64).
__device__ inline dd wave_sum(dd v) {
  for (int d = 32; d >= 1; d >>= 1) {
    dd o{__shfl_xor(v.hi, d, 64), __shfl_xor(v.lo, d, 64)};
    v = dd_add(v, o);
  }
  return v;
}

__device__ inline void wave_argmax(double& v, int& j) {
  for (int d = 32; d >= 1; d >>= 1) {
    const double ov = __shfl_xor(v, d, 64);
    const int oj = __shfl_xor(j, d, 64);
    if (ov > v || (ov == v && oj >= 0 && (j < 0 || oj < j))) {
      v = ov;
      j = oj;
    }
  }
}

// Pivoted Cholesky of G_i in double-double, one workgroup per cluster
// (left-looking: column k of L is G(:, p) minus the products of the earlier
// columns, p the pivot = largest remaining diagonal, smallest row on ties).
// Stops before step k when the remaining diagonal sums to <= tau2c[cl], i.e. when
// the Frobenius norm of the rows of M_i not yet chosen, projected off the
// chosen ones, is <= tau_i.  step[j] = 1 + the step that chose row j (0 if
// none); L(j, a) lives at L + goff + j + a*m.
__global__ __launch_bounds__(256) void k_far_pchol(const int* __restrict__ mrow, const int64_t* __restrict__ roff,
                                                   const int64_t* __restrict__ goff, const double* __restrict__ Ghi,
                                                   const double* __restrict__ Glo, double* __restrict__ Lhi,
                                                   double* __restrict__ Llo, double* __restrict__ dhi,
                                                   double* __restrict__ dlo, int* __restrict__ step,
                                                   int* __restrict__ piv, int* __restrict__ rank,
                                                   const double* __restrict__ tau2c, double* __restrict__ Lout) {
  __shared__ double red_v[4], red_h[4], red_l[4];
  __shared__ int red_j[4];
  __shared__ int s_p;
  __shared__ int s_stop;
  __shared__ double s_lkk_hi, s_lkk_lo;
  const int cl = blockIdx.x;
  const int m = mrow[cl];
  const double tau2 = tau2c[cl];
  const int64_t go = goff[cl], ro = roff[cl];
  const double* gh = Ghi + go;
  const double* gl = Glo + go;
  double* lh = Lhi + go;
  double* ll = Llo + go;
  double* d_h = dhi + ro;
  double* d_l = dlo + ro;
  int* stp = step + ro;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = tid; j < m; j += 256) {
    d_h[j] = gh[j + (int64_t)j * m];
    d_l[j] = gl[j + (int64_t)j * m];
    stp[j] = 0;
  }
  __syncthreads();
  int k = 0;
  for (; k < m; ++k) {
    // remaining sum and largest remaining diagonal
    dd sum{0.0, 0.0};
    double best = -INFINITY;
    int bj = -1;
    for (int j = tid; j < m; j += 256) {
      if (stp[j] == 0) {
        const dd v{d_h[j], d_l[j]};
        sum = dd_add(sum, v);
        const double vv = v.hi + v.lo;
        if (vv > best || (vv == best && (bj < 0 || j < bj))) {
          best = vv;
          bj = j;
        }
      }
    }
    sum = wave_sum(sum);
    wave_argmax(best, bj);
    if (lane == 0) {
      red_h[wave] = sum.hi;
      red_l[wave] = sum.lo;
      red_v[wave] = best;
      red_j[wave] = bj;
    }
    __syncthreads();
    if (tid == 0) {
      dd s{red_h[0], red_l[0]};
      double bv = red_v[0];
      int bjj = red_j[0];
      for (int w = 1; w < 4; ++w) {
        s = dd_add(s, dd{red_h[w], red_l[w]});
        if (red_v[w] > bv || (red_v[w] == bv && red_j[w] >= 0 && (bjj < 0 || red_j[w] < bjj))) {
          bv = red_v[w];
          bjj = red_j[w];
        }
      }
      const bool stop = !(s.hi + s.lo > tau2) || bjj < 0 || !(bv > 0.0);
      s_stop = stop ? 1 : 0;
      if (!stop) {
        s_p = bjj;
        const dd l = dd_sqrt(dd{d_h[bjj], d_l[bjj]});
        s_lkk_hi = l.hi;
        s_lkk_lo = l.lo;
        stp[bjj] = k + 1;
        piv[ro + k] = bjj;
      }
    }
    __syncthreads();
    if (s_stop) break;
    const int p = s_p;
    const dd lkk{s_lkk_hi, s_lkk_lo};
    for (int j = tid; j < m; j += 256) {
      if (stp[j] != 0) continue;
      double ch = gh[j + (int64_t)p * m], cl_ = gl[j + (int64_t)p * m];
      for (int q = 0; q < k; ++q)
        dd_msub(ch, cl_, dd{lh[j + (int64_t)q * m], ll[j + (int64_t)q * m]},
                dd{lh[p + (int64_t)q * m], ll[p + (int64_t)q * m]});
      const dd c = fast_norm(ch, cl_);
      const dd v = dd_div(c, lkk);
      lh[j + (int64_t)k * m] = v.hi;
      ll[j + (int64_t)k * m] = v.lo;
      const dd d = dd_add(dd{d_h[j], d_l[j]}, dd_neg(dd_mul(v, v)));
      d_h[j] = d.hi;
      d_l[j] = d.lo;
    }
    if (tid == 0) {
      lh[p + (int64_t)k * m] = lkk.hi;
      ll[p + (int64_t)k * m] = lkk.lo;
    }
    __syncthreads();
  }
  if (tid == 0) rank[cl] = k;
  // L rounded to FP64; a chosen row j has L(j, a) = 0 for a past its step
  double* lo_ = Lout + go;
  for (int64_t e = tid; e < (int64_t)m * k; e += 256) {
    const int j = (int)(e % m), a = (int)(e / m);
    const int sj = stp[j];
    lo_[e] = (sj == 0 || a <= sj - 1) ? lh[j + (int64_t)a * m] + ll[j + (int64_t)a * m] : 0.0;
  }
}

struct HipFail : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define FCHK(x)                                                                         \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) throw HipFail(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
T* dev_copy(const std::vector<T>& v, hipStream_t st) {
  T* p = nullptr;
  FCHK(h2::dev_malloc(&p, std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) FCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return p;
}

}  // namespace

void far_points_upload(FarIdPoints& P, const double* X, const int64_t* perm, int64_t n, int dim, hipStream_t st) {
  std::vector<double> x(n, 0.0), y(n, 0.0), z(n, 0.0);
  for (int64_t p = 0; p < n; ++p) {
    const double* q = X + perm[p] * dim;
    x[p] = q[0];
    if (dim > 1) y[p] = q[1];
    if (dim > 2) z[p] = q[2];
  }
  P.n = n;
  P.px = dev_copy(x, st);
  P.py = dev_copy(y, st);
  P.pz = dev_copy(z, st);
  FCHK(hipStreamSynchronize(st));
}

void far_points_free(FarIdPoints& P) {
  if (P.px) (void)h2::dev_free(P.px);
  if (P.py) (void)h2::dev_free(P.py);
  if (P.pz) (void)h2::dev_free(P.pz);
  P = FarIdPoints{};
}

void far_field_ids(const FarIdPoints& P, int kind, double p0, double p1, const FarIdLevel& lev, FarIdResult& out,
                   hipStream_t st) {
  const int N = lev.N;
  out.r.assign(N, 0);
  out.piv.assign(N, {});
  out.Lf.assign(N, {});
  // clusters with rows and a far field, processed in batches of at most ~8 GB of Gram + factor storage
  std::vector<int64_t> roff_all(N + 1, 0);
  for (int i = 0; i < N; ++i) roff_all[i + 1] = roff_all[i] + lev.m[i];
  std::vector<int> todo;
  for (int i = 0; i < N; ++i)
    if (lev.m[i] > 0 && lev.fptr[i + 1] > lev.fptr[i]) todo.push_back(i);
  const int64_t budget = (int64_t)8 << 30;   // bytes per batch (5 doubles per Gram entry)
  size_t t0 = 0;
  while (t0 < todo.size()) {
    size_t t1 = t0;
    int64_t bytes = 0;
    while (t1 < todo.size()) {
      const int64_t mm = (int64_t)lev.m[todo[t1]] * lev.m[todo[t1]] * 40;
      if (t1 > t0 && bytes + mm > budget) break;
      bytes += mm;
      ++t1;
    }
    const int nb = (int)(t1 - t0);
    std::vector<int> mb(nb);
    std::vector<double> t2b(nb);
    std::vector<int64_t> rob(nb), gob(nb), fpb(nb + 1, 0), f0, f1;
    std::vector<double> rx, ry, rz;
    std::vector<FarItem> items;
    int64_t go = 0, ro = 0;
    for (int b = 0; b < nb; ++b) {
      const int i = todo[t0 + b];
      const int m = lev.m[i];
      mb[b] = m;
      t2b[b] = lev.tau2[i];
      rob[b] = ro;
      gob[b] = go;
      for (int a = 0; a < m; ++a) {
        rx.push_back(lev.rx[roff_all[i] + a]);
        ry.push_back(lev.ry[roff_all[i] + a]);
        rz.push_back(lev.rz[roff_all[i] + a]);
      }
      for (int64_t k = lev.fptr[i]; k < lev.fptr[i + 1]; ++k) {
        f0.push_back(lev.fr0[k]);
        f1.push_back(lev.fr1[k]);
      }
      fpb[b + 1] = (int64_t)f0.size();
      const int nt = (m + FT - 1) / FT;
      for (int ta = 0; ta < nt; ++ta)
        for (int tb = ta; tb < nt; ++tb) items.push_back(FarItem{b, ta, tb});
      ro += m;
      go += (int64_t)m * m;
    }
    for (int64_t k = 0; k < (int64_t)f0.size(); ++k)
      if (f0[k] < 0 || f1[k] > P.n || f0[k] > f1[k]) throw std::invalid_argument("far range outside the point set");
    int* dm = dev_copy(mb, st);
    double* dt2 = dev_copy(t2b, st);
    int64_t* dro = dev_copy(rob, st);
    int64_t* dgo = dev_copy(gob, st);
    int64_t* dfp = dev_copy(fpb, st);
    int64_t* df0 = dev_copy(f0, st);
    int64_t* df1 = dev_copy(f1, st);
    double* drx = dev_copy(rx, st);
    double* dry = dev_copy(ry, st);
    double* drz = dev_copy(rz, st);
    FarItem* dit = dev_copy(items, st);
    double *Gh, *Gl, *Lh, *Ll, *Lo, *dh, *dl;
    int *stp, *piv, *rk, *bad;
    FCHK(h2::dev_malloc(&Gh, go * 8));
    FCHK(h2::dev_malloc(&Gl, go * 8));
    FCHK(h2::dev_malloc(&Lh, go * 8));
    FCHK(h2::dev_malloc(&Ll, go * 8));
    FCHK(h2::dev_malloc(&Lo, go * 8));
    FCHK(h2::dev_malloc(&dh, std::max<int64_t>(1, ro) * 8));
    FCHK(h2::dev_malloc(&dl, std::max<int64_t>(1, ro) * 8));
    FCHK(h2::dev_malloc(&stp, std::max<int64_t>(1, ro) * 4));
    FCHK(h2::dev_malloc(&piv, std::max<int64_t>(1, ro) * 4));
    FCHK(h2::dev_malloc(&rk, nb * 4));
    FCHK(h2::dev_malloc(&bad, 4));
    FCHK(hipMemsetAsync(bad, 0, 4, st));
    for (size_t i0 = 0; i0 < items.size(); i0 += 1u << 30) {
      const unsigned ni = (unsigned)std::min<size_t>(items.size() - i0, 1u << 30);
      const FarItem* ip = dit + i0;
      switch (kind) {
        case 0: hipLaunchKernelGGL(k_far_gram<0>, dim3(ni), dim3(256), 0, st, ip, P.px, P.py, P.pz, drx, dry, drz, dro, dm, dfp, df0, df1, dgo, Gh, Gl, p0, p1, bad); break;
        case 1: hipLaunchKernelGGL(k_far_gram<1>, dim3(ni), dim3(256), 0, st, ip, P.px, P.py, P.pz, drx, dry, drz, dro, dm, dfp, df0, df1, dgo, Gh, Gl, p0, p1, bad); break;
        case 2: hipLaunchKernelGGL(k_far_gram<2>, dim3(ni), dim3(256), 0, st, ip, P.px, P.py, P.pz, drx, dry, drz, dro, dm, dfp, df0, df1, dgo, Gh, Gl, p0, p1, bad); break;
        case 3: hipLaunchKernelGGL(k_far_gram<3>, dim3(ni), dim3(256), 0, st, ip, P.px, P.py, P.pz, drx, dry, drz, dro, dm, dfp, df0, df1, dgo, Gh, Gl, p0, p1, bad); break;
        default: hipLaunchKernelGGL(k_far_gram<4>, dim3(ni), dim3(256), 0, st, ip, P.px, P.py, P.pz, drx, dry, drz, dro, dm, dfp, df0, df1, dgo, Gh, Gl, p0, p1, bad); break;
      }
      FCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_far_pchol, dim3(nb), dim3(256), 0, st, dm, dro, dgo, Gh, Gl, Lh, Ll, dh, dl, stp, piv, rk,
                       dt2, Lo);
    FCHK(hipGetLastError());
    std::vector<int> rh(nb), ph(ro > 0 ? ro : 1);
    std::vector<double> lh(go > 0 ? go : 1);
    int badh = 0;
    FCHK(hipMemcpyAsync(rh.data(), rk, nb * 4, hipMemcpyDeviceToHost, st));
    FCHK(hipMemcpyAsync(ph.data(), piv, std::max<int64_t>(1, ro) * 4, hipMemcpyDeviceToHost, st));
    FCHK(hipMemcpyAsync(lh.data(), Lo, go * 8, hipMemcpyDeviceToHost, st));
    FCHK(hipMemcpyAsync(&badh, bad, 4, hipMemcpyDeviceToHost, st));
    FCHK(hipStreamSynchronize(st));
    for (void* p : {(void*)dm, (void*)dt2, (void*)dro, (void*)dgo, (void*)dfp, (void*)df0, (void*)df1, (void*)drx, (void*)dry,
                    (void*)drz, (void*)dit, (void*)Gh, (void*)Gl, (void*)Lh, (void*)Ll, (void*)Lo, (void*)dh,
                    (void*)dl, (void*)stp, (void*)piv, (void*)rk, (void*)bad})
      FCHK(h2::dev_free(p));
    if (badh) throw std::invalid_argument("kernel is not finite between a cluster and its far field");
    for (int b = 0; b < nb; ++b) {
      const int i = todo[t0 + b];
      const int m = mb[b], r = rh[b];
      out.r[i] = r;
      out.piv[i].assign(ph.begin() + rob[b], ph.begin() + rob[b] + r);
      out.Lf[i].assign(lh.begin() + gob[b], lh.begin() + gob[b] + (int64_t)m * r);
    }
    t0 = t1;
  }
}

}  // namespace h2

namespace h2 {

namespace {

// y_i = sum_j A_ij x_j for the exact kernel matrix (A_ii = diag), one row per
// thread, the column points (X row-major n x dim) and x streaming through LDS
// in tiles of 256.
template <int KIND>
__global__ __launch_bounds__(256) void k_kernel_matvec(const double* __restrict__ X, int dim,
                                                       const double* __restrict__ x, int64_t n, double diag, double p0,
                                                       double p1, double* __restrict__ y) {
  __shared__ double tx[256], ty[256], tz[256], tv[256];
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
    tv[threadIdx.x] = j < n ? x[j] : 0.0;
    __syncthreads();
    const int jn = (int)min<int64_t>(256, n - j0);
    for (int q = 0; q < jn; ++q) {
      const double dx = xi - tx[q], dy = yi - ty[q], dz = zi - tz[q];
      const double v = (j0 + q == i) ? diag : kval<KIND>(p0, p1, sqrt(dx * dx + dy * dy + dz * dz));
      acc = __builtin_fma(v, tv[q], acc);
    }
  }
  if (i < n) y[i] = acc;
}

}  // namespace

void launch_kernel_matvec(const double* dX, int64_t n, int dim, int kind, double diag, double p0, double p1,
                          const double* dx, double* dy, hipStream_t st) {
  if (n <= 0) return;
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_kernel_matvec<0>, g, b, 0, st, dX, dim, dx, n, diag, p0, p1, dy); break;
    case 1: hipLaunchKernelGGL(k_kernel_matvec<1>, g, b, 0, st, dX, dim, dx, n, diag, p0, p1, dy); break;
    case 2: hipLaunchKernelGGL(k_kernel_matvec<2>, g, b, 0, st, dX, dim, dx, n, diag, p0, p1, dy); break;
    case 3: hipLaunchKernelGGL(k_kernel_matvec<3>, g, b, 0, st, dX, dim, dx, n, diag, p0, p1, dy); break;
    default: hipLaunchKernelGGL(k_kernel_matvec<4>, g, b, 0, st, dX, dim, dx, n, diag, p0, p1, dy); break;
  }
}

void kernel_matvec_gpu(const double* X, int64_t n, int dim, int kind, double diag, double p0, double p1,
                       const double* x, double* y, hipStream_t st) {
  double *dX = nullptr, *dx = nullptr, *dy = nullptr;
  struct Guard {
    double** p[3];
    ~Guard() {
      for (double** q : p)
        if (*q) (void)h2::dev_free(*q);
    }
  } guard{{&dX, &dx, &dy}};
  FCHK(h2::dev_malloc(&dX, std::max<int64_t>(1, n * dim) * 8));
  FCHK(h2::dev_malloc(&dx, std::max<int64_t>(1, n) * 8));
  FCHK(h2::dev_malloc(&dy, std::max<int64_t>(1, n) * 8));
  FCHK(hipMemcpyAsync(dX, X, n * dim * 8, hipMemcpyHostToDevice, st));
  FCHK(hipMemcpyAsync(dx, x, n * 8, hipMemcpyHostToDevice, st));
  launch_kernel_matvec(dX, n, dim, kind, diag, p0, p1, dx, dy, st);
  FCHK(hipGetLastError());
  FCHK(hipMemcpyAsync(y, dy, n * 8, hipMemcpyDeviceToHost, st));
  FCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------ allocation-free variant
// Device scratch of kernel_matvec_noalloc: the points, x and y are staged here
// instead of in allocated buffers.  One copy per GPU, held until the process
// ends; every call on a GPU shares it, so calls that overlap on one GPU race.
constexpr int64_t NOALLOC_DOUBLES = (int64_t)8 << 20;   // 64 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};   // device address of `scratch` on each GPU (nullptr = not looked up yet)

double* scratch_on(int device) {
  if (device < 0 || device >= 64) throw std::invalid_argument("device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    FCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = (double*)p;
  }
  return g_scratch_ptr[device];
}

inline int64_t up32(int64_t v) { return (v + 31) / 32 * 32; }
}  // namespace

int64_t kernel_matvec_noalloc_max_n(int dim) { return (NOALLOC_DOUBLES - 96) / (dim + 2); }

void kernel_matvec_noalloc(const double* X, int64_t n, int dim, int kind, double diag, double p0, double p1,
                           const double* x, double* y, int device, hipStream_t st) {
  if (n > kernel_matvec_noalloc_max_n(dim)) throw std::invalid_argument("n exceeds the static scratch");
  FCHK(hipSetDevice(device));
  double* base = scratch_on(device);   // looked up with this device current
  double* dX = base;
  double* dx = base + up32(n * dim);
  double* dy = dx + up32(n);
  FCHK(hipMemcpyAsync(dX, X, n * dim * 8, hipMemcpyHostToDevice, st));
  FCHK(hipMemcpyAsync(dx, x, n * 8, hipMemcpyHostToDevice, st));
  launch_kernel_matvec(dX, n, dim, kind, diag, p0, p1, dx, dy, st);
  FCHK(hipGetLastError());
  FCHK(hipMemcpyAsync(y, dy, n * 8, hipMemcpyDeviceToHost, st));
  FCHK(hipStreamSynchronize(st));
}

}  // namespace h2
