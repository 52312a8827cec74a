// Level engine and C ABI of the H^2 k-th eigenvalue library.
//
// h2_build: host construction (tree, bases, couplings, static schedule), then the
//   leaf near blocks in skeleton coordinates Q_i^T A_ij Q_j (Eq. dense_skeleton)
//   are evaluated and rotated on the GPU and stay resident with the couplings and
//   transfer matrices.
// h2_inertia: batched generalized H^2-LDL of A~ - sigma_s I on the GPU, level by
//   level, colour class by colour class (Secs. 3.2-3.4), returning
//   nu_s = #{lambda < sigma_s} (Sec. 2, Sec. 4).
// h2_kth_eig: Algorithm 1 for every requested index; the midpoints of all open
//   brackets form one batch per bisection step, and every (mu, nu) record narrows
//   every open bracket (inertia reuse, Sec. 4.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/h2eig.h"
#include "construct.hpp"
#include "devmem.hpp"
#include "host.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "records.hpp"

using namespace h2;

namespace {

thread_local std::string g_err;

h2_status fail(h2_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipError {
  hipError_t e;
  std::string where;
};

#define HIPCHK(x)                                                   \
  do {                                                              \
    hipError_t e_ = (x);                                            \
    if (e_ != hipSuccess) throw HipError{e_, std::string(#x)};      \
  } while (0)

struct NoMem {
  std::string what;
};

// H2EIG_POISON=1: every workspace byte is set to 0xFF (a NaN in every double)
// when it is allocated and before every factorization, so that a read of
// memory the call did not write changes the result (a test of the kernels'
// initialisation).  Read at every call.
bool poison_on() {
  const char* e = std::getenv("H2EIG_POISON");
  return e && e[0] == '1';
}

// Device buffer that only grows.
struct Arena {
  void* p = nullptr;
  size_t cap = 0;
  void poison(hipStream_t st) {
    if (p) HIPCHK(hipMemsetAsync(p, 0xFF, cap, st));
  }
  void ensure(size_t bytes, hipStream_t st) {
    if (bytes <= cap) return;
    if (p) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(h2::dev_free(p));
      p = nullptr;
      cap = 0;
    }
    size_t want = bytes + bytes / 32 + 4096;
    if (h2::dev_malloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw NoMem{"device allocation of " + std::to_string(want) + " bytes failed"};
    }
    cap = want;
    if (poison_on()) poison(st);
  }
  void release() {
    if (p) (void)h2::dev_free(p);
    p = nullptr;
    cap = 0;
  }
};

// Host blob of plan arrays uploaded in one copy.
struct Blob {
  std::vector<char> h;
  template <class T>
  size_t put(const std::vector<T>& v) {
    size_t off = (h.size() + 255) & ~(size_t)255;
    h.resize(off + v.size() * sizeof(T) + 1);
    if (!v.empty()) std::memcpy(h.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

struct DevList {
  size_t items = 0, terms = 0;
  int n = 0;
};

struct DevColour {
  size_t clusters = 0;
  int ncl = 0;
  DevList pc_upd, ut_s, ut_t, ut_x, ut_u, ut_w, ldl_upd, inv_t, inv_x;
  DevList rot_rows, rot_cols, rot_cols_t, trsm;
  size_t rr_copy = 0, rc_copy = 0, tr_copy = 0, rr_copyt = 0, rct_copy = 0;
  DevList schur, gm, gt, gg;
  size_t gp_items = 0, gp_src = 0;
  int ngp = 0;
};

struct DevLevel {
  std::vector<DevColour> colours;
  size_t diag_blk = 0, r0 = 0, pr0 = 0, gather = 0, mirror = 0;
  int ngather = 0, nmirror = 0;
  DevList gram_init, gram_init_t, fill, tr1, tr2;
};

// Kernel classes of the level engine, for the diagnostic profiler.
enum ProfClass {
  PC_INIT = 0, PC_PCHOL, PC_PCHOL_UPD, PC_HQR, PC_HQR_UPD, PC_WFORM, PC_ROTATE, PC_LDL, PC_LDL_UPD, PC_LDL_INV,
  PC_LDL_OP, PC_ELIM, PC_COPY, PC_SCHUR, PC_GRAM, PC_MERGE, PC_MERGE_FILL, PC_MERGE_E, PC_N
};
const char* const kProfNames[PC_N] = {"init", "recompress_pchol", "recompress_pchol_update", "recompress_hqr",
                                      "recompress_hqr_update", "recompress_w", "rotate", "pivot_ldl",
                                      "pivot_ldl_update", "pivot_ldl_inverse", "pivot_ldl_operator", "elimination",
                                      "copyback", "schur", "fillin_gram", "merge_gather", "merge_fillin",
                                      "merge_transfer"};
// per-kernel totals of the GEMM kernels by operand layout (GemmKind order):
// 64 x 64 tiles FP64, FP32, then 128 x 128 tiles FP64, FP32
constexpr int PROF_N = PC_N + 16;
const char* const kGemmNames[16] = {
    "kernel:k_gemm<false, false>",        "kernel:k_gemm<false, true>",
    "kernel:k_gemm<true, false>",         "kernel:k_gemm<true, true>",
    "kernel:k_gemm_f32<false, false>",    "kernel:k_gemm_f32<false, true>",
    "kernel:k_gemm_f32<true, false>",     "kernel:k_gemm_f32<true, true>",
    "kernel:k_gemm128<false, false>",     "kernel:k_gemm128<false, true>",
    "kernel:k_gemm128<true, false>",      "kernel:k_gemm128<true, true>",
    "kernel:k_gemm128_f32<false, false>", "kernel:k_gemm128_f32<false, true>",
    "kernel:k_gemm128_f32<true, false>",  "kernel:k_gemm128_f32<true, true>"};
// classes whose contractions run in FP32 in an FP32 factorization (rotation,
// elimination, Schur, merge); recompression and the pivot LDL stay FP64
inline bool f32_class(int cls) {
  return cls == PC_ROTATE || cls == PC_ELIM || cls == PC_SCHUR || cls == PC_MERGE_FILL || cls == PC_MERGE_E;
}

// Brackets kernel launches with HIP events on the handle's stream and keeps a
// device array of per-class algorithmic flop counters.
struct Profiler {
  bool on = false;
  bool gemm_only = false;            // events only around GEMM launches (kernel symbols)
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> recs;
  int level = 0;                     // level of the records being made (for the per-level table)
  double ms_level[PROF_N][32] = {{0}};
  double ms[PROF_N] = {0};              // classes, then the GEMM kernel symbols
  long long launches[PROF_N] = {0};
  unsigned long long flops[PROF_N] = {0};
  unsigned long long bytes[PROF_N] = {0};   // algorithmic bytes (GEMM kernel symbols)
  unsigned long long* d_fc = nullptr;       // flop counters [PROF_N], then byte counters [PROF_N]
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    for (int c = 0; c < PROF_N; ++c) {
      ms[c] = 0; launches[c] = 0; flops[c] = 0; bytes[c] = 0;
      for (int l = 0; l < 32; ++l) ms_level[c][l] = 0;
    }
  }
  // after the stream is synchronized: fold the recorded pairs into the totals
  void collect() {
    for (auto& r : recs) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, r.second.first, r.second.second));
      const int cls = r.first & 0xFFFF, lev = r.first >> 16;
      ms[cls] += t;
      ms_level[cls][lev & 31] += t;
      launches[cls] += 1;
    }
    recs.clear();
    used = 0;
    if (d_fc) {
      unsigned long long h[2 * PROF_N];
      HIPCHK(hipMemcpy(h, d_fc, sizeof(h), hipMemcpyDeviceToHost));
      for (int c = 0; c < PROF_N; ++c) {
        flops[c] += h[c];
        bytes[c] += h[PROF_N + c];
      }
      HIPCHK(hipMemset(d_fc, 0, sizeof(h)));
    }
  }
  void release() {
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
    if (d_fc) (void)h2::dev_free(d_fc);
    d_fc = nullptr;
  }
};

}  // namespace

struct h2_matrix_s {
  std::atomic<int> busy{0};
  Tree T;
  Basis B;
  KernelSpec kern;
  double eps = 0, normA = 0, tau = 0;
  std::vector<LevelPlan> plan;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  int leafcap = 0;
  int device = 0;
  // resident device data
  double* d_bres = nullptr;
  std::vector<double*> d_cpl;    // per level
  std::vector<double*> d_emat;   // per level l: parents of level l+1 (index l)
  std::vector<int> emat_ld;
  char* d_plan = nullptr;
  std::vector<DevLevel> dlev;
  size_t leaf_m0 = 0, leaf_blkdiag = 0;
  int64_t resident = 0;
  // workspace
  Arena sf[2], lvl, mrg, small, rs;
  Arena tab[2];   // block offset / leading-dimension tables of the blocks in sf[0] / sf[1]
  Arena stab;     // offset / leading-dimension tables of the current level's fill-in Gram slots
  // slicing cache (FP64 inertia records, sorted by shift, runs of equal counts
  // compacted) and statistics
  std::vector<h2::Record> cache;
  bool have_gersh = false;
  double mixed_rel = 0.0;
  std::vector<std::vector<int64_t>> lstats;   // per level, per shift of the last factorization: sum t, sum m, max m, sum R
  int lstats_shifts = 0;
  std::vector<int32_t> last_cap;   // block capacity of each level in the last factorization (0 = not reached)   // h2_kth_eig: FP32 steps while a bracket is >= mixed_rel * normA wide
  double g_lo = 0, g_hi = 0;
  h2_stats_t st{};
  int max_shifts = 0;
  double ws_per_shift = 0.0;   // workspace bytes per shift, from the arenas and the batch they were sized for
  int arena_shifts = 0;        // largest batch factored since the arenas were last released
  int max_list = 1;        // longest GEMM list of the plan (tile-count scratch)
  int* d_prefix = nullptr;  // per-shift tile counts of the current GEMM launch (in the small arena)
  Profiler prof;
  int* d_more = nullptr;   // per-iteration "more panels needed" counters + colour maxima
  std::vector<double*> d_tau2;   // per level: squared truncation budget tau^2 * |cluster| / n of every cluster
  std::vector<double*> d_tau2_f32;   // the same for FP32 factorizations, with tau = max(eps, EPS_F32) * normA
  int* h_more = nullptr;   // pinned host copy (4 ints)

  template <class T>
  const T* dp(size_t off) const { return reinterpret_cast<const T*>(d_plan + off); }
  template <class T>
  T* dpm(size_t off) const { return reinterpret_cast<T*>(d_plan + off); }
};

namespace {

struct Busy {
  h2_matrix A;
  bool ok;
  explicit Busy(h2_matrix a) : A(a) {
    int z = 0;
    ok = A->busy.compare_exchange_strong(z, 1);
  }
  ~Busy() {
    if (ok) A->busy.store(0);
  }
};

// longest GEMM list of the plan being uploaded (per thread: builds may run
// concurrently): sizes the per-shift tile-count scratch
thread_local int g_max_list = 1;

DevList put_list(Blob& b, const GList& g) {
  DevList d;
  d.items = b.put(g.items);
  d.terms = b.put(g.terms);
  d.n = (int)g.items.size();
  g_max_list = std::max(g_max_list, d.n);
  return d;
}

void upload_plan(h2_matrix A) {
  Blob b;
  g_max_list = 1;
  int L = A->T.L;
  A->dlev.assign(L + 1, {});
  for (int l = 0; l <= L; ++l) {
    const LevelPlan& lp = A->plan[l];
    DevLevel& dl = A->dlev[l];
    dl.diag_blk = b.put(lp.diag_blk);
    dl.r0 = b.put(lp.r0);
    dl.colours.resize(lp.colours.size());
    for (size_t c = 0; c < lp.colours.size(); ++c) {
      const ColourPlan& cp = lp.colours[c];
      DevColour& dc = dl.colours[c];
      dc.clusters = b.put(cp.clusters);
      dc.ncl = (int)cp.clusters.size();
      dc.pc_upd = put_list(b, cp.pc_upd);
      dc.ut_s = put_list(b, cp.ut_s);
      dc.ut_t = put_list(b, cp.ut_t);
      dc.ut_x = put_list(b, cp.ut_x);
      dc.ut_u = put_list(b, cp.ut_u);
      dc.ut_w = put_list(b, cp.ut_w);
      dc.ldl_upd = put_list(b, cp.ldl_upd);
      dc.inv_t = put_list(b, cp.inv_t);
      dc.inv_x = put_list(b, cp.inv_x);
      dc.rot_rows = put_list(b, cp.rot_rows);
      dc.rot_cols = put_list(b, cp.rot_cols);
      dc.rot_cols_t = put_list(b, cp.rot_cols_t);
      dc.rct_copy = b.put(cp.rot_cols_t_copy);
      dc.trsm = put_list(b, cp.trsm);
      dc.rr_copy = b.put(cp.rot_rows_copy);
      dc.rr_copyt = b.put(cp.rot_rows_copyt);
      dc.rc_copy = b.put(cp.rot_cols_copy);
      dc.tr_copy = b.put(cp.trsm_copy);
      dc.schur = put_list(b, cp.schur);
      dc.gm = put_list(b, cp.gram_m);
      dc.gt = put_list(b, cp.gram_t);
      dc.gg = put_list(b, cp.gram_g);
      dc.gp_items = b.put(cp.gram_p.items);
      dc.gp_src = b.put(cp.gram_p.src);
      dc.ngp = (int)cp.gram_p.items.size();
    }
    dl.gram_init = put_list(b, lp.gram_init);
    dl.gram_init_t = put_list(b, lp.gram_init_t);
    if (l >= 1) {
      const MergePlan& mp = lp.merge;
      dl.pr0 = b.put(mp.pr0);
      dl.gather = b.put(mp.gather);
      dl.ngather = (int)mp.gather.size();
      dl.mirror = b.put(mp.mirror);
      dl.nmirror = (int)mp.mirror.size();
      dl.fill = put_list(b, mp.fill);
      dl.tr1 = put_list(b, mp.tr1);
      dl.tr2 = put_list(b, mp.tr2);
    }
  }
  // leaf: dimensions and diagonal flags
  const LevelPlan& lf = A->plan[L];
  std::vector<int> m0(lf.N), bdm(lf.nblk(), 0);
  for (int i = 0; i < lf.N; ++i) {
    m0[i] = A->B.m[L][i];
    bdm[lf.diag_blk[i]] = m0[i];
  }
  A->leaf_m0 = b.put(m0);
  A->leaf_blkdiag = b.put(bdm);
  A->max_list = g_max_list;
  HIPCHK(h2::dev_malloc(&A->d_plan, b.h.size()));
  HIPCHK(hipMemcpy(A->d_plan, b.h.data(), b.h.size(), hipMemcpyHostToDevice));
  A->resident += (int64_t)b.h.size();
}

// Leaf near blocks B_ij = Q_i^T A_ij Q_j on the GPU.
void build_near_blocks(h2_matrix A) {
  const Tree& T = A->T;
  int L = T.L;
  const LevelPlan& lf = A->plan[L];
  int cap = A->leafcap;
  int N = lf.N, nblk = lf.nblk();
  hipStream_t st = A->stream;
  size_t bsz = (size_t)cap * cap;
  HIPCHK(h2::dev_malloc(&A->d_bres, std::max<size_t>(1, (size_t)nblk * bsz * sizeof(double))));
  A->resident += (int64_t)nblk * bsz * 8;
  // points in leaf order, starts, sizes, bases
  std::vector<double> Xl((size_t)T.n * T.dim);
  for (int64_t p = 0; p < T.n; ++p)
    for (int d = 0; d < T.dim; ++d) Xl[p * T.dim + d] = T.X[T.perm[p] * T.dim + d];
  std::vector<int64_t> start(N);
  std::vector<int> msz(N);
  for (int i = 0; i < N; ++i) {
    start[i] = T.start[L][i];
    msz[i] = (int)T.size[L][i];
  }
  std::vector<double> Q((size_t)N * bsz, 0.0);
  for (int i = 0; i < N; ++i) {
    int m = msz[i];
    const auto& q = A->B.Q[L][i];
    for (int c = 0; c < m; ++c)
      for (int r = 0; r < m; ++r) Q[(size_t)i * bsz + r + (size_t)c * cap] = q[r + (size_t)c * m];
  }
  double *dX = nullptr, *dQ = nullptr;
  int64_t* dstart = nullptr;
  int *dm = nullptr, *dbad = nullptr;
  HIPCHK(h2::dev_malloc(&dX, std::max<size_t>(8, Xl.size() * 8)));
  HIPCHK(h2::dev_malloc(&dQ, Q.size() * 8));
  HIPCHK(h2::dev_malloc(&dstart, N * 8));
  HIPCHK(h2::dev_malloc(&dm, N * 4));
  HIPCHK(h2::dev_malloc(&dbad, 4));
  HIPCHK(hipMemcpy(dX, Xl.data(), Xl.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dQ, Q.data(), Q.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dstart, start.data(), N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dm, msz.data(), N * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(dbad, 0, 4));
  // chunked: kernel blocks -> HAT ; TMP = Q_i^T HAT ; BRES = TMP Q_j
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nblk, (int64_t)(2LL << 30) / (int64_t)(bsz * 8)));
  double *dA = nullptr, *dT = nullptr;
  HIPCHK(h2::dev_malloc(&dA, (size_t)chunk * bsz * 8));
  HIPCHK(h2::dev_malloc(&dT, (size_t)chunk * bsz * 8));
  std::vector<int> bi(nblk), bj(nblk);
  for (int i = 0; i < N; ++i)
    for (int k = lf.near_ptr[i]; k < lf.near_ptr[i + 1]; ++k) {
      bi[k] = i;
      bj[k] = lf.near_idx[k];
    }
  int *dbi = nullptr, *dbj = nullptr;
  HIPCHK(h2::dev_malloc(&dbi, std::max(1, nblk) * 4));
  HIPCHK(h2::dev_malloc(&dbj, std::max(1, nblk) * 4));
  HIPCHK(hipMemcpy(dbi, bi.data(), nblk * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dbj, bj.data(), nblk * 4, hipMemcpyHostToDevice));
  int zero_int = 0;
  SizeTab sz{};
  sz.N = 1;
  sz.Np = 1;
  sz.m = sz.R = sz.t = sz.pm = sz.pR = &zero_int;  // never dereferenced: constant sizes only
  for (int b0 = 0; b0 < nblk; b0 += chunk) {
    int nb = std::min(chunk, nblk - b0);
    launch_kernel_blocks(dA, bsz, cap, dbi + b0, dbj + b0, nb, dstart, dm, dX, T.dim, A->kern.kind, A->kern.diag,
                         A->kern.p0, A->kern.p1, dbad, st);
    GList g1, g2;
    for (int k = 0; k < nb; ++k) {
      int i = bi[b0 + k], j = bj[b0 + k];
      Ref q{B_V, i, 0, 0, 0, 0}, a{B_HAT, k, 0, 0, 0, 0}, t{B_TMP, k, 0, 0, 0, 0}, o{B_BRES, b0 + k, 0, 0, 0, 0};
      Ref none{-1, 0, 0, 0, 0, 0};
      GItem it1{t, none, msz[i], msz[j], 0, 0, 1.0, 0.0, -1, 0, 0};
      g1.add(it1, {GTerm{q, a, msz[i], -1, 0}});
      GItem it2{o, none, msz[i], msz[j], 0, 0, 1.0, 0.0, -1, 0, 0};
      g2.add(it2, {GTerm{t, Ref{B_V, j, 0, 0, 0, 0}, msz[j], -1, 0}});
    }
    GItem *di1, *di2;
    GTerm *dt1, *dt2;
    HIPCHK(h2::dev_malloc(&di1, g1.items.size() * sizeof(GItem)));
    HIPCHK(h2::dev_malloc(&di2, g2.items.size() * sizeof(GItem)));
    HIPCHK(h2::dev_malloc(&dt1, g1.terms.size() * sizeof(GTerm)));
    HIPCHK(h2::dev_malloc(&dt2, g2.terms.size() * sizeof(GTerm)));
    HIPCHK(hipMemcpy(di1, g1.items.data(), g1.items.size() * sizeof(GItem), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(di2, g2.items.data(), g2.items.size() * sizeof(GItem), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dt1, g1.terms.data(), g1.terms.size() * sizeof(GTerm), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dt2, g2.terms.data(), g2.terms.size() * sizeof(GTerm), hipMemcpyHostToDevice));
    BufTab bt{};
    for (int k = 0; k < NBUF; ++k) { bt.p[k] = nullptr; bt.ss[k] = 0; bt.bs[k] = (int64_t)bsz; bt.ld[k] = cap; }
    bt.p[B_V] = dQ;   // leaf bases
    bt.p[B_HAT] = dA;
    bt.p[B_TMP] = dT;
    bt.p[B_BRES] = A->d_bres;
    int* dpre = nullptr;
    HIPCHK(h2::dev_malloc(&dpre, (size_t)(nb + 1) * sizeof(int)));
    launch_gemm(GEMM_TN, di1, nb, dt1, bt, sz, cap, cap, 1, dpre, st);
    launch_gemm(GEMM_NN, di2, nb, dt2, bt, sz, cap, cap, 1, dpre, st);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(h2::dev_free(dpre));
    HIPCHK(h2::dev_free(di1));
    HIPCHK(h2::dev_free(di2));
    HIPCHK(h2::dev_free(dt1));
    HIPCHK(h2::dev_free(dt2));
  }
  int bad = 0;
  HIPCHK(hipMemcpy(&bad, dbad, 4, hipMemcpyDeviceToHost));
  HIPCHK(h2::dev_free(dA));
  HIPCHK(h2::dev_free(dT));
  HIPCHK(h2::dev_free(dX));
  HIPCHK(h2::dev_free(dQ));
  HIPCHK(h2::dev_free(dstart));
  HIPCHK(h2::dev_free(dm));
  HIPCHK(h2::dev_free(dbad));
  HIPCHK(h2::dev_free(dbi));
  HIPCHK(h2::dev_free(dbj));
  if (bad) throw std::invalid_argument("kernel is not finite for a pair of distinct points (coincident points?)");
}

void upload_resident(h2_matrix A) {
  int L = A->T.L;
  A->d_cpl.assign(L + 1, nullptr);
  A->d_emat.assign(L + 1, nullptr);
  A->emat_ld.assign(L + 1, 1);
  for (int l = 1; l <= L; ++l) {
    const LevelPlan& lp = A->plan[l];
    int rm = std::max(1, lp.rmax);
    size_t nsl = lp.far_idx.size();
    std::vector<double> h(std::max<size_t>(1, nsl) * rm * rm, 0.0);
    for (int i = 0; i < lp.N; ++i) {
      int ri = A->B.r[l][i];
      for (auto& pr : A->B.C[l][i]) {
        int j = pr.first, rj = A->B.r[l][j];
        int slot = lp.cslot(i, j);
        for (int c = 0; c < rj; ++c)
          for (int r = 0; r < ri; ++r) h[(size_t)slot * rm * rm + r + (size_t)c * rm] = pr.second[r + (size_t)c * ri];
      }
    }
    HIPCHK(h2::dev_malloc(&A->d_cpl[l], h.size() * 8));
    HIPCHK(hipMemcpy(A->d_cpl[l], h.data(), h.size() * 8, hipMemcpyHostToDevice));
    A->resident += (int64_t)h.size() * 8;
    // transfer matrices of the parents (level l-1), stored with level l-1
    const MergePlan& mp = lp.merge;
    int em = std::max(1, mp.emax);
    std::vector<double> e((size_t)mp.Np * em * em, 0.0);
    for (int p = 0; p < mp.Np; ++p) {
      int d = mp.emat_dim[p];
      const auto& Q = A->B.Q[l - 1][p];
      for (int c = 0; c < d; ++c)
        for (int r = 0; r < d; ++r) e[(size_t)p * em * em + r + (size_t)c * em] = Q[r + (size_t)c * d];
    }
    HIPCHK(h2::dev_malloc(&A->d_emat[l - 1], e.size() * 8));
    HIPCHK(hipMemcpy(A->d_emat[l - 1], e.data(), e.size() * 8, hipMemcpyHostToDevice));
    A->emat_ld[l - 1] = em;
    A->resident += (int64_t)e.size() * 8;
  }
}

// ------------------------------------------------------------ factorization
struct Work {
  int S = 0;
  int *m = nullptr, *R = nullptr, *t = nullptr, *pm = nullptr, *pR = nullptr, *status = nullptr;
  int *a0 = nullptr, *a1 = nullptr;
  unsigned long long* nu = nullptr;
  double* sigma = nullptr;
};

inline int round_cap(int v) { return std::max(8, (v + 7) & ~7); }

// Truncation budget of FP32 factorizations, relative to normA.  They serve
// bisection steps on brackets at least switch_rel * normA wide (1e-4 by
// default), whose decisions a perturbation of the matrix by about 1e-6 * normA
// changes only for shifts that close to an eigenvalue; the FP64 counts taken
// at the switch repair such decisions.  A budget near the FP32 rounding level
// of the contractions (about 1e-7 of the fill-in) would make recompression
// keep rounding noise as new directions.
constexpr double EPS_F32 = 1e-6;

// Counters of the blocked factorizations: one "more panels needed" slot per
// iteration (zeroed once per loop, read back only every few iterations, so
// that the host rarely waits for the device), then two slots for colour maxima.
constexpr int MORE_SLOTS = 4096;

// Read back n ints at d (synchronously).
void read_back(h2_matrix A, const int* d, int n, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(A->h_more, d, n * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

int debug_level() {
  static int v = [] {
    const char* e = std::getenv("H2EIG_DEBUG");
    return e ? std::atoi(e) : 0;
  }();
  return v;
}

// Diagnostic print (H2EIG_DEBUG=1): sizes of the first shift after a level.
void debug_dump_level(int l, int N, int S, const Work& w, hipStream_t st) {
  std::vector<int> m((size_t)S * N), R((size_t)S * N), t((size_t)S * N), stv(S);
  std::vector<unsigned long long> nu(S);
  HIPCHK(hipMemcpyAsync(m.data(), w.m, m.size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(R.data(), w.R, R.size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(t.data(), w.t, t.size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nu.data(), w.nu, S * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(stv.data(), w.status, S * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int mmax = 0, tmax = 0;
  for (int v : m) mmax = std::max(mmax, v);
  for (int v : t) tmax = std::max(tmax, v);
  double ms = 0, rs = 0, ts = 0;
  for (int i = 0; i < N; ++i) { ms += m[i]; rs += R[i]; ts += t[i]; }
  std::fprintf(stderr, "[h2eig] level %d: nu[0]=%llu status[0]=%d max m %d max t %d mean m %.1f R %.1f t %.1f\n", l,
               nu[0], stv[0], mmax, tmax, ms / N, rs / N, ts / N);
  std::fprintf(stderr, "[h2eig]   m:");
  for (int i = 0; i < std::min(N, 32); ++i) std::fprintf(stderr, " %d", m[i]);
  std::fprintf(stderr, "\n[h2eig]   R:");
  for (int i = 0; i < std::min(N, 32); ++i) std::fprintf(stderr, " %d", R[i]);
  std::fprintf(stderr, "\n[h2eig]   t:");
  for (int i = 0; i < std::min(N, 32); ++i) std::fprintf(stderr, " %d", t[i]);
  std::fprintf(stderr, "\n");
}

// Factor S shifts; nu/status are host outputs.
void factor_batch(h2_matrix A, const double* sig, int S, bool f32, int64_t* nu_out, int32_t* st_out,
                  double* flops_out, int* maxdim_out) {
  const Tree& T = A->T;
  const int L = T.L;
  hipStream_t st = A->stream;
  const int Nmax = 1 << L;
  // small arena: sizes tables + sigma + nu + status
  size_t nsz = (size_t)S * Nmax;
  size_t off_m = 0, off_R = off_m + nsz * 4, off_t = off_R + nsz * 4, off_pm = off_t + nsz * 4,
         off_pR = off_pm + nsz * 4, off_a0 = off_pR + nsz * 4, off_a1 = off_a0 + nsz * 4, off_st = off_a1 + nsz * 4,
         off_sig = ((off_st + S * 4 + 255) / 256) * 256, off_nu = off_sig + S * 8,
         off_pre = off_nu + S * 8, total = off_pre + (size_t)S * (A->max_list + 1) * 4;
  A->small.ensure(total, st);
  if (poison_on()) {
    for (auto& a : A->sf) a.poison(st);
    A->lvl.poison(st);
    A->mrg.poison(st);
    A->rs.poison(st);
    A->small.poison(st);
    HIPCHK(hipMemsetAsync(A->d_more, 0xFF, (MORE_SLOTS + 4) * sizeof(int), st));
  }
  char* base = (char*)A->small.p;
  int* const dpre = (int*)(base + off_pre);
  Work w;
  w.S = S;
  w.m = (int*)(base + off_m);
  w.R = (int*)(base + off_R);
  w.t = (int*)(base + off_t);
  w.pm = (int*)(base + off_pm);
  w.pR = (int*)(base + off_pR);
  w.a0 = (int*)(base + off_a0);
  w.a1 = (int*)(base + off_a1);
  w.status = (int*)(base + off_st);
  w.sigma = (double*)(base + off_sig);
  w.nu = (unsigned long long*)(base + off_nu);
  HIPCHK(hipMemcpyAsync(w.sigma, sig, S * 8, hipMemcpyHostToDevice, st));
  launch_fill_int(w.status, S, 0, st);
  launch_fill_int((int*)w.nu, 2 * S, 0, st);

  int cap = A->leafcap;
  int cur = 0;  // which sf arena holds the current level
  // per arena: byte offsets in tab[] of (S offsets, F offsets, S lds, F lds),
  // and the elements per shift of the S and F blocks
  size_t blk_tab[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  int64_t blk_tot[2][2] = {{0, 0}, {0, 0}};
  double flops = 0.0;
  int maxdim = cap;
  std::vector<int> hpm;
  A->last_cap.assign(L + 1, 0);
  A->lstats.assign(L + 1, {});
  A->lstats_shifts = S;
  // per-cluster bound on the dimension m over the shifts of the batch at the
  // current level (the merge sets it for the next level)
  std::vector<int> mb(A->plan[L].N, cap);
  for (int l = L; l >= 0; --l) {
    const LevelPlan& lp = A->plan[l];
    const DevLevel& dl = A->dlev[l];
    const int N = lp.N;
    A->prof.level = l;
    A->last_cap[l] = cap;
    if (cap > hqr_max_rows())
      throw NoMem{"cluster dimension " + std::to_string(cap) + " exceeds the supported maximum " +
                  std::to_string(hqr_max_rows())};
    const size_t bsz = (size_t)cap * cap;
    // level buffers: at the leaves every block is cap x cap; above, each block
    // (i, j) is cap_i x cap_j (tables written by the merge below)
    const size_t perS = l == L ? (size_t)lp.nblk() * bsz : (size_t)blk_tot[cur][0];
    const size_t perF = l == L ? (size_t)lp.nfblk() * bsz : (size_t)blk_tot[cur][1];
    size_t nS = (size_t)S * perS, nF = (size_t)S * perF;
    if (l == L) A->sf[cur].ensure((nS + nF) * 8 + 64, st);
    double* dS = (double*)A->sf[cur].p;
    double* dF = dS + nS;
    // Scratch slots of the fill-in Gram, per colour class, each sized by its
    // clusters: an M slot (j,i) and a P slot (k,i) hold R_i x R_i, a T slot
    // (k,i) R_k x R_i, and R <= m - r0 before and after the recompression.
    // Offsets run over one region per shift shared by the three buffers.
    std::vector<int64_t> soff;
    std::vector<int> sld, cslot0(lp.colours.size());
    int64_t mpt = 1;
    for (size_t c = 0; c < lp.colours.size(); ++c) {
      const ColourPlan& cp = lp.colours[c];
      cslot0[c] = (int)soff.size();
      auto rt = [&](int i) { return std::max(1, mb[i] - lp.r0[i]); };
      int64_t o = 0;
      for (int i : cp.slot_m_i) { soff.push_back(o); sld.push_back(rt(i)); o += (int64_t)rt(i) * rt(i); }
      for (int i : cp.slot_p_i) { soff.push_back(o); sld.push_back(rt(i)); o += (int64_t)rt(i) * rt(i); }
      for (size_t q = 0; q < cp.slot_p_k.size(); ++q) {
        const int k = cp.slot_p_k[q], i = cp.slot_p_i[q];
        soff.push_back(o);
        sld.push_back(rt(k));
        o += (int64_t)rt(k) * rt(i);
      }
      mpt = std::max(mpt, o);
    }
    const size_t soff_b = (soff.size() * 8 + 255) & ~(size_t)255;
    A->stab.ensure(soff_b + sld.size() * 4 + 64, st);
    if (!soff.empty()) {
      HIPCHK(hipMemcpyAsync(A->stab.p, soff.data(), soff.size() * 8, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync((char*)A->stab.p + soff_b, sld.data(), sld.size() * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));   // the host vectors go out of scope
    }
    const int64_t* d_soff = (const int64_t*)A->stab.p;
    const int* d_sld = (const int*)((const char*)A->stab.p + soff_b);
    size_t nG = (size_t)S * N * bsz, nMPT = (size_t)S * mpt, nSg = (size_t)S * N * cap;
    A->lvl.ensure((4 * nG + nMPT + nSg) * 8 + 64, st);
    if (debug_level())
      std::fprintf(stderr, "[h2eig] level %d sizes GB: S %.2f F %.2f G/V/W/Z %.2f M/P/T %.2f (N %d cap %d, %d shifts)\n", l,
                   nS * 8e-9, nF * 8e-9, 4.0 * nG * 8e-9, nMPT * 8e-9, N, cap, S);
    double* dG = (double*)A->lvl.p;
    double* dV = dG + nG;
    double* dW = dV + nG;
    double* dZ = dW + nG;
    double* dMPT = dZ + nG;
    double* dSg = dMPT + nMPT;
    BufTab bt{};
    for (int k = 0; k < NBUF; ++k) { bt.p[k] = nullptr; bt.ss[k] = 0; bt.bs[k] = (int64_t)bsz; bt.ld[k] = cap; }
    auto setb = [&](int id, double* p, size_t perShift, size_t blk, int ld) {
      bt.p[id] = p;
      bt.ss[id] = (int64_t)perShift;
      bt.bs[id] = (int64_t)blk;
      bt.ld[id] = ld;
    };
    setb(B_S, dS, perS, bsz, cap);
    setb(B_F, dF, perF, bsz, cap);
    if (l < L) {
      const char* tb = (const char*)A->tab[cur].p;
      bt.boff[B_S] = (const int64_t*)(tb + blk_tab[cur][0]);
      bt.boff[B_F] = (const int64_t*)(tb + blk_tab[cur][1]);
      bt.bld[B_S] = (const int*)(tb + blk_tab[cur][2]);
      bt.bld[B_F] = (const int*)(tb + blk_tab[cur][3]);
    }
    setb(B_G, dG, (size_t)N * bsz, bsz, cap);
    setb(B_V, dV, (size_t)N * bsz, bsz, cap);
    setb(B_W, dW, (size_t)N * bsz, bsz, cap);
    setb(B_Z, dZ, (size_t)N * bsz, bsz, cap);
    setb(B_M, dMPT, (size_t)mpt, 0, 0);
    setb(B_P, dMPT, (size_t)mpt, 0, 0);
    setb(B_T, dMPT, (size_t)mpt, 0, 0);
    setb(B_SIGN, dSg, (size_t)N * cap, (size_t)cap, cap);
    if (l >= 1) {
      const LevelPlan& lpl = A->plan[l];
      setb(B_CPL, A->d_cpl[l], 0, (size_t)std::max(1, lpl.rmax) * std::max(1, lpl.rmax), std::max(1, lpl.rmax));
    }
    Profiler& prof = A->prof;
    // profiled region: class cls, and for GEMM launches also the kernel symbol
    // (tag = GEMM layout), whose totals are kept beside the classes
    auto run = [&](int cls, auto&& fn, int tag = -1) {
      bt.f32 = (f32 && f32_class(cls)) ? 1 : 0;
      if (tag >= 0 && bt.f32) tag += 4;   // the FP32 kernel symbols follow the FP64 ones
      bt.fc = prof.on ? prof.d_fc + cls : nullptr;
      bt.fck = prof.on && tag >= 0 ? prof.d_fc + PC_N + tag : nullptr;
      bt.fbk = prof.on && tag >= 0 ? prof.d_fc + PROF_N + PC_N + tag : nullptr;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool ev = prof.on && (!prof.gemm_only || tag >= 0);
      if (ev) {
        e0 = prof.get();
        HIPCHK(hipEventRecord(e0, st));
      }
      fn();
      if (ev) {
        e1 = prof.get();
        HIPCHK(hipEventRecord(e1, st));
        prof.recs.push_back({cls | (prof.level << 16), {e0, e1}});
        if (tag >= 0) prof.recs.push_back({(PC_N + tag) | (prof.level << 16), {e0, e1}});
      }
      bt.fc = nullptr;
      bt.fck = nullptr;
      bt.fbk = nullptr;
      bt.f32 = 0;
    };
    SizeTab sz{};
    sz.m = w.m;
    sz.R = w.R;
    sz.t = w.t;
    sz.r0 = A->dp<int>(dl.r0);
    sz.pm = w.pm;
    sz.pR = w.pR;
    sz.a0 = w.a0;
    sz.a1 = w.a1;
    sz.N = N;
    sz.Np = std::max(1, N >> 1);
    sz.pr0 = l >= 1 ? A->dp<int>(dl.pr0) : nullptr;
    if (l == L) {
      bt.p[B_BRES] = A->d_bres;
      bt.ss[B_BRES] = 0;
      bt.bs[B_BRES] = (int64_t)bsz;
      bt.ld[B_BRES] = cap;
      run(PC_INIT, [&] { launch_sizes_init(sz, A->dp<int>(A->leaf_m0), S, st); });
      run(PC_INIT, [&] { launch_leaf_init(bt, lp.nblk(), A->dp<int>(A->leaf_blkdiag), w.sigma, cap, S, st); });
    }
    run(PC_INIT, [&] { launch_fill(dG, nG, 0.0, st); });
    run(PC_INIT, [&] { launch_fill(dSg, nSg, 0.0, st); });
    // one GEMM launch of class cls: launch parameters from the tuning table,
    // profiled under its kernel symbol (layout, precision, tile size)
    auto gemm = [&](int cls, int kind, const GItem* items, int n, const GTerm* terms, int mcap, int ncap) {
      if (n <= 0) return;
      const int f = (f32 && f32_class(cls)) ? 1 : 0;
      get_gemm_tuning(kind, f, gemm_bucket(std::max(mcap, ncap)), &bt.grid, &bt.group_m, &bt.tile);
      run(cls, [&] { launch_gemm(kind, items, n, terms, bt, sz, mcap, ncap, S, dpre, st); },
          kind + (bt.tile == 128 ? 8 : 0));
      bt.grid = bt.group_m = bt.tile = 0;
    };
    gemm(PC_GRAM, GEMM_NT, A->dp<GItem>(dl.gram_init.items), dl.gram_init.n, A->dp<GTerm>(dl.gram_init.terms), cap,
         cap);
    gemm(PC_GRAM, GEMM_TN, A->dp<GItem>(dl.gram_init_t.items), dl.gram_init_t.n,
         A->dp<GTerm>(dl.gram_init_t.terms), cap, cap);
    // scratch slots of the out-of-place products: about 2 GB per shift at most
    int max_items = 1;
    for (const DevColour& dc : dl.colours)
      max_items = std::max({max_items, dc.rot_rows.n, dc.rot_cols.n, dc.rot_cols_t.n, dc.trsm.n});
    const int CH = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)max_items, 65535,
                                                                (int64_t)(2LL << 30) / (int64_t)(bsz * 8)}));
    A->rs.ensure((size_t)S * CH * bsz * 8 + 64, st);
    if (debug_level()) std::fprintf(stderr, "[h2eig]   scratch slots GB: %.2f (%d slots)\n", S * CH * bsz * 8e-9, CH);
    setb(B_RS, (double*)A->rs.p, (size_t)CH * bsz, bsz, cap);
    // out-of-place products in chunks of CH scratch slots, each chunk copied
    // back (plain copies and/or transposed copies, parallel to the items)
    auto chunked = [&](int cls, int kind, const DevList& gl, size_t copies, size_t tcopies = 0, bool plain = true) {
      for (int c0 = 0; c0 < gl.n; c0 += CH) {
        int nc = std::min(CH, gl.n - c0);
        gemm(cls, kind, A->dp<GItem>(gl.items) + c0, nc, A->dp<GTerm>(gl.terms), cap, cap);
        if (plain) run(PC_COPY, [&] { launch_copyback(A->dp<CopyItem>(copies) + c0, nc, bt, sz, cap, S, st); });
        if (tcopies) run(PC_COPY, [&] { launch_copyback_t(A->dp<CopyItem>(tcopies) + c0, nc, bt, sz, S, st); });
      }
    };
    for (size_t c = 0; c < dl.colours.size(); ++c) {
      const DevColour& dc = dl.colours[c];
      {   // this class's Gram slots
        const ColourPlan& cp = lp.colours[c];
        const int m0 = cslot0[c], p0 = m0 + (int)cp.slot_m_i.size(), t0 = p0 + (int)cp.slot_p_i.size();
        bt.boff[B_M] = d_soff + m0;
        bt.bld[B_M] = d_sld + m0;
        bt.boff[B_P] = d_soff + p0;
        bt.bld[B_P] = d_sld + p0;
        bt.boff[B_T] = d_soff + t0;
        bt.bld[B_T] = d_sld + t0;
      }
      const int* cl = A->dp<int>(dc.clusters);
      auto gl = [&](int cls, int kind, const DevList& L, int mcap = 0, int ncap = 0) {
        const int mc = mcap > 0 ? mcap : cap, nc = ncap > 0 ? ncap : cap;
        gemm(cls, kind, A->dp<GItem>(L.items), L.n, A->dp<GTerm>(L.terms), mc, nc);
      };
      // pivoted Cholesky of the fill-in Gram, panel by panel (finished clusters
      // make a panel a no-op, so the counters are read back every 4 panels)
      run(PC_PCHOL, [&] { launch_pchol_init(cl, dc.ncl, bt, sz, S, st); });
      {
        const int nit = std::min(MORE_SLOTS, cap / PCHOL_NB + 2);
        HIPCHK(hipMemsetAsync(A->d_more, 0, nit * sizeof(int), st));
        for (int it = 0; it < nit; ++it) {
          run(PC_PCHOL, [&] {
            launch_pchol_panel(cl, dc.ncl, bt, sz, f32 ? A->d_tau2_f32[l] : A->d_tau2[l], A->d_more + it, cap, S, st);
          });
          gl(PC_PCHOL_UPD, GEMM_NT, dc.pc_upd);
          if (it % 4 == 3 || it == nit - 1) {
            read_back(A, A->d_more + it, 1, st);
            if (A->h_more[0] == 0) break;
          }
        }
      }
      run(PC_PCHOL, [&] { launch_pchol_finish(cl, dc.ncl, bt, sz, S, st); });
      // largest t and R of the class: exact launch counts from here on
      int* dmx = A->d_more + MORE_SLOTS;
      HIPCHK(hipMemsetAsync(dmx, 0, 3 * sizeof(int), st));
      run(PC_PCHOL, [&] { launch_colour_max(cl, dc.ncl, sz, dmx, S, st); });
      read_back(A, dmx, 3, st);
      const int tmax = A->h_more[0], rmax = A->h_more[1], nhqr = A->h_more[2];
      // Householder QR of the kept columns, panel by panel (LDS-resident panels)
      for (int it = 0; it < nhqr; ++it) {
        run(PC_HQR, [&] { launch_hqr_panel(cl, dc.ncl, bt, sz, it, dmx, S, st); });
        run(PC_HQR_UPD, [&] { launch_hqr_apply(cl, dc.ncl, bt, sz, tmax, S, st); });
      }
      // W = I - Y T Y^T (UT transform)
      if (tmax > 0) {
        gl(PC_WFORM, GEMM_TN, dc.ut_s);
        run(PC_WFORM, [&] { launch_ut_prep(cl, dc.ncl, bt, sz, cap, S, st); });
        run(PC_WFORM, [&] { launch_ut_diag_inv(cl, dc.ncl, bt, sz, cap, S, st); });
        for (int ib = 1; ib * inv_block() < tmax; ++ib) {
          run(PC_WFORM, [&] { launch_set_block(cl, dc.ncl, sz, ib, 1, S, st); });
          gl(PC_WFORM, GEMM_NN, dc.ut_t, 0, inv_block());
          gl(PC_WFORM, GEMM_NN, dc.ut_x, 0, inv_block());
        }
        gl(PC_WFORM, GEMM_NN, dc.ut_u);
        run(PC_WFORM, [&] { launch_eye(cl, dc.ncl, bt, sz, cap, S, st); });
        gl(PC_WFORM, GEMM_NT, dc.ut_w);
      }
      chunked(PC_ROTATE, GEMM_TN, dc.rot_rows, dc.rr_copy, dc.rr_copyt);
      chunked(PC_ROTATE, GEMM_NN, dc.rot_cols, dc.rc_copy);
      chunked(PC_ROTATE, GEMM_TT, dc.rot_cols_t, 0, dc.rct_copy, false);
      // pivot LDL, panel by panel (each panel takes at least ldl_panel_min()
      // pivots unless it reaches R), then the elimination operator
      run(PC_LDL, [&] { launch_ldl_init(cl, dc.ncl, bt, sz, S, st); });
      for (int it = 0; it * ldl_panel_min(cap) < rmax; ++it) {
        run(PC_LDL, [&] { launch_ldl_panel(cl, dc.ncl, A->dp<int>(dl.diag_blk), bt, sz, w.status, dmx, S, st); });
        gl(PC_LDL_UPD, GEMM_NT, dc.ldl_upd);
      }
      run(PC_LDL_OP, [&] { launch_ldl_prep(cl, dc.ncl, A->dp<int>(dl.diag_blk), bt, sz, w.nu, S, st); });
      // X = L^{-1}: diagonal blocks, then block rows by GEMMs
      run(PC_LDL_OP, [&] { launch_zero_clusters(cl, dc.ncl, bt, B_V, cap, S, st); });
      run(PC_LDL_OP, [&] { launch_diag_inv(cl, dc.ncl, A->dp<int>(dl.diag_blk), bt, sz, cap, S, st); });
      for (int ib = 1; ib * inv_block() < rmax; ++ib) {
        run(PC_LDL_OP, [&] { launch_set_block(cl, dc.ncl, sz, ib, 0, S, st); });
        gl(PC_LDL_INV, GEMM_NN, dc.inv_t, inv_block());
        gl(PC_LDL_INV, GEMM_NN, dc.inv_x, inv_block());
      }
      run(PC_LDL_OP, [&] { launch_kform(cl, dc.ncl, bt, sz, cap, S, st); });
      chunked(PC_ELIM, GEMM_NT, dc.trsm, dc.tr_copy);
      gl(PC_SCHUR, GEMM_NT, dc.schur);
      gl(PC_GRAM, GEMM_TN, dc.gm);
      if (dc.ngp)
        run(PC_GRAM, [&] { launch_matsum(A->dp<SumItem>(dc.gp_items), dc.ngp, A->dp<int>(dc.gp_src), bt, sz, cap, S, st); });
      gl(PC_GRAM, GEMM_NN, dc.gt);
      gl(PC_GRAM, GEMM_NT, dc.gg);
    }
    HIPCHK(hipGetLastError());
    // per-level statistics of the factorization (rank growth): m, R and t of
    // every cluster, read back with the merge sizes below
    std::vector<int> lm((size_t)S * N), lR((size_t)S * N), lt((size_t)S * N);
    HIPCHK(hipMemcpyAsync(lm.data(), w.m, lm.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(lR.data(), w.R, lR.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(lt.data(), w.t, lt.size() * 4, hipMemcpyDeviceToHost, st));
    auto record_stats = [&]() {
      A->lstats[l].assign((size_t)S * 4, 0);
      for (int s2 = 0; s2 < S; ++s2) {
        int64_t* o = &A->lstats[l][(size_t)s2 * 4];
        for (int i = 0; i < N; ++i) {
          const size_t k = (size_t)s2 * N + i;
          o[0] += lt[k];
          o[1] += lm[k];
          o[2] = std::max<int64_t>(o[2], lm[k]);
          o[3] += lR[k];
        }
      }
    };
    if (debug_level()) {
      debug_dump_level(l, N, S, w, st);
      std::fprintf(stderr, "[h2eig]   cap %d arenas GB: sf %.2f %.2f lvl %.2f mrg %.2f\n", cap, A->sf[0].cap / 1e9,
                   A->sf[1].cap / 1e9, A->lvl.cap / 1e9, A->mrg.cap / 1e9);
    }
    if (l == 0) {
      HIPCHK(hipStreamSynchronize(st));
      record_stats();
      break;
    }
    // ---- merge into level l-1
    const LevelPlan& pp = A->plan[l - 1];
    const int Np = N >> 1;
    run(PC_MERGE, [&] { launch_merge_sizes(sz, Np, S, st); });
    hpm.resize((size_t)S * Np);
    HIPCHK(hipMemcpyAsync(hpm.data(), w.pm, (size_t)S * Np * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    record_stats();
    int pmax = 0;
    for (int v : hpm) pmax = std::max(pmax, v);
    if (pmax == 0) break;  // nothing left above this level
    maxdim = std::max(maxdim, pmax);
    const int pcap = round_cap(pmax);
    const size_t pbsz = (size_t)pcap * pcap;
    const int other = 1 - cur;
    // each parent block (p, q) is cap_p x cap_q, cap_p the rounded largest
    // dimension of p over the shifts of the batch
    std::vector<int> pc(Np, 8);
    for (int s2 = 0; s2 < S; ++s2)
      for (int p = 0; p < Np; ++p) pc[p] = std::max(pc[p], round_cap(hpm[(size_t)s2 * Np + p]));
    mb = pc;
    std::vector<int64_t> offS(std::max(1, pp.nblk())), offF(std::max(1, pp.nfblk()));
    std::vector<int> ldS(std::max(1, pp.nblk())), ldF(std::max(1, pp.nfblk()));
    int64_t totS = 0, totF = 0;
    for (int p = 0; p < Np; ++p) {
      for (int k = pp.near_ptr[p]; k < pp.near_ptr[p + 1]; ++k) {
        offS[k] = totS;
        ldS[k] = pc[p];
        totS += (int64_t)pc[p] * pc[pp.near_idx[k]];
      }
      for (int k = pp.f_ptr[p]; k < pp.f_ptr[p + 1]; ++k) {
        offF[k] = totF;
        ldF[k] = pc[p];
        totF += (int64_t)pc[p] * pc[pp.f_idx[k]];
      }
    }
    {
      const size_t o0 = 0, o1 = (offS.size() * 8 + 255) & ~(size_t)255;
      const size_t o2 = o1 + ((offF.size() * 8 + 255) & ~(size_t)255);
      const size_t o3 = o2 + ((ldS.size() * 4 + 255) & ~(size_t)255);
      const size_t o4 = o3 + ((ldF.size() * 4 + 255) & ~(size_t)255);
      A->tab[other].ensure(o4, st);
      char* tb = (char*)A->tab[other].p;
      HIPCHK(hipMemcpyAsync(tb + o0, offS.data(), offS.size() * 8, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(tb + o1, offF.data(), offF.size() * 8, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(tb + o2, ldS.data(), ldS.size() * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(tb + o3, ldF.data(), ldF.size() * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));   // the host vectors go out of scope
      blk_tab[other][0] = o0;
      blk_tab[other][1] = o1;
      blk_tab[other][2] = o2;
      blk_tab[other][3] = o3;
      blk_tot[other][0] = std::max<int64_t>(totS, 1);
      blk_tot[other][1] = std::max<int64_t>(totF, 1);
    }
    size_t nSN = (size_t)S * blk_tot[other][0], nFN = (size_t)S * blk_tot[other][1];
    A->sf[other].ensure((nSN + nFN) * 8 + 64, st);
    double* dSN = (double*)A->sf[other].p;
    double* dFN = dSN + nSN;
    const MergePlan& mp = lp.merge;
    const int nslot = std::max(1, std::min(mp.nhat, MERGE_CHUNK));
    const int emax = std::max(1, mp.emax);
    const size_t ebsz = (size_t)emax * emax;
    size_t nH = (size_t)S * nslot * pbsz, nTm = (size_t)S * nslot * ebsz;
    A->mrg.ensure((nH + nTm) * 8 + 64, st);
    if (debug_level())
      std::fprintf(stderr, "[h2eig] merge %d -> %d sizes GB: next S %.2f F %.2f, hat %.2f tmp %.2f (pcap %d, %d slots)\n", l,
                   l - 1, nSN * 8e-9, nFN * 8e-9, nH * 8e-9, nTm * 8e-9, pcap, nslot);
    double* dH = (double*)A->mrg.p;
    double* dTm = dH + nH;
    setb(B_HAT, dH, (size_t)nslot * pbsz, pbsz, pcap);
    setb(B_TMP, dTm, (size_t)nslot * ebsz, ebsz, emax);
    setb(B_SN, dSN, (size_t)blk_tot[other][0], pbsz, pcap);
    setb(B_FN, dFN, (size_t)blk_tot[other][1], pbsz, pcap);
    {
      const char* tb = (const char*)A->tab[other].p;
      bt.boff[B_SN] = (const int64_t*)(tb + blk_tab[other][0]);
      bt.boff[B_FN] = (const int64_t*)(tb + blk_tab[other][1]);
      bt.bld[B_SN] = (const int*)(tb + blk_tab[other][2]);
      bt.bld[B_FN] = (const int*)(tb + blk_tab[other][3]);
    }
    setb(B_EMAT, A->d_emat[l - 1], 0, (size_t)A->emat_ld[l - 1] * A->emat_ld[l - 1], A->emat_ld[l - 1]);
    for (const MergeChunk& ch : mp.chunks) {
      run(PC_MERGE, [&] { launch_gather(A->dp<GatherItem>(dl.gather) + ch.g0, ch.g1 - ch.g0, bt, sz, pcap, S, st); });
      gemm(PC_MERGE_FILL, GEMM_NT, A->dp<GItem>(dl.fill.items) + ch.f0, ch.f1 - ch.f0, A->dp<GTerm>(dl.fill.terms),
           pcap, pcap);
      run(PC_MERGE, [&] { launch_merge_nn(A->dp<GatherItem>(dl.gather) + ch.g0, ch.g1 - ch.g0, bt, sz, pcap, S, st); });
      gemm(PC_MERGE_E, GEMM_NN, A->dp<GItem>(dl.tr1.items) + ch.a0, ch.a1 - ch.a0, A->dp<GTerm>(dl.tr1.terms), pcap,
           emax);
      gemm(PC_MERGE_E, GEMM_TN, A->dp<GItem>(dl.tr2.items) + ch.b0, ch.b1 - ch.b0, A->dp<GTerm>(dl.tr2.terms), emax,
           pcap);
    }
    // parent blocks (p,q), q < p: transposed copies of the finished (q,p)
    if (dl.nmirror) run(PC_MERGE, [&] { launch_copyback_t(A->dp<CopyItem>(dl.mirror), dl.nmirror, bt, sz, S, st); });
    run(PC_MERGE, [&] { launch_next_sizes(sz, S, st); });
    HIPCHK(hipGetLastError());
    cur = other;
    cap = pcap;
  }
  std::vector<unsigned long long> hnu(S);
  std::vector<int> hst(S);
  HIPCHK(hipMemcpyAsync(hnu.data(), w.nu, S * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hst.data(), w.status, S * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (A->prof.on) A->prof.collect();
  for (int s = 0; s < S; ++s) {
    nu_out[s] = hst[s] ? -1 : (int64_t)hnu[s];
    if (st_out) st_out[s] = hst[s] ? H2_ENUMERIC : H2_OK;
  }
  if (flops_out) *flops_out = flops;
  if (maxdim_out) *maxdim_out = maxdim;
}

// Gershgorin interval [min_i A_ii - rad_i, max_i A_ii + rad_i] of the kernel
// matrix, rad_i = sum_{j != i} |A_ij| over all n points, computed on the device
// once per handle.
void ensure_gershgorin(h2_matrix A) {
  if (A->have_gersh) return;
  const Tree& T = A->T;
  const int64_t n = T.n;
  hipStream_t st = A->stream;
  double *dX = nullptr, *drad = nullptr;
  struct Guard {
    double** a;
    double** b;
    ~Guard() {
      if (*a) (void)h2::dev_free(*a);
      if (*b) (void)h2::dev_free(*b);
    }
  } guard{&dX, &drad};
  HIPCHK(h2::dev_malloc(&dX, (size_t)n * T.dim * 8));
  HIPCHK(h2::dev_malloc(&drad, (size_t)n * 8));
  HIPCHK(hipMemcpyAsync(dX, T.X.data(), (size_t)n * T.dim * 8, hipMemcpyHostToDevice, st));
  launch_row_abs_sum(dX, n, T.dim, A->kern.kind, A->kern.p0, A->kern.p1, drad, st);
  HIPCHK(hipGetLastError());
  std::vector<double> rad(n);
  HIPCHK(hipMemcpyAsync(rad.data(), drad, (size_t)n * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double rmax = *std::max_element(rad.begin(), rad.end());
  A->g_lo = A->kern.diag - rmax;
  A->g_hi = A->kern.diag + rmax;
  A->have_gersh = true;
}

int auto_max_shifts(h2_matrix A) {
  if (A->max_shifts > 0) return A->max_shifts;
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) {
    (void)hipGetLastError();
    return 4;
  }
  if (A->ws_per_shift > 0) {
    // measured: the workspace of the last factorization per shift, against the
    // free memory plus what the handle's arenas already hold
    const double held = (double)(A->sf[0].cap + A->sf[1].cap + A->lvl.cap + A->mrg.cap + A->rs.cap);
    const int s = (int)std::floor(0.92 * ((double)freeb + held) / (1.04 * A->ws_per_shift));
    return std::max(1, std::min(s, 64));
  }
  const LevelPlan& lf = A->plan[A->T.L];
  double per = (double)A->leafcap * A->leafcap * 8.0 * (lf.nblk() + 4.0 * lf.N + lf.max_slot_m + 2.0 * lf.max_slot_p);
  per *= 2.2;  // upper levels and merge buffers
  int s = (int)std::floor(0.7 * (double)freeb / std::max(per, 1.0));
  return std::max(1, std::min(s, 64));
}

// nu(sigma_s) for every shift, in batches of at most the handle's capacity;
// FP64 counts join the handle's record cache, FP32 counts (f32) do not.
h2_status run_inertia(h2_matrix A, const double* sigma, int64_t ns, bool f32, int64_t* nu, int32_t* status) {
  int maxs = auto_max_shifts(A);
  bool anybad = false;
  auto t0 = std::chrono::steady_clock::now();
  for (int64_t s0 = 0; s0 < ns;) {
    int S = (int)std::min<int64_t>(maxs, ns - s0);
    try {
      int md = 0;
      factor_batch(A, sigma + s0, S, f32, nu + s0, status ? status + s0 : nullptr, nullptr, &md);
      A->arena_shifts = std::max(A->arena_shifts, S);
      A->st.last_rank_max = std::max(A->st.last_rank_max, md);
    } catch (NoMem&) {
      if (S == 1) throw;
      maxs = std::max(1, S / 2);
      A->max_shifts = maxs;
      for (auto& a : A->sf) a.release();
      A->lvl.release();
      A->mrg.release();
      A->rs.release();
      for (auto& a : A->tab) a.release();
      A->stab.release();
      A->arena_shifts = 0;
      continue;
    }
    for (int k = 0; k < S; ++k) {
      if (nu[s0 + k] < 0) anybad = true;
      else if (!f32) h2::record_insert(A->cache, sigma[s0 + k], nu[s0 + k]);
    }
    if (!f32) h2::record_compact(A->cache);
    int32_t& cnt = f32 ? A->st.evals_f32 : A->st.evals_f64;
    cnt = (int32_t)std::min<int64_t>(INT32_MAX, (int64_t)cnt + S);
    s0 += S;
  }
  (void)t0;
  int64_t ws = (int64_t)(A->sf[0].cap + A->sf[1].cap + A->lvl.cap + A->mrg.cap + A->small.cap + A->rs.cap);
  A->st.last_work_bytes = ws;
  if (A->arena_shifts > 0) A->ws_per_shift = (double)ws / (double)A->arena_shifts;
  return anybad ? H2_ENUMERIC : H2_OK;
}

}  // namespace

// error message of the calling thread, shared with the serving loop
namespace h2 {
void set_last_error(const std::string& msg) { g_err = msg; }

// ------------------------------------------------------- device allocations
namespace {
struct AllocHook {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
std::mutex g_alloc_mu;
AllocHook g_hook;                                     // the allocator for new blocks
std::atomic<bool> g_hook_used{false};                 // a hook was ever installed
std::unordered_map<void*, AllocHook> g_hook_blocks;   // blocks from a hook, by address
}  // namespace

hipError_t dev_malloc_bytes(void** p, size_t bytes) {
  AllocHook h;
  {
    std::lock_guard<std::mutex> g(g_alloc_mu);
    h = g_hook;
  }
  if (!h.alloc) return hipMalloc(p, bytes);
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  void* q = h.alloc(bytes, h.ctx);
  if (!q) return hipErrorOutOfMemory;
  std::lock_guard<std::mutex> g(g_alloc_mu);
  g_hook_blocks[q] = h;
  *p = q;
  return hipSuccess;
}

hipError_t dev_free(void* p) {
  if (!p) return hipSuccess;
  AllocHook h;
  bool hooked = false;
  if (g_hook_used.load()) {
    std::lock_guard<std::mutex> g(g_alloc_mu);
    auto it = g_hook_blocks.find(p);
    if (it != g_hook_blocks.end()) {
      h = it->second;
      g_hook_blocks.erase(it);
      hooked = true;
    }
  }
  if (!hooked) return hipFree(p);
  const hipError_t e = hipDeviceSynchronize();   // as hipFree: no queued kernel may still use the block
  h.release(p, h.ctx);
  return e;
}
}  // namespace h2

// =================================================================== C ABI
static h2_status inertia_impl(h2_matrix A, const double* sigma, int64_t nshift, bool f32, int64_t* nu, int32_t* status) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  if (nshift < 0 || (nshift > 0 && (!sigma || !nu))) return fail(H2_EINVAL, "bad shift arrays");
  for (int64_t s = 0; s < nshift; ++s)
    if (!std::isfinite(sigma[s])) return fail(H2_EINVAL, "non-finite shift");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  if (nshift == 0) return H2_OK;
  try {
    HIPCHK(hipSetDevice(A->device));
    h2_status r = run_inertia(A, sigma, nshift, f32, nu, status);
    if (r != H2_OK) return fail(r, "singular or non-finite pivot block for at least one shift");
    return H2_OK;
  } catch (HipError& e) {
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (NoMem& e) {
    return fail(H2_ENOMEM, e.what);
  }
}

extern "C" {

const char* h2_last_error(void) { return g_err.c_str(); }

h2_status h2_build(const double* points, int64_t n, int32_t dim, h2_kernel kern, int32_t leaf, double eta, double eps,
                   const h2_opts* opts, h2_matrix* out) {
  if (!out) return fail(H2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!points || n < 1) return fail(H2_EINVAL, "n must be >= 1 and points non-NULL");
  if (opts && (opts->reserved0 != 0 || opts->reserved1 != 0)) return fail(H2_EINVAL, "reserved options must be 0");
  if (dim < 1 || dim > 3) return fail(H2_EINVAL, "dim must be 1, 2 or 3");
  if (leaf < 2 && n > 1) return fail(H2_EINVAL, "leaf must be >= 2");
  if (!(eta > 0.0) || !(eps > 0.0)) return fail(H2_EINVAL, "eta and eps must be > 0");
  if (kern.kind < 0 || kern.kind > 4) return fail(H2_EINVAL, "unknown kernel kind");
  if (!std::isfinite(kern.diag) || !std::isfinite(kern.p0) || !std::isfinite(kern.p1))
    return fail(H2_EINVAL, "non-finite kernel parameter");
  if ((kern.kind == H2_K_GAUSS_DAMPED || kern.kind == H2_K_TRIDIAG_1D) && !(kern.p0 > 0.0))
    return fail(H2_EINVAL, "kernel parameter p0 must be > 0");
  for (int64_t i = 0; i < n * dim; ++i)
    if (!std::isfinite(points[i])) return fail(H2_EINVAL, "non-finite point coordinate");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(H2_EDEVICE, "no HIP device available");
  }
  h2_matrix A = new h2_matrix_s();
  auto t0 = std::chrono::steady_clock::now();
  try {
    HIPCHK(hipGetDevice(&A->device));
    HIPCHK(hipStreamCreateWithFlags(&A->own_stream, hipStreamNonBlocking));
    A->stream = A->own_stream;
    A->kern = KernelSpec{kern.kind, kern.diag, kern.p0, kern.p1};
    A->eps = eps;
    build_tree(A->T, points, n, dim, leaf, eta);
    A->normA = estimate_norm(A->T, A->kern);
    A->tau = eps * A->normA;
    BuildParams P;
    P.kern = A->kern;
    P.eps = eps;
    if (opts && opts->max_shifts > 0) A->max_shifts = opts->max_shifts;
    build_basis(A->T, P, A->tau, A->B, A->stream);
    A->plan = build_plan(A->T, A->B);
    int L = A->T.L;
    A->leafcap = 0;
    for (int i = 0; i < (1 << L); ++i) A->leafcap = std::max<int>(A->leafcap, (int)A->T.size[L][i]);
    A->leafcap = round_cap(A->leafcap);
    HIPCHK(h2::dev_malloc(&A->d_more, (MORE_SLOTS + 4) * sizeof(int)));
    A->d_tau2.assign(L + 1, nullptr);
    A->d_tau2_f32.assign(L + 1, nullptr);
    const double tau32 = std::max(eps, EPS_F32) * A->normA;
    for (int l = 0; l <= L; ++l) {
      std::vector<double> t2(1 << l), t32(1 << l);
      for (int i = 0; i < (1 << l); ++i) {
        const double share = (double)A->T.size[l][i] / (double)A->T.n;
        t2[i] = A->tau * A->tau * share;
        t32[i] = tau32 * tau32 * share;
      }
      HIPCHK(h2::dev_malloc(&A->d_tau2[l], t2.size() * sizeof(double)));
      HIPCHK(hipMemcpy(A->d_tau2[l], t2.data(), t2.size() * sizeof(double), hipMemcpyHostToDevice));
      HIPCHK(h2::dev_malloc(&A->d_tau2_f32[l], t32.size() * sizeof(double)));
      HIPCHK(hipMemcpy(A->d_tau2_f32[l], t32.data(), t32.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    HIPCHK(hipHostMalloc(&A->h_more, 4 * sizeof(int)));
    upload_plan(A);
    upload_resident(A);
    build_near_blocks(A);
    HIPCHK(hipStreamSynchronize(A->stream));
  } catch (HipError& e) {
    h2_free(A);
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (NoMem& e) {
    h2_free(A);
    return fail(H2_ENOMEM, e.what);
  } catch (std::invalid_argument& e) {
    h2_free(A);
    return fail(H2_EINVAL, e.what());
  } catch (std::bad_alloc&) {
    h2_free(A);
    return fail(H2_ENOMEM, "host allocation failed");
  } catch (std::runtime_error& e) {
    h2_free(A);
    return fail(H2_EDEVICE, e.what());
  }
  const Tree& T = A->T;
  A->st.n = T.n;
  A->st.levels = T.L;
  A->st.leaf_max = A->leafcap;
  int rmax = 0, nmax = 0;
  for (int l = 0; l <= T.L; ++l) {
    for (int v : A->B.r[l]) rmax = std::max(rmax, v);
    for (auto& v : T.near[l]) nmax = std::max(nmax, (int)v.size());
  }
  A->st.rank_max = rmax;
  A->st.near_max = nmax;
  A->st.near_blocks = A->plan[T.L].nblk();
  A->st.resident_bytes = A->resident;
  A->st.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = A;
  return H2_OK;
}


h2_status h2_inertia(h2_matrix A, const double* sigma, int64_t nshift, int64_t* nu, int32_t* status) {
  return inertia_impl(A, sigma, nshift, false, nu, status);
}

h2_status h2_inertia_f32(h2_matrix A, const double* sigma, int64_t nshift, int64_t* nu, int32_t* status) {
  return inertia_impl(A, sigma, nshift, true, nu, status);
}

h2_status h2_set_mixed(h2_matrix A, double switch_rel) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  if (!(switch_rel >= 0.0) || !std::isfinite(switch_rel)) return fail(H2_EINVAL, "switch_rel must be finite and >= 0");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  A->mixed_rel = switch_rel;
  return H2_OK;
}

h2_status h2_kth_eig(h2_matrix A, const int64_t* k, int64_t nk, double tol, const double* ab, double* lambda,
                     double* bracket) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  if (nk < 0 || (nk > 0 && (!k || !lambda))) return fail(H2_EINVAL, "bad index arrays");
  if (!(tol > 0.0)) return fail(H2_EINVAL, "tol must be > 0");
  const int64_t n = A->T.n;
  for (int64_t j = 0; j < nk; ++j)
    if (k[j] < 1 || k[j] > n) return fail(H2_EINVAL, "k out of range [1, n]");
  double a0, b0;
  if (ab) {
    a0 = ab[0];
    b0 = ab[1];
    if (!(std::isfinite(a0) && std::isfinite(b0) && a0 < b0)) return fail(H2_EINVAL, "bad interval ab");
  } else {
    double iv[2];
    const h2_status r = h2_interval(A, iv);
    if (r != H2_OK) return r;
    a0 = iv[0];
    b0 = iv[1];
  }
  if (nk == 0) return H2_OK;
  // mixed precision: FP32 steps while a bracket is at least thr wide
  const double thr = A->mixed_rel > 0.0 ? A->mixed_rel * A->normA : 0.0;
  std::vector<double> lo(nk, a0), hi(nk, b0), sp(nk);
  // split point of bracket j: the midpoint, moved by nudge[j]/64 of the width
  // after a shift there met an exactly singular pivot (any point strictly
  // inside the bracket keeps bisection correct)
  std::vector<int> nudge(nk, 0);
  // phase of bracket j: 0 FP32 steps; 1 switched to FP64, its ends (set by
  // FP32 counts) get FP64 counts this step; 2 FP64 steps on a bracket whose
  // ends all have FP64 counts
  std::vector<int> phase(nk, thr > 0.0 ? 0 : 2);
  // FP64 counts narrow every bracket, FP32 counts only brackets in phase 0
  auto narrow = [&](double mu, int64_t v, bool fp32) {
    for (int64_t j = 0; j < nk; ++j) {
      if (fp32 && phase[j] != 0) continue;
      if (!(mu > lo[j] && mu < hi[j])) continue;
      if (v >= k[j]) hi[j] = mu;
      else lo[j] = mu;
    }
  };
  auto has64 = [&](double mu) { return h2::record_has(A->cache, mu); };
  // the bracket of j from FP64 counts alone: the largest shift below k
  // eigenvalues, then the smallest shift above it with at least k
  auto rebuild = [&](int64_t j) { h2::record_bracket(A->cache, k[j], a0, b0, &lo[j], &hi[j]); };
  for (auto& rec : A->cache) narrow(rec.first, rec.second, false);
  const char* pe = std::getenv("H2EIG_PROGRESS");
  const bool progress = pe && pe[0] == '1';
  for (int step = 1;; ++step) {
    std::vector<double> m32, m64;
    std::vector<char> act(nk, 0), verify(nk, 0);
    for (int64_t j = 0; j < nk; ++j) {
      // to FP64 below thr, or before the bracket would end at tol with ends
      // that only FP32 counts set (tol >= thr)
      if (phase[j] == 0 && hi[j] - lo[j] < std::max(thr, tol)) phase[j] = 1;
      if (phase[j] == 1) {
        if (lo[j] != a0 && !has64(lo[j])) m64.push_back(lo[j]), verify[j] = 1;
        if (hi[j] != b0 && !has64(hi[j])) m64.push_back(hi[j]), verify[j] = 1;
        if (verify[j]) continue;
        rebuild(j);
        phase[j] = 2;
      }
      sp[j] = lo[j] + (hi[j] - lo[j]) * (0.5 + nudge[j] / 64.0);
      // active while wider than tol and still splittable in double precision
      if (hi[j] - lo[j] >= tol && sp[j] > lo[j] && sp[j] < hi[j]) {
        act[j] = 1;
        (phase[j] == 0 ? m32 : m64).push_back(sp[j]);
      }
    }
    if (m32.empty() && m64.empty()) break;
    for (auto* v : {&m32, &m64}) {
      std::sort(v->begin(), v->end());
      v->erase(std::unique(v->begin(), v->end()), v->end());
    }
    std::vector<int64_t> n32(m32.size()), n64(m64.size());
    std::vector<int32_t> s32(m32.size()), s64(m64.size());
    if (!m64.empty()) {
      h2_status r = h2_inertia(A, m64.data(), (int64_t)m64.size(), n64.data(), s64.data());
      if (r != H2_OK && r != H2_ENUMERIC) return r;
    }
    if (!m32.empty()) {
      h2_status r = h2_inertia_f32(A, m32.data(), (int64_t)m32.size(), n32.data(), s32.data());
      if (r != H2_OK && r != H2_ENUMERIC) return r;
    }
    for (int64_t j = 0; j < nk; ++j) {
      if (!act[j]) continue;
      const auto& m = phase[j] == 0 ? m32 : m64;
      const auto& sv = phase[j] == 0 ? s32 : s64;
      const size_t q = std::lower_bound(m.begin(), m.end(), sp[j]) - m.begin();
      if (sv[q] == H2_OK) {
        nudge[j] = 0;
      } else if (++nudge[j] > 8) {
        return fail(H2_ENUMERIC, "singular pivot block at every split point tried");
      }
    }
    if (progress) {
      int64_t open = 0;
      for (int64_t j = 0; j < nk; ++j) open += act[j] || verify[j];
      std::fprintf(stderr, "[h2eig] kth_eig step %d: %zu FP64 + %zu FP32 shifts for %lld open brackets\n", step,
                   m64.size(), m32.size(), (long long)open);
    }
    for (size_t q = 0; q < m64.size(); ++q)
      if (s64[q] == H2_OK) narrow(m64[q], n64[q], false);
    for (size_t q = 0; q < m32.size(); ++q)
      if (s32[q] == H2_OK) narrow(m32[q], n32[q], true);
    // brackets whose ends were just counted in FP64: rebuilt from FP64 counts
    for (int64_t j = 0; j < nk; ++j)
      if (verify[j]) {
        rebuild(j);
        phase[j] = 2;
      }
  }
  for (int64_t j = 0; j < nk; ++j) {
    lambda[j] = 0.5 * (lo[j] + hi[j]);
    if (bracket) {
      bracket[2 * j] = lo[j];
      bracket[2 * j + 1] = hi[j];
    }
  }
  return H2_OK;
}

h2_status h2_interval(h2_matrix A, double* ab) {
  if (!A || !ab) return fail(H2_EINVAL, "NULL argument");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  try {
    HIPCHK(hipSetDevice(A->device));
    ensure_gershgorin(A);
  } catch (HipError& e) {
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  const double mg = 10.0 * A->eps * A->normA;
  ab[0] = A->g_lo - mg;
  ab[1] = A->g_hi + mg;
  return H2_OK;
}

h2_status h2_release_workspace(h2_matrix A) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  try {
    HIPCHK(hipSetDevice(A->device));
    HIPCHK(hipStreamSynchronize(A->stream));
  } catch (HipError& e) {
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  for (auto& a : A->sf) a.release();
  A->lvl.release();
  A->mrg.release();
  A->rs.release();
  for (auto& a : A->tab) a.release();
  A->stab.release();
  A->arena_shifts = 0;
  return H2_OK;
}

h2_status h2_count(h2_matrix A, double a, double b, int64_t* count) {
  if (!A || !count) return fail(H2_EINVAL, "NULL argument");
  if (!(std::isfinite(a) && std::isfinite(b) && a <= b)) return fail(H2_EINVAL, "need finite a <= b");
  const double sig[2] = {a, b};
  int64_t nu[2];
  const h2_status r = h2_inertia(A, sig, 2, nu, nullptr);
  if (r != H2_OK) return r;
  *count = nu[1] - nu[0];
  return H2_OK;
}

h2_status h2_eigs_in(h2_matrix A, double a, double b, double tol, int64_t cap, double* lambda, int64_t* count) {
  if (!A || !count || (cap > 0 && !lambda)) return fail(H2_EINVAL, "NULL argument");
  if (!(std::isfinite(a) && std::isfinite(b) && a < b)) return fail(H2_EINVAL, "need finite a < b");
  if (!(tol > 0.0)) return fail(H2_EINVAL, "tol must be > 0");
  const double sig[2] = {a, b};
  int64_t nu[2];
  h2_status r = h2_inertia(A, sig, 2, nu, nullptr);
  if (r != H2_OK) return r;
  *count = nu[1] - nu[0];
  if (*count > cap) return fail(H2_EINVAL, "more eigenvalues in [a, b) than cap (count returned)");
  if (*count == 0) return H2_OK;
  std::vector<int64_t> ks((size_t)*count);
  for (int64_t j = 0; j < *count; ++j) ks[j] = nu[0] + 1 + j;
  const double ab[2] = {a, b};
  return h2_kth_eig(A, ks.data(), *count, tol, ab, lambda, nullptr);
}

h2_status h2_gap(h2_matrix A, int64_t k, double tol, double* lambda2, double* gap) {
  if (!A || !gap) return fail(H2_EINVAL, "NULL argument");
  if (k < 1 || k >= A->T.n) return fail(H2_EINVAL, "k must be in [1, n-1]");
  const int64_t ks[2] = {k, k + 1};
  double lam[2];
  const h2_status r = h2_kth_eig(A, ks, 2, tol, nullptr, lam, nullptr);
  if (r != H2_OK) return r;
  if (lambda2) {
    lambda2[0] = lam[0];
    lambda2[1] = lam[1];
  }
  *gap = lam[1] - lam[0];
  return H2_OK;
}

h2_status h2_set_gemm_tuning(int32_t layout, int32_t f32, int32_t bucket, int32_t grid, int32_t group_m,
                             int32_t tile) {
  if (layout < 0 || layout > 3 || f32 < 0 || f32 > 1 || bucket < 0 || bucket >= GEMM_BUCKETS)
    return fail(H2_EINVAL, "layout, f32 or bucket out of range");
  if (grid != 0 && (grid < 8 || grid > 65536 || grid % 8 != 0))
    return fail(H2_EINVAL, "grid must be 0 or a multiple of 8 in [8, 65536]");
  if (group_m < 0 || group_m > 64) return fail(H2_EINVAL, "group_m must be in [0, 64]");
  if (tile != 0 && tile != 64 && tile != 128) return fail(H2_EINVAL, "tile must be 0, 64 or 128");
  set_gemm_tuning(layout, f32, bucket, grid, group_m, tile);
  return H2_OK;
}

h2_status h2_get_gemm_tuning(int32_t layout, int32_t f32, int32_t bucket, int32_t* grid, int32_t* group_m,
                             int32_t* tile) {
  if (layout < 0 || layout > 3 || f32 < 0 || f32 > 1 || bucket < 0 || bucket >= GEMM_BUCKETS || !grid || !group_m ||
      !tile)
    return fail(H2_EINVAL, "layout, f32 or bucket out of range, or NULL output");
  int g = 0, gm = 0, t = 0;
  get_gemm_tuning(layout, f32, bucket, &g, &gm, &t);
  *grid = g;
  *group_m = gm;
  *tile = t;
  return H2_OK;
}

h2_status h2_level_dims(h2_matrix A, int32_t nlev, int32_t* cap) {
  if (!A || !cap || nlev < 0) return fail(H2_EINVAL, "NULL argument or nlev < 0");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  for (int32_t l = 0; l < nlev; ++l) cap[l] = l < (int32_t)A->last_cap.size() ? A->last_cap[l] : 0;
  return H2_OK;
}

h2_status h2_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (release == nullptr)) return fail(H2_EINVAL, "alloc and release must both be set or both be NULL");
  std::lock_guard<std::mutex> g(h2::g_alloc_mu);
  h2::g_hook.alloc = alloc;
  h2::g_hook.release = release;
  h2::g_hook.ctx = alloc ? ctx : nullptr;
  if (alloc) h2::g_hook_used.store(true);
  return H2_OK;
}

h2_status h2_set_max_shifts(h2_matrix A, int32_t max_shifts) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  if (max_shifts < 0) return fail(H2_EINVAL, "max_shifts must be >= 0");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  A->max_shifts = max_shifts;
  return H2_OK;
}

h2_status h2_capacity(h2_matrix A, int32_t* max_shifts) {
  if (!A || !max_shifts) return fail(H2_EINVAL, "NULL argument");
  try {
    HIPCHK(hipSetDevice(A->device));
    *max_shifts = auto_max_shifts(A);
  } catch (HipError& e) {
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  return H2_OK;
}

h2_status h2_norm(h2_matrix A, double* normA) {
  if (!A || !normA) return fail(H2_EINVAL, "NULL argument");
  *normA = A->normA;
  return H2_OK;
}

h2_status h2_stats(h2_matrix A, h2_stats_t* out) {
  if (!A || !out) return fail(H2_EINVAL, "NULL argument");
  *out = A->st;
  return H2_OK;
}

h2_status h2_set_stream(h2_matrix A, void* hip_stream) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  A->stream = hip_stream ? (hipStream_t)hip_stream : A->own_stream;
  return H2_OK;
}

h2_status h2_tree_perm(h2_matrix A, int64_t* perm) {
  if (!A || !perm) return fail(H2_EINVAL, "NULL argument");
  std::copy(A->T.perm.begin(), A->T.perm.end(), perm);
  return H2_OK;
}

h2_status h2_level_stats(h2_matrix A, int32_t shift, int32_t nlev, int64_t* out) {
  if (!A || !out) return fail(H2_EINVAL, "NULL argument");
  if (shift < 0 || shift >= A->lstats_shifts) return fail(H2_EINVAL, "shift out of range of the last factorization");
  for (int l = 0; l < nlev; ++l)
    for (int k = 0; k < 4; ++k)
      out[l * 4 + k] = (l <= A->T.L && (size_t)shift * 4 + k < A->lstats[l].size()) ? A->lstats[l][(size_t)shift * 4 + k]
                                                                                : 0;
  return H2_OK;
}

h2_status h2_basis_ranks(h2_matrix A, int32_t level, int32_t* r) {
  if (!A || !r) return fail(H2_EINVAL, "NULL argument");
  if (level < 0 || level > A->T.L) return fail(H2_EINVAL, "level out of range");
  for (int i = 0; i < (1 << level); ++i) r[i] = A->B.r[level][i];
  return H2_OK;
}

h2_status h2_matvec(h2_matrix A, const double* x, double* y) {
  if (!A || !x || !y) return fail(H2_EINVAL, "NULL argument");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  try {
    h2_matvec_host(A->T, A->kern, A->B, x, y);
  } catch (std::bad_alloc&) {
    return fail(H2_ENOMEM, "host allocation failed");
  }
  return H2_OK;
}

h2_status h2_kernel_matvec(h2_matrix A, const double* x, double* y) {
  if (!A || !x || !y) return fail(H2_EINVAL, "NULL argument");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  try {
    HIPCHK(hipSetDevice(A->device));
    kernel_matvec_gpu(A->T.X.data(), A->T.n, A->T.dim, A->kern.kind, A->kern.diag, A->kern.p0, A->kern.p1, x, y,
                      A->stream);
  } catch (HipError& e) {
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  } catch (std::runtime_error& e) {
    return fail(H2_EDEVICE, e.what());
  }
  return H2_OK;
}

h2_status h2_kernel_matvec_noalloc(h2_matrix A, const double* x, double* y) {
  if (!A || !x || !y) return fail(H2_EINVAL, "NULL argument");
  if (A->T.n > kernel_matvec_noalloc_max_n(A->T.dim))
    return fail(H2_EINVAL, "n = " + std::to_string(A->T.n) + " exceeds the static scratch (at most " +
                               std::to_string(kernel_matvec_noalloc_max_n(A->T.dim)) + " points)");
  Busy b(A);
  if (!b.ok) return fail(H2_EBUSY, "handle in use by another thread");
  try {
    kernel_matvec_noalloc(A->T.X.data(), A->T.n, A->T.dim, A->kern.kind, A->kern.diag, A->kern.p0, A->kern.p1, x, y,
                          A->device, A->stream);
  } catch (std::invalid_argument& e) {
    return fail(H2_EINVAL, e.what());
  } catch (std::runtime_error& e) {
    return fail(H2_EDEVICE, e.what());
  }
  return H2_OK;
}

h2_status h2_profile_enable(h2_matrix A, int32_t enable) {
  if (!A) return fail(H2_EINVAL, "NULL handle");
  try {
    HIPCHK(hipSetDevice(A->device));
    if (enable && !A->prof.d_fc) {
      HIPCHK(h2::dev_malloc(&A->prof.d_fc, 2 * PROF_N * sizeof(unsigned long long)));
      HIPCHK(hipMemset(A->prof.d_fc, 0, 2 * PROF_N * sizeof(unsigned long long)));
    }
  } catch (HipError& e) {
    return fail(H2_EDEVICE, e.where + ": " + hipGetErrorString(e.e));
  }
  A->prof.on = enable != 0;
  A->prof.gemm_only = enable == 2;
  A->prof.reset();
  return H2_OK;
}

int32_t h2_profile_classes(void) { return PROF_N; }

const char* h2_profile_class_name(int32_t cls) {
  if (cls >= 0 && cls < PC_N) return kProfNames[cls];
  if (cls >= PC_N && cls < PROF_N) return kGemmNames[cls - PC_N];
  return "";
}

h2_status h2_profile_read(h2_matrix A, int32_t cls, int64_t* launches, double* ms, double* flops) {
  if (!A || cls < 0 || cls >= PROF_N) return fail(H2_EINVAL, "bad handle or class");
  if (launches) *launches = A->prof.launches[cls];
  if (ms) *ms = A->prof.ms[cls];
  if (flops) *flops = (double)A->prof.flops[cls];
  return H2_OK;
}

h2_status h2_profile_bytes(h2_matrix A, int32_t cls, double* bytes) {
  if (!A || cls < 0 || cls >= PROF_N || !bytes) return fail(H2_EINVAL, "bad arguments");
  *bytes = (double)A->prof.bytes[cls];
  return H2_OK;
}

h2_status h2_profile_level_ms(h2_matrix A, int32_t cls, int32_t level, double* ms) {
  if (!A || cls < 0 || cls >= PROF_N || level < 0 || level >= 32 || !ms) return fail(H2_EINVAL, "bad arguments");
  *ms = A->prof.ms_level[cls][level];
  return H2_OK;
}

void h2_free(h2_matrix A) {
  if (!A) return;
  (void)hipSetDevice(A->device);
  if (A->stream) (void)hipStreamSynchronize(A->stream);
  for (auto& a : A->sf) a.release();
  A->lvl.release();
  A->mrg.release();
  A->small.release();
  A->rs.release();
  for (auto& a : A->tab) a.release();
  A->stab.release();
  if (A->d_bres) (void)h2::dev_free(A->d_bres);
  for (auto p : A->d_cpl)
    if (p) (void)h2::dev_free(p);
  for (auto p : A->d_emat)
    if (p) (void)h2::dev_free(p);
  if (A->d_plan) (void)h2::dev_free(A->d_plan);
  A->prof.release();
  if (A->d_more) (void)h2::dev_free(A->d_more);
  for (double* p : A->d_tau2)
    if (p) (void)h2::dev_free(p);
  for (double* p : A->d_tau2_f32)
    if (p) (void)h2::dev_free(p);
  if (A->h_more) (void)hipHostFree(A->h_more);
  if (A->own_stream) (void)hipStreamDestroy(A->own_stream);
  delete A;
}

}  // extern "C"
