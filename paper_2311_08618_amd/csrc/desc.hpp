// Work descriptors of the level-by-level factorization.  They are built once
// per matrix on the host (the block structure does not depend on the shift)
// and resolved on the device per shift, because the redundant/skeleton split of
// every cluster depends on the shift through fill-in recompression.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#define __device__
#endif
#endif

namespace h2 {

// ---------------------------------------------------------- size expressions
// A size expression is (kind << 24) | arg, evaluated per shift on the device.
enum DimKind : int {
  DK_CONST = 0,  // arg
  DK_M = 1,      // m(c): current dimension of cluster c at this level
  DK_R = 2,      // R(c): current redundant count
  DK_S = 3,      // m(c) - R(c): skeleton count (after elimination: kept part)
  DK_T = 4,      // t(c): directions added by this level's recompression of c
  DK_RT = 5,     // R(c) + t(c): redundant count before the recompression
  DK_R0 = 6,     // r0(c): skeleton rank of the construction
  DK_PM = 7,     // parent dimension m(p) (merge)
  DK_PR = 8,     // parent redundant count R(p) (merge)
  DK_A0 = 9,     // a0(c): panel start of the current blocked factorization step
  DK_A1 = 10,    // a1(c): panel width of the current step
  DK_TMA0 = 11,  // t(c) - a0(c)
  DK_TREM = 12,  // t(c) - a0(c) - a1(c): columns to the right of the panel
  DK_RTMA0 = 13, // R(c) + t(c) - a0(c)
  DK_RMK = 14,   // R(c) - a0(c) - a1(c): trailing rows of a pivot block
  DK_TN = 15,    // t(2c) + t(2c+1): new directions of the children of parent c (merge)
};

__host__ __device__ inline int dx(int kind, int arg) { return (kind << 24) | arg; }
__host__ __device__ inline int dconst(int v) { return v; }

// --------------------------------------------------------------- buffers
enum BufId : int {
  B_S = 0,    // near blocks of the current level        [shift][pair][mcap x mcap]
  B_F,        // carried fill-in of the current level    [shift][pair][mcap x mcap]
  B_G,        // per cluster: Gram G -> compact-WY factor T -> elimination operator K
  B_V,        // per cluster: pivoted Cholesky columns -> Householder vectors Y
  B_W,        // per cluster: rotation W = I - Y T Y^T
  B_Z,        // per cluster scratch: Y T
  B_M,        // per colour scratch: Y^T Y                [shift][slot][mcap^2]
  B_P,        // per colour scratch: sums of Y^T Y
  B_T,        // per colour scratch: Y^R sign P
  B_SIGN,     // per cluster signs of the scaled pivots   [shift][cluster][mcap]
  B_HAT,      // merge: children skeleton blocks, permuted [shift][slot][pcap^2]
  B_TMP,      // merge: old-old part times E_q             [shift][slot][emax^2]
  B_SN,       // next level near blocks
  B_FN,       // next level carried fill-in
  B_BRES,     // resident leaf near blocks (shift independent)
  B_CPL,      // resident couplings of the current level
  B_EMAT,     // resident transfer matrices of the parent level
  B_RS,       // per launch scratch for out-of-place products (slot = item index in the launch)
  NBUF
};

struct BufTab {
  double* p[NBUF];
  int64_t ss[NBUF];  // shift stride (elements)
  int64_t bs[NBUF];  // block stride (elements)
  int ld[NBUF];      // leading dimension
  // Blocks sized by their own clusters (the near and carried fill-in blocks of
  // the levels above the leaves): block blk starts boff[buf][blk] elements
  // into the shift's part and has leading dimension bld[buf][blk].  Null:
  // every block is bs elements with leading dimension ld.
  const int64_t* boff[NBUF];
  const int* bld[NBUF];
  unsigned long long* fc;   // algorithmic flop counter of the launch's kernel class (or null)
  unsigned long long* fck;  // second counter, per kernel symbol (GEMM layouts), or null
  unsigned long long* fbk;  // algorithmic bytes per kernel symbol (GEMM layouts), or null
  int f32;                  // GEMMs of this launch multiply in FP32 (operands rounded, FP32 accumulation)
  int grid;                 // GEMM workgroups per shift (0 = from the tuning table), a multiple of 8
  int group_m;              // GEMM tile order inside an item: groups of group_m tile rows,
                            // column by column inside a group (<= 1: row by row)
  int tile;                 // GEMM output tile 64 or 128 (set together with grid)
};

struct SizeTab {
  int* m;          // [S][N]
  int* R;          // [S][N]
  int* t;          // [S][N]
  int* a0;         // [S][N] panel state of the blocked per-cluster factorizations
  int* a1;         // [S][N]
  const int* r0;   // [N]
  int* pm;         // [S][Np]
  int* pR;         // [S][Np]
  const int* pr0;  // [Np]
  int N, Np;
};

__host__ __device__ inline int dev_eval(int e, const SizeTab& z, int s) {
  int k = (int)((unsigned)e >> 24), a = e & 0xFFFFFF;
  switch (k) {
    case DK_CONST: return a;
    case DK_M: return z.m[s * z.N + a];
    case DK_R: return z.R[s * z.N + a];
    case DK_S: return z.m[s * z.N + a] - z.R[s * z.N + a];
    case DK_T: return z.t[s * z.N + a];
    case DK_RT: return z.R[s * z.N + a] + z.t[s * z.N + a];
    case DK_R0: return z.r0[a];
    case DK_PM: return z.pm[s * z.Np + a];
    case DK_PR: return z.pR[s * z.Np + a];
    case DK_A0: return z.a0[s * z.N + a];
    case DK_A1: return z.a1[s * z.N + a];
    case DK_TMA0: return z.t[s * z.N + a] - z.a0[s * z.N + a];
    case DK_TREM: return z.t[s * z.N + a] - z.a0[s * z.N + a] - z.a1[s * z.N + a];
    case DK_RTMA0: return z.R[s * z.N + a] + z.t[s * z.N + a] - z.a0[s * z.N + a];
    case DK_RMK: return z.R[s * z.N + a] - z.a0[s * z.N + a] - z.a1[s * z.N + a];
    case DK_TN: return z.t[s * z.N + 2 * a] + z.t[s * z.N + 2 * a + 1];
  }
  return 0;
}

// A sub-block origin: row = eval(r0) + eval(r1), col = eval(c0) + eval(c1).
struct Ref {
  int buf, blk;
  int r0, r1, c0, c1;
};

// GEMM term: op(A) (M x K) * diag(w) * op(B) (K x N)
struct GTerm {
  Ref a, b;
  int K;            // size expression
  int wbuf, wblk;   // weights (B_SIGN, cluster) or wbuf = -1
};

// One output block: C = beta*C + alpha * sum_t op(A_t) diag(w_t) op(B_t)
// optional C2 = beta*C2 + alpha*(...)^T (the transposed twin of a symmetric pair)
// Segmented output (c2.buf == SEG_OUT): rows [0, rsplit) go to the origin of c,
// rows [rsplit, M) to the row origin c2.r0 + c2.r1; columns likewise with
// csplit and c2.c0 + c2.c1 (same buffer and block as c).
constexpr int SEG_OUT = -2;

struct GItem {
  Ref c, c2;        // c2.buf = -1 when absent; c.blk = -1: scratch slot of the item
  int M, N;         // size expressions
  int t0, nt;       // term range
  double alpha, beta;
  int guard;        // size expression; the item is skipped when it evaluates to 0 (-1: none)
  int rsplit, csplit;  // size expressions of a segmented output
};

// Copy of a scratch slot back into a block: X[r0 + a][c0 + b] = RS[slot][a][b]
struct CopyItem {
  Ref x;
  int M, N;
  int guard;
  Ref src{-1, 0, 0, 0, 0, 0};   // source block of a transposed copy (buf < 0: the item's scratch slot)
};

// Matrix sum: C[M x N] = sum_t A_t[M x N] (all at origin)
struct SumItem {
  int cbuf, cblk, M, N;
  int t0, nt;       // into an int array of (buf, blk) pairs
};

// In-place rotation of the first RT(i) rows (side 0) or columns (side 1) of a
// block by the cluster's rotation W (in B_W): rows <- W^T rows; cols <- cols W.
struct RotItem {
  int buf, blk, cluster, side;
  int other;        // size expression: number of columns (side 0) / rows (side 1)
};

// In-place right multiplication of rows [row0, row0+nrows) x cols [0, R(i))
// of a near block by the elimination operator K_i (in B_G).
struct TrsmItem {
  int blk, cluster;
  int row0, nrows;  // size expressions
};

// Merge gather: parent block (p, q) from the 2x2 children skeleton blocks, in
// the order [new c1 | new c2 | old c1 | old c2] for rows and columns.
struct GatherItem {
  int out_blk;              // slot in B_HAT
  int dst_buf, dst_blk;     // output block (B_SN or B_FN): receives the new-new part
  int p, q;                 // parent clusters
  int src_kind[4];          // 0 none, 1 near block (B_S), 2 carried fill-in (B_F), 3 carried fill-in
                            // stored as the other orientation (read transposed)
  int src_blk[4];
  int cpl_blk[4];           // coupling slot in B_CPL or -1
};

}  // namespace h2
