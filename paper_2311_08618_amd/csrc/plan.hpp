// Static schedule of the generalized H^2-LDL: for every level, the colour
// classes of the near graph and, per class, the descriptor lists of each
// kernel; then the merge into the parent level (Secs. 3.2-3.4).
#pragma once
#include <vector>

#include "desc.hpp"
#include "host.hpp"

namespace h2 {

struct GList {
  std::vector<GItem> items;
  std::vector<GTerm> terms;
  void add(const GItem& it, const std::vector<GTerm>& ts) {
    GItem x = it;
    x.t0 = (int)terms.size();
    x.nt = (int)ts.size();
    items.push_back(x);
    terms.insert(terms.end(), ts.begin(), ts.end());
  }
};

struct SumList {
  std::vector<SumItem> items;
  std::vector<int> src;  // pairs (buf, blk)
};

struct ColourPlan {
  std::vector<int> clusters;
  GList pc_upd;                // NT: G -= L_p L_p^T after a pivoted-Cholesky panel
  GList ut_s;                  // TN: S = Y^T Y (into B_G)
  GList ut_t;                  // NN: B_W = T[0:a0, 0:a0] S[0:a0, block]
  GList ut_x;                  // NN: T[0:a0, block] = -B_W T_block
  GList ut_u;                  // NN: U = Y T (into B_G)
  GList ut_w;                  // NT: W -= U Y^T
  GList ldl_upd;               // NT: A_trail -= L_p W_p^T after an LDL panel
  GList inv_t;                 // NN: T = L[rows of block ib, 0:a0] X[0:a0, 0:a0]
  GList inv_x;                 // NN: X[block ib, 0:a0] = -X_ii T
  GList rot_rows, rot_cols;    // TN: RS = W^T X ; NN: RS = X W
  std::vector<CopyItem> rot_rows_copy, rot_cols_copy;
  std::vector<CopyItem> rot_rows_copyt;   // transposed copies into the mirror blocks (parallel to rot_rows)
  // carried fill-in blocks are stored once, as F(q,i) with q < i: the columns
  // of F(q,i) that belong to i are rotated as RS = W^T F(q,i)^T (TT), copied
  // back transposed
  GList rot_cols_t;
  std::vector<CopyItem> rot_cols_t_copy;
  GList trsm;                  // NT: RS = X (K^T)^T, operator stored transposed
  std::vector<CopyItem> trsm_copy;
  GList schur;                 // NT, alpha -1
  GList gram_m;                // TN
  SumList gram_p;
  GList gram_t;                // NN
  GList gram_g;                // NT
  int nslot_m = 0, nslot_p = 0;
  // the clusters behind the scratch slots, which size them per level: M slot
  // (j,i) and P slot (k,i) are R_i x R_i, T slot (k,i) is R_k x R_i
  std::vector<int> slot_m_i, slot_p_k, slot_p_i;
};

// Merge outputs are processed in chunks of MERGE_CHUNK parent blocks, which
// share the B_HAT / B_TMP slots (slot = output index % MERGE_CHUNK).
constexpr int MERGE_CHUNK = 64;

struct MergeChunk {
  int g0, g1, f0, f1, a0, a1, b0, b1;   // item ranges in gather, fill, tr1, tr2
};

struct MergePlan {
  int Np = 0;
  int nhat = 0;
  std::vector<MergeChunk> chunks;
  std::vector<GatherItem> gather;
  GList fill;                  // NT into B_HAT / the output's new-new part
  GList tr1;                   // NN: out[new, old] = HAT[new, old] E_q ; TMP = HAT[old, old] E_q
  GList tr2;                   // TN: out[old, new] = E_p^T HAT[old, new] ; out[old, old] = E_p^T TMP
  std::vector<int> pr0;        // parent construction ranks
  std::vector<int> emat_dim;   // r0_c1 + r0_c2 per parent
  std::vector<CopyItem> mirror;   // near (p,q), q < p: the transpose of the finished (q,p), after all chunks
  int emax = 0;
};

struct LevelPlan {
  int l = 0, N = 0;
  std::vector<int> near_ptr, near_idx;   // CSR, sorted, includes self
  std::vector<int> diag_blk;
  std::vector<int> f_ptr, f_idx;         // carried fill-in partners j > i (CSR): one stored block per pair
  std::vector<int> far_ptr, far_idx;     // interaction list I_l (CSR) = coupling slots
  std::vector<int> r0;
  std::vector<int> colour;
  int rmax = 0;
  std::vector<ColourPlan> colours;
  GList gram_init;                       // NT: G_p += F F^T over carried fill-in F(p,q), q > p
  GList gram_init_t;                     // TN: G_p += F^T F over carried fill-in F(q,p), q < p
  MergePlan merge;                       // into level l-1 (unused at l = 0)
  int max_slot_m = 0, max_slot_p = 0;

  int nblk() const { return near_ptr.back(); }
  int nfblk() const { return f_ptr.back(); }
  int blk(int i, int j) const;           // near pair block index, -1 if not near
  int fblk(int i, int j) const;          // carried pair block index for i < j, -1 if none
  int cslot(int i, int j) const;         // coupling slot, -1 if not admissible
};

std::vector<LevelPlan> build_plan(const Tree& T, const Basis& B);

}  // namespace h2
