// Builds the static schedule.  For a level l with colour classes c = 0..C-1
// (clusters of one class are pairwise non-near, so eliminating them together
// gives the same result as eliminating them one after the other in index
// order), each class runs, in this order:
//   recompress -> rotate rows -> rotate columns -> pivot LDL -> elimination
//   (right-multiplication by the LDL operator) -> Schur updates of near blocks
//   -> Gram of the fill-in products for the not yet eliminated neighbours.
// Then the merge into level l-1 and the Gram of carried fill-in.
#include "plan.hpp"

#include <algorithm>
#include <map>
#include <set>

namespace h2 {

static int find_in(const std::vector<int>& ptr, const std::vector<int>& idx, int i, int j) {
  auto b = idx.begin() + ptr[i], e = idx.begin() + ptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it != e && *it == j) return (int)(it - idx.begin());
  return -1;
}

int LevelPlan::blk(int i, int j) const { return find_in(near_ptr, near_idx, i, j); }
int LevelPlan::fblk(int i, int j) const { return find_in(f_ptr, f_idx, i, j); }
int LevelPlan::cslot(int i, int j) const { return find_in(far_ptr, far_idx, i, j); }

static Ref ref(int buf, int blk, int r0 = 0, int c0 = 0, int r1 = 0, int c1 = 0) {
  Ref x;
  x.buf = buf; x.blk = blk; x.r0 = r0; x.r1 = r1; x.c0 = c0; x.c1 = c1;
  return x;
}
static Ref noref() { Ref x = ref(-1, 0); return x; }

static GTerm term(Ref a, Ref b, int K, int wbuf = -1, int wblk = 0) {
  GTerm t;
  t.a = a; t.b = b; t.K = K; t.wbuf = wbuf; t.wblk = wblk;
  return t;
}

static GItem item(Ref c, Ref c2, int M, int N, double alpha, double beta) {
  GItem g;
  g.c = c; g.c2 = c2; g.M = M; g.N = N; g.alpha = alpha; g.beta = beta; g.t0 = 0; g.nt = 0; g.guard = -1;
  g.rsplit = 0; g.csplit = 0;
  return g;
}

std::vector<LevelPlan> build_plan(const Tree& T, const Basis& B) {
  int L = T.L;
  std::vector<LevelPlan> P(L + 1);
  // carried fill-in partners per level, bottom-up
  std::vector<std::vector<std::set<int>>> carried(L + 1);
  for (int l = 0; l <= L; ++l) carried[l].assign(1 << l, {});
  for (int l = L; l >= 1; --l) {
    int N = 1 << l;
    // fill pairs at level l: non-near pairs with a common near neighbour, or carried
    std::vector<std::set<int>> fill(N);
    for (int i = 0; i < N; ++i)
      for (int c : T.near[l][i])
        for (int d : T.near[l][i])
          if (!T.is_near(l, c, d)) fill[c].insert(d);
    for (int c = 0; c < N; ++c)
      for (int d : carried[l][c]) fill[c].insert(d);
    for (int c = 0; c < N; ++c)
      for (int d : fill[c]) {
        int p = c >> 1, q = d >> 1;
        if (!T.is_near(l - 1, p, q)) carried[l - 1][p].insert(q);
      }
  }
  for (int l = L; l >= 0; --l) {
    LevelPlan& lp = P[l];
    int N = 1 << l;
    lp.l = l;
    lp.N = N;
    lp.near_ptr.assign(1, 0);
    lp.f_ptr.assign(1, 0);
    lp.far_ptr.assign(1, 0);
    for (int i = 0; i < N; ++i) {
      for (int j : T.near[l][i]) lp.near_idx.push_back(j);
      lp.near_ptr.push_back((int)lp.near_idx.size());
      for (int j : carried[l][i])
        if (j > i) lp.f_idx.push_back(j);
      lp.f_ptr.push_back((int)lp.f_idx.size());
      for (int j : T.far[l][i]) lp.far_idx.push_back(j);
      lp.far_ptr.push_back((int)lp.far_idx.size());
    }
    lp.diag_blk.resize(N);
    for (int i = 0; i < N; ++i) lp.diag_blk[i] = lp.blk(i, i);
    lp.r0 = B.r[l];
    lp.colour = T.colour[l];
    lp.rmax = 0;
    for (int v : lp.r0) lp.rmax = std::max(lp.rmax, v);

    const auto& col = T.colour[l];
    int C = T.ncolour[l];
    lp.colours.assign(C, {});
    for (int c = 0; c < C; ++c) {
      ColourPlan& cp = lp.colours[c];
      for (int i = 0; i < N; ++i)
        if (col[i] == c) cp.clusters.push_back(i);
      auto done = [&](int k) { return col[k] <= c; };  // eliminated before or in this class
      auto row0 = [&](int k) { return done(k) ? dx(DK_R, k) : dconst(0); };
      auto nrows = [&](int k) { return done(k) ? dx(DK_S, k) : dx(DK_M, k); };
      for (int i : cp.clusters) {
        const int a0 = dx(DK_A0, i), a1 = dx(DK_A1, i);
        GItem g;
        // pivoted Cholesky: G -= V[:, a0:t] V[:, a0:t]^T
        g = item(ref(B_G, i), noref(), dx(DK_R, i), dx(DK_R, i), -1.0, 1.0);
        g.guard = dx(DK_TMA0, i);
        cp.pc_upd.add(g, {term(ref(B_V, i, 0, a0), ref(B_V, i, 0, a0), dx(DK_TMA0, i))});
        // W = I - Y T Y^T with T^{-1} = striu(Y^T Y) + diag(1/beta)
        const int ti = dx(DK_T, i), rti = dx(DK_RT, i);
        g = item(ref(B_G, i), noref(), ti, ti, 1.0, 0.0);
        g.guard = ti;
        cp.ut_s.add(g, {term(ref(B_V, i), ref(B_V, i), rti)});
        g = item(ref(B_W, i), noref(), a0, a1, 1.0, 0.0);
        g.guard = a1;
        cp.ut_t.add(g, {term(ref(B_Z, i), ref(B_G, i, 0, a0), a0)});
        g = item(ref(B_Z, i, 0, a0), noref(), a0, a1, -1.0, 0.0);
        g.guard = a1;
        cp.ut_x.add(g, {term(ref(B_W, i), ref(B_Z, i, a0, a0), a1)});
        g = item(ref(B_G, i), noref(), rti, ti, 1.0, 0.0);
        g.guard = ti;
        cp.ut_u.add(g, {term(ref(B_V, i), ref(B_Z, i), ti)});
        g = item(ref(B_W, i), noref(), rti, rti, -1.0, 1.0);
        g.guard = ti;
        cp.ut_w.add(g, {term(ref(B_G, i), ref(B_V, i), ti)});
        // LDL trailing update A[k:R, k:R] -= L_p W_p^T, k = a0 + a1
        const int db = lp.blk(i, i);
        g = item(ref(B_S, db, a0, a0, a1, a1), noref(), dx(DK_RMK, i), dx(DK_RMK, i), -1.0, 1.0);
        g.guard = a1;
        cp.ldl_upd.add(g, {term(ref(B_S, db, a0, a0, a1, 0), ref(B_W, i, a0, 0, a1, 0), a1)});
        // blocked L^{-1}: T = L[a0:a0+a1, 0:a0] X[0:a0, 0:a0] ; X[a0:a0+a1, 0:a0] = -X_ii T
        g = item(ref(B_W, i), noref(), a1, a0, 1.0, 0.0);
        g.guard = a1;
        cp.inv_t.add(g, {term(ref(B_S, db, a0, 0), ref(B_V, i), a0)});
        g = item(ref(B_V, i, a0, 0), noref(), a1, a0, -1.0, 0.0);
        g.guard = a1;
        cp.inv_x.add(g, {term(ref(B_V, i, a0, a0), ref(B_W, i), a1)});
      }
      // rotation by W (rows, then columns) and elimination by K, each as an
      // out-of-place product into a scratch slot followed by a copy back
      // Both orientations of a block are stored and (k,i) = (i,k)^T, so the
      // columns of (k,i) receive the transpose of the rotated rows of (i,k).
      // Blocks whose row and column clusters are rotated in the same class
      // (the diagonal block, and fill-in blocks between two clusters of one
      // colour) are rotated on both sides by products instead.
      auto rot = [&](int buf, int blk_row, int blk_col, int i, int other, bool both_sides) {
        const bool diag = both_sides;
        GItem g = item(ref(B_RS, -1), noref(), dx(DK_RT, i), other, 1.0, 0.0);
        g.guard = dx(DK_T, i);
        cp.rot_rows.add(g, {term(ref(B_W, i), ref(buf, blk_row), dx(DK_RT, i))});
        CopyItem cr{ref(buf, blk_row), dx(DK_RT, i), other, dx(DK_T, i)};
        cp.rot_rows_copy.push_back(cr);
        CopyItem ct{ref(buf, blk_col), other, dx(DK_RT, i), diag ? dconst(0) : dx(DK_T, i)};
        cp.rot_rows_copyt.push_back(ct);
        if (diag) {
          GItem h = item(ref(B_RS, -1), noref(), other, dx(DK_RT, i), 1.0, 0.0);
          h.guard = dx(DK_T, i);
          cp.rot_cols.add(h, {term(ref(buf, blk_col), ref(B_W, i), dx(DK_RT, i))});
          CopyItem cc{ref(buf, blk_col), other, dx(DK_RT, i), dx(DK_T, i)};
          cp.rot_cols_copy.push_back(cc);
        }
      };
      // Carried fill-in is stored once per pair, as F(i,q) with i < q: its rows
      // are rotated when i is, its columns when q is, each by one product (the
      // two passes run one after the other, so blocks between two clusters of
      // one class receive both).
      auto rot_f = [&](int i, int q) {
        if (i < q) {
          const int fb = lp.fblk(i, q);
          GItem g = item(ref(B_RS, -1), noref(), dx(DK_RT, i), dx(DK_M, q), 1.0, 0.0);
          g.guard = dx(DK_T, i);
          cp.rot_rows.add(g, {term(ref(B_W, i), ref(B_F, fb), dx(DK_RT, i))});
          cp.rot_rows_copy.push_back(CopyItem{ref(B_F, fb), dx(DK_RT, i), dx(DK_M, q), dx(DK_T, i)});
          cp.rot_rows_copyt.push_back(CopyItem{ref(B_F, fb), dx(DK_M, q), dx(DK_RT, i), dconst(0)});   // no mirror
        } else {
          const int fb = lp.fblk(q, i);
          GItem g = item(ref(B_RS, -1), noref(), dx(DK_RT, i), dx(DK_M, q), 1.0, 0.0);
          g.guard = dx(DK_T, i);
          cp.rot_cols_t.add(g, {term(ref(B_W, i), ref(B_F, fb), dx(DK_RT, i))});
          cp.rot_cols_t_copy.push_back(CopyItem{ref(B_F, fb), dx(DK_M, q), dx(DK_RT, i), dx(DK_T, i)});
        }
      };
      for (int i : cp.clusters) {
        for (int k : T.near[l][i]) rot(B_S, lp.blk(i, k), lp.blk(k, i), i, dx(DK_M, k), k == i);
        for (int q : carried[l][i]) rot_f(i, q);
        for (int k : T.near[l][i]) {
          GItem g = item(ref(B_RS, -1), noref(), nrows(k), dx(DK_R, i), 1.0, 0.0);
          g.guard = dx(DK_R, i);
          // operator stored transposed (K^T in B_G): NT product
          cp.trsm.add(g, {term(ref(B_S, lp.blk(k, i), row0(k), 0), ref(B_G, i), dx(DK_R, i))});
          CopyItem ct{ref(B_S, lp.blk(k, i), row0(k), 0), nrows(k), dx(DK_R, i), dx(DK_R, i)};
          cp.trsm_copy.push_back(ct);
        }
      }
      // Schur updates, aggregated per target pair (j <= k)
      std::map<std::pair<int, int>, std::vector<int>> tgt;
      for (int i : cp.clusters)
        for (int j : T.near[l][i])
          for (int k : T.near[l][i])
            if (j <= k && T.is_near(l, j, k)) tgt[{j, k}].push_back(i);
      for (auto& kv : tgt) {
        int j = kv.first.first, k = kv.first.second;
        Ref c = ref(B_S, lp.blk(j, k), row0(j), row0(k));
        Ref c2 = j != k ? ref(B_S, lp.blk(k, j), row0(k), row0(j)) : noref();
        std::vector<GTerm> ts;
        for (int i : kv.second)
          ts.push_back(term(ref(B_S, lp.blk(j, i), row0(j), 0), ref(B_S, lp.blk(k, i), row0(k), 0),
                            dx(DK_R, i), B_SIGN, i));
        cp.schur.add(item(c, c2, nrows(j), nrows(k), -1.0, 1.0), ts);
      }
      // Gram of fill-in products for not-yet-eliminated neighbours k of i
      std::map<std::pair<int, int>, int> slot_m, slot_p;   // (j,i) -> slot ; (k,i) -> slot
      std::map<int, std::vector<int>> gtarget;             // k -> contributing i
      for (int i : cp.clusters)
        for (int k : T.near[l][i]) {
          if (done(k)) continue;
          std::vector<int> J;
          for (int j : T.near[l][i])
            if (!T.is_near(l, j, k)) J.push_back(j);
          if (J.empty()) continue;
          int sp = (int)slot_p.size();
          slot_p[{k, i}] = sp;
          cp.slot_p_k.push_back(k);
          cp.slot_p_i.push_back(i);
          std::vector<int> src;
          for (int j : J) {
            auto key = std::make_pair(j, i);
            if (!slot_m.count(key)) {
              int sm = (int)slot_m.size();
              slot_m[key] = sm;
              cp.slot_m_i.push_back(i);
              Ref a = ref(B_S, lp.blk(j, i), row0(j), 0);
              cp.gram_m.add(item(ref(B_M, sm), noref(), dx(DK_R, i), dx(DK_R, i), 1.0, 0.0),
                            {term(a, a, nrows(j))});
            }
            cp.gram_p.src.push_back(B_M);
            cp.gram_p.src.push_back(slot_m[key]);
          }
          SumItem s;
          s.cbuf = B_P; s.cblk = sp; s.M = dx(DK_R, i); s.N = dx(DK_R, i);
          s.nt = (int)J.size();
          s.t0 = (int)cp.gram_p.src.size() / 2 - s.nt;
          cp.gram_p.items.push_back(s);
          cp.gram_t.add(item(ref(B_T, sp), noref(), dx(DK_R, k), dx(DK_R, i), 1.0, 0.0),
                        {term(ref(B_S, lp.blk(k, i)), ref(B_P, sp), dx(DK_R, i), B_SIGN, i)});
          gtarget[k].push_back(i);
        }
      for (auto& kv : gtarget) {
        int k = kv.first;
        std::vector<GTerm> ts;
        for (int i : kv.second)
          ts.push_back(term(ref(B_T, slot_p[{k, i}]), ref(B_S, lp.blk(k, i)), dx(DK_R, i), B_SIGN, i));
        cp.gram_g.add(item(ref(B_G, k), noref(), dx(DK_R, k), dx(DK_R, k), 1.0, 1.0), ts);
      }
      cp.nslot_m = (int)slot_m.size();
      cp.nslot_p = (int)slot_p.size();
      lp.max_slot_m = std::max(lp.max_slot_m, cp.nslot_m);
      lp.max_slot_p = std::max(lp.max_slot_p, cp.nslot_p);
    }
    // Gram of carried fill-in at the start of the level: F(p,q) F(p,q)^T for
    // the blocks stored with p as row cluster, F(q,p)^T F(q,p) for the others
    for (int p = 0; p < N; ++p) {
      if (carried[l][p].empty()) continue;
      std::vector<GTerm> up, lo;
      for (int q : carried[l][p]) {
        if (q > p) {
          Ref a = ref(B_F, lp.fblk(p, q));
          up.push_back(term(a, a, dx(DK_M, q)));
        } else {
          Ref a = ref(B_F, lp.fblk(q, p));
          lo.push_back(term(a, a, dx(DK_M, q)));
        }
      }
      if (!up.empty()) lp.gram_init.add(item(ref(B_G, p), noref(), dx(DK_R, p), dx(DK_R, p), 1.0, 1.0), up);
      if (!lo.empty()) lp.gram_init_t.add(item(ref(B_G, p), noref(), dx(DK_R, p), dx(DK_R, p), 1.0, 1.0), lo);
    }
  }
  // merge plans (need both levels' CSR)
  for (int l = L; l >= 1; --l) {
    LevelPlan& lp = P[l];
    const LevelPlan& pp = P[l - 1];
    MergePlan& mp = lp.merge;
    int Np = 1 << (l - 1);
    mp.Np = Np;
    mp.pr0 = B.r[l - 1];
    mp.emat_dim.assign(Np, 0);
    for (int p = 0; p < Np; ++p) {
      mp.emat_dim[p] = B.r[l][2 * p] + B.r[l][2 * p + 1];
      mp.emax = std::max(mp.emax, mp.emat_dim[p]);
    }
    int h = 0;
    auto add_out = [&](int p, int q, bool is_near) {
      if (h % MERGE_CHUNK == 0) {
        MergeChunk ch;
        ch.g0 = (int)mp.gather.size();
        ch.f0 = (int)mp.fill.items.size();
        ch.a0 = (int)mp.tr1.items.size();
        ch.b0 = (int)mp.tr2.items.size();
        ch.g1 = ch.f1 = ch.a1 = ch.b1 = 0;
        mp.chunks.push_back(ch);
      }
      const int slot = h % MERGE_CHUNK;
      // Parent coordinates [new c1 | new c2 | E^T (old c1, old c2)]: the new
      // directions pass through, only the old skeleton coordinates meet E.
      // The children block is gathered into its slot of B_HAT in the permuted
      // order [new c1 | new c2 | old c1 | old c2]; once the fill-in is added
      // its new-new part is final and is copied to the output block.
      const int obuf = is_near ? B_SN : B_FN;
      const int oblk = is_near ? pp.blk(p, q) : pp.fblk(p, q);
      const int tnp = dx(DK_TN, p), tnq = dx(DK_TN, q);
      const int edp = mp.emat_dim[p], edq = mp.emat_dim[q];
      GatherItem g;
      g.out_blk = slot;
      g.p = p;
      g.q = q;
      g.dst_buf = obuf;
      g.dst_blk = oblk;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          int c = 2 * p + a, d = 2 * q + b, s = 2 * a + b;
          g.src_kind[s] = 0;
          g.src_blk[s] = 0;
          g.cpl_blk[s] = -1;
          if (lp.blk(c, d) >= 0) { g.src_kind[s] = 1; g.src_blk[s] = lp.blk(c, d); }
          else if (c < d && lp.fblk(c, d) >= 0) { g.src_kind[s] = 2; g.src_blk[s] = lp.fblk(c, d); }
          else if (c > d && lp.fblk(d, c) >= 0) { g.src_kind[s] = 3; g.src_blk[s] = lp.fblk(d, c); }
          if (is_near && lp.cslot(c, d) >= 0) g.cpl_blk[s] = lp.cslot(c, d);
          if (lp.blk(c, d) < 0) {
            // generator fill-in from common near neighbours of c and d
            std::vector<int> cn;
            std::set_intersection(T.near[l][c].begin(), T.near[l][c].end(), T.near[l][d].begin(),
                                  T.near[l][d].end(), std::back_inserter(cn));
            if (!cn.empty()) {
              // one product per child pair, its rows and columns scattered to
              // the new and old segments of the permuted layout
              const int rn = a ? dx(DK_T, 2 * p) : 0, ro = a ? dconst(B.r[l][2 * p]) : 0;
              const int cnn = b ? dx(DK_T, 2 * q) : 0, co = b ? dconst(B.r[l][2 * q]) : 0;
              std::vector<GTerm> ts;
              for (int i : cn)
                ts.push_back(term(ref(B_S, lp.blk(c, i), dx(DK_R, c), 0), ref(B_S, lp.blk(d, i), dx(DK_R, d), 0),
                                  dx(DK_R, i), B_SIGN, i));
              GItem it = item(ref(B_HAT, slot, rn, cnn), noref(), dx(DK_S, c), dx(DK_S, d), -1.0, 1.0);
              it.c2 = ref(SEG_OUT, slot, tnp, tnq, ro, co);
              it.rsplit = dx(DK_T, c);
              it.csplit = dx(DK_T, d);
              mp.fill.add(it, ts);
            }
          }
        }
      mp.gather.push_back(g);
      // new rows x old columns, and the old rows' right product, by E_q
      mp.tr1.add(item(ref(obuf, oblk, 0, tnq), noref(), tnp, dconst(edq), 1.0, 0.0),
                 {term(ref(B_HAT, slot, 0, tnq), ref(B_EMAT, q), dconst(edq))});
      mp.tr1.add(item(ref(B_TMP, slot), noref(), dconst(edp), dconst(edq), 1.0, 0.0),
                 {term(ref(B_HAT, slot, tnp, tnq), ref(B_EMAT, q), dconst(edq))});
      // old rows: E_p^T on the left
      mp.tr2.add(item(ref(obuf, oblk, tnp, 0), noref(), dconst(edp), tnq, 1.0, 0.0),
                 {term(ref(B_EMAT, p), ref(B_HAT, slot, tnp, 0), dconst(edp))});
      mp.tr2.add(item(ref(obuf, oblk, tnp, tnq), noref(), dconst(edp), dconst(edq), 1.0, 0.0),
                 {term(ref(B_EMAT, p), ref(B_TMP, slot), dconst(edp))});
      MergeChunk& ch = mp.chunks.back();
      ch.g1 = (int)mp.gather.size();
      ch.f1 = (int)mp.fill.items.size();
      ch.a1 = (int)mp.tr1.items.size();
      ch.b1 = (int)mp.tr2.items.size();
      ++h;
    };
    // Both orientations of a near parent pair are stored and (p,q) = (q,p)^T:
    // the products run for q >= p only, and (p,q) with q < p is a transposed
    // copy of the finished (q,p).  Carried fill-in has one block per pair
    // (q > p) and no mirror.
    auto mirror_of = [&](int p, int q) {
      const int dst = pp.blk(p, q), src = pp.blk(q, p);
      if (src < 0) {
        add_out(p, q, true);
        return;
      }
      CopyItem c{ref(B_SN, dst), dx(DK_PM, p), dx(DK_PM, q), -1};
      c.src = ref(B_SN, src);
      mp.mirror.push_back(c);
    };
    for (int p = 0; p < Np; ++p) {
      for (int q : T.near[l - 1][p]) {
        if (q >= p) add_out(p, q, true);
        else mirror_of(p, q);
      }
      for (int k = pp.f_ptr[p]; k < pp.f_ptr[p + 1]; ++k) add_out(p, pp.f_idx[k], false);
    }
    mp.nhat = h;
  }
  return P;
}

}  // namespace h2
