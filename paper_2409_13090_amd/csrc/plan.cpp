// Lowering of the symbolic structure of RLB (Section 2.2.2, Alg. 5) into the
// flat work lists the device kernels consume.
//
// Factor storage: Lnz(J) is an m_J x w_J column-major block (ld = m_J) whose
// row r holds global row glbind(J)[r] (Section 2.1.2); the blocks of all
// supernodes live in one FP64 buffer, each starting on a 64-byte boundary.
//
// Schedule: supernodes are grouped by their height in the supernodal
// elimination tree; every level runs, for column block k = 0, 1, ... of its
// supernodes (blocks of 64 columns):
//   * a PANEL launch: cdiv of block k -- POTRF of the 64x64 diagonal tile
//     fused with the TRSM of every row below it (Alg. 5 line 4);
//   * an UPDATE launch holding (a) the trailing update of the columns right of
//     block k inside the same supernode, and (b) for every supernode whose last
//     column block was k, all of its SYRK/GEMM updates written straight into
//     the ancestors' factor storage (Alg. 5 lines 7-18).
// Siblings of one level may write the same target entries; a tile is marked
// atomic exactly when another supernode of its launch touches one of its
// target columns.
#include <algorithm>
#include <cmath>

#include "symbolic.h"

namespace rlb {

namespace {
constexpr int NB = 64;   // column block of the panel kernel
constexpr int TM = 64;   // update tile rows
constexpr int TN = 64;   // update tile columns
constexpr int FLAG_DIAG = 1;
constexpr int FLAG_ATOMIC = 2;

// One rectangle of the ancestor update: target rows [r0, r0+mr) and columns
// [c0, c0+nc) of Lnz(P); source rows [sx, ..) and [sy, ..) of Lnz(J).
struct Rect {
  int64_t P, r0, c0, mr, nc, sx, sy;
  bool diag;
};

// entries a tile writes: the full rectangle, or its lower triangle part when
// the tile sits on the diagonal of a SYRK target
double tile_entries(int64_t m, int64_t n, bool diag) {
  if (!diag) return (double)m * (double)n;
  double e = 0;
  for (int64_t c = 0; c < n; ++c) e += (double)std::max<int64_t>(0, m - c);
  return e;
}

void cut_rect(const Symbolic& s, Plan& p, int64_t J, const Rect& r, int32_t atomic,
              std::vector<UpdTile>& out, double& flops) {
  int64_t mP = s.gl_ptr[r.P + 1] - s.gl_ptr[r.P];
  int64_t mJ = s.gl_ptr[J + 1] - s.gl_ptr[J];
  int64_t wJ = s.sn_ptr[J + 1] - s.sn_ptr[J];
  for (int64_t tj = 0; tj < r.nc; tj += TN) {
    int64_t tn = std::min<int64_t>(TN, r.nc - tj);
    for (int64_t ti = r.diag ? tj : 0; ti < r.mr; ti += TM) {
      int64_t tm = std::min<int64_t>(TM, r.mr - ti);
      UpdTile t;
      t.c = p.off[r.P] + (r.c0 + tj) * mP + (r.r0 + ti);
      t.x = p.off[J] + r.sx + ti;
      t.y = p.off[J] + r.sy + tj;
      t.ldc = (int32_t)mP;
      t.lds = (int32_t)mJ;
      t.m = (int32_t)tm;
      t.n = (int32_t)tn;
      t.k = (int32_t)wJ;
      t.flags = ((r.diag && ti == tj) ? FLAG_DIAG : 0) | atomic;
      t.src = (int32_t)J;
      out.push_back(t);
      flops += 2.0 * (double)tm * (double)tn * (double)wJ;
      p.flops_upd_alg += 2.0 * (double)wJ * tile_entries(tm, tn, r.diag && ti == tj);
    }
  }
}

}  // namespace

int build_plan(Symbolic& s, std::string& err) {
  Plan& p = s.plan;
  p = Plan();
  const int64_t n = s.n;
  const int64_t S = (int64_t)s.sn_ptr.size() - 1;
  auto W = [&](int64_t J) { return s.sn_ptr[J + 1] - s.sn_ptr[J]; };
  auto M = [&](int64_t J) { return s.gl_ptr[J + 1] - s.gl_ptr[J]; };

  // factor storage
  p.off.assign(S + 1, 0);
  int64_t run = 0;
  for (int64_t J = 0; J < S; ++J) {
    p.off[J] = run;
    run += M(J) * W(J);
    run = (run + 7) & ~int64_t(7);
  }
  p.off[S] = run;
  p.l_elems = run;

  std::vector<int64_t> snode(n), inv(n);
  for (int64_t J = 0; J < S; ++J)
    for (int64_t j = s.sn_ptr[J]; j < s.sn_ptr[J + 1]; ++j) snode[j] = J;
  for (int64_t k = 0; k < n; ++k) inv[s.perm[k]] = k;

  // A-load map: input entry (i, j) -> its slot in Lnz of the column's supernode
  p.amap.resize(s.nnz_a);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t e = s.colptr[j]; e < s.colptr[j + 1]; ++e) {
      int64_t a = inv[s.rowidx[e]], b = inv[j];
      int64_t r = std::max(a, b), c = std::min(a, b);
      int64_t J = snode[c];
      const int32_t* g = s.gl.data() + s.gl_ptr[J];
      const int32_t* it = std::lower_bound(g, g + M(J), (int32_t)r);
      if (it == g + M(J) || *it != r) {
        err = "internal: entry of A outside the supernodal structure";
        return -1;
      }
      p.amap[e] = p.off[J] + (c - s.sn_ptr[J]) * M(J) + (it - g);
    }

  // levels: height in the supernodal elimination tree
  p.level.assign(S, 0);
  for (int64_t J = 0; J < S; ++J) {
    int64_t P = s.sn_parent[J];
    if (P >= 0) p.level[P] = std::max(p.level[P], p.level[J] + 1);
  }
  p.nlevels = 0;
  for (int64_t J = 0; J < S; ++J) p.nlevels = std::max<int32_t>(p.nlevels, p.level[J] + 1);
  p.lvl_ptr.assign(p.nlevels + 1, 0);
  for (int64_t J = 0; J < S; ++J) p.lvl_ptr[p.level[J] + 1]++;
  for (int32_t h = 0; h < p.nlevels; ++h) p.lvl_ptr[h + 1] += p.lvl_ptr[h];
  p.lvl_sn.resize(S);
  {
    std::vector<int64_t> fill(p.lvl_ptr.begin(), p.lvl_ptr.end() - 1);
    for (int64_t J = 0; J < S; ++J) p.lvl_sn[fill[p.level[J]]++] = (int32_t)J;
  }

  // ancestor-update rectangles of every supernode, from its blocks and relindB
  std::vector<std::vector<Rect>> rects(S);
  for (int64_t J = 0; J < S; ++J) {
    int64_t wJ = W(J);
    int64_t nb = s.blk_ptr[J + 1] - s.blk_ptr[J];
    if (nb == 0) continue;
    std::vector<int64_t> bsize(nb), bsrc(nb);
    int64_t q = wJ;
    for (int64_t b = 0; b < nb; ++b) {
      bsize[b] = s.blk[s.blk_ptr[J] + b];
      bsrc[b] = q;
      q += bsize[b];
    }
    int64_t first_block = 0;
    for (int64_t pi = s.rbp_ptr[J]; pi < s.rbp_ptr[J + 1]; ++pi) {
      int64_t P = s.rbp_anc[pi];
      const int32_t* rb = s.rbv.data() + s.rbv_ptr[pi];  // blocks first_block..nb-1
      int64_t mP = M(P), wP = W(P);
      int64_t cnt = nb - first_block;
      std::vector<int64_t> pos(cnt);
      for (int64_t b = 0; b < cnt; ++b) pos[b] = mP - 1 - rb[b];
      int64_t inP = 0;
      while (inP < cnt && pos[inP] < wP) inP++;
      for (int64_t bi = 0; bi < inP; ++bi) {
        int64_t B = first_block + bi;
        // rows from B downwards, in runs that are contiguous in Lnz(P):
        // the first run is the SYRK (B,B) extended by any block directly
        // below it; every later run is one "maximal" GEMM block B'
        int64_t b = bi;
        bool first = true;
        while (b < cnt) {
          int64_t e = b + 1;
          if (s.opt.maximal_blocks)
            while (e < cnt && pos[e] == pos[e - 1] + bsize[first_block + e - 1]) e++;
          int64_t rows = 0;
          for (int64_t t = b; t < e; ++t) rows += bsize[first_block + t];
          Rect r;
          r.P = P;
          r.r0 = pos[b];
          r.c0 = pos[bi];
          r.mr = rows;
          r.nc = bsize[B];
          r.sx = bsrc[first_block + b];
          r.sy = bsrc[B];
          r.diag = first;
          rects[J].push_back(r);
          first = false;
          b = e;
        }
      }
      first_block += inP;
    }
    if (first_block != nb) {
      err = "internal: blocks not consumed by ancestors";
      return -1;
    }
  }

  // launches
  std::vector<int32_t> colcnt(n, 0);
  p.flops_tiles = 0;
  for (int32_t h = 0; h < p.nlevels; ++h) {
    int64_t steps = 0;
    for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q)
      steps = std::max<int64_t>(steps, (W(p.lvl_sn[q]) + NB - 1) / NB);
    for (int64_t k = 0; k < steps; ++k) {
      // POTRF (and the TRSM of blocks with at most one row tile), then the
      // TRSM row tiles of the taller blocks against their factored tiles
      Launch lp{LAUNCH_POTRF, h, (int32_t)k, 0, (int64_t)p.panels.size(), 0};
      std::vector<PanelTile> trsm;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        if (k * NB >= w) continue;
        int64_t c0 = k * NB, nb = std::min<int64_t>(NB, w - c0), nrows = m - c0;
        int64_t below = nrows - nb;
        // POTRF of the nb x nb tile (sum over its columns of (count)^2 with
        // counts nb..1) plus TRSM of the rows below (nb^2 per row)
        for (int64_t t = 0; t < nb; ++t) p.flops_panel += (double)(nb - t) * (double)(nb - t);
        p.flops_panel += (double)below * (double)nb * (double)nb;
        int64_t nt = (below + 63) / 64;  // TRSM row tiles of 64 rows
        PanelTile pt;
        pt.diag = p.off[J] + c0 * m + c0;
        pt.ld = (int32_t)m;
        pt.nb = (int32_t)nb;
        pt.nrows = (int32_t)nrows;
        pt.row0 = (int32_t)nb;
        pt.col = (int32_t)(s.sn_ptr[J] + c0);
        pt.slot = 0;
        pt.pad = 0;
        pt.mode = 1;
        p.panels.push_back(pt);
        if (nt > 0) {
          for (int64_t t = 0; t < nt; ++t) {
            PanelTile tt = pt;
            tt.mode = 2;
            tt.row0 = (int32_t)(nb + 64 * t);
            trsm.push_back(tt);
          }
        }
      }
      lp.count = (int64_t)p.panels.size() - lp.start;
      if (lp.count) p.launches.push_back(lp);
      if (!trsm.empty()) {
        Launch lt{LAUNCH_TRSM, h, (int32_t)k, 0, (int64_t)p.panels.size(), (int64_t)trsm.size()};
        p.panels.insert(p.panels.end(), trsm.begin(), trsm.end());
        p.launches.push_back(lt);
      }
      // UPDATE: trailing updates of step k, ancestor updates of finished supernodes
      Launch lu{LAUNCH_UPDATE, h, (int32_t)k, 0, (int64_t)p.updates.size(), 0};
      std::vector<int64_t> finished;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        if (k * NB >= w) continue;
        int64_t c0 = k * NB, nb = std::min<int64_t>(NB, w - c0), c1 = c0 + nb;
        if (c1 < w) {
          for (int64_t tj0 = c1; tj0 < w; tj0 += TN) {
            int64_t tn = std::min<int64_t>(TN, w - tj0);
            for (int64_t ti0 = tj0; ti0 < m; ti0 += TM) {
              int64_t tm = std::min<int64_t>(TM, m - ti0);
              UpdTile t;
              t.c = p.off[J] + tj0 * m + ti0;
              t.x = p.off[J] + c0 * m + ti0;
              t.y = p.off[J] + c0 * m + tj0;
              t.ldc = (int32_t)m;
              t.lds = (int32_t)m;
              t.m = (int32_t)tm;
              t.n = (int32_t)tn;
              t.k = (int32_t)nb;
              t.flags = (ti0 == tj0) ? FLAG_DIAG : 0;
              t.src = (int32_t)J;
              p.updates.push_back(t);
              p.flops_tiles += 2.0 * tm * tn * nb;
              p.flops_upd_alg += 2.0 * (double)nb * tile_entries(tm, tn, ti0 == tj0);
            }
          }
        } else {
          finished.push_back(J);
        }
      }
      // conflicts: columns of an ancestor touched by two supernodes of this launch
      for (int64_t J : finished)
        for (const Rect& r : rects[J])
          if (r.diag)
            for (int64_t c = 0; c < r.nc; ++c) colcnt[s.sn_ptr[r.P] + r.c0 + c]++;
      for (int64_t J : finished)
        for (const Rect& r : rects[J]) {
          int32_t atomic = 0;
          for (int64_t c = 0; c < r.nc; ++c)
            if (colcnt[s.sn_ptr[r.P] + r.c0 + c] > 1) {
              atomic = FLAG_ATOMIC;
              break;
            }
          size_t before = p.updates.size();
          cut_rect(s, p, J, r, atomic, p.updates, p.flops_tiles);
          if (atomic) p.n_atomic_tiles += (int64_t)(p.updates.size() - before);
        }
      for (int64_t J : finished)
        for (const Rect& r : rects[J])
          if (r.diag)
            for (int64_t c = 0; c < r.nc; ++c) colcnt[s.sn_ptr[r.P] + r.c0 + c] = 0;
      lu.count = (int64_t)p.updates.size() - lu.start;
      if (lu.count) p.launches.push_back(lu);
    }
  }
  // full symmetric A in the original order, CSR, with the source entry of each value
  p.a_rowptr.assign(n + 1, 0);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t e = s.colptr[j]; e < s.colptr[j + 1]; ++e) {
      int64_t i = s.rowidx[e];
      p.a_rowptr[i + 1]++;
      if (i != j) p.a_rowptr[j + 1]++;
    }
  for (int64_t i = 0; i < n; ++i) p.a_rowptr[i + 1] += p.a_rowptr[i];
  p.a_col.resize(p.a_rowptr[n]);
  p.a_src.resize(p.a_rowptr[n]);
  {
    std::vector<int64_t> fill(p.a_rowptr.begin(), p.a_rowptr.end() - 1);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t e = s.colptr[j]; e < s.colptr[j + 1]; ++e) {
        int64_t i = s.rowidx[e];
        p.a_col[fill[i]] = (int32_t)j;
        p.a_src[fill[i]++] = e;
        if (i != j) {
          p.a_col[fill[j]] = (int32_t)i;
          p.a_src[fill[j]++] = e;
        }
      }
  }
  return 0;
}

}  // namespace rlb
