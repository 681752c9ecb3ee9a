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
//     fused with the TRSM of every row below it (Alg. 5);
//   * an UPDATE launch holding (a) the trailing update of the columns right of
//     block k inside the same supernode, and (b) for every supernode whose last
//     column block was k, all of its SYRK/GEMM updates written straight into
//     the ancestors' factor storage (Alg. 5).
// Siblings of one level may write the same target entries: the update launch
// gives every 64x64 target tile to one workgroup, which sums the
// contributions of all supernodes that touch the tile and writes it once.
#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <tuple>

#include "symbolic.h"

namespace rlb {

namespace {
constexpr int NB = 64;   // column block of the panel kernel
constexpr int TM = 64;   // update tile rows
constexpr int TN = 64;   // update tile columns
constexpr int FLAG_DIAG = 1;
constexpr int FLAG_ATOMIC = 2;
constexpr int FLAG_ASSIGN = 4;  // the tile is written with -(sum), not read (RL's U_J)
constexpr int KCH = 16;        // K chunk of the update kernel
constexpr double HYB_PASSES_PER_US = 1024 / 2.3;  // hybrid method's cost model
constexpr double HYB_BYTES_PER_US = 2.0e6;
// panel launch cost model by width class (1, 2, 4 blocks of 16 columns):
// microseconds per workgroup, resident workgroups on the device, and the
// fixed cost of a launch (measured orders of magnitude on MI355X)
constexpr double PANEL_US[3] = {6.0, 10.0, 16.0};
constexpr int64_t PANEL_SLOTS[3] = {3 * 256, 2 * 256, 256};
constexpr double LAUNCH_US = 4.0;
constexpr int WG_CHUNKS = 16;  // K chunks one update workgroup takes before a tile is split
// Two-level blocking of wide supernodes (options.outer_block, 256 by
// default): the trailing update of the columns right of an outer block is
// applied once, with k = the outer block's width, after its last 64-column
// panel; inside the outer block every panel updates only the outer block's
// remaining columns (k = 64). The long updates of a step go to 128x128
// target tiles (k_update_big) when there are at least options.big_tile_min
// of them (256 by default: about one per compute unit).
constexpr int64_t BIG = 128;
constexpr int64_t XCD_ORDER_MIN = 1024;  // tiles of a launch ordered for the XCDs from this many
// fusion of a step's trailing update into the next panel launch: compute
// units of the device, and short update tiles one unit runs while the panel
// workgroups factor (one resident workgroup per unit in a fused launch)
constexpr int64_t DEVICE_CUS = 256;
// rows of a backward-solve workgroup against ancestor rows: each 64-row block
// of them waits on a dependent pair of loads (the row's index, then x), so
// the blocks a workgroup walks through are kept few
constexpr int64_t FWD_ROWS = 64;  // rows of a forward-solve workgroup below its chunk
constexpr int64_t FWD_ROWS_BIG = 256;     // the same in launches of many workgroups
constexpr int64_t FWD_BIG_LAUNCH = 2048;
#ifndef BELOW_ROWS
#define BELOW_ROWS 64
#endif
constexpr int64_t FUSE_TILES_PER_CU = 4;
// deterministic load balance of an update launch of its own (an option,
// split_chunks < 0; off by default, since it adds working storage that
// Algorithm 5 does without): a launch lasts at least as long as its heaviest
// target tile, which one workgroup sums. When that tile has more K chunks
// than SPLIT_TRIGGER times the launch's
// balanced share (its chunks over min(tiles, resident workgroups)), every
// tile of more than SPLIT_SHARE times the share, and of at least
// SPLIT_MIN_CHUNKS, is cut along its contribution list into parts of about
// half the share (at least SPLIT_MIN_PART chunks, at most SPLIT_MAX_PARTS
// parts); each part is a workgroup that writes its sum into a 64x64 block of
// the workspace, and a reduce launch right after adds the parts into the
// tile in part order, so the result does not depend on timing. (Launches
// with a milder tail do not win back the reduce launch.)
constexpr int64_t RESIDENT_UPDATE_WGS = 4 * DEVICE_CUS;
constexpr double SPLIT_TRIGGER = 2.0;
constexpr double SPLIT_SHARE = 1.0;
constexpr int64_t SPLIT_MIN_CHUNKS = 64;
constexpr int64_t SPLIT_MIN_PART = 32;
constexpr int64_t SPLIT_MAX_PARTS = 64;
constexpr int FLAG_PART = 8;  // planner only: a part's target is relative to the part region

// the update work of one step before it is placed: target tiles with their
// contributions; `next` marks the trailing tiles of the column block right
// after the step's block, which the next panel launch can apply itself
struct PendingUpdate {
  bool valid = false;
  int32_t level = 0, step = 0;
  std::vector<UpdTile> tiles;               // seg0 relative to `segs`
  std::vector<UpdSeg> segs;
  std::vector<char> next;
  std::vector<double> alg;                  // algorithmic flops of each tile
};

// One rectangle of the ancestor update: target rows [r0, r0+mr) and columns
// [c0, c0+nc) of Lnz(P); source rows [sx, ..) and [sy, ..) of Lnz(J).
struct Rect {
  int64_t P, r0, c0, mr, nc, sx, sy;
  bool diag;
};

// entries a contribution writes: its full rectangle, or the part with
// row >= col when the target tile sits on the diagonal of its supernode
double seg_entries(int64_t ra, int64_t rb, int64_t ca, int64_t cb, bool diag) {
  if (!diag) return (double)(rb - ra) * (double)(cb - ca);
  double e = 0;
  for (int64_t c = ca; c < cb; ++c) e += (double)std::max<int64_t>(0, rb - std::max(ra, c));
  return e;
}

// flops the kernel executes for a contribution: the 16x16 blocks of the
// 64x64 tile that meet its rectangle, over k rounded up to the K chunk
double seg_exec_flops(int64_t ra, int64_t rb, int64_t ca, int64_t cb, int64_t k) {
  int64_t br = (rb - 1) / 16 - ra / 16 + 1, bc = (cb - 1) / 16 - ca / 16 + 1;
  int64_t kp = (k + 15) / 16 * 16;
  return 2.0 * (double)(br * 16) * (double)(bc * 16) * (double)kp;
}

}  // namespace

int32_t tile_variant(const UpdTile* tiles, int64_t count, const UpdSeg* segs) {
  // chunk rounds of the three ways of staging K: KCH-deep chunks of every
  // contribution; chunks shaped to the contribution's rectangle (64-row
  // windows KCH deep, 32- and 16-row windows 2 and 4 times deeper); the
  // contributions of a tile end to end (each padded to a multiple of 4), KCH
  // deep
  int64_t rounds = 0, rounds_win = 0, rounds_pack = 0;
  for (int64_t i = 0; i < count; ++i) {
    const UpdTile& t = tiles[i];
    int64_t kt = 0;
    for (int32_t e = 0; e < t.nseg; ++e) {
      const UpdSeg& g = segs[t.seg0 + e];
      const bool r16 = (g.ra >> 4) == ((g.rb - 1) >> 4) && (g.ca >> 4) == ((g.cb - 1) >> 4);
      const bool r32 = (g.ra >> 5) == ((g.rb - 1) >> 5) && (g.ca >> 5) == ((g.cb - 1) >> 5);
      const int64_t kc = KCH * (r16 ? 4 : (r32 ? 2 : 1));
      rounds += (g.k + KCH - 1) / KCH;
      rounds_win += (g.k + kc - 1) / kc;
      kt += (g.k + 3) & ~3;
    }
    rounds_pack += (kt + KCH - 1) / KCH;
  }
  // another staging only when it saves at least 30 % of the rounds
  const int64_t best = std::min(rounds_win, rounds_pack);
  if (10 * best > 7 * rounds) return UPD_TILE;
  return rounds_pack < rounds_win ? UPD_TILE_PACK : UPD_TILE_WIN;
}

int build_plan(Symbolic& s, std::string& err) {
  Plan& p = s.plan;
  p = Plan();
  if (s.opt.outer_block < NB || s.opt.outer_block % NB) {
    err = "outer_block must be a positive multiple of 64";
    return -1;
  }
  const int64_t NBO = s.opt.outer_block;
  const int64_t MIN_BIG_TILES =
      s.opt.big_tile_min > 0 ? s.opt.big_tile_min : std::numeric_limits<int64_t>::max();
  const int64_t MIN_TALL_TILES =
      s.opt.tall_tile_min > 0 ? s.opt.tall_tile_min : std::numeric_limits<int64_t>::max();
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

  // scale slots of the 16-bit update forms: one per 64-column block of every
  // supernode (its rows below the block's diagonal tile), then one per
  // supernode (its rows below its diagonal block)
  std::vector<int32_t> sbase(S + 1, 0);
  for (int64_t J = 0; J < S; ++J) sbase[J + 1] = sbase[J] + (int32_t)((W(J) + NB - 1) / NB) + 1;
  p.n_scale_slots = sbase[S];
  auto anc_slot = [&](int64_t J) { return sbase[J + 1] - 1; };
  // input entry of the diagonal of every factored column
  p.diag_src.assign(n, -1);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t e = s.colptr[j]; e < s.colptr[j + 1]; ++e)
      if (s.rowidx[e] == j) p.diag_src[inv[j]] = e;

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
  // hybrid method, a model of the time (us) the update-matrix route saves for
  // supernode J: written in place its ancestor updates take one K pass per
  // (rectangle, 64x64 target tile) pair they meet, through RL one per 64x64
  // tile of U_J, and the assembly moves 32 bytes per entry of U_J (written,
  // read, target read and written); K passes run at about 1024 resident tiles
  // per 2.3 us round, the assembly at about 2 TB/s (half the rate it moves
  // its bytes at: a margin for what the model leaves out)
  auto rl_gain_us = [&](int64_t J) {
    const int64_t r = M(J) - W(J);
    if (r <= 0) return 0.0;
    int64_t pieces = 0;
    for (const Rect& q : rects[J]) {
      const int64_t nr = (q.r0 + q.mr - 1) / TM - q.r0 / TM + 1;
      const int64_t nc = (q.c0 + q.nc - 1) / TN - q.c0 / TN + 1;
      pieces += nr * nc;
    }
    const int64_t t = (r + TM - 1) / TM;
    const double passes = (double)(pieces - t * (t + 1) / 2) * (double)((W(J) + KCH - 1) / KCH);
    return passes / HYB_PASSES_PER_US - 32.0 * 0.5 * (double)r * (double)(r + 1) / HYB_BYTES_PER_US;
  };
  // Where a wide supernode switches from outer blocks to per-step trailing
  // updates: once its trailing region holds few enough 64x64 tiles to run
  // beside the next panel launch (the fused form), every step updates all of
  // it (k = 64) and that work overlaps the panels; before that, the trailing
  // columns right of an outer block are updated once per outer block. The
  // switch falls on an outer-block boundary, where the outer block's update
  // has brought every trailing column up to date. It is one column for all
  // supernodes of a level: the previous-block update is a property of a whole
  // panel launch, so at every step the level's supernodes must agree on
  // whether their next block still needs it. The budget follows the fusion
  // rule below: FUSE_TILES_PER_CU tiles per compute unit left free by the
  // level's panel workgroups.
  std::vector<int64_t> sw(S, 0);
  for (int32_t h = 0; h < p.nlevels; ++h) {
    int64_t wmax = 0;
    for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q)
      wmax = std::max<int64_t>(wmax, W(p.lvl_sn[q]));
    if (wmax <= NBO) continue;
    int64_t sl = (wmax + NBO - 1) / NBO * NBO;
    for (int64_t c = 0; c < wmax; c += NBO) {
      int64_t tiles = 0, rowt = 0;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        const int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        if (w <= c) continue;
        const int64_t a = (w - c + TN - 1) / TN, b = (m - c + TM - 1) / TM;
        tiles += a * b - a * (a - 1) / 2;
        rowt += b;
      }
      if (tiles <= FUSE_TILES_PER_CU * std::max<int64_t>(0, DEVICE_CUS - rowt)) {
        sl = c;
        break;
      }
    }
    for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) sw[p.lvl_sn[q]] = sl;
  }

  // launches
  p.flops_tiles = 0;
  // places a step's update work in p.updates, heaviest workgroups first: into
  // a launch of its own, or as the fused part of panel launch `fused_into`
  // (the tiles not marked next, followed by the next ones, which that
  // launch's panels apply themselves and which stay listed for the unfused
  // form)
  // the deterministic split of a launch's heaviest tiles (SPLIT_SHARE above):
  // false when no tile is cut; otherwise `out` holds the launch's tiles with
  // every cut tile replaced by its parts (targets: 64x64 blocks at 4096 *
  // slot, relative to the part region until the plan is complete) and `reds`
  // one record per cut tile
  auto split_heavy = [&](const PendingUpdate& u, PendingUpdate& out,
                         std::vector<PartReduce>& reds) -> bool {
    if (!s.opt.deterministic || s.opt.split_chunks == 0) return false;
    const size_t nt = u.tiles.size();
    if (nt == 0) return false;
    std::vector<int64_t> ch(nt, 0);
    int64_t total = 0;
    for (size_t i = 0; i < nt; ++i) {
      for (int32_t e = 0; e < u.tiles[i].nseg; ++e)
        ch[i] += (u.segs[u.tiles[i].seg0 + e].k + KCH - 1) / KCH;
      total += ch[i];
    }
    int64_t thr, part;
    if (s.opt.split_chunks > 0) {
      thr = part = s.opt.split_chunks;
    } else {
      const double share =
          (double)total / (double)std::min<int64_t>((int64_t)nt, RESIDENT_UPDATE_WGS);
      if ((double)*std::max_element(ch.begin(), ch.end()) <= SPLIT_TRIGGER * share) return false;
      thr = std::max<int64_t>(SPLIT_MIN_CHUNKS, (int64_t)std::ceil(SPLIT_SHARE * share));
      part = std::max<int64_t>(SPLIT_MIN_PART, (int64_t)std::ceil(0.5 * share));
    }
    auto eligible = [&](size_t i) {
      const UpdTile& t = u.tiles[i];
      return ch[i] > thr && t.n > NARROW_COLS && !(t.flags & (FLAG_ATOMIC | FLAG_ASSIGN));
    };
    bool any = false;
    for (size_t i = 0; i < nt && !any; ++i) any = eligible(i);
    if (!any) return false;
    out = PendingUpdate();
    out.valid = true;
    out.level = u.level;
    out.step = u.step;
    int64_t slot = 0;
    for (size_t i = 0; i < nt; ++i) {
      const UpdTile& t = u.tiles[i];
      if (!eligible(i)) {
        UpdTile c = t;
        c.seg0 = (int32_t)out.segs.size();
        out.segs.insert(out.segs.end(), u.segs.begin() + t.seg0,
                        u.segs.begin() + t.seg0 + t.nseg);
        out.tiles.push_back(c);
        out.next.push_back(u.next[i]);
        out.alg.push_back(u.alg[i]);
        continue;
      }
      const int64_t np = std::min<int64_t>(SPLIT_MAX_PARTS, (ch[i] + part - 1) / part);
      const int64_t per = (ch[i] + np - 1) / np;  // K chunks of a part
      const bool diag = (t.flags & FLAG_DIAG) != 0;
      PartReduce r;
      r.c = t.c;
      r.pbase = slot * NB * NB;
      r.ldc = t.ldc;
      r.m = t.m;
      r.n = t.n;
      r.flags = diag ? 1 : 0;
      r.nparts = 0;
      r.pad = 0;
      std::vector<UpdSeg> piece;
      int64_t used = 0;
      double a = 0;
      auto emit = [&]() {
        UpdTile pt = t;
        pt.c = (slot + r.nparts) * NB * NB;
        pt.ldc = (int32_t)NB;
        pt.flags = (diag ? FLAG_DIAG : 0) | FLAG_ASSIGN | FLAG_PART;
        pt.seg0 = (int32_t)out.segs.size();
        pt.nseg = (int32_t)piece.size();
        out.segs.insert(out.segs.end(), piece.begin(), piece.end());
        out.tiles.push_back(pt);
        out.next.push_back(u.next[i]);
        out.alg.push_back(a);
        r.nparts++;
        piece.clear();
        used = 0;
        a = 0;
      };
      // consecutive pieces of the contribution list, cut inside a
      // contribution's k range at a multiple of the K chunk where needed
      for (int32_t e = 0; e < t.nseg; ++e) {
        const UpdSeg& g = u.segs[t.seg0 + e];
        for (int64_t q0 = 0; q0 < g.k;) {
          const int64_t take = std::min<int64_t>(g.k - q0, (per - used) * KCH);
          UpdSeg pc = g;
          pc.x += q0 * g.lds;
          pc.y += q0 * g.lds;
          pc.k = (int32_t)take;
          piece.push_back(pc);
          a += 2.0 * (double)take * seg_entries(g.ra, g.rb, g.ca, g.cb, diag);
          used += (take + KCH - 1) / KCH;
          q0 += take;
          if (used >= per) emit();
        }
      }
      if (!piece.empty()) emit();
      slot += r.nparts;
      p.n_split_tiles += r.nparts;
      reds.push_back(r);
    }
    p.part_elems = std::max(p.part_elems, slot * NB * NB);
    return true;
  };
  auto commit = [&](const PendingUpdate& u_in, int64_t fused_into) {
    PendingUpdate cut_u;
    std::vector<PartReduce> reds;
    const bool cut = fused_into < 0 && split_heavy(u_in, cut_u, reds);
    const PendingUpdate& u = cut ? cut_u : u_in;
    const int64_t start = (int64_t)p.updates.size();
    int64_t nwave = 0;
    bool shortk = true;
    int64_t counts[2] = {0, 0};
    for (int part = 0; part < 2; ++part) {
      if (part == 1 && fused_into < 0) break;
      std::vector<std::pair<int64_t, size_t>> order;
      for (size_t i = 0; i < u.tiles.size(); ++i) {
        if (fused_into >= 0 && (u.next[i] != 0) != (part == 1)) continue;
        int64_t ch = 0;
        for (int32_t e = 0; e < u.tiles[i].nseg; ++e)
          ch += (u.segs[u.tiles[i].seg0 + e].k + KCH - 1) / KCH;
        order.push_back({-ch, i});
      }
      std::stable_sort(order.begin(), order.end(),
                       [](const std::pair<int64_t, size_t>& x, const std::pair<int64_t, size_t>& y) {
                         return x.first < y.first;
                       });
      // a launch of its own in 8x8 blocks of neighbouring tiles (each target
      // supernode's tiles by column-block and row-tile band), read by the
      // kernel as a contiguous eighth per XCD
      const bool by_xcd = fused_into < 0 && s.opt.tile_order == 1 && order.size() >= XCD_ORDER_MIN;
      if (by_xcd) {
        auto key = [&](size_t i) {
          const UpdTile& t = u.tiles[i];
          const int64_t P = std::upper_bound(p.off.begin(), p.off.end() - 1, t.c) - p.off.begin() - 1;
          const int64_t rel = t.c - p.off[P];
          const int64_t cb = rel / t.ldc / NB, rt = rel % t.ldc / NB;
          return std::make_tuple(P, cb / 8, rt / 8, cb, rt);
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](const std::pair<int64_t, size_t>& x,
                             const std::pair<int64_t, size_t>& y) {
                           return key(x.second) < key(y.second);
                         });
      }
      // a launch of its own with enough narrow tiles puts them last
      if (fused_into < 0 && !by_xcd) {
        int64_t nn = 0;
        for (auto& o : order) nn += u.tiles[o.second].n <= NARROW_COLS;
        if (nn >= WAVE_SPLIT_MIN) {
          std::stable_partition(order.begin(), order.end(),
                                [&](const std::pair<int64_t, size_t>& o) {
                                  return u.tiles[o.second].n > NARROW_COLS;
                                });
          nwave = nn;
        }
      }
      for (auto& o : order) {
        UpdTile t = u.tiles[o.second];
        const int32_t s0 = t.seg0;
        t.seg0 = (int32_t)p.segs.size();
        for (int32_t e = 0; e < t.nseg; ++e) p.segs.push_back(u.segs[s0 + e]);
        if (t.nseg != 1 || (t.flags & FLAG_ATOMIC) || u.segs[s0].k > 64) shortk = false;
        if (fused_into < 0) p.flops_upd_launch += u.alg[o.second];
        p.updates.push_back(t);
      }
      counts[part] = (int64_t)order.size();
    }
    if (fused_into >= 0) {
      p.launches[fused_into].ustart = start;
      p.launches[fused_into].ucount = counts[0];
      p.launches[fused_into].ncount = counts[1];
    } else if (counts[0]) {
      const int32_t var = shortk ? UPD_SHORT
                          : (s.opt.tile_order == 1 && counts[0] >= XCD_ORDER_MIN)
                              ? UPD_TILE_XCD
                              : tile_variant(p.updates.data() + start, counts[0], p.segs.data());
      Launch lu{LAUNCH_UPDATE, u.level, u.step, var, start, counts[0], 0, (int32_t)nwave, 0, 0, 0};
      p.launches.push_back(lu);
      if (cut) {
        const int64_t r0 = (int64_t)p.reduces.size();
        p.reduces.insert(p.reduces.end(), reds.begin(), reds.end());
        p.launches.push_back(Launch{LAUNCH_REDUCE, u.level, u.step, 0, r0, (int64_t)reds.size(), 0,
                                    0, 0, 0, 0});
      }
    }
  };
  for (int32_t h = 0; h < p.nlevels; ++h) {
    int64_t steps = 0;
    for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q)
      steps = std::max<int64_t>(steps, (W(p.lvl_sn[q]) + NB - 1) / NB);
    PendingUpdate pend;
    for (int64_t k = 0; k < steps; ++k) {
      // PANEL: one group per supernode with a column block k, one workgroup
      // per 64 rows below the diagonal tile (a single one when there are
      // none); in launches with more than panel_spread row tiles a
      // workgroup takes several consecutive row tiles, so that the redundant
      // factorization of the diagonal tile is not repeated needlessly
      int64_t ntiles = 0;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        if (k * NB >= w) continue;
        int64_t c0 = k * NB, nb = std::min<int64_t>(NB, w - c0);
        ntiles += std::max<int64_t>(1, (m - c0 - nb + 63) / 64);
      }
      const int64_t spread = std::max(1, s.opt.panel_spread);
      const int64_t per = std::max<int64_t>(1, (ntiles + spread - 1) / spread);
      // one launch per width class of the diagonal tiles (1, 2 or 4 blocks of 16)
      std::vector<PanelTile> cls[3];
      int32_t ngroups[3] = {0, 0, 0};
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        if (k * NB >= w) continue;
        int64_t c0 = k * NB, nb = std::min<int64_t>(NB, w - c0), nrows = m - c0;
        int64_t below = nrows - nb;
        // POTRF of the nb x nb tile (sum over its columns of (count)^2 with
        // counts nb..1) plus TRSM of the rows below (nb^2 per row)
        for (int64_t t = 0; t < nb; ++t) p.flops_panel += (double)(nb - t) * (double)(nb - t);
        p.flops_panel += (double)below * (double)nb * (double)nb;
        const int ci = nb <= 16 ? 0 : (nb <= 32 ? 1 : 2);
        int64_t nt = (below + 63) / 64;  // row tiles
        int64_t nwg = std::max<int64_t>(1, (nt + per - 1) / per);
        PanelTile pt;
        pt.diag = p.off[J] + c0 * m + c0;
        pt.ld = (int32_t)m;
        pt.nb = (int32_t)nb;
        pt.nrows = (int32_t)nrows;
        pt.col = (int32_t)(s.sn_ptr[J] + c0);
        pt.slot = 0;
        pt.grp = ngroups[ci]++;
        pt.gcnt = (int32_t)nwg;
        pt.s_step = sbase[J] + (int32_t)k;
        pt.s_anc = anc_slot(J);
        pt.rw = (int32_t)(w - c0);
        for (int64_t g = 0; g < nwg; ++g) {
          pt.row0 = (int32_t)(nb + 64 * per * g);
          pt.nrt = (int32_t)std::min<int64_t>(per, std::max<int64_t>(0, nt - per * g));
          cls[ci].push_back(pt);
        }
      }
      // a narrow class gets a launch of its own unless running its tiles in
      // the next wider class's launch is estimated cheaper: workgroup rounds
      // (workgroups over resident slots) times a per-workgroup time, plus a
      // fixed cost per launch
      auto rounds = [](int64_t wgs, int64_t slots) { return (wgs + slots - 1) / slots; };
      for (int ci = 0; ci < 2; ++ci)
        if (!cls[ci].empty()) {
          const int64_t nn = (int64_t)cls[ci].size(), nw = (int64_t)cls[ci + 1].size();
          const double tw = PANEL_US[ci + 1], tn = PANEL_US[ci];
          const int64_t sw = PANEL_SLOTS[ci + 1], sn = PANEL_SLOTS[ci];
          const double sep = (nw ? rounds(nw, sw) * tw + LAUNCH_US : 0.0) + rounds(nn, sn) * tn +
                             LAUNCH_US;
          const double fold = rounds(nn + nw, sw) * tw + LAUNCH_US;
          if (fold > sep) continue;
          for (PanelTile& t : cls[ci]) t.grp += ngroups[ci + 1];
          cls[ci + 1].insert(cls[ci + 1].end(), cls[ci].begin(), cls[ci].end());
          ngroups[ci + 1] += ngroups[ci];
          ngroups[ci] = 0;
          cls[ci].clear();
        }
      // the previous step's update: its trailing tiles of this column block
      // go into this step's panel workgroups (pre-update) and the rest runs
      // as extra workgroups of this step's 64-column panel launch, when the
      // rest is all short single-contribution tiles few enough to run beside
      // the panel workgroups; otherwise it keeps a launch of its own, before
      // this step's panels
      bool fuse = false;
      if (pend.valid) {
        int64_t rest = 0, npw = 0;
        bool short_rest = true, has_next = false;
        for (size_t i = 0; i < pend.tiles.size(); ++i) {
          has_next = has_next || pend.next[i];
          if (pend.next[i]) continue;
          ++rest;
          const UpdTile& t = pend.tiles[i];
          if (t.nseg != 1 || (t.flags & FLAG_ATOMIC) || pend.segs[t.seg0].k > 64)
            short_rest = false;
        }
        for (int ci = 0; ci < 3; ++ci) npw += (int64_t)cls[ci].size();
        // (the update tiles ride on the 64-column class launch)
        // (after an outer block the next block's update came with the long
        // part, so no panel of this step has a previous-block update to apply)
        fuse = has_next && short_rest && !cls[2].empty() &&
               rest <= FUSE_TILES_PER_CU * std::max<int64_t>(0, DEVICE_CUS - npw);
        if (!fuse) commit(pend, -1);
      }
      const int32_t cls_nbb[3] = {1, 2, 4};
      int64_t widest = -1;
      for (int ci = 0; ci < 3; ++ci) {
        if (cls[ci].empty()) continue;
        Launch lp{LAUNCH_PANEL, h, (int32_t)k, cls_nbb[ci], (int64_t)p.panels.size(),
                  (int64_t)cls[ci].size(), fuse ? 1 : 0, 0, 0, 0, 0};
        p.panels.insert(p.panels.end(), cls[ci].begin(), cls[ci].end());
        widest = (int64_t)p.launches.size();
        p.launches.push_back(lp);
        p.max_groups = std::max(p.max_groups, ngroups[ci]);
      }
      if (fuse) commit(pend, widest);
      // UPDATE work of step k, in two parts. The short part (pend): the
      // trailing update by block k of the columns of its own 256-column outer
      // block (k = 64; the next panel launch may apply the tiles of block k+1
      // itself). The long part: for a supernode whose block k closes an outer
      // block, the update of every column right of it by the whole outer
      // block (k = 256), and for a supernode whose last block is k, all of its
      // SYRK/GEMM updates written straight into the ancestors. The long part
      // is cut into 128x128 target tiles when that gives enough of them to
      // fill the device, and then runs as a launch of its own; otherwise it
      // joins the short part in 64x64 tiles.
      pend = PendingUpdate();
      pend.valid = true;
      pend.level = h;
      pend.step = (int32_t)k;
      auto add_tile = [&](UpdTile t, const std::vector<UpdSeg>& gs, size_t g0, size_t g1,
                          bool next) {
        t.seg0 = (int32_t)pend.segs.size();
        t.nseg = (int32_t)(g1 - g0);
        pend.segs.insert(pend.segs.end(), gs.begin() + g0, gs.begin() + g1);
        double alg = 0;
        for (size_t i = g0; i < g1; ++i)
          alg += 2.0 * (double)gs[i].k *
                 seg_entries(gs[i].ra, gs[i].rb, gs[i].ca, gs[i].cb, (t.flags & FLAG_DIAG) != 0);
        pend.tiles.push_back(t);
        pend.next.push_back(next ? 1 : 0);
        pend.alg.push_back(alg);
      };
      std::vector<int64_t> finished;
      struct Outer {
        int64_t J, c1, ob0;  // trailing columns from c1 on, outer block [ob0, c1)
      };
      std::vector<Outer> outer;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        if (k * NB >= w) continue;
        int64_t c0 = k * NB, nb = std::min<int64_t>(NB, w - c0), c1 = c0 + nb;
        if (c1 >= w) {
          finished.push_back(J);
          continue;
        }
        const int64_t ob0 = c0 / NBO * NBO;
        const int64_t ob1 = c0 >= sw[J] ? w : std::min<int64_t>(w, ob0 + NBO);
        if (c1 == ob1) {
          outer.push_back(Outer{J, c1, ob0});
          continue;
        }
        for (int64_t tj0 = c1; tj0 < ob1; tj0 += TN) {
          int64_t tn = std::min<int64_t>(TN, ob1 - tj0);
          for (int64_t ti0 = tj0; ti0 < m; ti0 += TM) {
            int64_t tm = std::min<int64_t>(TM, m - ti0);
            bool diag = ti0 == tj0;
            UpdTile t;
            t.c = p.off[J] + tj0 * m + ti0;
            t.ldc = (int32_t)m;
            t.m = (int32_t)tm;
            t.n = (int32_t)tn;
            t.flags = diag ? FLAG_DIAG : 0;
            UpdSeg g;
            g.x = p.off[J] + c0 * m + ti0;
            g.y = p.off[J] + c0 * m + tj0;
            g.lds = (int32_t)m;
            g.k = (int32_t)nb;
            g.ra = 0;
            g.rb = (int32_t)tm;
            g.ca = 0;
            g.cb = (int32_t)tn;
            g.src = (int32_t)J;
            g.sslot = sbase[J] + (int32_t)k;
            add_tile(t, std::vector<UpdSeg>{g}, 0, 1, tj0 == c1);
            p.flops_tiles += seg_exec_flops(0, tm, 0, tn, nb);
            p.flops_upd_alg += 2.0 * (double)nb * seg_entries(0, tm, 0, tn, diag);
          }
        }
      }
      // the supernodes whose ancestor updates go through an update matrix:
      // all finished ones in RL; in the hybrid method those whose rectangles
      // would fill the MFMA blocks of the target tiles poorly
      std::vector<int64_t> via_u;
      if (s.opt.method == 1) {
        via_u.swap(finished);
      } else if (s.opt.method == 2) {
        // the supernodes the route saves time for, when together they save
        // more than the step's two extra launches (SYRK and assembly) cost
        std::vector<int64_t> keep;
        double saved = 0;
        for (int64_t J : finished) {
          const double g = rl_gain_us(J);
          if (g > 0) {
            via_u.push_back(J);
            saved += g;
          } else {
            keep.push_back(J);
          }
        }
        if (saved > s.opt.hybrid_step_us)
          finished.swap(keep);
        else
          via_u.clear();
      }
      if (!via_u.empty()) {
        // RL (Algorithm 4): for every supernode J whose cdiv ends at this
        // step, one SYRK forms its update matrix U_J = -L_{R,J} L_{R,J}^T
        // (R: the r_J rows below the diagonal block; lower triangle, r_J x r_J
        // column-major, in working storage after the factor), then every
        // column of U_J is added into the ancestor supernode that owns that
        // column, at the rows its relative indices give (the rows of J below
        // the column all lie in the ancestor's index list, eq. (1)). The
        // working storage is reused by the next step.
        std::vector<UpdTile> ut;
        std::vector<UpdSeg> ug;
        double alg = 0;
        bool shortk = true;
        int64_t uo = 0;
        const int64_t ac0 = (int64_t)p.asmcols.size();
        for (int64_t J : via_u) {
          const int64_t w = W(J), m = M(J), r = m - w;
          if (r == 0) continue;
          const int64_t ub = p.l_elems + uo;
          for (int64_t tj0 = 0; tj0 < r; tj0 += TN) {
            const int64_t tn = std::min<int64_t>(TN, r - tj0);
            for (int64_t ti0 = tj0; ti0 < r; ti0 += TM) {
              const int64_t tm = std::min<int64_t>(TM, r - ti0);
              const bool diag = ti0 == tj0;
              UpdTile t;
              t.c = ub + tj0 * r + ti0;
              t.ldc = (int32_t)r;
              t.m = (int32_t)tm;
              t.n = (int32_t)tn;
              t.flags = (diag ? FLAG_DIAG : 0) | FLAG_ASSIGN;
              t.seg0 = (int32_t)ug.size();
              t.nseg = 1;
              UpdSeg g;
              g.x = p.off[J] + w + ti0;
              g.y = p.off[J] + w + tj0;
              g.lds = (int32_t)m;
              g.k = (int32_t)w;
              g.ra = 0;
              g.rb = (int32_t)tm;
              g.ca = 0;
              g.cb = (int32_t)tn;
              g.src = (int32_t)J;
              g.sslot = anc_slot(J);
              ut.push_back(t);
              ug.push_back(g);
              p.flops_tiles += seg_exec_flops(0, tm, 0, tn, w);
              alg += 2.0 * (double)w * seg_entries(0, tm, 0, tn, diag);
            }
          }
          if (w > 64) shortk = false;
          // assembly: the columns of U_J grouped by the ancestor owning them
          const int32_t* gJ = s.gl.data() + s.gl_ptr[J];
          for (int64_t j0 = 0; j0 < r;) {
            const int64_t P = snode[gJ[w + j0]];
            int64_t j1 = j0 + 1;
            while (j1 < r && snode[gJ[w + j1]] == P) ++j1;
            const int32_t* gP = s.gl.data() + s.gl_ptr[P];
            const int64_t mP = M(P);
            const int64_t rp0 = (int64_t)p.asm_rows.size();
            for (int64_t i = j0; i < r; ++i) {
              const int32_t* it = std::lower_bound(gP, gP + mP, gJ[w + i]);
              if (it == gP + mP || *it != gJ[w + i]) {
                err = "internal: a row of an update matrix outside its ancestor's structure";
                return -1;
              }
              p.asm_rows.push_back((int32_t)(it - gP));
            }
            for (int64_t j = j0; j < j1; ++j)
              p.asmcols.push_back(AsmCol{ub + j * r + j,
                                         p.off[P] + (gJ[w + j] - s.sn_ptr[P]) * mP,
                                         (int32_t)(rp0 + (j - j0)), (int32_t)(r - j)});
            j0 = j1;
          }
          uo += r * r;
          uo = (uo + 7) & ~int64_t(7);
        }
        if (p.asm_rows.size() > (size_t)INT32_MAX) {
          err = "RL assembly lists too large";
          return -1;
        }
        // the step's columns grouped by target column, in source order
        std::stable_sort(p.asmcols.begin() + ac0, p.asmcols.end(),
                         [](const AsmCol& x, const AsmCol& y) { return x.dst < y.dst; });
        p.u_elems = std::max(p.u_elems, uo);
        if (!ut.empty()) {
          const int64_t start = (int64_t)p.updates.size();
          for (UpdTile t : ut) {
            const UpdSeg g = ug[t.seg0];
            t.seg0 = (int32_t)p.segs.size();
            p.segs.push_back(g);
            p.updates.push_back(t);
          }
          p.launches.push_back(Launch{LAUNCH_UPDATE, h, (int32_t)k, shortk ? UPD_SHORT : UPD_TILE,
                                      start, (int64_t)ut.size(), 0, 0, 0, 0, 0});
          p.launches.push_back(Launch{LAUNCH_ASSEMBLE, h, (int32_t)k, 0, ac0,
                                      (int64_t)p.asmcols.size() - ac0, 0, 0, 0, 0, 0});
          p.flops_upd_alg += alg;
          p.flops_upd_launch += alg;
        }
      }
      // the long part cut by a target tile grid of side T; every tile keeps
      // its contributions in ascending source order
      struct LongPart {
        std::vector<UpdTile> tiles;  // seg0 relative to segs
        std::vector<UpdSeg> segs;
        std::vector<double> alg;
        double exec = 0, alg_total = 0;
        int64_t merged = 0, split = 0, whole = 0;
      };
      // (target tiles of TR rows and TC columns; in column block TJ of a
      // target the row tiles start at its diagonal row TJ * TC, so the first
      // holds the diagonal block and the rows below it)
      auto build_long = [&](int64_t TR, int64_t TC) {
        LongPart lp;
        auto put = [&](UpdTile t, const std::vector<UpdSeg>& gs) {
          const bool diag = (t.flags & FLAG_DIAG) != 0;
          double alg = 0;
          for (const UpdSeg& g : gs) {
            lp.exec += seg_exec_flops(g.ra, g.rb, g.ca, g.cb, g.k);
            alg += 2.0 * (double)g.k * seg_entries(g.ra, g.rb, g.ca, g.cb, diag);
          }
          lp.alg_total += alg;
          lp.whole++;
          // one workgroup while the tile's K chunks fit the budget (always in
          // the deterministic form); otherwise consecutive pieces of its
          // contribution list (cut inside a contribution's k range where
          // needed), each added atomically
          int64_t chunks = 0;
          for (const UpdSeg& g : gs) chunks += (g.k + KCH - 1) / KCH;
          auto emit = [&](UpdTile tt, const std::vector<UpdSeg>& part) {
            double a = 0;
            for (const UpdSeg& g : part)
              a += 2.0 * (double)g.k * seg_entries(g.ra, g.rb, g.ca, g.cb, diag);
            tt.seg0 = (int32_t)lp.segs.size();
            tt.nseg = (int32_t)part.size();
            lp.segs.insert(lp.segs.end(), part.begin(), part.end());
            lp.tiles.push_back(tt);
            lp.alg.push_back(a);
          };
          if (chunks <= WG_CHUNKS || s.opt.deterministic) {
            emit(t, gs);
            return;
          }
          t.flags |= FLAG_ATOMIC;
          std::vector<UpdSeg> part;
          int64_t used = 0;
          for (const UpdSeg& g : gs) {
            for (int64_t q0 = 0; q0 < g.k;) {
              int64_t take = std::min<int64_t>(g.k - q0, (WG_CHUNKS - used) * KCH);
              UpdSeg piece = g;
              piece.x += q0 * g.lds;
              piece.y += q0 * g.lds;
              piece.k = (int32_t)take;
              part.push_back(piece);
              used += (take + KCH - 1) / KCH;
              q0 += take;
              if (used >= WG_CHUNKS) {
                emit(t, part);
                lp.split++;
                part.clear();
                used = 0;
              }
            }
          }
          if (!part.empty()) {
            emit(t, part);
            lp.split++;
          }
        };
        // trailing update by a whole outer block: one contribution per
        // 64-column block of it (each with its own scale slot in the 16-bit
        // forms), tiles anchored at the first column right of the block
        for (const Outer& o : outer) {
          const int64_t J = o.J, w = W(J), m = M(J);
          for (int64_t tj0 = o.c1; tj0 < w; tj0 += TC) {
            const int64_t tn = std::min<int64_t>(TC, w - tj0);
            for (int64_t ti0 = tj0; ti0 < m; ti0 += TR) {
              const int64_t tm = std::min<int64_t>(TR, m - ti0);
              UpdTile t;
              t.c = p.off[J] + tj0 * m + ti0;
              t.ldc = (int32_t)m;
              t.m = (int32_t)tm;
              t.n = (int32_t)tn;
              t.flags = ti0 == tj0 ? FLAG_DIAG : 0;
              t.seg0 = t.nseg = 0;
              std::vector<UpdSeg> gs;
              for (int64_t b0 = o.ob0; b0 < o.c1; b0 += NB) {
                UpdSeg g;
                g.x = p.off[J] + b0 * m + ti0;
                g.y = p.off[J] + b0 * m + tj0;
                g.lds = (int32_t)m;
                g.k = (int32_t)std::min<int64_t>(NB, o.c1 - b0);
                g.ra = 0;
                g.rb = (int32_t)tm;
                g.ca = 0;
                g.cb = (int32_t)tn;
                g.src = (int32_t)J;
                g.sslot = sbase[J] + (int32_t)(b0 / NB);
                gs.push_back(g);
              }
              put(t, gs);
            }
          }
        }
        // ancestor updates: every rectangle cut by the T x T tile grid of its
        // target supernode, the pieces grouped by target tile (key: target,
        // tile column, tile row), in ascending source order
        std::map<std::tuple<int64_t, int64_t, int64_t>, std::vector<UpdSeg>> by_tile;
        for (int64_t J : finished) {
          int64_t mJ = M(J), wJ = W(J);
          for (const Rect& r : rects[J]) {
            int64_t mP = M(r.P), wP = W(r.P);
            for (int64_t TJ = r.c0 / TC; TJ * TC < r.c0 + r.nc; ++TJ) {
              const int64_t cs = TJ * TC;
              for (int64_t TI = r.r0 > cs ? (r.r0 - cs) / TR : 0; cs + TI * TR < r.r0 + r.mr; ++TI) {
                const int64_t rs = cs + TI * TR;
                int64_t rlo = std::max(r.r0, rs), rhi = std::min({r.r0 + r.mr, rs + TR, mP});
                int64_t clo = std::max(r.c0, cs), chi = std::min({r.c0 + r.nc, cs + TC, wP});
                if (rlo >= rhi || clo >= chi) continue;
                if (TI == 0 && rhi - 1 < clo) continue;  // entirely above the diagonal
                UpdSeg g;
                g.x = p.off[J] + r.sx + (rlo - r.r0);
                g.y = p.off[J] + r.sy + (clo - r.c0);
                g.lds = (int32_t)mJ;
                g.k = (int32_t)wJ;
                g.ra = (int32_t)(rlo - rs);
                g.rb = (int32_t)(rhi - rs);
                g.ca = (int32_t)(clo - cs);
                g.cb = (int32_t)(chi - cs);
                g.src = (int32_t)J;
                g.sslot = anc_slot(J);
                by_tile[std::make_tuple(r.P, TJ, TI)].push_back(g);
              }
            }
          }
        }
        for (auto& kv : by_tile) {
          int64_t P = std::get<0>(kv.first), TJ = std::get<1>(kv.first), TI = std::get<2>(kv.first);
          int64_t mP = M(P), wP = W(P);
          UpdTile t;
          const int64_t cs = TJ * TC, rs = cs + TI * TR;
          t.c = p.off[P] + cs * mP + rs;
          t.ldc = (int32_t)mP;
          t.m = (int32_t)std::min<int64_t>(TR, mP - rs);
          t.n = (int32_t)std::min<int64_t>(TC, wP - cs);
          t.flags = TI == 0 ? FLAG_DIAG : 0;
          t.seg0 = t.nseg = 0;
          if (kv.second.size() > 1) lp.merged++;
          put(t, kv.second);
        }
        return lp;
      };
      // the long part: a launch of its own in 128x128 tiles when there are
      // enough of them (with the same work in 64x64 tiles kept for the forms
      // whose kernels take only those, the 16-bit update forms); otherwise it
      // joins the short part in 64x64 tiles
      auto place = [&](const LongPart& part) {
        const int64_t start = (int64_t)p.updates.size();
        std::vector<std::pair<int64_t, size_t>> order;
        for (size_t i = 0; i < part.tiles.size(); ++i) {
          int64_t ch = 0;
          for (int32_t e = 0; e < part.tiles[i].nseg; ++e)
            ch += (part.segs[part.tiles[i].seg0 + e].k + KCH - 1) / KCH;
          order.push_back({-ch * part.tiles[i].m * part.tiles[i].n, i});
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<int64_t, size_t>& x,
                            const std::pair<int64_t, size_t>& y) { return x.first < y.first; });
        for (auto& o : order) {
          UpdTile t = part.tiles[o.second];
          const int32_t s0 = t.seg0;
          t.seg0 = (int32_t)p.segs.size();
          for (int32_t e = 0; e < t.nseg; ++e) p.segs.push_back(part.segs[s0 + e]);
          p.updates.push_back(t);
        }
        return start;
      };
      LongPart lp = build_long(BIG, BIG);
      if (lp.whole >= MIN_BIG_TILES) {
        LongPart alt = build_long(TM, TN);
        Launch lb{LAUNCH_UPDATE, h, (int32_t)k, UPD_BIG, place(lp), (int64_t)lp.tiles.size(),
                  0, 0, 0, 0, 0};
        lb.alt_start = place(alt);
        lb.alt_count = (int64_t)alt.tiles.size();
        p.launches.push_back(lb);
        p.flops_tiles += lp.exec;
        p.flops_upd_alg += lp.alg_total;
        p.flops_upd_launch += lp.alg_total;
        p.n_merged_tiles += lp.merged;
        p.n_split_tiles += lp.split;
      } else {
        // 128x64 target tiles for a long part of enough of them (the same work
        // in 64x64 tiles kept for the forms other than FP64)
        LongPart tp;
        if (MIN_TALL_TILES < std::numeric_limits<int64_t>::max()) tp = build_long(2 * TM, TN);
        if (tp.whole >= MIN_TALL_TILES) {
          LongPart alt = build_long(TM, TN);
          Launch lt{LAUNCH_UPDATE, h, (int32_t)k, UPD_TALL, place(tp), (int64_t)tp.tiles.size(),
                    0, 0, 0, 0, 0};
          lt.alt_start = place(alt);
          lt.alt_count = (int64_t)alt.tiles.size();
          p.launches.push_back(lt);
          p.flops_tiles += tp.exec;
          p.flops_upd_alg += tp.alg_total;
          p.flops_upd_launch += tp.alg_total;
          p.n_merged_tiles += tp.merged;
          p.n_split_tiles += tp.split;
        } else {
          LongPart sp = build_long(TM, TN);
          for (size_t i = 0; i < sp.tiles.size(); ++i) {
            const UpdTile& t = sp.tiles[i];
            add_tile(t, sp.segs, t.seg0, t.seg0 + t.nseg, false);
          }
          p.flops_tiles += sp.exec;
          p.flops_upd_alg += sp.alg_total;
          p.n_merged_tiles += sp.merged;
          p.n_split_tiles += sp.split;
        }
      }
    }
    if (pend.valid) commit(pend, -1);
  }
  // the part blocks follow the update matrices in the workspace
  const int64_t part_base = p.l_elems + p.u_elems;
  for (UpdTile& t : p.updates)
    if (t.flags & FLAG_PART) {
      t.c += part_base;
      t.flags &= ~FLAG_PART;
    }
  for (PartReduce& r : p.reduces) r.pbase += part_base;
  p.ws_elems = part_base + p.part_elems;
  // diagonal tiles of every 64-column step, inverted after the factorization,
  // grouped by width class
  for (int ci = 0; ci < 3; ++ci) {
    p.dt_ptr[ci] = (int64_t)p.dtiles.size();
    for (int64_t J = 0; J < S; ++J)
      for (int64_t c0 = 0; c0 < W(J); c0 += NB) {
        int64_t nb = std::min<int64_t>(NB, W(J) - c0);
        if ((nb <= 16 ? 0 : (nb <= 32 ? 1 : 2)) != ci) continue;
        p.dtiles.push_back(DiagTile{p.off[J] + c0 * M(J) + c0, (int32_t)M(J), (int32_t)nb});
      }
  }
  p.dt_ptr[3] = (int64_t)p.dtiles.size();
  // diagonal blocks of the two-chunk solve steps that have a second chunk
  for (int64_t J = 0; J < S; ++J)
    for (int64_t c0 = 0; c0 < W(J); c0 += 2 * NB) {
      int64_t nb = std::min<int64_t>(2 * NB, W(J) - c0);
      if (nb > NB) p.ptiles.push_back(DiagTile{p.off[J] + c0 * M(J) + c0, (int32_t)M(J), (int32_t)nb});
    }
  // solves: forward by level and step of two 64-column chunks (row tiles of
  // FWD_ROWS below them, for each chunk), backward by level from the root: first
  // every 64-column chunk against the ancestor rows (segments of BELOW_ROWS rows),
  // then the steps of two chunks from the last down, each chunk pushing into
  // the earlier 64-column chunks of its supernode
  {
    constexpr int64_t SB = 2 * NB;  // columns of a solve step
    auto base_tile = [&](int64_t J) {
      SolveTile t;
      t.off = p.off[J];
      t.ld = (int32_t)M(J);
      t.f = (int32_t)s.sn_ptr[J];
      t.w = (int32_t)W(J);
      t.gl = (int32_t)s.gl_ptr[J];
      t.c0 = t.nb = t.r0 = t.r1 = t.flags = 0;
      t.cslot = -1;
      return t;
    };
    auto push_launch = [&](int32_t kind, int32_t h, int64_t start, int32_t chain) {
      int64_t cnt = (int64_t)p.stiles.size() - start;
      if (cnt) p.slaunches.push_back(SolveLaunch{kind, h, start, cnt, chain, 0});
    };
    p.sneed.clear();
    p.nchains = 0;
    // A level of several steps runs as one chained launch: its supernodes of
    // two or more steps get a counter per step. Returns the counter base of
    // supernode J (or -1).
    auto chain_slots = [&](int64_t J) -> int32_t {
      const int64_t steps = (W(J) + SB - 1) / SB;
      if (steps < 2) return -1;
      const int32_t base = (int32_t)p.sneed.size();
      p.sneed.resize(p.sneed.size() + steps, 0);
      return base;
    };
    for (int32_t h = 0; h < p.nlevels; ++h) {
      int64_t steps = 0;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q)
        steps = std::max<int64_t>(steps, (W(p.lvl_sn[q]) + SB - 1) / SB);
      const bool chain = steps >= 2;
      std::vector<int32_t> cslot(p.lvl_ptr[h + 1] - p.lvl_ptr[h], -1);
      if (chain)
        for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q)
          cslot[q - p.lvl_ptr[h]] = chain_slots(p.lvl_sn[q]);
      const int64_t lstart = (int64_t)p.stiles.size();
      for (int64_t k = 0; k < steps; ++k) {
        int64_t start = (int64_t)p.stiles.size();
        // rows per workgroup: FWD_ROWS, or FWD_ROWS_BIG when the step would
        // otherwise hold more than FWD_BIG_LAUNCH workgroups (then each
        // workgroup's chunk solve serves more rows)
        int64_t nwg = 0;
        for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
          int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
          if (k * SB >= w) continue;
          const int64_t nb = std::min<int64_t>(SB, w - k * SB), lo = k * SB + nb;
          nwg += (nb > NB ? 2 : 1) * std::max<int64_t>(1, (m - lo + FWD_ROWS - 1) / FWD_ROWS);
        }
        const int64_t rows = nwg > FWD_BIG_LAUNCH ? FWD_ROWS_BIG : FWD_ROWS;
        for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
          int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
          if (k * SB >= w) continue;
          SolveTile t = base_tile(J);
          t.cslot = cslot[q - p.lvl_ptr[h]];
          t.c0 = (int32_t)(k * SB);
          t.nb = (int32_t)std::min<int64_t>(SB, w - k * SB);
          int64_t lo = t.c0 + t.nb;
          int64_t nt = std::max<int64_t>(1, (m - lo + rows - 1) / rows);
          for (int32_t half = 0; half < (t.nb > NB ? 2 : 1); ++half)
            for (int64_t i = 0; i < nt; ++i) {
              t.r0 = (int32_t)std::min<int64_t>(m, lo + rows * i);
              t.r1 = (int32_t)std::min<int64_t>(m, lo + rows * (i + 1));
              t.flags = (i == 0 ? 1 : 0) | (half << 1);
              p.stiles.push_back(t);
              // the later steps of J whose columns its rows meet wait for it
              if (t.cslot >= 0 && t.r0 < t.w) {
                const int64_t s0 = t.r0 / SB, s1 = (std::min(t.r1, t.w) - 1) / SB;
                for (int64_t st = std::max<int64_t>(s0, k + 1); st <= s1; ++st) ++p.sneed[t.cslot + st];
              }
            }
        }
        if (!chain) push_launch(SOLVE_FWD, h, start, -1);
      }
      if (chain) push_launch(SOLVE_FWD, h, lstart, p.nchains++);
    }
    for (int32_t h = p.nlevels - 1; h >= 0; --h) {
      int64_t start = (int64_t)p.stiles.size();
      int64_t steps = 0;
      for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
        int64_t J = p.lvl_sn[q], w = W(J), m = M(J);
        steps = std::max<int64_t>(steps, (w + SB - 1) / SB);
        for (int64_t c0 = 0; c0 < w && m > w; c0 += NB)
          for (int64_t r = w; r < m; r += BELOW_ROWS) {
            SolveTile t = base_tile(J);
            t.c0 = (int32_t)c0;
            t.nb = (int32_t)std::min<int64_t>(NB, w - c0);
            t.r0 = (int32_t)r;
            t.r1 = (int32_t)std::min<int64_t>(m, r + BELOW_ROWS);
            p.stiles.push_back(t);
          }
      }
      push_launch(SOLVE_BELOW, h, start, -1);
      const bool chain = steps >= 2;
      std::vector<int32_t> cslot(p.lvl_ptr[h + 1] - p.lvl_ptr[h], -1);
      if (chain)
        for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q)
          cslot[q - p.lvl_ptr[h]] = chain_slots(p.lvl_sn[q]);
      const int64_t lstart = (int64_t)p.stiles.size();
      for (int64_t k = steps - 1; k >= 0; --k) {
        start = (int64_t)p.stiles.size();
        for (int64_t q = p.lvl_ptr[h]; q < p.lvl_ptr[h + 1]; ++q) {
          int64_t J = p.lvl_sn[q], w = W(J);
          if (k * SB >= w) continue;
          SolveTile t = base_tile(J);
          t.cslot = cslot[q - p.lvl_ptr[h]];
          t.c0 = (int32_t)(k * SB);
          t.nb = (int32_t)std::min<int64_t>(SB, w - k * SB);
          const int64_t earlier = k * SB / NB;  // 64-column chunks before the step
          for (int32_t half = 0; half < (t.nb > NB ? 2 : 1); ++half)
            for (int64_t j = 0; j < std::max<int64_t>(earlier, 1); ++j) {
              t.r0 = (int32_t)(j * NB);
              t.r1 = (int32_t)(earlier == 0 ? 0 : j * NB + NB);  // an empty range: only the solve
              t.flags = (j == 0 ? 1 : 0) | (half << 1);
              p.stiles.push_back(t);
              // the earlier step whose columns it pushes into waits for it
              if (t.cslot >= 0 && t.r1 > t.r0) ++p.sneed[t.cslot + t.r0 / SB];
            }
        }
        if (!chain) push_launch(SOLVE_BWD, h, start, -1);
      }
      if (chain) push_launch(SOLVE_BWD, h, lstart, p.nchains++);
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
