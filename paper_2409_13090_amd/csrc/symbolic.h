// Host symbolic analysis and numeric plan for right-looking blocked (RLB)
// supernodal Cholesky. Internal header of the rlb library (not installed).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace rlb {

struct AnalyzeOptions {
  int ordering = 1;  // 0 natural, 1 grid nested dissection, 2 user permutation
  const int64_t* user_perm = nullptr;
  int64_t grid[4] = {0, 0, 0, 1};
  double merge_cap = 0.125;
  int reorder = 1;
  int maximal_blocks = 1;
  int precision = 0;
  int panel_spread = 512;  // row tiles a panel launch spreads over workgroups
  int deterministic = 1;   // 1: no floating-point atomics in the factorization (every
                           // target tile has one owner); 0: heavy tiles split, parts
                           // added atomically
  int outer_block = 256;   // columns of the outer block of wide supernodes (a multiple
                           // of 64; 64 = every panel updates all trailing columns)
  int big_tile_min = 0;    // the long updates of a step take 128x128 target tiles when
                           // there are at least this many (<= 0: never)
  int method = 0;          // 0: RLB (Algorithm 5); 1: RL (Algorithm 4), the updates of a
                           // supernode into its ancestors through an update matrix
  double hybrid_step_us = 30.0;  // hybrid method: least modelled saving of a step (us)
  int tall_tile_min = 0;   // the long updates of a step take 128x64 target tiles (FP64)
                           // when there are at least this many (<= 0: never)
  int tile_order = 0;      // 0: heaviest tiles first; 1: 8x8 blocks of neighbouring
                           // tiles, a contiguous eighth of the order per XCD
  int split_chunks = 0;    // deterministic form: target tiles cut into parts that write
                           // into workspace blocks, summed in a fixed order by a reduce
                           // launch (0: never -- every update written straight into its
                           // target, as Algorithm 5; < 0: the tiles far heavier than their
                           // launch's balanced share; > 0: every tile of more K chunks than
                           // this, in parts of this many)
};

// One 64x64 (or smaller) target tile of factor storage and the list of its
// contributions C -= X * Y^T in one update launch. A target tile of a launch
// is normally owned by one workgroup, which sums all contributions (from the
// trailing update of the tile's own supernode, or from the SYRK/GEMM updates
// of every supernode of the launch that touches the tile) and writes the tile
// once; a tile with more work than one workgroup should take is cut into
// several entries that add their parts atomically. Offsets are element
// offsets into the factor buffer.
struct UpdTile {
  int64_t c;     // target tile origin
  int32_t ldc;   // leading dimension of the target panel
  int32_t m, n;  // tile rows, tile columns
  int32_t flags; // bit0: tile on the diagonal of its supernode (write only row >= col);
                 // bit1: one of several workgroups of a split tile (adds atomically)
  int32_t seg0;  // first contribution
  int32_t nseg;  // number of contributions
};
static_assert(sizeof(UpdTile) == 32, "UpdTile layout");

// One source supernode's contribution to a target tile: tile rows [ra, rb)
// and columns [ca, cb) receive X * Y^T, where X row r is source row
// x + (r - ra) and Y row c is source row y + (c - ca), over k source columns.
struct UpdSeg {
  int64_t x;     // source offset of the X row that meets tile row ra, column 0
  int64_t y;     // source offset of the Y row that meets tile column ca, column 0
  int32_t lds;   // leading dimension of the source panel
  int32_t k;     // inner dimension (source columns)
  int32_t ra, rb, ca, cb;
  int32_t src;   // source supernode
  int32_t sslot; // scale slot of the source panel (16-bit update forms)
};
static_assert(sizeof(UpdSeg) == 48, "UpdSeg layout");

// Work item of the cdiv of a <=64-wide column block (see k_panel).
struct PanelTile {
  int64_t diag;       // offset of the diagonal tile's top-left element
  int32_t ld;         // leading dimension of the panel
  int32_t nb;         // columns in the block (1..64)
  int32_t nrows;      // rows from the diagonal tile down to the panel bottom
  int32_t row0;       // first row handled here, relative to the diagonal tile
  int32_t col;        // factored-order index of the block's first column
  int32_t slot;       // status slot (matrix index in a batch)
  int32_t grp;        // counter of the group of tiles sharing this diagonal tile
  int32_t gcnt;       // number of tiles in the group
  int32_t s_step;     // scale slot of this column block (16-bit update forms)
  int32_t s_anc;      // scale slot of the supernode's rows below its diagonal block
  int32_t rw;         // first row, relative to the diagonal tile, below the diagonal block
  int32_t nrt;        // 64-row tiles handled, from row0 on
};
static_assert(sizeof(PanelTile) == 56, "PanelTile layout");

// A diagonal tile of the factor (see k_tile_inverse).
struct DiagTile {
  int64_t diag;  // offset of its top-left element
  int32_t ld;
  int32_t nb;
};
static_assert(sizeof(DiagTile) == 16, "DiagTile layout");

// Work item of the supernodal solves, one workgroup each (see k_fwd_step,
// k_bwd_below, k_bwd_step). Columns and rows are relative to the supernode.
struct SolveTile {
  int64_t off;   // Lnz(J) offset in factor storage
  int32_t ld;    // m_J
  int32_t f;     // first column of J (factored order)
  int32_t w;     // w_J
  int32_t gl;    // offset of glbind(J)
  int32_t c0;    // first column of the chunk solved here
  int32_t nb;    // chunk width (<= 64)
  int32_t r0;    // forward / below: first row handled; backward step: first column
  int32_t r1;    //   of the earlier chunk updated here (end of the range)
  int32_t flags; // bit0: writes the chunk's solution
  int32_t cslot; // in a chained launch: the first step counter of the supernode, else -1
};
static_assert(sizeof(SolveTile) == 48, "SolveTile layout");

constexpr int32_t SOLVE_FWD = 0;    // forward step: chunk solve + rows below
constexpr int32_t SOLVE_BELOW = 1;  // backward: columns against the ancestor rows
constexpr int32_t SOLVE_BWD = 2;    // backward step: chunk solve + earlier chunks

// chain >= 0: every step of the level in one launch whose workgroups take
// their tiles in order by ticket (ticket counter `chain`); a tile with
// cslot >= 0 first waits until the step counter cslot + (its step) has
// received sneed[...] signals, one from each earlier tile of the launch that
// writes into the columns of that step, and signals the counters of the
// steps it writes into itself
struct SolveLaunch {
  int32_t kind;
  int32_t level;
  int64_t start;
  int64_t count;
  int32_t chain;
  int32_t pad;
};

// launch kinds, in execution order inside one (level, step)
constexpr int32_t LAUNCH_PANEL = 0;
constexpr int32_t LAUNCH_UPDATE = 1;
constexpr int32_t LAUNCH_ASSEMBLE = 2;  // RL: update matrices scatter-added into ancestors
constexpr int32_t LAUNCH_REDUCE = 3;    // the parts of split target tiles summed into them

// A target tile of an update launch cut into nparts parts along its
// contribution list (load balance in the deterministic form): part p wrote
// -(its sum) into the 64x64 block at pbase + 4096 p of the workspace (column
// major, ld 64); the reduce adds the parts, in part order, into the tile
// (rows < m, columns < n; on the diagonal only row >= col).
struct PartReduce {
  int64_t c;      // target tile origin
  int64_t pbase;  // first part's block
  int32_t ldc, m, n, flags;  // flags bit0: diagonal tile
  int32_t nparts;
  int32_t pad;
};
static_assert(sizeof(PartReduce) == 40, "PartReduce layout");

// RL (Algorithm 4): one column of an update matrix U_J, assembled into column
// `dst` of an ancestor's factor storage: entry i of the column (the U_J
// entry src + i) is added at dst + rows[rp + i].
struct AsmCol {
  int64_t src;  // U_J(j, j): the column's first entry on or below the diagonal
  int64_t dst;  // the target column's first entry in Lnz(P)
  int32_t rp;   // offset of the column's target row positions in the row list
  int32_t len;  // entries (rows j .. r_J - 1 of U_J)
};
static_assert(sizeof(AsmCol) == 24, "AsmCol layout");

// Narrow update tiles (at most NARROW_COLS columns) run one per wavefront
// (k_update_w, FP64) when a launch holds at least WAVE_SPLIT_MIN of them;
// fewer do not repay a launch of their own. Panel launches of at least
// WAVE_SPLIT_MIN column blocks of at most 16 columns likewise run one group
// member per wavefront (k_panel_w).
constexpr int32_t NARROW_COLS = 16;
constexpr int64_t WAVE_SPLIT_MIN = 1024;

// update launch variants: 64x64 target tiles (k_update), 64x64 tiles that all
// hold one contribution with k <= 64 and one owner (k_update_short), 128x128
// target tiles (k_update_big)
constexpr int32_t UPD_TILE = 0;
constexpr int32_t UPD_SHORT = 1;
constexpr int32_t UPD_BIG = 2;
constexpr int32_t UPD_TILE_WIN = 4;  // UPD_TILE with K chunks shaped to the contributions'
                                     // rectangles (tiles of many small contributions)
constexpr int32_t UPD_TALL = 6;  // 128x64 target tiles (the long updates), FP64; the
                                 // launch's alt list holds the same work in 64x64 tiles
constexpr int32_t UPD_TILE_PACK = 5;  // UPD_TILE with the contributions of a tile end to end
                                      // along K (tiles of many contributions of small k)
constexpr int32_t UPD_TILE_XCD = 3;  // UPD_TILE, workgroup b takes the tile at position
                                     // (b % 8) * (count / 8) + min(b % 8, count % 8) + b / 8

struct Launch {
  int32_t kind;   // LAUNCH_*
  int32_t level;
  int32_t step;   // column block index inside the level
  int32_t variant; // update: UPD_*; panel: 16-column blocks of its widest tile (1, 2 or 4)
  int64_t start;  // first tile
  int64_t count;  // number of tiles
  int32_t pre;    // panel: its tiles first apply the previous block's trailing update
  int32_t nwave;  // update: its last nwave tiles are narrow (<= 16 columns), run one per
                  // wavefront in the FP64 form
  int64_t ustart; // panel: update tiles of the previous step run in the same launch
  int64_t ucount; //   (single-contribution tiles, k <= 64); the ncount tiles after
  int64_t ncount; //   them are the ones pre applies (kept for the unfused form)
  int64_t alt_start = 0;  // UPD_BIG: the same work cut into 64x64 tiles, for the
  int64_t alt_count = 0;  //   forms whose update kernels take only those (16-bit)
};

struct Plan {
  // factor storage: Lnz(J) is m_J x w_J column-major at off[J], ld = m_J
  std::vector<int64_t> off;
  int64_t l_elems = 0;
  // RL: the update matrices of the supernodes whose cdiv ends in one step,
  // r_J x r_J column-major each, reused from step to step; they follow the
  // factor storage in the workspace (ws_elems = l_elems + u_elems)
  int64_t u_elems = 0;
  // the parts of split target tiles (64x64 blocks, reused from launch to
  // launch) follow the update matrices: ws_elems = l_elems + u_elems + part_elems
  int64_t part_elems = 0;
  std::vector<PartReduce> reduces;
  int64_t ws_elems = 0;
  std::vector<AsmCol> asmcols;
  std::vector<int32_t> asm_rows;
  std::vector<int64_t> amap;  // input CSC entry -> position in factor storage
  std::vector<PanelTile> panels;
  std::vector<UpdTile> updates;
  std::vector<UpdSeg> segs;
  int32_t n_scale_slots = 0;     // per column block of every supernode, plus one per supernode
  std::vector<int64_t> diag_src; // input entry of the diagonal of every factored column
  std::vector<DiagTile> dtiles;       // every 64-column step's diagonal tile, by width class
  int64_t dt_ptr[4] = {0, 0, 0, 0};   // classes of 1, 2 and 4 16-column blocks
  std::vector<DiagTile> ptiles;       // diagonal blocks of the two-chunk solve steps (nb > 64)
  std::vector<SolveTile> stiles;      // solve work items, launch by launch
  std::vector<SolveLaunch> slaunches; // forward levels upwards, then backward downwards
  std::vector<int32_t> sneed;         // signals each step counter of a chained launch waits for
  int32_t nchains = 0;                // chained launches (ticket counters)
  std::vector<Launch> launches;
  int32_t nlevels = 0;
  std::vector<int32_t> level;       // height of every supernode
  std::vector<int64_t> lvl_ptr;     // supernodes grouped by level
  std::vector<int32_t> lvl_sn;
  // full symmetric A in the factored order, CSR, values gathered from the input
  std::vector<int64_t> a_rowptr;
  std::vector<int32_t> a_col;
  std::vector<int64_t> a_src;
  int64_t n_merged_tiles = 0;  // target tiles that sum contributions of several supernodes
  int64_t n_split_tiles = 0;   // workgroups of target tiles split for load balance
  int32_t max_groups = 0;  // largest number of tile groups in one panel launch
  double flops_tiles = 0;  // flops the update tiles execute (the 16x16 MFMA blocks they touch)
  double flops_upd_alg = 0;  // algorithmic flops of the update tiles (entries written x 2k)
  double flops_panel = 0;    // flops of the POTRF + TRSM column blocks
  double flops_upd_launch = 0;  // flops_upd_alg of the tiles run by update launches of their own
};

struct Symbolic {
  int64_t n = 0;
  int64_t nnz_a = 0;
  AnalyzeOptions opt;
  std::vector<int64_t> colptr, rowidx;  // copy of the input pattern
  std::vector<int64_t> perm;       // final: perm[new] = old
  std::vector<int64_t> perm_nd;    // after the fill-reducing ordering
  std::vector<int64_t> perm_post;  // after the postorder
  std::vector<int64_t> etree_post; // column etree under perm_post
  std::vector<int64_t> etree;      // column etree under perm
  std::vector<int64_t> fund_ptr;   // fundamental supernodes (perm_post numbering)
  std::vector<int64_t> sn_ptr;     // merged supernodes
  std::vector<int64_t> sn_parent;
  std::vector<int64_t> gl_ptr;     // glbind(J), final numbering
  std::vector<int32_t> gl;
  std::vector<int64_t> rel_ptr;    // relind(J, p(J)) for every row below the diagonal block
  std::vector<int32_t> rel;
  std::vector<int64_t> blk_ptr;    // block sizes, top to bottom
  std::vector<int32_t> blk;
  std::vector<int64_t> rbp_ptr;    // per J: its (J, P) pairs
  std::vector<int32_t> rbp_anc;    // ancestor P of each pair
  std::vector<int64_t> rbv_ptr;    // per pair: relindB(J, P) values
  std::vector<int32_t> rbv;
  std::vector<int64_t> colcount;   // exact column counts, final numbering
  int64_t merge_added = 0, merge_base = 0;
  int64_t nnz_exact = 0, nnz_stored = 0;
  double flops_exact = 0, flops_padded = 0;
  int64_t n_blocks = 0, n_pairs = 0, n_calls = 0;  // blocks, (J,P) pairs, SYRK+GEMM calls
  Plan plan;
};

// Returns 0 or a negative rlb status; fills `err` with a message on failure.
int analyze(int64_t n, const int64_t* colptr, const int64_t* rowidx,
            const AnalyzeOptions& opt, Symbolic& out, std::string& err);

int build_plan(Symbolic& s, std::string& err);
// Kernel variant (UPD_TILE, UPD_TILE_WIN or UPD_TILE_PACK) of an update launch
// over the given tiles, from the chunk rounds each way of staging K takes.
int32_t tile_variant(const UpdTile* tiles, int64_t count, const UpdSeg* segs);

}  // namespace rlb
