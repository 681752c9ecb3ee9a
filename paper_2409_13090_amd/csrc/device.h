// Host-side launch wrappers of the device kernels (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "symbolic.h"

namespace rlb {


constexpr int SOLVE_MAXRHS = 16;

// capacity of each of the three work vectors of the allocation-free solve
// (n * nrhs doubles): 2^21, e.g. n = 262144 with 8 right-hand sides; 48 MiB
// in all per GPU
constexpr int64_t NOALLOC_SOLVE_ELEMS = int64_t(1) << 21;

// device address of the allocation-free solve's work vectors on the current
// device (looked up once per device)
hipError_t noalloc_solve_scratch(double** out);

// the counters of a chained solve launch (tick == nullptr: a plain launch,
// one tile per workgroup in grid order)
struct ChainArgs {
  int* tick;        // ticket counter of the launch
  int* cnt;         // step counters
  const int* need;  // signals each step counter waits for
  int* err;         // set when a wait times out
};
void launch_zero_i32(int* p, int64_t n, hipStream_t st);

// one coefficient per right-hand-side column, passed by value
struct ColCoef {
  double v[SOLVE_MAXRHS];
};

void launch_fill(double* p, int64_t n, double v, hipStream_t st);
void launch_init_status(int* status, int count, int* counters, int ncounters, hipStream_t st);
void launch_scatter_a(const double* vals, const int64_t* amap, int64_t nnz, double* L,
                      hipStream_t st);
void launch_scatter_batch(const double* const* vals, const int64_t* nnz_ptr, int32_t count,
                          int64_t total, const int64_t* amap, double* L, hipStream_t st);
// cdiv of the tiles of one panel launch; pre: apply the previous block's
// trailing update of each column block first; the ucount tiles of utiles (the
// rest of that trailing update, short single-contribution tiles) run as extra
// workgroups of the same launch in the FP64 and FP32 forms (precision 0, 1);
// with precision 2 the caller launches them separately
void launch_panel(const PanelTile* tiles, int64_t count, double* L, int* status, int* counters,
                  int precision, int nbb, bool pre, const double* thr,
                  const unsigned long long* amax, double ufix, unsigned long long* smax,
                  unsigned int* nfixed, const UpdTile* utiles, const UpdSeg* usegs,
                  int64_t ucount, hipStream_t st, float* Ls = nullptr,
                  int64_t wave_min = WAVE_SPLIT_MIN);
// variant: UPD_TILE, UPD_SHORT or UPD_BIG (128x128 tiles; FP64 and FP32 forms)
// Ls: the FP32 copy of the finished factor entries (operands of the FP32 form)
void launch_update(const UpdTile* tiles, const UpdSeg* segs, int64_t count, double* L,
                   int precision, const unsigned long long* smax, int variant, hipStream_t st,
                   int64_t nwave = 0, const float* Ls = nullptr,
                   int64_t wave_min = WAVE_SPLIT_MIN);
void launch_tile_inverse(const DiagTile* tiles, int64_t count, int nbb, double* L,
                         hipStream_t st);
// RL: update-matrix columns added into their ancestors (atomic adds)
void launch_part_reduce(const PartReduce* recs, int64_t count, double* L, hipStream_t st);
void launch_assemble(const AsmCol* cols, int64_t count, const int32_t* rows, double* L,
                     hipStream_t st);
// the off-diagonal inverse blocks of the two-chunk solve steps (after
// launch_tile_inverse)
void launch_pair_inverse(const DiagTile* tiles, int64_t count, double* L, hipStream_t st);
void launch_pivthr(const double* vals, const int64_t* dsrc, int64_t n, double u, double* thr,
                   unsigned long long* amax, hipStream_t st);
void launch_fwd_step(const SolveTile* tiles, int64_t count, const int32_t* gl, const double* L,
                     double* y, double* z, int nrhs, int64_t ldy, hipStream_t st, ChainArgs ca);
void launch_bwd_below(const SolveTile* tiles, int64_t count, const int32_t* gl, const double* L,
                      const double* x, double* z, int nrhs, int64_t ldy, hipStream_t st);
void launch_bwd_step(const SolveTile* tiles, int64_t count, const double* L, double* z, double* x,
                     int nrhs, int64_t ldy, hipStream_t st, ChainArgs ca);
void launch_perm_in(const int64_t* perm, const double* b, int64_t ldb, double* y, int64_t ldy,
                    int64_t n, int nrhs, hipStream_t st);
void launch_perm_out(const int64_t* perm, const double* y, int64_t ldy, double* x, int64_t ldx,
                     int64_t n, int nrhs, hipStream_t st);
void launch_residual(int64_t n, const int64_t* rp, const int32_t* ci, const int64_t* src,
                     const double* vals, const double* x, int64_t ldx, const double* b,
                     int64_t ldb, double* r, int64_t ldr, int nrhs, hipStream_t st);
void launch_absmax(const double* v, int64_t n, int64_t ld, int nrhs, unsigned long long* out,
                   hipStream_t st);
void launch_anorm(int64_t n, const int64_t* rp, const int64_t* src, const double* vals,
                  unsigned long long* out, hipStream_t st);
void launch_axpy(double* x, int64_t ldx, const double* d, int64_t ldd, int64_t n, int nrhs,
                 hipStream_t st);
void launch_dot_cols(const double* x, int64_t ldx, const double* y, int64_t ldy, int64_t n,
                     int nrhs, double* out, hipStream_t st);
void launch_axpby_cols(double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, int nrhs,
                       const ColCoef& a, const ColCoef& b, hipStream_t st);
void launch_zero_u64(unsigned long long* p, int count, hipStream_t st);

}  // namespace rlb
