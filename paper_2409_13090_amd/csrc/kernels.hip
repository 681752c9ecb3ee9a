// CDNA4 (gfx950) kernels of the RLB numeric phase, its solves and the FP64
// refinement residual.
//
// Factor storage: Lnz(J) is m_J x w_J column-major (ld = m_J), one FP64 buffer.
//  * k_fill / k_scatter_a  -- A-load: zero the factor storage, then place A's
//    lower-triangle values (Alg. 5 input: Lnz(J) holds A_{*,J} on entry).
//  * k_potrf / k_trsm      -- cdiv of one <=64-wide column block (Alg. 5 line 4):
//    POTRF of the 64x64 diagonal tile in the registers of one wavefront, then
//    TRSM of the rows below it, one row per lane.
//  * k_update<T>           -- C -= X * Y^T on a 64x64 tile of factor storage:
//    the in-supernode trailing update and the SYRK/GEMM updates written
//    directly into ancestors (Alg. 5 lines 11-16), on MFMA 16x16x4 (FP64, or
//    FP32 operands with FP32 accumulation in the mixed form).
//  * solves, SpMV residual, norms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace rlb {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_init_status(int* status, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) status[i] = 0x7fffffff;
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// A-load of many matrices: entry e of the concatenated entry space belongs to
// the matrix k with nnz_ptr[k] <= e < nnz_ptr[k+1]
__global__ void k_scatter_batch(const double* const* __restrict__ vals,
                                const int64_t* __restrict__ nnz_ptr, int32_t count, int64_t total,
                                const int64_t* __restrict__ amap, double* __restrict__ L) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = count;  // largest k with nnz_ptr[k] <= e
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (nnz_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  L[amap[e]] = vals[lo][e - nnz_ptr[lo]];
}

__global__ void k_scatter_a(const double* __restrict__ vals, const int64_t* __restrict__ amap,
                            int64_t nnz, double* __restrict__ L) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nnz; i += stride) L[amap[i]] = vals[i];
}

// ---------------------------------------------------------------------------
// cdiv of a column block (Alg. 5 line 4) in two launches.
//
// k_potrf (one wavefront per block): blocked Cholesky of the <=64x64 diagonal
// tile T in LDS with 16-column steps. Only the 16x16 base blocks pivot in
// registers (lane = row, row c reaches every lane through readlane); the
// block TRSM and the trailing SYRK of each step are 16x16x16 products on FP64
// MFMA. The kernel also forms inv(L) of the tile -- inverses of the base blocks
// by substitution, then a block forward substitution on MFMA -- and stores its
// strict lower part transposed in the tile's unused strict upper triangle
// (the diagonal of inv(L) is 1/L(i,i)). No floating-point working storage
// beyond factor storage is used.
//
// k_trsm (four wavefronts per 64 rows below the tile): X = A * inv(L)^T as one
// 64x64x64 MFMA product, written over A.

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

constexpr int TP = 65;  // LDS row pitch of a 64x64 tile (doubles)

// D += A * B for 16x16 blocks in LDS. A(i,k) = A[i*ar + k*ac], B(k,j) = B[k*br + j*bc].
__device__ __forceinline__ v4d mma16(const double* A, int ar, int ac, const double* B, int br,
                                     int bc, v4d acc, int lane) {
#pragma unroll
  for (int kq = 0; kq < 4; ++kq) {
    const int k = kq * 4 + (lane >> 4);
    const double a = A[(lane & 15) * ar + k * ac];
    const double b = B[k * br + (lane & 15) * bc];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// element v of lane l of a 16x16 FP64 MFMA result is D(4v + l/16, l%16)
__device__ __forceinline__ void st16(double* D, const v4d& acc, int lane, double scale) {
#pragma unroll
  for (int v = 0; v < 4; ++v) D[(4 * v + (lane >> 4)) * TP + (lane & 15)] = scale * acc[v];
}

__global__ __launch_bounds__(64) void k_potrf(const PanelTile* __restrict__ tiles,
                                              double* __restrict__ L, int* __restrict__ status) {
  const PanelTile t = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  const int nb = t.nb;
  const int ldi = t.ld;
  double* D = L + t.diag;
  __shared__ double T[64 * TP];   // the tile, row-major: T[i*TP + j]
  __shared__ double I[64 * TP];   // inv(L), row-major
  // stage the lower triangle (identity beyond nb); unconditional clamped loads
  {
    const int li = min(lane, nb - 1);
    double v[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) v[j] = D[min(j, nb - 1) * ldi + li];  // all loads in flight
#pragma unroll
    for (int j = 0; j < 64; ++j)
      T[lane * TP + j] = (lane < nb && j < nb && j <= lane) ? v[j] : (j == lane ? 1.0 : 0.0);
  }
  __syncthreads();
  int bad = 0x7fffffff;
  const int nbb = (nb + 15) >> 4;  // base blocks that hold columns of the tile
  for (int b = 0; b < nbb; ++b) {
    const int o = 16 * b;
    // (1) base POTRF of T[o:o+16, o:o+16]: lanes 0..15 hold its rows
    // (lanes 16..63 mirror them). Left-looking, four partial sums per dot
    // product; the column below each pivot is scaled by 1/L(c,c) from one rsq
    // with two Newton steps, while L(c,c) itself is the correctly rounded sqrt.
    const int r = lane & 15;
    double blk[16], rinv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) blk[j] = T[(o + r) * TP + o + j];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
      for (int k = 0; k + 3 < c; k += 4) {
        p0 += blk[k] * lane_bcast(blk[k], c);
        p1 += blk[k + 1] * lane_bcast(blk[k + 1], c);
        p2 += blk[k + 2] * lane_bcast(blk[k + 2], c);
        p3 += blk[k + 3] * lane_bcast(blk[k + 3], c);
      }
#pragma unroll
      for (int k = c & ~3; k < c; ++k) p0 += blk[k] * lane_bcast(blk[k], c);
      const double v = blk[c] - ((p0 + p1) + (p2 + p3));
      double piv = lane_bcast(v, c);
      if (!(piv > 0.0)) {
        if (o + c < nb) bad = min(bad, t.col + o + c + 1);
        piv = 1.0;
      }
      double y = __builtin_amdgcn_rsq(piv);
      y = fma(0.5 * y, fma(-piv * y, y, 1.0), y);
      y = fma(0.5 * y, fma(-piv * y, y, 1.0), y);
      rinv[c] = y;
      blk[c] = (r == c) ? sqrt(piv) : (r > c ? v * y : 0.0);
    }
    // (2) base inverse: lane j < 16 forms column j of inv(L_bb) by substitution
    double yv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double q0 = (i == r) ? 1.0 : 0.0, q1 = 0.0;
#pragma unroll
      for (int k = 0; k + 1 < i; k += 2) {
        q0 -= lane_bcast(blk[k], i) * yv[k];
        q1 -= lane_bcast(blk[k + 1], i) * yv[k + 1];
      }
      if (i & 1) q0 -= lane_bcast(blk[i - 1], i) * yv[i - 1];
      yv[i] = (q0 + q1) * rinv[i];
    }
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < 16; ++j) T[(o + r) * TP + o + j] = blk[j];
#pragma unroll
      for (int i = 0; i < 16; ++i) I[(o + i) * TP + o + r] = yv[i];
    }
    __syncthreads();
    // (3) panel below the base block: L(q, bb) = T(q, bb) * inv(L_bb)^T
    for (int qb = b + 1; qb < nbb; ++qb) {
      v4d acc = {0, 0, 0, 0};
      acc = mma16(&T[(16 * qb) * TP + o], TP, 1, &I[o * TP + o], 1, TP, acc, lane);
      __syncthreads();
      st16(&T[(16 * qb) * TP + o], acc, lane, 1.0);
    }
    __syncthreads();
    // (4) trailing SYRK: T(q, p) -= L(q, bb) * L(p, bb)^T for b < p <= q
    for (int qb = b + 1; qb < nbb; ++qb)
      for (int pb = b + 1; pb <= qb; ++pb) {
        v4d acc = {0, 0, 0, 0};
        acc = mma16(&T[(16 * qb) * TP + o], TP, 1, &T[(16 * pb) * TP + o], 1, TP, acc, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          T[(16 * qb + 4 * v + (lane >> 4)) * TP + 16 * pb + (lane & 15)] -= acc[v];
      }
    __syncthreads();
  }
  // (5) block forward substitution for the off-diagonal blocks of inv(L):
  //     inv(L)(i,j) = -inv(L_ii) * sum_{j<=k<i} L(i,k) * inv(L)(k,j)
  for (int jb = 0; jb + 1 < nbb; ++jb)
    for (int ib = jb + 1; ib < nbb; ++ib) {
      v4d s = {0, 0, 0, 0};
      for (int kb = jb; kb < ib; ++kb)
        s = mma16(&T[(16 * ib) * TP + 16 * kb], TP, 1, &I[(16 * kb) * TP + 16 * jb], TP, 1, s,
                  lane);
      __syncthreads();
      // stage S into the (ib, jb) block of I, then multiply by -inv(L_ii)
      st16(&I[(16 * ib) * TP + 16 * jb], s, lane, 1.0);
      __syncthreads();
      v4d u = {0, 0, 0, 0};
      u = mma16(&I[(16 * ib) * TP + 16 * ib], TP, 1, &I[(16 * ib) * TP + 16 * jb], TP, 1, u, lane);
      __syncthreads();
      st16(&I[(16 * ib) * TP + 16 * jb], u, lane, -1.0);
      __syncthreads();
    }
  if (lane == 0 && bad != 0x7fffffff) atomicMin(status + t.slot, bad);
  // (6) L to the lower triangle, strict lower of inv(L) transposed to the
  //     strict upper triangle (only inside the nb x nb tile)
  {
    double w[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) w[j] = (j <= lane) ? T[lane * TP + j] : I[j * TP + lane];
    if (lane < nb) {
#pragma unroll
      for (int j = 0; j < 64; ++j)
        if (j < nb) D[j * ldi + lane] = w[j];
    }
  }
}

// X = A * inv(L)^T for up to 64 rows below the diagonal tile, in place.
__global__ __launch_bounds__(256) void k_trsm(const PanelTile* __restrict__ tiles,
                                              double* __restrict__ L) {
  const PanelTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = t.nb;
  const int ldi = t.ld;
  const int nr = min(64, t.nrows - t.row0);
  if (nr <= 0) return;
  double* D = L + t.diag;
  __shared__ double sA[64][64];   // sA[k][r] = A(row0 + r, k)
  __shared__ double sV[64][64];   // sV[k][j] = inv(L)(j, k)
  for (int e = tid; e < 64 * 64; e += 256) {
    const int k = e >> 6, r = e & 63;  // consecutive threads: consecutive rows
    const double a = D[min(k, nb - 1) * ldi + t.row0 + min(r, nr - 1)];
    sA[k][r] = (k < nb && r < nr) ? a : 0.0;
  }
  for (int e = tid; e < 64 * 64; e += 256) {
    const int j = e >> 6, k = e & 63;  // inv(L)(j,k) for j > k sits at D[j*ld + k]
    const int jj = min(j, nb - 1), kk = min(k, nb - 1);
    const double u = D[jj * ldi + kk];
    double v = 0.0;
    if (j < nb && k < nb) v = (j > k) ? u : (j == k ? 1.0 / u : 0.0);
    sV[k][j] = v;
  }
  __syncthreads();
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0, 0, 0, 0};
#pragma unroll 4
  for (int kq = 0; kq < 16; ++kq) {
    const int k = kq * 4 + (lane >> 4);
    const double a0 = sV[k][wc + (lane & 15)], a1 = sV[k][wc + 16 + (lane & 15)];
    const double b0 = sA[k][wr + (lane & 15)], b1 = sA[k][wr + 16 + (lane & 15)];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  // D = V * A^T: element v of lane l of block (bj, bi) is X(row wr+16bi+l%16,
  // column wc+16bj+4v+l/16)
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + 4 * v + (lane >> 4);
        if (row < nr && col < nb) D[col * ldi + t.row0 + row] = acc[bj][bi][v];
      }
}

// ---------------------------------------------------------------------------
// C -= X * Y^T on one <=64x64 tile. 256 threads = 4 wavefronts in a 2x2
// arrangement, each owning a 32x32 quarter = 2x2 MFMA 16x16 blocks. K is
// staged through LDS in chunks of 16 (column-major, as in factor storage).
//
// MFMA 16x16x4 operand layout (lane l): A[l%16][l/16] and B[l/16][l%16]. The
// accumulator layout differs by type: for FP64 element v of lane l is
// D[4*v + l/16][l%16]; for FP32 it is D[4*(l/16) + v][l%16]. The kernel computes
// D = Y * X^T, so D's column index is the target row: for fixed v, 16 lanes
// cover 16 consecutive rows of one target column, which keeps the
// read-modify-write of column-major storage coalesced.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int KC = 16;  // K chunk staged per LDS buffer

template <typename T>
__global__ __launch_bounds__(256) void k_update(const UpdTile* __restrict__ tiles,
                                                double* __restrict__ L) {
  typedef typename Mfma<T>::acc_t acc_t;
  const UpdTile t = tiles[blockIdx.x];
  __shared__ T sX[2][KC][64];
  __shared__ T sY[2][KC][64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32;   // rows of this wave's quarter
  const int wc = (wave >> 1) * 32;  // columns of this wave's quarter
  const double* __restrict__ X = L + t.x;
  const double* __restrict__ Y = L + t.y;
  const int64_t lds = t.lds;
  const int K = t.k;
  const int lr = tid & 63;  // row this thread stages
  const int lk = tid >> 6;  // first k this thread stages (then +4, +8, +12)

  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  double xr[4], yr[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + lk + 4 * q;
      xr[q] = (k < K && lr < t.m) ? X[(int64_t)k * lds + lr] : 0.0;
      yr[q] = (k < K && lr < t.n) ? Y[(int64_t)k * lds + lr] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sX[buf][lk + 4 * q][lr] = (T)xr[q];
      sY[buf][lk + 4 * q][lr] = (T)yr[q];
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += KC) {
    const bool more = k0 + KC < K;
    if (more) fetch(k0 + KC);
#pragma unroll
    for (int kq = 0; kq < KC / 4; ++kq) {
      const int kk = kq * 4 + (lane >> 4);
      const T a0 = sY[buf][kk][wc + (lane & 15)];
      const T a1 = sY[buf][kk][wc + 16 + (lane & 15)];
      const T b0 = sX[buf][kk][wr + (lane & 15)];
      const T b1 = sX[buf][kk][wr + 16 + (lane & 15)];
      acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
    }
    if (more) {
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  // epilogue: acc[bj][bi][v] is the update of target row wr+16*bi+(lane&15),
  // target column wc+16*bj+drow(lane,v)
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<T>::drow(lane, v);
        if (row < t.m && col < t.n && (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          const double u = (double)acc[bj][bi][v];
          if (atomic)
            atomicAdd(p, -u);
          else
            *p -= u;
        }
      }
}

template __global__ void k_update<double>(const UpdTile*, double*);
template __global__ void k_update<float>(const UpdTile*, double*);

// ---------------------------------------------------------------------------
// supernodal solves, one workgroup per supernode of a level.
// y is n x nrhs column-major (ld = ldy) in the factored order.

static_assert(sizeof(SnMeta) == 24, "SnMeta layout");

constexpr int SB = 64;  // columns per in-LDS triangular chunk of the solves
constexpr int MAXRHS = SOLVE_MAXRHS;

// Stage the nb x nb diagonal chunk of L at (c0, c0) into Ld (identity beyond nb).
__device__ __forceinline__ void stage_chunk(double (*Ld)[SB + 1], const double* Lj, int64_t ld,
                                            int c0, int nb, int tid) {
  for (int e = tid; e < SB * SB; e += 256) {
    const int col = e / SB, row = e % SB;
    double v = (row == col) ? 1.0 : 0.0;
    if (row < nb && col < nb && row >= col) v = Lj[(int64_t)(c0 + col) * ld + c0 + row];
    Ld[row][col] = v;
  }
}

// Forward solve L y = b for the supernodes of one level, one workgroup each.
// Per 64-column chunk: triangle in LDS (one wavefront per right-hand side,
// lane = row, pivots broadcast with readlane), then a coalesced GEMV for every
// row below the chunk (own rows plainly, ancestor rows with atomics).
__global__ __launch_bounds__(256) void k_fwd(const int32_t* __restrict__ sns,
                                             const SnMeta* __restrict__ meta,
                                             const int32_t* __restrict__ gl,
                                             const double* __restrict__ L,
                                             double* __restrict__ y, int nrhs, int64_t ldy) {
  const SnMeta s = meta[sns[blockIdx.x]];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Lj = L + s.off;
  const int64_t ld = s.m;
  const int32_t* g = gl + s.gl;
  __shared__ double Ld[SB][SB + 1];
  __shared__ double xs[MAXRHS][SB];
  for (int c0 = 0; c0 < s.w; c0 += SB) {
    const int nb = min(SB, s.w - c0);
    stage_chunk(Ld, Lj, ld, c0, nb, tid);
    for (int e = tid; e < SB * nrhs; e += 256) {
      const int c = e % SB, r = e / SB;
      xs[r][c] = c < nb ? y[(int64_t)r * ldy + s.f + c0 + c] : 0.0;
    }
    __syncthreads();
    for (int r = wave; r < nrhs; r += 4) {
      double yj = xs[r][lane];
      for (int c = 0; c < nb; ++c) {
        const double xc = lane_bcast(yj, c) / Ld[c][c];
        if (lane == c) yj = xc;
        if (lane > c) yj -= Ld[lane][c] * xc;
      }
      xs[r][lane] = yj;
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int c = e % nb, r = e / nb;
      y[(int64_t)r * ldy + s.f + c0 + c] = xs[r][c];
    }
    const int q0 = c0 + nb;
    for (int q = q0 + tid; q < s.m + 255; q += 256) {
      // one row per thread; all 64 column loads in flight (coalesced across
      // threads), clamped to valid slots
      const int qq = min(q, s.m - 1);
      const double* lq = Lj + qq;
      double l[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c) l[c] = lq[(int64_t)(c0 + min(c, nb - 1)) * ld];
      if (q < s.m) {
        const int gq = g[q];
        for (int r = 0; r < nrhs; ++r) {
          double a0 = 0.0, a1 = 0.0;
#pragma unroll
          for (int c = 0; c < SB; c += 2) {
            a0 += l[c] * xs[r][c];         // xs is 0 beyond nb
            a1 += l[c + 1] * xs[r][c + 1];
          }
          const double acc = a0 + a1;
          if (q < s.w)
            y[(int64_t)r * ldy + gq] -= acc;
          else
            atomicAdd(&y[(int64_t)r * ldy + gq], -acc);
        }
      }
    }
    __syncthreads();
  }
}

// Backward solve L^T x = y, levels from the root down, one workgroup per
// supernode. Chunks from the last: every column of the chunk first subtracts
// its dot product with the already final x of all rows below the chunk (own
// rows and ancestors alike, both read through glbind), one wavefront per
// column with a wave reduction; then the chunk's triangle is solved in LDS.
__global__ __launch_bounds__(256) void k_bwd(const int32_t* __restrict__ sns,
                                             const SnMeta* __restrict__ meta,
                                             const int32_t* __restrict__ gl,
                                             const double* __restrict__ L,
                                             double* __restrict__ y, int nrhs, int64_t ldy) {
  const SnMeta s = meta[sns[blockIdx.x]];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Lj = L + s.off;
  const int64_t ld = s.m;
  const int32_t* g = gl + s.gl;
  __shared__ double Ld[SB][SB + 1];
  __shared__ double xs[MAXRHS][SB];
  __shared__ double part[4][MAXRHS][SB];
  const int nchunks = (s.w + SB - 1) / SB;
  for (int ch = nchunks - 1; ch >= 0; --ch) {
    const int c0 = ch * SB, nb = min(SB, s.w - c0), q0 = c0 + nb;
    stage_chunk(Ld, Lj, ld, c0, nb, tid);
    // column dot products over the rows below the chunk: lane = column, each
    // wave walks a quarter of the rows (8 rows in flight per iteration); the
    // four partial sums meet in LDS
    {
      const int c = min(lane, nb - 1);
      const double* col = Lj + (int64_t)(c0 + c) * ld;
      const int rows = s.m - q0;
      const int per = (rows + 3) / 4;
      const int qa = q0 + wave * per, qe = min(s.m, qa + per);
      double acc[MAXRHS];
#pragma unroll
      for (int r = 0; r < MAXRHS; ++r) acc[r] = 0.0;
      for (int q = qa; q < qe; q += 8) {
        double l[8];
        int gq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int qq = min(q + u, qe - 1);
          l[u] = (q + u < qe) ? col[qq] : 0.0;
          gq[u] = g[qq];
        }
#pragma unroll
        for (int r = 0; r < MAXRHS; ++r) {
          if (r < nrhs) {
            double yv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) yv[u] = y[(int64_t)r * ldy + gq[u]];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[r] += l[u] * yv[u];
          }
        }
      }
      for (int r = 0; r < nrhs; ++r) part[wave][r][lane] = acc[r];
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int c = e % nb, r = e / nb;
      const double d = (part[0][r][c] + part[1][r][c]) + (part[2][r][c] + part[3][r][c]);
      xs[r][c] = y[(int64_t)r * ldy + s.f + c0 + c] - d;
    }
    __syncthreads();
    for (int r = wave; r < nrhs; r += 4) {
      double yj = lane < nb ? xs[r][lane] : 0.0;
      for (int c = nb - 1; c >= 0; --c) {
        const double xc = lane_bcast(yj, c) / Ld[c][c];
        if (lane == c) yj = xc;
        if (lane < c) yj -= Ld[c][lane] * xc;
      }
      if (lane < nb) xs[r][lane] = yj;
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int c = e % nb, r = e / nb;
      y[(int64_t)r * ldy + s.f + c0 + c] = xs[r][c];
    }
    __syncthreads();
  }
}

// y[k] = b[perm[k]] (gather into the factored order) and back
__global__ void k_perm_in(const int64_t* __restrict__ perm, const double* __restrict__ b,
                          int64_t ldb, double* __restrict__ y, int64_t ldy, int64_t n, int nrhs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i % n, r = i / n;
  y[r * ldy + k] = b[r * ldb + perm[k]];
}

__global__ void k_perm_out(const int64_t* __restrict__ perm, const double* __restrict__ y,
                           int64_t ldy, double* __restrict__ x, int64_t ldx, int64_t n, int nrhs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i % n, r = i / n;
  x[r * ldx + perm[k]] = y[r * ldy + k];
}

// r = b - A x in the original order (full symmetric CSR, values gathered
// from the caller's lower-triangle array)
__global__ void k_residual(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const int64_t* __restrict__ src, const double* __restrict__ vals,
                           const double* __restrict__ x, int64_t ldx, const double* __restrict__ b,
                           int64_t ldb, double* __restrict__ r, int64_t ldr, int nrhs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t row = i % n, k = i / n;
  double acc = 0.0;
  for (int64_t e = rp[row]; e < rp[row + 1]; ++e) acc += vals[src[e]] * x[k * ldx + ci[e]];
  r[k * ldr + row] = b[k * ldb + row] - acc;
}

// out[k] = max(out[k], max_i |v[i + k*ld]|) via the ordering of non-negative
// doubles as unsigned integers
__global__ void k_absmax(const double* __restrict__ v, int64_t n, int64_t ld, int nrhs,
                         unsigned long long* __restrict__ out) {
  const int k = blockIdx.y;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(v[k * ld + i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out + k, (unsigned long long)__double_as_longlong(m));
}

// infinity norm of A: max over rows of sum |a_ij|
__global__ void k_anorm(int64_t n, const int64_t* __restrict__ rp, const int64_t* __restrict__ src,
                        const double* __restrict__ vals, unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s += fabs(vals[src[e]]);
    m = fmax(m, s);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_axpy(double* __restrict__ x, int64_t ldx, const double* __restrict__ d,
                       int64_t ldd, int64_t n, int nrhs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t row = i % n, k = i / n;
  x[k * ldx + row] += d[k * ldd + row];
}

// ---------------------------------------------------------------------------
// launch wrappers

static inline unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, n, v);
}
void launch_init_status(int* status, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_init_status, dim3(grid_for(count, 256)), dim3(256), 0, st, status, count);
}
void launch_zero_u64(unsigned long long* p, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(count, 256)), dim3(256), 0, st, p, count);
}
void launch_scatter_a(const double* vals, const int64_t* amap, int64_t nnz, double* L,
                      hipStream_t st) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_scatter_a, dim3(grid_for(nnz, 256, 16384)), dim3(256), 0, st, vals, amap,
                     nnz, L);
}
void launch_scatter_batch(const double* const* vals, const int64_t* nnz_ptr, int32_t count,
                          int64_t total, const int64_t* amap, double* L, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_scatter_batch, dim3(grid_for(total, 256, INT32_MAX)), dim3(256), 0, st,
                     vals, nnz_ptr, count, total, amap, L);
}
void launch_potrf(const PanelTile* tiles, int64_t count, double* L, int* status, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_potrf, dim3((unsigned)count), dim3(64), 0, st, tiles, L, status);
}
void launch_trsm(const PanelTile* tiles, int64_t count, double* L, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_trsm, dim3((unsigned)count), dim3(256), 0, st, tiles, L);
}
void launch_update(const UpdTile* tiles, int64_t count, double* L, int precision,
                   hipStream_t st) {
  if (count <= 0) return;
  if (precision == 1)
    hipLaunchKernelGGL(k_update<float>, dim3((unsigned)count), dim3(256), 0, st, tiles, L);
  else
    hipLaunchKernelGGL(k_update<double>, dim3((unsigned)count), dim3(256), 0, st, tiles, L);
}
void launch_fwd(const int32_t* sns, int64_t count, const SnMeta* meta, const int32_t* gl,
                const double* L, double* y, int nrhs, int64_t ldy, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fwd, dim3((unsigned)count), dim3(256), 0, st, sns, meta, gl, L, y, nrhs,
                     ldy);
}
void launch_bwd(const int32_t* sns, int64_t count, const SnMeta* meta, const int32_t* gl,
                const double* L, double* y, int nrhs, int64_t ldy, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_bwd, dim3((unsigned)count), dim3(256), 0, st, sns, meta, gl, L, y, nrhs,
                     ldy);
}
void launch_perm_in(const int64_t* perm, const double* b, int64_t ldb, double* y, int64_t ldy,
                    int64_t n, int nrhs, hipStream_t st) {
  int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_perm_in, dim3(grid_for(tot, 256, INT32_MAX)), dim3(256), 0, st, perm, b,
                     ldb, y, ldy, n, nrhs);
}
void launch_perm_out(const int64_t* perm, const double* y, int64_t ldy, double* x, int64_t ldx,
                     int64_t n, int nrhs, hipStream_t st) {
  int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_perm_out, dim3(grid_for(tot, 256, INT32_MAX)), dim3(256), 0, st, perm, y,
                     ldy, x, ldx, n, nrhs);
}
void launch_residual(int64_t n, const int64_t* rp, const int32_t* ci, const int64_t* src,
                     const double* vals, const double* x, int64_t ldx, const double* b,
                     int64_t ldb, double* r, int64_t ldr, int nrhs, hipStream_t st) {
  int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_residual, dim3(grid_for(tot, 256, INT32_MAX)), dim3(256), 0, st, n, rp,
                     ci, src, vals, x, ldx, b, ldb, r, ldr, nrhs);
}
void launch_absmax(const double* v, int64_t n, int64_t ld, int nrhs, unsigned long long* out,
                   hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(n, 256, 1024), nrhs), dim3(256), 0, st, v, n, ld,
                     nrhs, out);
}
void launch_anorm(int64_t n, const int64_t* rp, const int64_t* src, const double* vals,
                  unsigned long long* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_anorm, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, n, rp, src, vals,
                     out);
}
void launch_axpy(double* x, int64_t ldx, const double* d, int64_t ldd, int64_t n, int nrhs,
                 hipStream_t st) {
  int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(tot, 256, INT32_MAX)), dim3(256), 0, st, x, ldx, d,
                     ldd, n, nrhs);
}

}  // namespace rlb
