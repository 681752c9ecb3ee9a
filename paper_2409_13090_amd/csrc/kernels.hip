// CDNA4 (gfx950) kernels of the RLB numeric phase, its solves and the FP64
// refinement residual.
//
// Factor storage: Lnz(J) is m_J x w_J column-major (ld = m_J), one FP64 buffer.
//  * k_fill / k_scatter_a  -- A-load: zero the factor storage, then place A's
//    lower-triangle values (Alg. 5 input: Lnz(J) holds A_{*,J} on entry).
//  * k_panel               -- cdiv of one <=64-wide column block (Alg. 5 line 4):
//    the 64x64 diagonal tile is factored (POTRF) in registers of one
//    wavefront, then every lane solves one row below it (TRSM).
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
// cdiv of a column block: POTRF of the diagonal tile + TRSM of up to 64 rows.
// One wavefront per tile. Both steps are left-looking (Crout order): lane i
// keeps row i in registers and forms column c as a dot product with row c of
// the factor, which every lane reads from LDS as a broadcast.

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(64) void k_panel(const PanelTile* __restrict__ tiles,
                                              double* __restrict__ L, int* __restrict__ status) {
  const PanelTile t = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  __shared__ double sr[64][65];  // sr[i][k] = L(i, k) of the factored diagonal tile
  const int nb = t.nb;
  const int64_t ld = t.ld;
  double* D = L + t.diag;
  if (t.mode != 2) {
    int bad = 0x7fffffff;
    double row[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) {
      double v = (j == lane) ? 1.0 : 0.0;  // identity beyond nb
      if (lane < nb && j < nb && j <= lane) v = D[(int64_t)j * ld + lane];
      row[j] = v;
    }
#pragma unroll
    for (int c = 0; c < 64; ++c) {
      double v = row[c];
#pragma unroll
      for (int k = 0; k < c; ++k) v -= row[k] * sr[c][k];
      double piv = lane_bcast(v, c);
      if (!(piv > 0.0)) {
        if (c < nb) bad = min(bad, t.col + c + 1);
        piv = 1.0;
      }
      const double d = sqrt(piv);
      row[c] = (lane == c) ? d : (lane > c ? v / d : 0.0);
      sr[lane][c] = row[c];
      __syncthreads();
    }
    if (lane == 0 && bad != 0x7fffffff) atomicMin(status + t.slot, bad);
    if (lane < nb) {
#pragma unroll
      for (int j = 0; j < 64; ++j)
        if (j < nb && j <= lane) D[(int64_t)j * ld + lane] = row[j];
    }
    if (t.mode == 1) return;
  } else {
    // the diagonal tile was factored by this block's mode-1 item in an
    // earlier launch: stage it (identity beyond nb)
    for (int j = 0; j < 64; ++j) {
      double v = (j == lane) ? 1.0 : 0.0;
      if (lane < nb && j < nb && j <= lane) v = D[(int64_t)j * ld + lane];
      sr[lane][j] = v;
    }
    __syncthreads();
  }
  // TRSM: x * L^T = a for row r, x_c = (a_c - sum_{k<c} x_k L(c,k)) / L(c,c).
  // Loads are unconditional (clamped indices, 32-bit offsets from a uniform
  // base) and every column ends with an LDS store into the unused pad column:
  // both keep the register footprint at one 64-double row.
  if (t.row0 >= t.nrows) return;
  const bool live = t.row0 + lane < t.nrows;
  const int rr = live ? t.row0 + lane : t.row0;
  const int ldi = (int)ld;
  double x[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    const double v = D[min(c, nb - 1) * ldi + rr];
    x[c] = c < nb ? v : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    double v = x[c];
#pragma unroll
    for (int k = 0; k < c; ++k) v -= x[k] * sr[c][k];
    x[c] = v / sr[c][c];
    sr[lane][64] = x[c];
  }
  if (live) {
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < nb) D[j * ldi + rr] = x[j];
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

__global__ __launch_bounds__(256) void k_fwd(const int32_t* __restrict__ sns,
                                             const SnMeta* __restrict__ meta,
                                             const int32_t* __restrict__ gl,
                                             const double* __restrict__ L,
                                             double* __restrict__ y, int nrhs, int64_t ldy) {
  const SnMeta s = meta[sns[blockIdx.x]];
  const int tid = threadIdx.x;
  const double* Lj = L + s.off;
  const int64_t ld = s.m;
  const int32_t* g = gl + s.gl;
  __shared__ double xs[MAXRHS][SB];
  for (int c0 = 0; c0 < s.w; c0 += SB) {
    const int nb = min(SB, s.w - c0);
    // load the chunk of y into LDS
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int c = e % nb, r = e / nb;
      xs[r][c] = y[(int64_t)r * ldy + s.f + c0 + c];
    }
    __syncthreads();
    // in-chunk lower solve: one thread per right-hand side
    if (tid < nrhs) {
      for (int c = 0; c < nb; ++c) {
        const double x = xs[tid][c] / Lj[(int64_t)(c0 + c) * ld + c0 + c];
        xs[tid][c] = x;
        for (int q = c + 1; q < nb; ++q) xs[tid][q] -= Lj[(int64_t)(c0 + c) * ld + c0 + q] * x;
      }
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int c = e % nb, r = e / nb;
      y[(int64_t)r * ldy + s.f + c0 + c] = xs[r][c];
    }
    // rows below the chunk: own rows of the diagonal block, then ancestors
    const int below = s.m - c0 - nb;
    for (int e = tid; e < below * nrhs; e += 256) {
      const int q = c0 + nb + e % below, r = e / below;
      double acc = 0.0;
      for (int c = 0; c < nb; ++c) acc += Lj[(int64_t)(c0 + c) * ld + q] * xs[r][c];
      if (q < s.w)
        y[(int64_t)r * ldy + s.f + q] -= acc;
      else
        atomicAdd(&y[(int64_t)r * ldy + g[q]], -acc);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_bwd(const int32_t* __restrict__ sns,
                                             const SnMeta* __restrict__ meta,
                                             const int32_t* __restrict__ gl,
                                             const double* __restrict__ L,
                                             double* __restrict__ y, int nrhs, int64_t ldy) {
  const SnMeta s = meta[sns[blockIdx.x]];
  const int tid = threadIdx.x;
  const double* Lj = L + s.off;
  const int64_t ld = s.m;
  const int32_t* g = gl + s.gl;
  __shared__ double xs[MAXRHS][SB];
  // contributions of the rows below the diagonal block (ancestors are final)
  const int below = s.m - s.w;
  for (int e = tid; e < s.w * nrhs; e += 256) {
    const int c = e % s.w, r = e / s.w;
    double acc = 0.0;
    for (int q = 0; q < below; ++q)
      acc += Lj[(int64_t)c * ld + s.w + q] * y[(int64_t)r * ldy + g[s.w + q]];
    y[(int64_t)r * ldy + s.f + c] -= acc;
  }
  __syncthreads();
  const int nchunks = (s.w + SB - 1) / SB;
  for (int ch = nchunks - 1; ch >= 0; --ch) {
    const int c0 = ch * SB, nb = min(SB, s.w - c0), c1 = c0 + nb;
    // contributions of the already solved columns [c1, w) of the diagonal block
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int c = e % nb, r = e / nb;
      double acc = 0.0;
      for (int q = c1; q < s.w; ++q)
        acc += Lj[(int64_t)(c0 + c) * ld + q] * y[(int64_t)r * ldy + s.f + q];
      xs[r][c] = y[(int64_t)r * ldy + s.f + c0 + c] - acc;
    }
    __syncthreads();
    if (tid < nrhs) {
      for (int c = nb - 1; c >= 0; --c) {
        double v = xs[tid][c];
        for (int q = c + 1; q < nb; ++q) v -= Lj[(int64_t)(c0 + c) * ld + c0 + q] * xs[tid][q];
        xs[tid][c] = v / Lj[(int64_t)(c0 + c) * ld + c0 + c];
      }
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
void launch_panel(const PanelTile* tiles, int64_t count, double* L, int* status, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_panel, dim3((unsigned)count), dim3(64), 0, st, tiles, L, status);
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
