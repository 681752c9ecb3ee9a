// CDNA4 (gfx950) kernels of the RLB numeric phase, its solves and the FP64
// refinement residual.
//
// Factor storage: Lnz(J) is m_J x w_J column-major (ld = m_J), one FP64 buffer.
//  * k_fill / k_scatter_a  -- A-load: zero the factor storage, then place A's
//    lower-triangle values (Alg. 5 input: Lnz(J) holds A_{*,J} on entry).
//  * k_panel               -- cdiv of one <=64-wide column block (Alg. 5):
//    POTRF of the diagonal tile in LDS fused with the TRSM of the rows below.
//  * k_update<T>           -- C -= sum of X * Y^T on a 64x64 tile of factor
//    storage: the in-supernode trailing update and the SYRK/GEMM updates
//    written directly into ancestors (Alg. 5), on MFMA 16x16x4
//    (FP64, or FP32 operands with FP32 accumulation in the mixed form).
//  * k_update_w / k_panel_w / k_tile_inverse_w -- the same work for narrow
//    items (at most 16 columns), one wavefront each, four per workgroup, for
//    launches that hold many of them (the batched form).
//  * k_tile_inverse / k_pair_inverse -- inverses of the diagonal tiles and of
//    the two-chunk solve steps' diagonal blocks, for the solves.
//  * k_fwd_step / k_bwd_below / k_bwd_step -- supernodal solves in steps of
//    two 64-column chunks, the diagonal block as a product with its inverse.
//  * SpMV residual, norms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "device.h"

namespace rlb {

// Work vectors of the allocation-free solve (rlb_solve_noalloc): three n x
// nrhs column-major blocks (right-hand side in the factored order, forward
// solution, backward solution) of at most NOALLOC_SOLVE_ELEMS doubles each.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, never the device memory:
// only the address hipGetSymbolAddress returns for the current device is
// passed to kernels.
static __device__ __align__(256) double scratch[3 * NOALLOC_SOLVE_ELEMS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_solve_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_init_status(int* status, int count, int* counters, int ncounters) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) status[i] = 0x7fffffff;
  if (i < ncounters) counters[i] = 0;
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// A-load of many matrices: entry e of the concatenated entry space belongs to
// the matrix k with nnz_ptr[k] <= e < nnz_ptr[k+1]
// every matrix's input entries into its factor storage: matrix k holds
// entries nnz_ptr[k] .. nnz_ptr[k+1]-1 of the concatenated list; the matrix
// of a workgroup's first entry is found once (every matrix has at least 256
// entries in practice, and a thread walks on past the ones it crosses)
__global__ __launch_bounds__(256) void k_scatter_batch(const double* const* __restrict__ vals,
                                                       const int64_t* __restrict__ nnz_ptr,
                                                       int32_t count, int64_t total,
                                                       const int64_t* __restrict__ amap,
                                                       double* __restrict__ L) {
  __shared__ int s_lo;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x;
  if (threadIdx.x == 0) {
    int lo = 0, hi = count;  // largest k with nnz_ptr[k] <= e0
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nnz_ptr[mid] <= e0) lo = mid; else hi = mid;
    }
    s_lo = lo;
  }
  __syncthreads();
  const int64_t e = e0 + threadIdx.x;
  if (e >= total) return;
  int lo = s_lo;
  while (lo + 1 < count && nnz_ptr[lo + 1] <= e) ++lo;
  L[amap[e]] = vals[lo][e - nnz_ptr[lo]];
}

__global__ void k_scatter_a(const double* __restrict__ vals, const int64_t* __restrict__ amap,
                            int64_t nnz, double* __restrict__ L) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nnz; i += stride) L[amap[i]] = vals[i];
}

// ---------------------------------------------------------------------------
// cdiv of one <=64-column block (Alg. 5): POTRF of the diagonal tile
// fused with the TRSM of every row below it, in one launch.
//
// A group is the set of workgroups that share one diagonal tile: one per 64
// rows below it (or a single one when there are none), or one per few
// consecutive 64-row tiles in launches that hold many. Every member stages
// the unfactored tile into LDS, factors it there redundantly and overwrites
// its own row tiles A with X = A * L^-T. After staging, each member
// increments the group's counter; the member that brings it to the group
// size is the last reader of the unfactored tile, and only it writes the
// factored tile back. It also resets the counter for the next launch.
//
// Factorization of the tile T (identity beyond nb) in 16-column rounds. In
// round r, wavefront 0 factors the 64 x 16 column block r in registers
// (lane = row, right-looking: the pivot and the next column's multiplier
// reach every lane through readlane, the other multipliers through
// same-address LDS reads of the finished column) while wavefronts 1-2 apply
// block r-1's updates to the column blocks right of r+1 and wavefront 3
// inverts the 16 x 16 diagonal block r-1; then all wavefronts update column
// block r+1 with block r on MFMA. The pivot reciprocal is an rsq with two
// Newton steps; the stored diagonal is the correctly rounded square root.
// The row tiles are solved by block forward substitution with the 16 x 16
// inverses, on MFMA. The inverse of the whole tile, which the solves use, is
// formed after the factorization by k_tile_inverse.

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}


__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A * B for 16x16 blocks in LDS, A(i,k) = A[i*ar + k*ac], B(k,j) = B[k*br + j*bc];
// two accumulation chains over the halves of k
__device__ __forceinline__ v4d mma16(const double* A, int ar, int ac, const double* B, int br,
                                     int bc, int lane) {
  v4d c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
#pragma unroll
  for (int kq = 0; kq < 4; kq += 2) {
    const int k0 = kq * 4 + (lane >> 4), k1 = k0 + 4;
    c0 = mfma64(A[(lane & 15) * ar + k0 * ac], B[k0 * br + (lane & 15) * bc], c0);
    c1 = mfma64(A[(lane & 15) * ar + k1 * ac], B[k1 * br + (lane & 15) * bc], c1);
  }
  return c0 + c1;
}

// A * S with A a 16x16 block in LDS and S a 16x16 MFMA result in registers:
// element kq of lane l of an FP64 result is S(4kq + l/16, l%16), which is
// exactly lane l's B operand of k-step kq
__device__ __forceinline__ v4d mma16r(const double* A, int ar, int ac, const v4d& S, int lane) {
  v4d c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
#pragma unroll
  for (int kq = 0; kq < 4; kq += 2) {
    const int k0 = kq * 4 + (lane >> 4), k1 = k0 + 4;
    c0 = mfma64(A[(lane & 15) * ar + k0 * ac], S[kq], c0);
    c1 = mfma64(A[(lane & 15) * ar + k1 * ac], S[kq + 1], c1);
  }
  return c0 + c1;
}

// element v of lane l of a 16x16 FP64 MFMA result is D(4v + l/16, l%16); row pitch tp
__device__ __forceinline__ void st16(double* D, int tp, const v4d& acc, int lane, double scale) {
#pragma unroll
  for (int v = 0; v < 4; ++v) D[(4 * v + (lane >> 4)) * tp + (lane & 15)] = scale * acc[v];
}

// T(q, p) -= L(q, b) * L(p, b)^T for 16x16 blocks of a tile with row pitch tp
__device__ __forceinline__ void syrk16(double* T, int tp, int q, int p, int b, int lane) {
  const v4d acc = mma16(&T[16 * q * tp + 16 * b], tp, 1, &T[16 * p * tp + 16 * b], 1, tp, lane);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    T[(16 * q + 4 * v + (lane >> 4)) * tp + 16 * p + (lane & 15)] -= acc[v];
}

// inverse of the 16x16 lower-triangular block at (o, o) of T (row pitch tp)
// into the 16x16 block Io (row pitch ip); lane r (< 16) forms column r by
// forward substitution, reading row i of L with same-address LDS loads
// NC < 16 (blocks whose rows from NC on are those of the identity): those
// rows of the inverse are the identity's and are not computed
template <int NC = 16>
__device__ __forceinline__ void inv16(const double* T, int tp, int o, double* Io, int ip,
                                      int lane) {
  const int r = lane & 15;
  const double rr = 1.0 / T[(o + r) * tp + o + r];
  const double* Lo = T + o * tp + o;
  double yv[16];
#pragma unroll
  for (int i = NC; i < 16; ++i) yv[i] = (i == r) ? 1.0 : 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    double q0 = (i == r) ? 1.0 : 0.0, q1 = 0.0;
#pragma unroll
    for (int k = 0; k + 1 < i; k += 2) {
      q0 = fma(-Lo[i * tp + k], yv[k], q0);
      q1 = fma(-Lo[i * tp + k + 1], yv[k + 1], q1);
    }
    if (i & 1) q0 = fma(-Lo[i * tp + i - 1], yv[i - 1], q0);
    yv[i] = (q0 + q1) * lane_bcast(rr, i);
  }
  if (lane < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) Io[i * ip + r] = yv[i];
  }
}

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

// a contribution record read by every lane alike (from LDS), made scalar so
// that the loop control and the addresses built from it stay uniform
__device__ __forceinline__ int32_t uni32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ UpdSeg uniform_seg(const UpdSeg& g) {
  UpdSeg u;
  u.x = uni64(g.x);
  u.y = uni64(g.y);
  u.lds = uni32(g.lds);
  u.k = uni32(g.k);
  u.ra = uni32(g.ra);
  u.rb = uni32(g.rb);
  u.ca = uni32(g.ca);
  u.cb = uni32(g.cb);
  u.src = uni32(g.src);
  u.sslot = uni32(g.sslot);
  return u;
}

// One FP64 element per lane from a buffer of `bytes` bytes at p (a uniform
// address): lanes whose byte offset lies outside it read zero (the buffer
// unit's range check), so ragged rows and columns need no masking.
constexpr int BUF_CONFIG = 0x00020000;  // raw buffer, 32-bit data format
__device__ __forceinline__ double load_range(const double* p, int bytes, uint32_t off) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, bytes, BUF_CONFIG);
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

constexpr int KC = 16;  // K chunk staged per LDS buffer

// Which of this thread's 16 accumulator elements of a 64x64 target tile lie in
// the rectangle of at least one of the tile's contributions: bit
// bj*8 + bi*4 + v for element (bj, bi, v) of a wavefront quarter at rows wr,
// columns wc (Lay gives the accumulator layout). Every other element receives
// no update, so it is neither read nor written: at the lower levels the
// rectangles of a target tile cover a quarter to a half of it. Tiles with more
// than COVER_SEGS contributions are taken as fully covered.
constexpr int COVER_SEGS = 32;
template <typename Lay>
__device__ __forceinline__ unsigned cover_bits(const UpdTile& t, const UpdSeg* __restrict__ segs,
                                               int wr, int wc, int lane) {
  if (t.nseg > COVER_SEGS) return 0xffffu;
  int row[2], col[2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) row[bi] = wr + 16 * bi + (lane & 15);
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) col[bj][v] = wc + 16 * bj + Lay::drow(lane, v);
  unsigned m = 0;
  for (int e = 0; e < t.nseg; ++e) {
    const UpdSeg& g = segs[t.seg0 + e];
    const int ra = uni32(g.ra), rb = uni32(g.rb), ca = uni32(g.ca), cb = uni32(g.cb);
    unsigned cbits = 0;  // bits bj*8 + v: column inside [ca, cb)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cbits |= (col[bj][v] >= ca && col[bj][v] < cb) ? 1u << (bj * 8 + v) : 0u;
    if (row[0] >= ra && row[0] < rb) m |= cbits;
    if (row[1] >= ra && row[1] < rb) m |= cbits << 4;
  }
  return m;
}


// One target tile of a launch whose tiles all hold a single contribution
// with k <= 64 and a single owner (the trailing updates of a step): every
// load of K is issued up front, so the tile waits for memory once. sX and sY
// are LDS stages of 2 x KC x 64 elements each.
template <typename T>
__device__ __forceinline__ void upd_short_tile(const UpdTile& t, const UpdSeg& g,
                                               double* __restrict__ L, const T* __restrict__ S,
                                               T (*sX)[KC][64], T (*sY)[KC][64]) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int lr = tid & 63, lk = tid >> 6;
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool assign = t.flags & 4;  // write -(sum) without reading the target
  const bool xin = lr >= g.ra && lr < g.rb, yin = lr >= g.ca && lr < g.cb;
  T xr[16], yr[16];
  if constexpr (sizeof(T) == 8) {
    // range-checked buffer loads: rows outside the rectangle and k past the
    // contribution's read zero
    const UpdSeg u = uniform_seg(g);
    const int kw = uni32(lk);
    const uint32_t xoff = (uint32_t)(lr - u.ra) << 3, yoff = (uint32_t)(lr - u.ca) << 3;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int kk = kw + 4 * q;
      const bool kin = kk < u.k;
      const int64_t ko = (int64_t)kk * u.lds;
      xr[q] = load_range(S + u.x + ko, kin ? (u.rb - u.ra) << 3 : 0, xoff);
      yr[q] = load_range(S + u.y + ko, kin ? (u.cb - u.ca) << 3 : 0, yoff);
    }
  } else {
    const int64_t xo = g.x + min(max(lr - g.ra, 0), g.rb - g.ra - 1);
    const int64_t yo = g.y + min(max(lr - g.ca, 0), g.cb - g.ca - 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t kk = min(lk + 4 * q, g.k - 1);
      xr[q] = S[xo + kk * g.lds];
      yr[q] = S[yo + kk * g.lds];
    }
  }
  double cv[2][2][4];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
        const int col = min(wc + 16 * bj + Mfma<T>::drow(lane, v), t.n - 1);
        cv[bj][bi][v] = assign ? 0.0 : C[(int64_t)col * ldc + row];
      }
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  const int nch = (g.k + KC - 1) / KC;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c < nch) {
      const int buf = c & 1;
#pragma unroll
      for (int u = 0; u < KC / 4; ++u) {
        const int q = 4 * c + u;
        if constexpr (sizeof(T) == 8) {
          sX[buf][lk + 4 * u][lr] = xr[q];
          sY[buf][lk + 4 * u][lr] = yr[q];
        } else {
          const bool kin = lk + 4 * q < g.k;
          sX[buf][lk + 4 * u][lr] = (kin && xin) ? xr[q] : T(0);
          sY[buf][lk + 4 * u][lr] = (kin && yin) ? yr[q] : T(0);
        }
      }
      __syncthreads();
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
    }
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<T>::drow(lane, v);
        if (row < t.m && col < t.n && (!diag || row >= col))
          C[(int64_t)col * ldc + row] = cv[bj][bi][v] - (double)acc[bj][bi][v];
      }
}

// right-looking factorization of the tr x 16 column block at column o of T
// (row pitch tp), one wavefront, lane = row (lanes >= tr idle); Lc (16 x 64)
// receives the scaled columns for the broadcasts. FIX (reduced-precision
// update forms): a pivot at or below thr (this lane's column threshold, u
// times the column's diagonal entry of A) is replaced by rep and counted in
// *nfix. Otherwise a non-positive pivot is not patched on the way (its NaN or
// Inf only reaches later columns of this supernode and its ancestors, whose
// column indices are larger); afterwards each pivot lane checks its own raw
// pivot and the smallest failing column (1-based, factored order) is
// returned, or INT_MAX.
template <bool FIX, int NC = 16>
__device__ __forceinline__ int panel16(double* T, int tp, int tr, double* Lc, int o, int nb,
                                       int col0, int lane, double thr, double rep, int* nfix) {
  const int lr = min(lane, tr - 1);
  double v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = T[lr * tp + o + j];
  double dg = 1.0;  // the pivot of this lane's row, for its diagonal entry
  double dn = lane_bcast(v[0], o);  // the next pivot, before any patching
  // Column c's update of the columns j >= c + 2 needs the multipliers of rows
  // o + j (through LDS); it is applied one pivot later, its LDS reads issued
  // before that pivot's square root, so the LDS round trip overlaps the
  // pivot chain. Every entry still takes the updates in pivot order, with the
  // same operands.
  double lp = 0.0;  // the previous column's multiplier of this lane's row
  double r[16];     // the previous column's multipliers of rows o + j
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    // NC < 16 (callers with nb <= o + NC): columns from nb on are the
    // identity with zeros below, they change nothing and are not visited
    if (c >= 1) {
#pragma unroll
      for (int j = c + 1; j < 16; ++j) r[j] = Lc[(c - 1) * 64 + o + j];
    }
    double d = dn;
    if (FIX) {
      if (d <= lane_bcast(thr, o + c) && o + c < nb) {
        d = rep;
        ++*nfix;
      }
    }
    dg = (lane == o + c) ? d : dg;
    double y = __builtin_amdgcn_rsq(d);
    y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
    const double l = v[c] * y;
    v[c] = l;
    if (c >= 1 && c < 15) v[c + 1] = fma(-lp, r[c + 1], v[c + 1]);
    if (c < 15) {
      // the pivot row's own entries give the next pivot without waiting for
      // the broadcast of its multiplier
      dn = lane_bcast(fma(-l, l, v[c + 1]), o + c + 1);
    }
    if (c >= 1) {
#pragma unroll
      for (int j = c + 2; j < 16; ++j) v[j] = fma(-lp, r[j], v[j]);
    }
    if (c < 15) {
      Lc[c * 64 + lane] = l;
      v[c + 1] = fma(-l, lane_bcast(l, o + c + 1), v[c + 1]);
    }
    lp = l;
  }
  // the last column's update of the columns past it (NC < 16)
#pragma unroll
  for (int j = NC + 1; j < 16; ++j) v[j] = fma(-lp, Lc[(NC - 1) * 64 + o + j], v[j]);
  const double sq = sqrt(dg);
  // rows from the diagonal block down; the rows above it lie in the tile's
  // unused upper part, which may hold other data (the 16x16 inverses)
  if (lane < tr && lane >= o) {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      T[lane * tp + o + j] = lane > o + j ? v[j] : (lane == o + j ? sq : 0.0);
  }
  const unsigned long long fails =
      __ballot(lane >= o && lane < o + 16 && lane < nb && !(dg > 0.0));
  return fails ? col0 + __ffsll((long long)fails) : 0x7fffffff;
}

constexpr int AP = 65;  // LDS pitch of the staged row tile: sA[k * AP + r] = A(r, k)

constexpr int IP = 17;  // LDS row pitch of the 16x16 inverse blocks

constexpr int YP = 66;  // LDS row pitch of the previous block's rows Y and X (row-major)

// The previous block's update of the tile and the row tile, K = 64: an FP64
// MFMA 16x16x4 sums over k in any order as long as both operands use the same
// one, so step kq takes k = 16 g + kq in lane group g = l/16; a lane's
// operands of a product are then consecutive doubles of one row of Y (or X),
// read as 16-byte LDS loads. The loads of the next two steps are issued
// before the products of the current two (a wave cannot issue past an MFMA
// that waits for the matrix pipe), and sched_barrier keeps that order.
__device__ __forceinline__ v4d pre_mma64(const double* Ra, const double* Rb, int lane) {
  const int kl = lane >> 4, il = lane & 15;
  const double* pa = Ra + il * YP + 16 * kl;
  const double* pb = Rb + il * YP + 16 * kl;
  double2 a = *reinterpret_cast<const double2*>(pa), b = *reinterpret_cast<const double2*>(pb);
  v4d c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
#pragma unroll
  for (int kq = 0; kq < 16; kq += 2) {
    double2 na = a, nb = b;
    if (kq + 2 < 16) {
      na = *reinterpret_cast<const double2*>(pa + kq + 2);
      nb = *reinterpret_cast<const double2*>(pb + kq + 2);
    }
    __builtin_amdgcn_sched_barrier(0);
    c0 = mfma64(a.x, b.x, c0);
    c1 = mfma64(a.y, b.y, c1);
    __builtin_amdgcn_sched_barrier(0);
    a = na;
    b = nb;
  }
  return c0 + c1;
}

// T(q, p) -= Y_q Y_p^T (sY row-major, pitch YP)
__device__ __forceinline__ void pre_syrk16(double* T, int tp, const double* sY, int q, int p,
                                           int lane) {
  const v4d acc = pre_mma64(sY + 16 * q * YP, sY + 16 * p * YP, lane);
  const int kl = lane >> 4, il = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) T[(16 * q + 4 * v + kl) * tp + 16 * p + il] -= acc[v];
}

// row blocks a0, a0+1 and column blocks b0, b0+1 (b0 only without TWO) of
// the k-major row tile sA (pitch AP) minus X_a Y_b^T (sX, sY row-major, pitch
// YP): each product is formed as Y_b X_a^T, whose MFMA result layout is sA's
// k-major layout; every operand loaded serves two of the products
template <bool TWO>
__device__ __forceinline__ void pre_gemm2x2(double* sA, const double* sX, const double* sY,
                                            int a0, int b0, int lane) {
  const int kl = lane >> 4, il = lane & 15;
  const double* y0 = sY + (16 * b0 + il) * YP + 16 * kl;
  const double* y1 = y0 + 16 * YP;
  const double* x0 = sX + (16 * a0 + il) * YP + 16 * kl;
  const double* x1 = x0 + 16 * YP;
  v4d c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;  // c[b][a]
  double2 ya = *reinterpret_cast<const double2*>(y0);
  double2 yb = TWO ? *reinterpret_cast<const double2*>(y1) : ya;
  double2 xa = *reinterpret_cast<const double2*>(x0);
  double2 xb = *reinterpret_cast<const double2*>(x1);
#pragma unroll
  for (int kq = 0; kq < 16; kq += 2) {
    double2 nya = ya, nyb = yb, nxa = xa, nxb = xb;
    if (kq + 2 < 16) {
      nya = *reinterpret_cast<const double2*>(y0 + kq + 2);
      if (TWO) nyb = *reinterpret_cast<const double2*>(y1 + kq + 2);
      nxa = *reinterpret_cast<const double2*>(x0 + kq + 2);
      nxb = *reinterpret_cast<const double2*>(x1 + kq + 2);
    }
    __builtin_amdgcn_sched_barrier(0);
    c00 = mfma64(ya.x, xa.x, c00);
    c01 = mfma64(ya.x, xb.x, c01);
    if (TWO) {
      c10 = mfma64(yb.x, xa.x, c10);
      c11 = mfma64(yb.x, xb.x, c11);
    }
    c00 = mfma64(ya.y, xa.y, c00);
    c01 = mfma64(ya.y, xb.y, c01);
    if (TWO) {
      c10 = mfma64(yb.y, xa.y, c10);
      c11 = mfma64(yb.y, xb.y, c11);
    }
    __builtin_amdgcn_sched_barrier(0);
    ya = nya;
    yb = nyb;
    xa = nxa;
    xb = nxb;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double* r0 = sA + (16 * b0 + 4 * v + kl) * AP + 16 * a0 + il;
    r0[0] -= c00[v];
    r0[16] -= c01[v];
    if (TWO) {
      double* r1 = r0 + 16 * AP;
      r1[0] -= c10[v];
      r1[16] -= c11[v];
    }
  }
}

template <int MODE>
struct PanelUpd {
  typedef double type;  // FP64 form
};
template <>
struct PanelUpd<1> {
  typedef float type;  // FP32 update operands
};

// resident workgroups per compute unit the register budget is sized for
constexpr int panel_occupancy(int nbb, bool pre) {
  return pre ? (nbb == 1 ? 2 : 1) : (nbb == 1 ? 3 : 2);
}

// MODE 0: FP64 form. MODE 1: reduced-precision updates (pivot patching).
// MODE 2: 16-bit updates (pivot patching, and the largest |entry| of the row
// tiles, overall and in the rows below the diagonal block, into the scale
// slots of the column block and of the supernode).
// NBB: 16-column blocks of the widest tile of the launch (1, 2 or 4); the
// tile and its LDS images are 16*NBB wide.
// PRE: the column block's own share of the trailing update of the previous
// (64-column) block of its supernode is applied here, before the
// factorization, in FP64 on MFMA: T -= Y Y^T on the diagonal tile and
// A -= X Y^T on each row tile, Y and X being the previous block's entries in
// the rows of the diagonal tile and of the row tile (they sit 64 columns to
// the left). Column block 0 of T is updated by all waves before the first
// pivot round, the other column blocks and the row tile by waves 1-3 while
// wave 0 factors.
// Workgroups blockIdx.x >= npanel (MODE 0 and 1, NBB 4) each run one tile of utiles:
// the rest of that previous block's trailing update (single-contribution
// tiles, k <= 64) in the update precision of the form; those tiles lie right
// of this column block, so the two kinds of work touch disjoint entries.
template <int MODE, int NBB, bool PRE>
__global__ __launch_bounds__(256, panel_occupancy(NBB, PRE)) void k_panel(
    const PanelTile* __restrict__ tiles, double* __restrict__ L, int* __restrict__ status,
    int* __restrict__ counters, const double* __restrict__ thr,
    const unsigned long long* __restrict__ amax, double ufix, unsigned long long* __restrict__ smax,
    unsigned int* __restrict__ nfixed, const UpdTile* __restrict__ utiles,
    const UpdSeg* __restrict__ usegs, int npanel, float* __restrict__ Ls) {
  constexpr int TR = 16 * NBB;  // tile rows and columns
  constexpr int TPn = TR + 1;   // LDS row pitch of the tile images
  // LDS carve (doubles): the tile T (row-major), the inverses of its 16x16
  // diagonal blocks, the row tile (k-major), the finished columns of the
  // current 16-column block, and for PRE the previous block's rows Y and X
  // with four column blocks the 16x16 inverses live in T's unused upper
  // blocks (0,1), (0,2), (0,3) and (1,3) (pitch TPn), else in a region of
  // their own (pitch IP)
  constexpr bool IUP = NBB == 4;
  constexpr int O_I = TR * TPn;
  constexpr int O_A = O_I + (IUP ? 0 : NBB * 16 * IP);
  constexpr int O_LC = O_A + TR * AP;
  constexpr int O_Y = O_LC + 16 * 64;
  constexpr int O_X = O_Y + (PRE ? TR * YP : 0);
  constexpr int N_PANEL = O_X + (PRE ? 64 * YP : 0);
  constexpr bool UROLE = MODE != 2 && NBB == 4;  // launches that carry update tiles
  constexpr int N_UPD = UROLE ? 4 * KC * 64 * (int)sizeof(typename PanelUpd<MODE>::type) / 8 : 0;
  constexpr int N_LDS = N_PANEL > N_UPD ? N_PANEL : N_UPD;
  __shared__ double smem[N_LDS];
  __shared__ int s_last;
  __shared__ unsigned long long s_max[2];
  if (UROLE && (int)blockIdx.x >= npanel) {
    typedef typename PanelUpd<MODE>::type UT;
    UT* su = reinterpret_cast<UT*>(smem);
    const UpdTile ut = utiles[blockIdx.x - npanel];
    // operands: the FP64 factor, or its FP32 copy in the FP32-update form
    const UT* S;
    if constexpr (MODE == 1)
      S = Ls;
    else
      S = L;
    upd_short_tile<UT>(ut, usegs[ut.seg0], L, S, reinterpret_cast<UT(*)[KC][64]>(su),
                       reinterpret_cast<UT(*)[KC][64]>(su + 2 * KC * 64));
    return;
  }
  double* const T = smem;
  double* const Ib = smem + O_I;
  constexpr int IPB = IUP ? TPn : IP;  // row pitch of the inverse blocks
  auto inv_blk = [&](int b) -> double* {
    if (IUP) return T + (b == 3 ? 16 * TPn + 48 : 16 * (b + 1));
    return Ib + b * 16 * IP;
  };
  double* const sA = smem + O_A;
  double* const Lc = smem + O_LC;
  double* const sY = smem + O_Y;
  double* const sX = smem + O_X;
  const PanelTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = t.nb, ldi = t.ld;
  const int nr = min(64, t.nrows - t.row0);  // rows of the first row tile (may be <= 0)
  double* D = L + t.diag;
  // stage: thread (row, cg) loads columns cg, cg+4, ..., all loads in flight;
  // addresses are clamped so every load is in bounds. With PRE the row tile
  // and its X rows are staged later, during the first pivot round.
  const int arow0 = min(t.row0 + max(0, min(lane, nr - 1)), t.nrows - 1);
  {
    const int row = lane, cg = wave;
    const int dr = min(row, nb - 1);
    double dv[4 * NBB], av[PRE ? 1 : 4 * NBB];
    double yv[PRE ? 16 : 1];
#pragma unroll
    for (int i = 0; i < 4 * NBB; ++i) {
      const int j = min(cg + 4 * i, nb - 1);
      dv[i] = D[(int64_t)j * ldi + dr];
      if (!PRE) av[i] = D[(int64_t)j * ldi + arow0];
    }
    if (PRE) {
#pragma unroll
      for (int i = 0; i < 16; ++i) yv[i] = D[(int64_t)(cg + 4 * i - 64) * ldi + dr];
    }
#pragma unroll
    for (int i = 0; i < 4 * NBB; ++i) {
      const int j = cg + 4 * i;
      if (row < TR)
        T[row * TPn + j] = (row < nb && j < nb && j <= row) ? dv[i] : (j == row ? 1.0 : 0.0);
      if (!PRE) sA[j * AP + row] = (row < nr && j < nb) ? av[i] : 0.0;
    }
    if (PRE && row < TR) {
#pragma unroll
      for (int i = 0; i < 16; ++i) sY[row * YP + cg + 4 * i] = row < nb ? yv[i] : 0.0;
    }
  }
  __syncthreads();
  const int nbb = (nb + 15) >> 4;
  int bad = 0x7fffffff;
  int nfix = 0;
  double cthr = 0.0, crep = 0.0;
  if (MODE >= 1) {
    cthr = thr[t.col + min(lane, nb - 1)];
    double am;
    __builtin_memcpy(&am, amax, sizeof(double));
    crep = ufix * am;
    if (tid < 2) s_max[tid] = 0ull;
  }
  if (PRE) {
    // the previous block's update of column block 0 of the tile (one 16x16
    // block per wave) while the first row tile and its X rows arrive
    const int row = lane, cg = wave;
    double av[4 * NBB], xv[16];
    if (t.nrt > 0) {
#pragma unroll
      for (int i = 0; i < 4 * NBB; ++i) av[i] = D[(int64_t)min(cg + 4 * i, nb - 1) * ldi + arow0];
#pragma unroll
      for (int i = 0; i < 16; ++i) xv[i] = D[(int64_t)(cg + 4 * i - 64) * ldi + arow0];
    }
    if (wave < nbb) pre_syrk16(T, TPn, sY, wave, 0, lane);
    if (t.nrt > 0) {
#pragma unroll
      for (int i = 0; i < 4 * NBB; ++i) {
        const int j = cg + 4 * i;
        sA[j * AP + row] = (row < nr && j < nb) ? av[i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) sX[row * YP + cg + 4 * i] = row < nr ? xv[i] : 0.0;
    }
    __syncthreads();
  }
  // row-tile work of the previous block's update: 2x2 groups of 16x16 blocks,
  // g = (row blocks 2(g&1).., column blocks 2(g>>1)..) for the later row
  // tiles (a 16-column tile image holds one column block); for the first row
  // tile halves of them, h = (row blocks 2(h&1).., column block h>>1), dealt
  // to waves 1-3 in the pivot rounds from the second on (slot 3(r-1) + w - 1
  // takes half h) so that no round's work outlasts its pivot chain, the rest
  // after the rounds
  const int ngrp = (PRE && t.nrt > 0) ? 2 * ((nbb + 1) >> 1) : 0;
  auto grp = [&](int g) { pre_gemm2x2<(NBB > 1)>(sA, sX, sY, 2 * (g & 1), 2 * (g >> 1), lane); };
  const int nhalf = (PRE && t.nrt > 0) ? 2 * nbb : 0;
  auto half = [&](int h) { pre_gemm2x2<false>(sA, sX, sY, 2 * (h & 1), h >> 1, lane); };
  for (int r = 0; r < nbb; ++r) {
    if (wave == 0) {
      bad = min(bad, panel16<(MODE >= 1)>(T, TPn, TR, Lc, 16 * r, nb, t.col, lane, cthr, crep,
                                          &nfix));
    } else {
      if (r >= 1) {
        if (wave == 3) {
          inv16(T, TPn, 16 * (r - 1), inv_blk(r - 1), IPB, lane);
        } else {
          // block r-1's updates of column blocks p >= r+1
          int idx = 0;
          for (int p = r + 1; p < nbb; ++p)
            for (int q = p; q < nbb; ++q, ++idx)
              if ((idx & 1) == wave - 1) syrk16(T, TPn, q, p, r - 1, lane);
        }
      }
      if (r == 0) {
        // group counter, on a wave that does not carry the pivot chain
        int old = 0;
        if (tid == 192) old = atomicAdd(&counters[t.grp], 1);
        if (PRE) {
          // the previous block's update of column blocks 1.. of the tile
          int idx = 0;
          for (int p = 1; p < nbb; ++p)
            for (int q = p; q < nbb; ++q, ++idx)
              if (idx % 3 == wave - 1) pre_syrk16(T, TPn, sY, q, p, lane);
        }
        if (tid == 192) {
          const int last = (old == t.gcnt - 1);
          if (last) atomicExch(&counters[t.grp], 0);
          s_last = last;
        }
      } else if (PRE) {
        const int h = 3 * (r - 1) + wave - 1;
        if (h < nhalf) half(h);
      }
    }
    __syncthreads();
    // column block r+1 from block r
    if (r + 1 < nbb && r + 1 + wave < nbb) syrk16(T, TPn, r + 1 + wave, r + 1, r, lane);
    __syncthreads();
  }
  if (PRE && 3 * (nbb - 1) < nhalf) {
    // halves the rounds had no room for
    if (wave >= 1)
      for (int h = 3 * (nbb - 1) + wave - 1; h < nhalf; h += 3) half(h);
    __syncthreads();
  }
  // the last base inverse (wave 3) alongside the first column blocks of the
  // row tiles' solves
  if (wave == 3) inv16(T, TPn, 16 * (nbb - 1), inv_blk(nbb - 1), IPB, lane);
  // the last reader writes the factored tile (lower triangle)
  if (s_last) {
    if (wave == 0 && lane == 0 && bad != 0x7fffffff) atomicMin(status + t.slot, bad);
    if (MODE >= 1 && wave == 0 && lane == 0 && nfix) atomicAdd(nfixed + t.slot, (unsigned)nfix);
    const int i = lane;
#pragma unroll
    for (int q = 0; q < 4 * NBB; ++q) {
      const int j = wave + 4 * q;
      if (i < nb && j < nb && i >= j) D[(int64_t)j * ldi + i] = T[i * TPn + j];
    }
  }
  // X = A * L^-T for each of this member's row tiles (the first was staged
  // with the diagonal tile), by block forward substitution over the column
  // blocks: X_b = (A_b - sum_{c<b} X_c L_bc^T) inv(L_bb)^T. Wave w owns rows
  // 16w..16w+15 of the tile and keeps its X_c^T blocks in MFMA result layout
  // (element v of lane l is X(16w + l%16, 16c + 4v + l/16)), which is also
  // the B-operand layout of the next products, so X never goes through LDS.
  const int rb = wave;
  double mx_step = 0.0, mx_anc = 0.0;
  for (int rt = 0; rt < t.nrt; ++rt) {
    const int row0 = t.row0 + 64 * rt;
    const int nrt_rows = min(64, t.nrows - row0);
    if (rt > 0) {
      __syncthreads();  // the previous tile's reads of sA are done
      const int row = lane, cg = wave;
      const int arow = row0 + min(row, nrt_rows - 1);
      double av[4 * NBB], xv[PRE ? 16 : 1];
#pragma unroll
      for (int i = 0; i < 4 * NBB; ++i) av[i] = D[(int64_t)min(cg + 4 * i, nb - 1) * ldi + arow];
      if (PRE) {
#pragma unroll
        for (int i = 0; i < 16; ++i) xv[i] = D[(int64_t)(cg + 4 * i - 64) * ldi + arow];
      }
#pragma unroll
      for (int i = 0; i < 4 * NBB; ++i) {
        const int j = cg + 4 * i;
        sA[j * AP + row] = (row < nrt_rows && j < nb) ? av[i] : 0.0;
      }
      if (PRE) {
#pragma unroll
        for (int i = 0; i < 16; ++i) sX[row * YP + cg + 4 * i] = row < nrt_rows ? xv[i] : 0.0;
      }
      __syncthreads();
      if (PRE) {
        for (int g = wave; g < ngrp; g += 4) grp(g);
        __syncthreads();
      }
    }
    v4d X[NBB];
#pragma unroll
    for (int b = 0; b < NBB; ++b) {
      if (b == nbb - 1 && rt == 0) __syncthreads();  // inv(L_bb) of the last block is ready
      X[b] = v4d{0, 0, 0, 0};
      if (b < nbb) {
        v4d r;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          r[v] = sA[(16 * b + 4 * v + (lane >> 4)) * AP + 16 * rb + (lane & 15)];
#pragma unroll
        for (int c = 0; c < b; ++c)
#pragma unroll
          for (int kq = 0; kq < 4; ++kq)
            r = mfma64(-T[(16 * b + (lane & 15)) * TPn + 16 * c + 4 * kq + (lane >> 4)], X[c][kq],
                       r);
        v4d x = {0, 0, 0, 0};
#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
          x = mfma64(inv_blk(b)[(lane & 15) * IPB + 4 * kq + (lane >> 4)], r[kq], x);
        X[b] = x;
        const int rr = 16 * rb + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * b + 4 * v + (lane >> 4);
          const bool ok = c < nb && rr < nrt_rows;
          if (ok) D[(int64_t)c * ldi + row0 + rr] = x[v];
          // the FP32-update form keeps an FP32 copy of every finished entry
          // below the diagonal tiles: the operands of all later updates
          if (MODE == 1 && ok) Ls[t.diag + (int64_t)c * ldi + row0 + rr] = (float)x[v];
          if (MODE == 2) {
            // |x| of a non-negative double orders like its bit pattern
            const double ax = ok ? fabs(x[v]) : 0.0;
            mx_step = fmax(mx_step, ax);
            mx_anc = fmax(mx_anc, row0 + rr >= t.rw ? ax : 0.0);
          }
        }
      }
    }
  }
  if (MODE == 2 && t.nrt > 0) {
    atomicMax(&s_max[0], (unsigned long long)__double_as_longlong(mx_step));
    atomicMax(&s_max[1], (unsigned long long)__double_as_longlong(mx_anc));
    __syncthreads();
    if (tid == 0) {
      atomicMax(smax + t.s_step, s_max[0]);
      if (s_max[1]) atomicMax(smax + t.s_anc, s_max[1]);
    }
  }
}

// LDS written by a wavefront is read back by other lanes of the same
// wavefront: order the accesses without a workgroup barrier
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The inverse of diagonal tiles of at most 16 columns, one wavefront per tile
// and four tiles per workgroup (small supernodes: one wavefront does all of
// the work), stored as k_tile_inverse stores it.
__global__ __launch_bounds__(256) void k_tile_inverse_w(const DiagTile* __restrict__ tiles,
                                                        double* __restrict__ L, int count) {
  constexpr int TP = 17;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double Ts[4][16 * TP];
  __shared__ double Is[4][16 * TP];
  const int ti = (int)blockIdx.x * 4 + wave;
  if (ti >= count) return;  // no workgroup barrier below
  const DiagTile t = tiles[ti];
  double* const T = Ts[wave];
  double* const I = Is[wave];
  const int nb = t.nb, ldi = t.ld;
  double* D = L + t.diag;
  {
    const int row = lane & 15, cg = lane >> 4;
    const int dr = min(row, nb - 1);
    double dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) dv[i] = D[(int64_t)min(cg + 4 * i, nb - 1) * ldi + dr];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = cg + 4 * i;
      T[row * TP + j] = (row < nb && j < nb && j <= row) ? dv[i] : (j == row ? 1.0 : 0.0);
    }
  }
  wave_sync_lds();
  if (nb <= 4)
    inv16<4>(T, TP, 0, I, TP, lane);
  else if (nb <= 8)
    inv16<8>(T, TP, 0, I, TP, lane);
  else
    inv16<16>(T, TP, 0, I, TP, lane);
  wave_sync_lds();
  // inv(i, j), i > j, at row j of column i
  for (int e = lane; e < 256; e += 64) {
    const int i = e >> 4, j = e & 15;
    if (i > j && i < nb) D[(int64_t)i * ldi + j] = I[i * TP + j];
  }
}

// k_panel for column blocks of at most 16 columns without a previous-block
// update, FP64 form, one wavefront per group member and four per workgroup
// (small supernodes leave most of a 256-thread workgroup idle): the
// wavefront factors the diagonal tile (pivot chain as in k_panel), the last
// reader of the group writes it back, and each 64-row tile is solved with
// the tile's inverse on MFMA, its operands read straight from factor storage.
__global__ __launch_bounds__(256, 3) void k_panel_w(const PanelTile* __restrict__ tiles,
                                                 double* __restrict__ L,
                                                 int* __restrict__ status,
                                                 int* __restrict__ counters, int count) {
  constexpr int TP = 17;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int il = lane & 15, kl = lane >> 4;
  __shared__ double Ts[4][16 * TP];
  __shared__ double Is[4][16 * TP];
  __shared__ double Lcs[4][16 * 64];
  const int ti = (int)blockIdx.x * 4 + wave;
  if (ti >= count) return;  // no workgroup barrier below
  const PanelTile t = tiles[ti];
  double* const T = Ts[wave];
  double* const I = Is[wave];
  const int nb = t.nb, ldi = t.ld;
  double* D = L + t.diag;
  {
    const int dr = min(il, nb - 1);
    double dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) dv[i] = D[(int64_t)min(kl + 4 * i, nb - 1) * ldi + dr];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = kl + 4 * i;
      T[il * TP + j] = (il < nb && j < nb && j <= il) ? dv[i] : (j == il ? 1.0 : 0.0);
    }
  }
  wave_sync_lds();
  // this member has read the unfactored tile
  int old = 0;
  if (lane == 0) old = atomicAdd(&counters[t.grp], 1);
  const bool last = __builtin_amdgcn_readfirstlane(old) == t.gcnt - 1;
  // the pivot chain visits the block's columns only (nb <= 4, 8 or 16)
  const int bad =
      nb <= 4 ? panel16<false, 4>(T, TP, 16, Lcs[wave], 0, nb, t.col, lane, 0.0, 0.0, nullptr)
      : nb <= 8 ? panel16<false, 8>(T, TP, 16, Lcs[wave], 0, nb, t.col, lane, 0.0, 0.0, nullptr)
                : panel16<false, 16>(T, TP, 16, Lcs[wave], 0, nb, t.col, lane, 0.0, 0.0, nullptr);
  wave_sync_lds();
  if (nb <= 4)
    inv16<4>(T, TP, 0, I, TP, lane);
  else if (nb <= 8)
    inv16<8>(T, TP, 0, I, TP, lane);
  else
    inv16<16>(T, TP, 0, I, TP, lane);
  if (last) {
    if (lane == 0) {
      atomicExch(&counters[t.grp], 0);
      if (bad != 0x7fffffff) atomicMin(status + t.slot, bad);
    }
    for (int e = lane; e < 256; e += 64) {
      const int i = e >> 4, j = e & 15;
      if (i < nb && j <= i) D[(int64_t)j * ldi + i] = T[i * TP + j];
    }
  }
  wave_sync_lds();
  // X = A inv(L)^T for the member's row tiles, 16 rows per MFMA block
  for (int rt = 0; rt < t.nrt; ++rt) {
    const int row0 = t.row0 + 64 * rt;
    const int nrows = min(64, t.nrows - row0);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      if (16 * rb >= nrows) break;
      const int rr = 16 * rb + il;
      const int ar = row0 + min(rr, nrows - 1);
      v4d r;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 4 * v + kl;
        const double a = D[(int64_t)min(c, nb - 1) * ldi + ar];
        r[v] = (rr < nrows && c < nb) ? a : 0.0;
      }
      v4d x = {0, 0, 0, 0};
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) x = mfma64(I[il * TP + 4 * kq + kl], r[kq], x);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 4 * v + kl;
        if (c < nb && rr < nrows) D[(int64_t)c * ldi + row0 + rr] = x[v];
      }
    }
  }
}

// Inverse of every diagonal tile of the factor, for the solves: inv(L_kk)
// of the <=64x64 tile goes, strict lower part transposed, into the tile's
// unused strict upper triangle (inv(L)(i,j), i > j, at row j of column i).
// One workgroup per tile: the 16x16 diagonal blocks are inverted by
// substitution (one wavefront each), then the 2 x 2 block formula
// [A 0; B C]^-1 = [A^-1 0; -C^-1 B A^-1  C^-1] joins them in two levels.
// NBB as in k_panel.
template <int NBB>
__global__ __launch_bounds__(256) void k_tile_inverse(const DiagTile* __restrict__ tiles,
                                                      double* __restrict__ L) {
  constexpr int TR = 16 * NBB, TPn = TR + 1;
  const DiagTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = t.nb, ldi = t.ld;
  double* D = L + t.diag;
  __shared__ double T[TR * TPn];
  __shared__ double I[TR * TPn];
  {
    const int row = lane, cg = wave;
    const int dr = min(row, nb - 1);
    double dv[4 * NBB];
#pragma unroll
    for (int i = 0; i < 4 * NBB; ++i) dv[i] = D[(int64_t)min(cg + 4 * i, nb - 1) * ldi + dr];
    if (row < TR) {
#pragma unroll
      for (int i = 0; i < 4 * NBB; ++i) {
        const int j = cg + 4 * i;
        T[row * TPn + j] = (row < nb && j < nb && j <= row) ? dv[i] : (j == row ? 1.0 : 0.0);
      }
    }
  }
  __syncthreads();
  const int nbb = (nb + 15) >> 4;
  if (wave < nbb) inv16(T, TPn, 16 * wave, &I[16 * wave * TPn + 16 * wave], TPn, lane);
  __syncthreads();
  if (NBB >= 2) {
    // level 1: blocks (1,0) and (3,2) = -inv(i,i) * (L(i,j) * inv(j,j))
    const int i1 = wave == 0 ? 1 : 3;
    if ((wave == 0 && nbb >= 2) || (wave == 1 && nbb >= 4)) {
      const v4d s = mma16(&T[16 * i1 * TPn + 16 * (i1 - 1)], TPn, 1,
                          &I[16 * (i1 - 1) * TPn + 16 * (i1 - 1)], TPn, 1, lane);
      const v4d u = mma16r(&I[16 * i1 * TPn + 16 * i1], TPn, 1, s, lane);
      st16(&I[16 * i1 * TPn + 16 * (i1 - 1)], TPn, u, lane, -1.0);
    }
    __syncthreads();
  }
  if (NBB >= 4) {
    // level 2 (nbb >= 3): for i in [2, nbb), j in {0, 1}: S(i,j) = L(i,0)
    // inv(0,j) + L(i,1) inv(1,j), kept in T's unused block (j, i), then
    // inv(i,j) = -sum_{2 <= l <= i} inv(i,l) S(l,j)
    const int i2 = 2 + (wave >> 1), j2 = wave & 1;
    const bool p2 = nbb >= 3 && i2 < nbb;
    if (p2) {
      v4d s = mma16(&T[16 * i2 * TPn + 16], TPn, 1, &I[16 * TPn + 16 * j2], TPn, 1, lane);
      if (j2 == 0) s += mma16(&T[16 * i2 * TPn], TPn, 1, &I[0], TPn, 1, lane);
      st16(&T[16 * j2 * TPn + 16 * i2], TPn, s, lane, 1.0);
    }
    __syncthreads();
    if (p2) {
      v4d u = {0, 0, 0, 0};
      for (int l = 2; l <= i2; ++l)
        u += mma16(&I[16 * i2 * TPn + 16 * l], TPn, 1, &T[16 * j2 * TPn + 16 * l], TPn, 1, lane);
      st16(&I[16 * i2 * TPn + 16 * j2], TPn, u, lane, -1.0);
    }
    __syncthreads();
  }
  const int i = lane;
  if (i < TR) {
#pragma unroll
    for (int q = 0; q < 4 * NBB; ++q) {
      const int j = wave + 4 * q;
      if (i < j && j < nb) D[(int64_t)j * ldi + i] = I[j * TPn + i];
    }
  }
}


// ---------------------------------------------------------------------------
// Update of one <=64x64 target tile: C -= sum over its contributions of
// X * Y^T. 256 threads = 4 wavefronts in a 2x2 arrangement, each owning a
// 32x32 quarter = 2x2 MFMA 16x16 blocks; K is staged through LDS in chunks of
// 16 in FP64 and 32 in FP32 (the same LDS bytes), column-major as in factor
// storage. The operand loads are issued two chunks ahead: two register sets
// alternate (chunk c is fetched into set c % 2 while chunk c - 3 is
// multiplied, and written to LDS while chunk c - 1 is), so a chunk's loads
// have two chunk times to arrive, which the tiles of many short
// contributions at the lower levels need; the register budget is held to
// four wavefronts per SIMD. A tile with one owner is read once at the start
// and written once at the end, only where a contribution's rectangle meets
// it; the parts of a split tile are added with atomics.
template <typename T>
__global__ __launch_bounds__(256, 4) void k_update(const UpdTile* __restrict__ tiles,
                                                   const UpdSeg* __restrict__ segs,
                                                   double* __restrict__ L, const T* __restrict__ S,
                                                   int count, int by_xcd) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int KC = 16 * (int)(sizeof(double) / sizeof(T));
  constexpr int NQ = KC / 4;
  // workgroups are dealt to the 8 XCDs round-robin as dispatched: with
  // by_xcd, the ones of XCD x take the x-th contiguous eighth of the list
  int b = (int)blockIdx.x;
  if (by_xcd) {
    const int x = b & 7, q = count >> 3, r = count & 7;
    b = x * q + min(x, r) + (b >> 3);
  }
  const UpdTile t = tiles[b];
  __shared__ T sX[2][KC][64];
  __shared__ T sY[2][KC][64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int lr = tid & 63, lk = tid >> 6;
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;
  const bool assign = t.flags & 4;
  auto seg_at = [&](int i) { return uniform_seg(segs[t.seg0 + i]); };

  // register sets: the loaded values and the masks of their chunk
  T xr[2][NQ], yr[2][NQ];
  bool xin[2] = {false, false}, yin[2] = {false, false};
  int kvalid[2] = {0, 0};
  // fetch cursor
  int fe = 0, fk = 0;
  UpdSeg gf = seg_at(0);
  auto fetch = [&](int set) {
    if constexpr (sizeof(T) == 8) {
      // FP64 operands through buffer loads whose range is the contribution's
      // rows (columns) of one source column: rows outside it, and k past the
      // contribution's, read as zero with no masking in the kernel
      const int kw = uni32(fk + lk);
      const uint32_t xoff = (uint32_t)(lr - gf.ra) << 3, yoff = (uint32_t)(lr - gf.ca) << 3;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int kk = kw + 4 * q;
        const bool kin = kk < gf.k;
        const int64_t ko = (int64_t)kk * gf.lds;
        xr[set][q] = load_range(S + gf.x + ko, kin ? (gf.rb - gf.ra) << 3 : 0, xoff);
        yr[set][q] = load_range(S + gf.y + ko, kin ? (gf.cb - gf.ca) << 3 : 0, yoff);
      }
    } else {
      xin[set] = lr >= gf.ra && lr < gf.rb;
      yin[set] = lr >= gf.ca && lr < gf.cb;
      kvalid[set] = gf.k - fk - lk;
      const int64_t xo = gf.x + min(max(lr - gf.ra, 0), gf.rb - gf.ra - 1);
      const int64_t yo = gf.y + min(max(lr - gf.ca, 0), gf.cb - gf.ca - 1);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int64_t kk = min(fk + lk + 4 * q, gf.k - 1);
        xr[set][q] = S[xo + kk * gf.lds];
        yr[set][q] = S[yo + kk * gf.lds];
      }
    }
    fk += KC;
    if (fk >= gf.k) {
      fk = 0;
      if (++fe < t.nseg) gf = seg_at(fe);
    }
  };
  auto stash = [&](int set, int buf) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if constexpr (sizeof(T) == 8) {
        sX[buf][lk + 4 * q][lr] = xr[set][q];
        sY[buf][lk + 4 * q][lr] = yr[set][q];
      } else {
        const bool kin = 4 * q < kvalid[set];
        sX[buf][lk + 4 * q][lr] = (kin && xin[set]) ? xr[set][q] : T(0);
        sY[buf][lk + 4 * q][lr] = (kin && yin[set]) ? yr[set][q] : T(0);
      }
    }
  };
  // chunks 0 and 1 in flight first, then the target values
  fetch(0);
  const bool two = fe < t.nseg;
  if (two) fetch(1);
  const unsigned cover = assign ? 0xffffu : cover_bits<Mfma<T>>(t, segs, wr, wc, lane);
  double cv[2][2][4] = {};
  if (!atomic && !assign) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
          const int col = min(wc + 16 * bj + Mfma<T>::drow(lane, v), t.n - 1);
          if ((cover >> (bj * 8 + bi * 4 + v)) & 1u) cv[bj][bi][v] = C[(int64_t)col * ldc + row];
        }
  }
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  stash(0, 0);
  if (fe < t.nseg) fetch(0);  // chunk 2
  __syncthreads();

  // compute cursor
  int e = 0, k0 = 0;
  UpdSeg g = seg_at(0);
  auto multiply = [&](int buf) {
    bool use[2][2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
        use[bj][bi] = wr + 16 * bi < g.rb && wr + 16 * bi + 16 > g.ra &&
                      wc + 16 * bj < g.cb && wc + 16 * bj + 16 > g.ca;
    const bool all4 = use[0][0] && use[0][1] && use[1][0] && use[1][1];
    if (all4) {
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) {
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
    } else if (use[0][0] || use[0][1] || use[1][0] || use[1][1]) {
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) {
        const int kk = kq * 4 + (lane >> 4);
        const T a0 = sY[buf][kk][wc + (lane & 15)];
        const T a1 = sY[buf][kk][wc + 16 + (lane & 15)];
        const T b0 = sX[buf][kk][wr + (lane & 15)];
        const T b1 = sX[buf][kk][wr + 16 + (lane & 15)];
        if (use[0][0]) acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
        if (use[0][1]) acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
        if (use[1][0]) acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
        if (use[1][1]) acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
      }
    }
    k0 += KC;
    if (k0 >= g.k) {
      k0 = 0;
      if (++e < t.nseg) g = seg_at(e);
    }
  };
  // chunk i (even) is in LDS buffer 0, its successor in register set 1
  for (;;) {
    multiply(0);
    if (e >= t.nseg) break;
    stash(1, 1);  // chunk i + 1
    if (fe < t.nseg) fetch(1);  // chunk i + 3
    __syncthreads();
    multiply(1);
    if (e >= t.nseg) break;
    stash(0, 0);  // chunk i + 2
    if (fe < t.nseg) fetch(0);  // chunk i + 4
    __syncthreads();
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<T>::drow(lane, v);
        if (((cover >> (bj * 8 + bi * 4 + v)) & 1u) && row < t.m && col < t.n &&
            (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          if (atomic)
            atomicAdd(p, -(double)acc[bj][bi][v]);
          else
            *p = cv[bj][bi][v] - (double)acc[bj][bi][v];
        }
      }
}

template __global__ void k_update<double>(const UpdTile*, const UpdSeg*, double*, const double*,
                                          int, int);

// k_update on target tiles of up to 128 rows and 64 columns (the long
// updates of the upper levels): eight wavefronts, wavefront w holding the
// 32x32 quarter at rows 32 (w & 3), columns 32 (w >> 2); each K chunk stages
// 128 rows of X and 64 of Y, 1.5 times the bytes of a 64x64 tile's chunk for
// twice its products. X row (w & 1) * 64 + lane of k (w >> 1) + 4q and Y row
// lane of k w + 8q are one wavefront's loads; FP64, range-checked buffer
// loads as in k_update.
__global__ __launch_bounds__(512, 2) void k_update_tall(const UpdTile* __restrict__ tiles,
                                                        const UpdSeg* __restrict__ segs,
                                                        double* __restrict__ L) {
  constexpr int KC = 16, NQX = 4, NQY = 2;
  const UpdTile t = tiles[blockIdx.x];
  __shared__ double sX[2][KC][128];
  __shared__ double sY[2][KC][64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = (wave & 3) * 32, wc = (wave >> 2) * 32;
  const int xrow = (wave & 1) * 64 + lane, xk = wave >> 1;
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;
  auto seg_at = [&](int i) { return uniform_seg(segs[t.seg0 + i]); };

  double xr[2][NQX], yr[2][NQY];
  int fe = 0, fk = 0;  // fetch cursor
  UpdSeg gf = seg_at(0);
  auto fetch = [&](int set) {
    const uint32_t xoff = (uint32_t)(xrow - gf.ra) << 3, yoff = (uint32_t)(lane - gf.ca) << 3;
    const int xrec = (gf.rb - gf.ra) << 3, yrec = (gf.cb - gf.ca) << 3;
#pragma unroll
    for (int q = 0; q < NQX; ++q) {
      const int kk = fk + xk + 4 * q;
      xr[set][q] = load_range(L + gf.x + (int64_t)kk * gf.lds, kk < gf.k ? xrec : 0, xoff);
    }
#pragma unroll
    for (int q = 0; q < NQY; ++q) {
      const int kk = fk + wave + 8 * q;
      yr[set][q] = load_range(L + gf.y + (int64_t)kk * gf.lds, kk < gf.k ? yrec : 0, yoff);
    }
    fk += KC;
    if (fk >= gf.k) {
      fk = 0;
      if (++fe < t.nseg) gf = seg_at(fe);
    }
  };
  auto stash = [&](int set, int buf) {
#pragma unroll
    for (int q = 0; q < NQX; ++q) sX[buf][xk + 4 * q][xrow] = xr[set][q];
#pragma unroll
    for (int q = 0; q < NQY; ++q) sY[buf][wave + 8 * q][lane] = yr[set][q];
  };
  // chunks 0 and 1 in flight first, then the target values
  fetch(0);
  if (fe < t.nseg) fetch(1);
  const unsigned cover = cover_bits<Mfma<double>>(t, segs, wr, wc, lane);
  double cv[2][2][4] = {};
  if (!atomic) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
          const int col = min(wc + 16 * bj + Mfma<double>::drow(lane, v), t.n - 1);
          if ((cover >> (bj * 8 + bi * 4 + v)) & 1u) cv[bj][bi][v] = C[(int64_t)col * ldc + row];
        }
  }
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  stash(0, 0);
  if (fe < t.nseg) fetch(0);  // chunk 2
  __syncthreads();

  int e = 0, k0 = 0;  // compute cursor
  UpdSeg g = seg_at(0);
  auto multiply = [&](int buf) {
    bool use[2][2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
        use[bj][bi] = wr + 16 * bi < g.rb && wr + 16 * bi + 16 > g.ra &&
                      wc + 16 * bj < g.cb && wc + 16 * bj + 16 > g.ca;
    if (use[0][0] || use[0][1] || use[1][0] || use[1][1]) {
      const bool all4 = use[0][0] && use[0][1] && use[1][0] && use[1][1];
#pragma unroll
      for (int kq = 0; kq < KC / 4; ++kq) {
        const int kk = kq * 4 + (lane >> 4);
        const double a0 = sY[buf][kk][wc + (lane & 15)];
        const double a1 = sY[buf][kk][wc + 16 + (lane & 15)];
        const double b0 = sX[buf][kk][wr + (lane & 15)];
        const double b1 = sX[buf][kk][wr + 16 + (lane & 15)];
        if (all4 || use[0][0]) acc[0][0] = mfma64(a0, b0, acc[0][0]);
        if (all4 || use[0][1]) acc[0][1] = mfma64(a0, b1, acc[0][1]);
        if (all4 || use[1][0]) acc[1][0] = mfma64(a1, b0, acc[1][0]);
        if (all4 || use[1][1]) acc[1][1] = mfma64(a1, b1, acc[1][1]);
      }
    }
    k0 += KC;
    if (k0 >= g.k) {
      k0 = 0;
      if (++e < t.nseg) g = seg_at(e);
    }
  };
  // chunk i (even) is in LDS buffer 0, its successor in register set 1
  for (;;) {
    multiply(0);
    if (e >= t.nseg) break;
    stash(1, 1);
    if (fe < t.nseg) fetch(1);
    __syncthreads();
    multiply(1);
    if (e >= t.nseg) break;
    stash(0, 0);
    if (fe < t.nseg) fetch(0);
    __syncthreads();
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<double>::drow(lane, v);
        if (((cover >> (bj * 8 + bi * 4 + v)) & 1u) && row < t.m && col < t.n &&
            (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          if (atomic)
            atomicAdd(p, -acc[bj][bi][v]);
          else
            *p = cv[bj][bi][v] - acc[bj][bi][v];
        }
      }
}
template __global__ void k_update<float>(const UpdTile*, const UpdSeg*, double*, const float*,
                                         int, int);

// k_update for launches whose tiles hold many contributions with small
// rectangles (the lower levels; irregular input): the K chunk takes the shape
// of the contribution, 64 rows x KC k when its rectangle spans more than one
// 32-row quarter, 32 x 2KC or 16 x 4KC when it lies inside an aligned 32- or
// 16-row window (rows and columns alike), so a contribution of a few rows and
// a long k takes a quarter of the chunk rounds (memory round trips) for the
// same staging bytes; the k steps of a chunk stop at the contribution's k.
// The planner picks it per launch when it saves enough rounds: on tiles of
// full 64-row contributions the general indexing costs a few percent.
template <typename T>
__global__ __launch_bounds__(256, 4) void k_update_win(const UpdTile* __restrict__ tiles,
                                                   const UpdSeg* __restrict__ segs,
                                                   double* __restrict__ L, const T* __restrict__ S,
                                                   int count, int by_xcd) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int KC = 16 * (int)(sizeof(double) / sizeof(T));
  constexpr int NQ = KC / 4;
  // workgroups are dealt to the 8 XCDs round-robin as dispatched: with
  // by_xcd, the ones of XCD x take the x-th contiguous eighth of the list
  int b = (int)blockIdx.x;
  if (by_xcd) {
    const int x = b & 7, q = count >> 3, r = count & 7;
    b = x * q + min(x, r) + (b >> 3);
  }
  const UpdTile t = tiles[b];
  // a stage holds ELEMS operand values of X and of Y: 64 rows x KC k for a
  // contribution whose rectangle spans more than one quarter, 32 x 2KC or
  // 16 x 4KC for one inside an aligned 32- or 16-row window (rows and
  // columns alike), laid out [k][row] with the window's row pitch
  constexpr int ELEMS = 64 * KC;
  __shared__ T sX[2][ELEMS];
  __shared__ T sY[2][ELEMS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;
  const bool assign = t.flags & 4;
  auto seg_at = [&](int i) { return uniform_seg(segs[t.seg0 + i]); };
  // log2 of the window of a contribution: 4, 5 or 6
  auto window_log = [](const UpdSeg& g) {
    const bool r16 = (g.ra >> 4) == ((g.rb - 1) >> 4) && (g.ca >> 4) == ((g.cb - 1) >> 4);
    const bool r32 = (g.ra >> 5) == ((g.rb - 1) >> 5) && (g.ca >> 5) == ((g.cb - 1) >> 5);
    return r16 ? 4 : (r32 ? 5 : 6);
  };

  // register sets: the loaded values and the masks of their chunk
  T xr[2][NQ], yr[2][NQ];
  bool xin[2] = {false, false}, yin[2] = {false, false};
  int kvalid[2] = {0, 0};
  int wlog[2] = {6, 6};  // window of the set's chunk
  // fetch cursor
  int fe = 0, fk = 0;
  UpdSeg gf = seg_at(0);
  int fwl = window_log(gf);
  auto fetch_w = [&](int set, int wl) {
    if constexpr (sizeof(T) == 8) {
      if (wl == 6) {
        // 64-row chunks: one k per wavefront and load, through range-checked
        // buffer loads (ragged rows and k past the contribution read zero)
        const int kw = uni32(fk + (tid >> 6));
        const uint32_t xoff = (uint32_t)(lane - gf.ra) << 3, yoff = (uint32_t)(lane - gf.ca) << 3;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int kk = kw + 4 * q;
          const bool kin = kk < gf.k;
          const int64_t ko = (int64_t)kk * gf.lds;
          xr[set][q] = load_range(S + gf.x + ko, kin ? (gf.rb - gf.ra) << 3 : 0, xoff);
          yr[set][q] = load_range(S + gf.y + ko, kin ? (gf.cb - gf.ca) << 3 : 0, yoff);
        }
        return;
      }
    }
    const int win = 1 << wl;
    const int r = tid & (win - 1), kb = tid >> wl, kstep = 256 >> wl;
    const int xrow = (gf.ra & ~(win - 1)) + r, ycol = (gf.ca & ~(win - 1)) + r;
    xin[set] = xrow >= gf.ra && xrow < gf.rb;
    yin[set] = ycol >= gf.ca && ycol < gf.cb;
    kvalid[set] = gf.k - fk - kb;
    const int64_t xo = gf.x + min(max(xrow - gf.ra, 0), gf.rb - gf.ra - 1);
    const int64_t yo = gf.y + min(max(ycol - gf.ca, 0), gf.cb - gf.ca - 1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int64_t kk = min(fk + kb + kstep * q, gf.k - 1);
      xr[set][q] = S[xo + kk * gf.lds];
      yr[set][q] = S[yo + kk * gf.lds];
    }
  };
  auto fetch = [&](int set) {
    const int wl = fwl;
    wlog[set] = wl;
    fetch_w(set, wl);
    fk += ELEMS >> wl;
    if (fk >= gf.k) {
      fk = 0;
      if (++fe < t.nseg) {
        gf = seg_at(fe);
        fwl = window_log(gf);
      }
    }
  };
  auto stash_w = [&](int set, int buf, int wl) {
    const int r = tid & ((1 << wl) - 1), kb = tid >> wl, kstep = 256 >> wl;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const bool kin = kstep * q < kvalid[set];
      const int pos = ((kb + kstep * q) << wl) + r;
      if (sizeof(T) == 8 && wl == 6) {
        sX[buf][pos] = xr[set][q];
        sY[buf][pos] = yr[set][q];
      } else {
        sX[buf][pos] = (kin && xin[set]) ? xr[set][q] : T(0);
        sY[buf][pos] = (kin && yin[set]) ? yr[set][q] : T(0);
      }
    }
  };
  auto stash = [&](int set, int buf) {
    if (wlog[set] == 6)
      stash_w(set, buf, 6);
    else
      stash_w(set, buf, wlog[set]);
  };
  // chunks 0 and 1 in flight first, then the target values
  fetch(0);
  const bool two = fe < t.nseg;
  if (two) fetch(1);
  const unsigned cover = assign ? 0xffffu : cover_bits<Mfma<T>>(t, segs, wr, wc, lane);
  double cv[2][2][4] = {};
  if (!atomic && !assign) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
          const int col = min(wc + 16 * bj + Mfma<T>::drow(lane, v), t.n - 1);
          if ((cover >> (bj * 8 + bi * 4 + v)) & 1u) cv[bj][bi][v] = C[(int64_t)col * ldc + row];
        }
  }
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  stash(0, 0);
  if (fe < t.nseg) fetch(0);  // chunk 2
  __syncthreads();

  // compute cursor
  int e = 0, k0 = 0;
  UpdSeg g = seg_at(0);
  int gwl = window_log(g);
  auto multiply = [&](int buf) {
    bool use[2][2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
        use[bj][bi] = wr + 16 * bi < g.rb && wr + 16 * bi + 16 > g.ra &&
                      wc + 16 * bj < g.cb && wc + 16 * bj + 16 > g.ca;
    // every block of the quarter, in the 64-row window (a rectangle that fills
    // one quarter has a 32-row window and takes the general form)
    const bool all4 = gwl == 6 && use[0][0] && use[0][1] && use[1][0] && use[1][1];
    if (all4) {
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) {
        const int kk = kq * 4 + (lane >> 4);
        const T a0 = sY[buf][kk * 64 + wc + (lane & 15)];
        const T a1 = sY[buf][kk * 64 + wc + 16 + (lane & 15)];
        const T b0 = sX[buf][kk * 64 + wr + (lane & 15)];
        const T b1 = sX[buf][kk * 64 + wr + 16 + (lane & 15)];
        acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
        acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
        acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
      }
    } else if (use[0][0] || use[0][1] || use[1][0] || use[1][1]) {
      // the blocks this wavefront uses lie inside the window (windows are
      // aligned to their size, blocks to 16); indices of the others are kept
      // in range and their values unused
      const int wl = gwl, win = 1 << wl;
      const int wx0 = g.ra & ~(win - 1), wy0 = g.ca & ~(win - 1);
      const int ya = (wc - wy0 + (lane & 15)) & (ELEMS - 1);
      const int xa = (wr - wx0 + (lane & 15)) & (ELEMS - 1);
      // 4-deep k steps of the chunk that the contribution's k reaches
      const int nq = min(ELEMS >> (wl + 2), (g.k - k0 + 3) >> 2);
      for (int kq0 = 0; kq0 < nq; kq0 += NQ) {
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
          if (kq0 + u >= nq) break;
          const int kk = (kq0 + u) * 4 + (lane >> 4);
          const int ko = kk << wl;
          const T a0 = sY[buf][(ko + ya) & (ELEMS - 1)];
          const T a1 = sY[buf][(ko + ya + 16) & (ELEMS - 1)];
          const T b0 = sX[buf][(ko + xa) & (ELEMS - 1)];
          const T b1 = sX[buf][(ko + xa + 16) & (ELEMS - 1)];
          if (use[0][0]) acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
          if (use[0][1]) acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
          if (use[1][0]) acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
          if (use[1][1]) acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
        }
      }
    }
    k0 += ELEMS >> gwl;
    if (k0 >= g.k) {
      k0 = 0;
      if (++e < t.nseg) {
        g = seg_at(e);
        gwl = window_log(g);
      }
    }
  };
  // chunk i (even) is in LDS buffer 0, its successor in register set 1
  for (;;) {
    multiply(0);
    if (e >= t.nseg) break;
    stash(1, 1);  // chunk i + 1
    if (fe < t.nseg) fetch(1);  // chunk i + 3
    __syncthreads();
    multiply(1);
    if (e >= t.nseg) break;
    stash(0, 0);  // chunk i + 2
    if (fe < t.nseg) fetch(0);  // chunk i + 4
    __syncthreads();
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<T>::drow(lane, v);
        if (((cover >> (bj * 8 + bi * 4 + v)) & 1u) && row < t.m && col < t.n &&
            (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          if (atomic)
            atomicAdd(p, -(double)acc[bj][bi][v]);
          else
            *p = cv[bj][bi][v] - (double)acc[bj][bi][v];
        }
      }
}

template __global__ void k_update_win<double>(const UpdTile*, const UpdSeg*, double*,
                                              const double*, int, int);

// k_update for launches whose tiles hold many contributions of a small k
// (the small supernodes of a batch of 2D grids: k of a few columns): the
// contributions of a tile are laid end to end along one K axis, each padded to
// a multiple of 4, and staged 16 k at a time, so a chunk round serves several
// of them. Each group of 4 consecutive k (one MFMA step) belongs to one
// contribution: its X rows outside that contribution's rectangle and its Y
// columns outside it are zero, and a wavefront runs the step only on the 16x16
// blocks of its quarter that the rectangle meets, so every target entry
// receives exactly the products of the contributions whose rectangles contain
// it, in no more MFMA steps than the contributions' own k take. Wavefront w
// stages k w, w+4, w+8, w+12 of each chunk, walking the contribution list
// (copied to LDS when it is short) with a cursor of its own. FP64 operands.
constexpr int PACK_SEGS = 21;  // contribution records staged in LDS (12 words each)
__global__ __launch_bounds__(256, 4) void k_update_pack(const UpdTile* __restrict__ tiles,
                                                        const UpdSeg* __restrict__ segs,
                                                        double* __restrict__ L) {
  constexpr int KC = 16, NQ = 4;
  const UpdTile t = tiles[blockIdx.x];
  __shared__ double sX[2][KC][64];
  __shared__ double sY[2][KC][64];
  __shared__ UpdSeg sSeg[PACK_SEGS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int lr = lane, lk = wave;
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;
  const bool assign = t.flags & 4;
  const int nseg = t.nseg;
  if (nseg <= 0) return;
  const bool in_lds = nseg <= PACK_SEGS;
  constexpr int SEG_WORDS = (int)(sizeof(UpdSeg) / 4);
  if (in_lds && tid < nseg * SEG_WORDS)
    reinterpret_cast<int32_t*>(sSeg)[tid] = reinterpret_cast<const int32_t*>(segs + t.seg0)[tid];
  __syncthreads();
  auto seg_at = [&](int i) {
    return in_lds ? uniform_seg(sSeg[i]) : uniform_seg(segs[t.seg0 + i]);
  };
  // total K of the tile, contributions padded to multiples of 4
  int kt = 0;
  for (int i = 0; i < nseg; ++i) kt += (seg_at(i).k + 3) & ~3;
  const int nch = (kt + KC - 1) / KC;

  // register sets of loaded values (range-checked buffer loads: a staged
  // element outside its contribution's rectangle or k reads zero) and the blocks
  // of this wavefront's quarter each MFMA step of the chunk meets (bit
  // 4 q + 2 bj + bi)
  double xr[2][NQ], yr[2][NQ];
  unsigned ub[2] = {0u, 0u};
  int fe = 0, fbase = 0, fc = 0;  // contribution fe starts at padded k fbase
  UpdSeg gf = seg_at(0);
  auto fetch = [&](int set) {
    unsigned u = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int v = fc * KC + lk + 4 * q;
      while (fe + 1 < nseg && v >= fbase + ((gf.k + 3) & ~3)) {
        fbase += (gf.k + 3) & ~3;
        gf = seg_at(++fe);
      }
      const int kk = v - fbase;
      const bool kin = kk < gf.k;
      const int64_t ko = (int64_t)kk * gf.lds;
      xr[set][q] = load_range(L + gf.x + ko, kin ? (gf.rb - gf.ra) << 3 : 0,
                              (uint32_t)(lr - gf.ra) << 3);
      yr[set][q] = load_range(L + gf.y + ko, kin ? (gf.cb - gf.ca) << 3 : 0,
                              (uint32_t)(lr - gf.ca) << 3);
      if (kk < ((gf.k + 3) & ~3)) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
            if (wr + 16 * bi < gf.rb && wr + 16 * bi + 16 > gf.ra && wc + 16 * bj < gf.cb &&
                wc + 16 * bj + 16 > gf.ca)
              u |= 1u << (4 * q + 2 * bj + bi);
      }
    }
    ub[set] = u;
    ++fc;
  };
  unsigned uu[2] = {0u, 0u};
  auto stash = [&](int set, int buf) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      sX[buf][lk + 4 * q][lr] = xr[set][q];
      sY[buf][lk + 4 * q][lr] = yr[set][q];
    }
    uu[buf] = ub[set];
  };
  fetch(0);
  if (fc < nch) fetch(1);
  const unsigned cover = assign ? 0xffffu : cover_bits<Mfma<double>>(t, segs, wr, wc, lane);
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  stash(0, 0);
  if (fc < nch) fetch(0);
  __syncthreads();

  auto multiply = [&](int buf) {
    // step kq of the chunk: the staging wavefronts wrote k kq*4 + w
    const unsigned u = __builtin_amdgcn_readfirstlane(uu[buf]);
    if (u == 0xffffu) {
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) {
        const int kk = kq * 4 + (lane >> 4);
        const double a0 = sY[buf][kk][wc + (lane & 15)];
        const double a1 = sY[buf][kk][wc + 16 + (lane & 15)];
        const double b0 = sX[buf][kk][wr + (lane & 15)];
        const double b1 = sX[buf][kk][wr + 16 + (lane & 15)];
        acc[0][0] = mfma64(a0, b0, acc[0][0]);
        acc[0][1] = mfma64(a0, b1, acc[0][1]);
        acc[1][0] = mfma64(a1, b0, acc[1][0]);
        acc[1][1] = mfma64(a1, b1, acc[1][1]);
      }
    } else {
#pragma unroll
      for (int kq = 0; kq < NQ; ++kq) {
        const unsigned m = (u >> (4 * kq)) & 15u;
        if (!m) continue;
        const int kk = kq * 4 + (lane >> 4);
        const double a0 = sY[buf][kk][wc + (lane & 15)];
        const double a1 = sY[buf][kk][wc + 16 + (lane & 15)];
        const double b0 = sX[buf][kk][wr + (lane & 15)];
        const double b1 = sX[buf][kk][wr + 16 + (lane & 15)];
        if (m & 1u) acc[0][0] = mfma64(a0, b0, acc[0][0]);
        if (m & 2u) acc[0][1] = mfma64(a0, b1, acc[0][1]);
        if (m & 4u) acc[1][0] = mfma64(a1, b0, acc[1][0]);
        if (m & 8u) acc[1][1] = mfma64(a1, b1, acc[1][1]);
      }
    }
  };
  // chunk c (even) is in LDS buffer 0, its successor in register set 1
  for (int c = 0;; c += 2) {
    multiply(0);
    if (c + 1 >= nch) break;
    stash(1, 1);
    if (fc < nch) fetch(1);
    __syncthreads();
    multiply(1);
    if (c + 2 >= nch) break;
    stash(0, 0);
    if (fc < nch) fetch(0);
    __syncthreads();
  }
  double cv[2][2][4] = {};
  if (!atomic && !assign) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
          const int col = min(wc + 16 * bj + Mfma<double>::drow(lane, v), t.n - 1);
          if ((cover >> (bj * 8 + bi * 4 + v)) & 1u) cv[bj][bi][v] = C[(int64_t)col * ldc + row];
        }
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<double>::drow(lane, v);
        if (((cover >> (bj * 8 + bi * 4 + v)) & 1u) && row < t.m && col < t.n &&
            (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          if (atomic)
            atomicAdd(p, -acc[bj][bi][v]);
          else
            *p = cv[bj][bi][v] - acc[bj][bi][v];
        }
      }
}

// Update of narrow target tiles (at most 64 rows and 16 columns: the targets
// in small supernodes), one wavefront per tile and four tiles per
// workgroup: C -= sum over the tile's contributions of X * Y^T, the MFMA
// operands read straight from factor storage (a wavefront's 16 lanes of one
// k read 16 consecutive source rows), no LDS and no barrier. Row block bi of
// the tile is MFMA block acc[bi]; NBI blocks cover the tile's rows (rows past
// the tile are clamped reads, not stored); rows and k outside a contribution
// read as 0.
template <int NBI>
__device__ __forceinline__ void update_w_tile(const UpdTile& t, const UpdSeg* __restrict__ segs,
                                              double* __restrict__ L, int lane) {
  const int il = lane & 15, kl = lane >> 4;
  double* __restrict__ C = L + t.c;
  const bool diag = t.flags & 1, atomic = t.flags & 2;
  double cv[NBI][4];
  if (!atomic) {
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = min(16 * bi + il, t.m - 1), col = min(4 * v + kl, t.n - 1);
        cv[bi][v] = C[(int64_t)col * t.ldc + row];
      }
  }
  v4d acc[NBI];
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi) acc[bi] = v4d{0, 0, 0, 0};
  // K in steps of 8 (two 4-deep MFMA steps) over the contributions in order;
  // the loads of a step are issued before the products of the one before
  // (two register sets), so a tile of many short contributions waits for
  // memory about once instead of once per contribution
  constexpr int KW = 8, NQW = KW / 4;
  double ya[2][NQW], xb[2][NQW][NBI];
  bool yin[2], xin[2][NBI];
  int kv[2], nq[2];
  int e = 0, k0 = 0;  // load cursor
  UpdSeg g = uniform_seg(segs[t.seg0]);
  auto load = [&](const int st) {
    yin[st] = il >= g.ca && il < g.cb;
    const int64_t yo = g.y + min(max(il - g.ca, 0), g.cb - g.ca - 1);
    int64_t xo[NBI];
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) {
      const int r = 16 * bi + il;
      xin[st][bi] = r >= g.ra && r < g.rb;
      xo[bi] = g.x + min(max(r - g.ra, 0), g.rb - g.ra - 1);
    }
    kv[st] = g.k - k0;
    nq[st] = min(NQW, (g.k - k0 + 3) >> 2);
#pragma unroll
    for (int q = 0; q < NQW; ++q) {
      if (q < nq[st]) {
        const int64_t kc = min(k0 + 4 * q + kl, g.k - 1);
        ya[st][q] = L[yo + kc * g.lds];
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi) xb[st][q][bi] = L[xo[bi] + kc * g.lds];
      }
    }
    k0 += KW;
    if (k0 >= g.k) {
      k0 = 0;
      if (++e < t.nseg) g = uniform_seg(segs[t.seg0 + e]);
    }
  };
  auto compute = [&](const int st) {
#pragma unroll
    for (int q = 0; q < NQW; ++q) {
      if (q < nq[st]) {
        const bool kin = 4 * q + kl < kv[st];
        const double a = (kin && yin[st]) ? ya[st][q] : 0.0;
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi)
          acc[bi] = mfma64(a, (kin && xin[st][bi]) ? xb[st][q][bi] : 0.0, acc[bi]);
      }
    }
  };
  if (t.nseg > 0) {
    load(0);
    for (;;) {
      const bool m1 = e < t.nseg;
      if (m1) load(1);
      compute(0);
      if (!m1) break;
      const bool m0 = e < t.nseg;
      if (m0) load(0);
      compute(1);
      if (!m0) break;
    }
  }
  // acc[bi][v] is the update of target row 16*bi + il, column 4*v + kl
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * bi + il, col = 4 * v + kl;
      if (row < t.m && col < t.n && (!diag || row >= col)) {
        double* p = C + (int64_t)col * t.ldc + row;
        if (atomic)
          atomicAdd(p, -acc[bi][v]);
        else
          *p = cv[bi][v] - acc[bi][v];
      }
    }
}

__global__ __launch_bounds__(256, 4) void k_update_w(const UpdTile* __restrict__ tiles,
                                                     const UpdSeg* __restrict__ segs,
                                                     double* __restrict__ L, int count) {
  const int lane = threadIdx.x & 63;
  const int ti = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + ((int)threadIdx.x >> 6));
  if (ti >= count) return;
  const UpdTile t = tiles[ti];
  if (t.m <= 16)
    update_w_tile<1>(t, segs, L, lane);
  else if (t.m <= 32)
    update_w_tile<2>(t, segs, L, lane);
  else
    update_w_tile<4>(t, segs, L, lane);
}

// RL (Algorithm 4) assembly: column j of an update matrix U_J added into the
// ancestor column that owns it, at the rows its relative indices give. The
// columns of a launch that target one ancestor column (from several update
// matrices of the step) are consecutive in the list, in source order; the
// wavefront of the first of them adds them all, one after the other, so
// every entry has one writer and the sums have a fixed order (no atomics).
// The target entries are read and written at agent scope (past the CU's L1)
// and each column's stores complete before the next column's reads.
__global__ __launch_bounds__(256) void k_assemble(const AsmCol* __restrict__ cols,
                                                  const int32_t* __restrict__ rows,
                                                  double* __restrict__ L, int count) {
  const int lane = threadIdx.x & 63;
  const int ci = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + ((int)threadIdx.x >> 6));
  if (ci >= count) return;
  const int64_t dst = uni64(cols[ci].dst);
  if (ci > 0 && uni64(cols[ci - 1].dst) == dst) return;  // not the first of its group
  for (int c = ci; c < count; ++c) {
    const AsmCol a = cols[c];
    if (uni64(a.dst) != dst) break;
    const int64_t src = uni64(a.src);
    const int32_t rp = uni32(a.rp), len = uni32(a.len);
    // 256 entries at a time: their row positions and values, then their
    // targets, then the sums, so each pass waits for memory twice
    for (int i0 = 0; i0 < len; i0 += 256) {
      int ro[4];
      double u[4], t[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = min(i0 + 64 * q + lane, len - 1);
        ro[q] = rows[rp + i];
        u[q] = L[src + i];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        t[q] = __hip_atomic_load(L + dst + ro[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i0 + 64 * q + lane < len)
          __hip_atomic_store(L + dst + ro[q], t[q] + u[q], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this column's stores are done
  }
}

// The parts of split target tiles added into them, one workgroup per tile:
// part p holds -(its sum) in the 64x64 block at pbase + 4096 p (column major,
// ld 64), and every entry of the tile receives the parts' values summed in
// part order, so the result does not depend on which part finished first.
__global__ __launch_bounds__(256) void k_part_reduce(const PartReduce* __restrict__ recs,
                                                     double* __restrict__ L) {
  const PartReduce r = recs[blockIdx.x];
  const bool diag = r.flags & 1;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int row = e & 63, col = e >> 6;
    if (row >= r.m || col >= r.n || (diag && row < col)) continue;
    const double* q = L + r.pbase + e;
    double sum = q[0];
    for (int pi = 1; pi < r.nparts; ++pi) sum += q[(int64_t)pi * 4096];
    L[r.c + (int64_t)col * r.ldc + row] += sum;
  }
}

// The trailing updates of a step as a launch of their own.
template <typename T>
__global__ __launch_bounds__(256) void k_update_short(const UpdTile* __restrict__ tiles,
                                                      const UpdSeg* __restrict__ segs,
                                                      double* __restrict__ L,
                                                      const T* __restrict__ S) {
  __shared__ T sX[2][KC][64];
  __shared__ T sY[2][KC][64];
  const UpdTile t = tiles[blockIdx.x];
  upd_short_tile<T>(t, segs[t.seg0], L, S, sX, sY);
}

template __global__ void k_update_short<double>(const UpdTile*, const UpdSeg*, double*,
                                                const double*);
template __global__ void k_update_short<float>(const UpdTile*, const UpdSeg*, double*,
                                               const float*);

// C -= sum of X * Y^T on a 128x128 target tile (the updates of launches with
// many long contributions: the trailing updates of wide supernodes after a
// 256-column outer block, and the SYRK/GEMM updates into ancestors at the
// upper levels). Against the 64x64 tile of k_update this halves the operand
// bytes per flop (16 flop per byte staged in FP64). Four wavefronts, each a
// 64x64 quadrant held as 4 x 4 MFMA 16x16 accumulators; K is staged through
// LDS in chunks of 16 (the next chunk's loads in flight during the current
// chunk's 64 MFMAs per wavefront); thread (row, k parity) stages one tile
// row for 8 values of k, a wavefront's loads of one k being 64 consecutive
// rows of a source column. Blocks of a quadrant outside a contribution's
// rectangle, and blocks of a diagonal tile above its diagonal, are skipped.
// The target is read and written once, in the epilogue (one owner), or its
// parts are added with atomics (a split tile).
constexpr int BT = 128;  // big target tile

template <typename T>
__global__ __launch_bounds__(256, 2) void k_update_big(const UpdTile* __restrict__ tiles,
                                                       const UpdSeg* __restrict__ segs,
                                                       double* __restrict__ L,
                                                       const T* __restrict__ S) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T sX[2][KC][BT];  // [k][tile row]
  __shared__ T sY[2][KC][BT];  // [k][tile column]
  const UpdTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;  // this wave's quadrant
  const int lr = tid & 127, lk = tid >> 7;                // staging: row lr, k = lk + 2q
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;

  acc_t acc[4][4];  // [column block][row block]
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  T xr[KC / 2], yr[KC / 2];
  bool xin = false, yin = false;
  int kvalid = 0;
  auto fetch = [&](const UpdSeg& g, int k0) {
    xin = lr >= g.ra && lr < g.rb;
    yin = lr >= g.ca && lr < g.cb;
    kvalid = g.k - k0 - lk;
    const int64_t xo = g.x + min(max(lr - g.ra, 0), g.rb - g.ra - 1);
    const int64_t yo = g.y + min(max(lr - g.ca, 0), g.cb - g.ca - 1);
#pragma unroll
    for (int q = 0; q < KC / 2; ++q) {
      const int64_t kk = min(k0 + lk + 2 * q, g.k - 1);
      xr[q] = S[xo + kk * g.lds];
      yr[q] = S[yo + kk * g.lds];
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < KC / 2; ++q) {
      const bool kin = 2 * q < kvalid;
      sX[buf][lk + 2 * q][lr] = (kin && xin) ? xr[q] : T(0);
      sY[buf][lk + 2 * q][lr] = (kin && yin) ? yr[q] : T(0);
    }
  };
  auto seg_at = [&](int i) { return uniform_seg(segs[t.seg0 + i]); };
  int e = 0, k0 = 0;
  UpdSeg g = seg_at(0);
  fetch(g, 0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (;;) {
    // the quadrant's 16-row and 16-column blocks that meet the rectangle
    const int bi0 = max(0, (g.ra - wr) >> 4), bi1 = min(4, (g.rb - wr + 15) >> 4);
    const int bj0 = max(0, (g.ca - wc) >> 4), bj1 = min(4, (g.cb - wc + 15) >> 4);
    // a diagonal tile: block (bj, bi) lies above the diagonal when its last
    // row is above its first column
    const bool full = bi0 == 0 && bi1 == 4 && bj0 == 0 && bj1 == 4 && (!diag || wr >= wc + 48);
    int ne = e, nk0 = k0 + KC;
    if (nk0 >= g.k) {
      ne = e + 1;
      nk0 = 0;
    }
    const bool more = ne < t.nseg;
    UpdSeg gn = g;
    if (more) {
      if (ne != e) gn = seg_at(ne);
      fetch(gn, nk0);
    }
    if (full) {
#pragma unroll
      for (int kq = 0; kq < KC / 4; ++kq) {
        const int kk = kq * 4 + (lane >> 4);
        T a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = sY[buf][kk][wc + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = sX[buf][kk][wr + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[j][i] = Mfma<T>::op(a[j], b[i], acc[j][i]);
      }
    } else if (bi0 < bi1 && bj0 < bj1) {
#pragma unroll
      for (int kq = 0; kq < KC / 4; ++kq) {
        const int kk = kq * 4 + (lane >> 4);
        T a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = sY[buf][kk][wc + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = sX[buf][kk][wr + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i >= bi0 && i < bi1 && j >= bj0 && j < bj1 &&
                (!diag || wr + 16 * i + 15 >= wc + 16 * j))
              acc[j][i] = Mfma<T>::op(a[j], b[i], acc[j][i]);
      }
    }
    if (!more) break;
    stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    e = ne;
    k0 = nk0;
    g = gn;
  }
  // epilogue, one column block at a time: acc[bj][bi][v] is the update of
  // target row wr+16*bi+(lane&15), column wc+16*bj+drow(lane,v)
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    if (diag && wr + 63 < wc + 16 * bj) continue;  // the whole column block is above
    double cv[4][4];
    if (!atomic) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
          const int col = min(wc + 16 * bj + Mfma<T>::drow(lane, v), t.n - 1);
          cv[bi][v] = C[(int64_t)col * ldc + row];
        }
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + Mfma<T>::drow(lane, v);
        if (row < t.m && col < t.n && (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          if (atomic)
            atomicAdd(p, -(double)acc[bj][bi][v]);
          else
            *p = cv[bi][v] - (double)acc[bj][bi][v];
        }
      }
  }
}

template __global__ void k_update_big<double>(const UpdTile*, const UpdSeg*, double*,
                                              const double*);
template __global__ void k_update_big<float>(const UpdTile*, const UpdSeg*, double*,
                                             const float*);

// 16-bit operand form of the update. Every contribution's X and Y are scaled
// by the power of two s = 2^e of its source panel (e chosen so that the
// panel's largest |entry| times s lies in [2^13, 2^14)), rounded to FP16 or
// BF16 (round to nearest even, through FP32) and multiplied on the gfx950
// MFMA 16x16x32 with FP32 accumulation; a contribution's sum is scaled back by
// 2^-2e into an FP64 accumulator before the next contribution starts. Staging
// as in k_update with K chunks of 32, each thread staging 8 consecutive k of
// one row, stored row-major so that a lane's 8-element MFMA operand (row
// l % 16, k 8 (l / 16) .. +7) is one 16-byte LDS read; the row pitch of 40
// elements (5 x 16 bytes) keeps the 16 rows of a read in distinct banks.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int P>
struct Half;
template <>
struct Half<3> {  // FP16
  typedef v8h vec;
  static __device__ __forceinline__ unsigned short cvt(double x) {
    const _Float16 h = (_Float16)(float)x;
    unsigned short b;
    __builtin_memcpy(&b, &h, 2);
    return b;
  }
  static __device__ __forceinline__ v4f op(vec a, vec b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Half<2> {  // BF16
  typedef v8bf vec;
  static __device__ __forceinline__ unsigned short cvt(double x) {
    const __bf16 h = (__bf16)(float)x;
    unsigned short b;
    __builtin_memcpy(&b, &h, 2);
    return b;
  }
  static __device__ __forceinline__ v4f op(vec a, vec b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// the scale exponent e of a panel from its largest |entry| (bit pattern)
__device__ __forceinline__ int panel_scale_exp(unsigned long long mbits) {
  if (mbits == 0ull) return 0;
  const int E = (int)((mbits >> 52) & 0x7ff) - 1023;  // floor(log2(max)) for normal max
  return min(max(13 - E, -960), 960);
}

constexpr int KC16 = 32;  // K chunk of the 16-bit stage
constexpr int KP16 = 40;  // LDS row pitch of the 16-bit stage (elements)

template <int P>
__global__ __launch_bounds__(256) void k_update16(const UpdTile* __restrict__ tiles,
                                                  const UpdSeg* __restrict__ segs,
                                                  double* __restrict__ L,
                                                  const unsigned long long* __restrict__ smax) {
  typedef typename Half<P>::vec vec;
  const UpdTile t = tiles[blockIdx.x];
  __shared__ __align__(16) unsigned short sX[2][64][KP16];  // [tile row][k]
  __shared__ __align__(16) unsigned short sY[2][64][KP16];  // [tile column][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int lr = tid & 63;  // row this thread stages
  const int lk = tid >> 6;  // it stages k = 8*lk .. 8*lk+7 of the chunk
  double* __restrict__ C = L + t.c;
  const int64_t ldc = t.ldc;
  const bool diag = t.flags & 1;
  const bool atomic = t.flags & 2;
  const bool assign = t.flags & 4;  // write -(sum) without reading the target
  // elements met by a contribution (the FP32 accumulator layout)
  const unsigned cover = assign ? 0xffffu : cover_bits<Mfma<float>>(t, segs, wr, wc, lane);
  double cv[2][2][4] = {};
  if (!atomic && !assign) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = min(wr + 16 * bi + (lane & 15), t.m - 1);
          const int col = min(wc + 16 * bj + 4 * (lane >> 4) + v, t.n - 1);
          if ((cover >> (bj * 8 + bi * 4 + v)) & 1u) cv[bj][bi][v] = C[(int64_t)col * ldc + row];
        }
  }
  v4f acc[2][2];
  double accd[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = v4f{0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[a][b][v] = 0.0;
    }
  constexpr int SEGS_LDS = 64;
  __shared__ UpdSeg sg[SEGS_LDS];
  {
    const int words = min(t.nseg, SEGS_LDS) * (int)(sizeof(UpdSeg) / 8);
    const int64_t* src = reinterpret_cast<const int64_t*>(segs + t.seg0);
    int64_t* dst = reinterpret_cast<int64_t*>(sg);
    for (int w = tid; w < words; w += 256) dst[w] = src[w];
  }
  __syncthreads();
  auto seg_at = [&](int i) { return uniform_seg(i < SEGS_LDS ? sg[i] : segs[t.seg0 + i]); };
  double xr[8], yr[8];
  bool xin = false, yin = false;
  int kvalid = 0;
  double fscale = 1.0;  // scale of the fetched chunk's contribution
  auto fetch = [&](const UpdSeg& g, int k0) {
    xin = lr >= g.ra && lr < g.rb;
    yin = lr >= g.ca && lr < g.cb;
    kvalid = g.k - k0 - 8 * lk;
    fscale = ldexp(1.0, panel_scale_exp(smax[g.sslot]));
    const int64_t xo = g.x + min(max(lr - g.ra, 0), g.rb - g.ra - 1);
    const int64_t yo = g.y + min(max(lr - g.ca, 0), g.cb - g.ca - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t kk = min(k0 + 8 * lk + q, g.k - 1);
      xr[q] = L[xo + kk * g.lds];
      yr[q] = L[yo + kk * g.lds];
    }
  };
  auto stash = [&](int buf) {
    uint4 px = {0, 0, 0, 0}, py = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool kin = q < kvalid;
      const unsigned hx = Half<P>::cvt((kin && xin) ? xr[q] * fscale : 0.0);
      const unsigned hy = Half<P>::cvt((kin && yin) ? yr[q] * fscale : 0.0);
      const int sh = 16 * (q & 1);
      if (q < 2) { px.x |= hx << sh; py.x |= hy << sh; }
      else if (q < 4) { px.y |= hx << sh; py.y |= hy << sh; }
      else if (q < 6) { px.z |= hx << sh; py.z |= hy << sh; }
      else { px.w |= hx << sh; py.w |= hy << sh; }
    }
    *reinterpret_cast<uint4*>(&sX[buf][lr][8 * lk]) = px;
    *reinterpret_cast<uint4*>(&sY[buf][lr][8 * lk]) = py;
  };
  int e = 0, k0 = 0;
  UpdSeg g = seg_at(0);
  fetch(g, 0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (;;) {
    int ne = e, nk0 = k0 + KC16;
    if (nk0 >= g.k) {
      ne = e + 1;
      nk0 = 0;
    }
    const bool more = ne < t.nseg;
    UpdSeg gn = g;
    if (more) {
      if (ne != e) gn = seg_at(ne);
      fetch(gn, nk0);
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const vec a = *reinterpret_cast<const vec*>(&sY[buf][wc + 16 * bj + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const vec b = *reinterpret_cast<const vec*>(&sX[buf][wr + 16 * bi + (lane & 15)][8 * (lane >> 4)]);
        acc[bj][bi] = Half<P>::op(a, b, acc[bj][bi]);
      }
    }
    if (ne != e || !more) {
      // end of a contribution: undo its scale into the FP64 accumulator
      const double inv2 = ldexp(1.0, -2 * panel_scale_exp(smax[g.sslot]));
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
          for (int v = 0; v < 4; ++v) accd[bj][bi][v] += (double)acc[bj][bi][v] * inv2;
          acc[bj][bi] = v4f{0, 0, 0, 0};
        }
    }
    if (!more) break;
    stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    e = ne;
    k0 = nk0;
    g = gn;
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * bi + (lane & 15);
        const int col = wc + 16 * bj + 4 * (lane >> 4) + v;
        if (((cover >> (bj * 8 + bi * 4 + v)) & 1u) && row < t.m && col < t.n &&
            (!diag || row >= col)) {
          double* p = C + (int64_t)col * ldc + row;
          if (atomic)
            atomicAdd(p, -accd[bj][bi][v]);
          else
            *p = cv[bj][bi][v] - accd[bj][bi][v];
        }
      }
}

template __global__ void k_update16<2>(const UpdTile*, const UpdSeg*, double*,
                                       const unsigned long long*);
template __global__ void k_update16<3>(const UpdTile*, const UpdSeg*, double*,
                                       const unsigned long long*);

// ---------------------------------------------------------------------------
// Supernodal solves L z = y and L^T x = z in the factored order (vectors
// n x nrhs column-major, nrhs <= 16), in the 64-column steps of the
// factorization. The diagonal chunk of a step is solved as a product with
// inv(L_kk), which the factorization left in the chunk's unused strict upper
// triangle (inv(L)(i,j), i > j, at row j of column i) together with 1/L(i,i).
// Every workgroup of a step forms the chunk's solution itself from the
// finished right-hand side, so the step needs no second launch; the first
// workgroup of the supernode also stores it.

constexpr int MAXRHS = SOLVE_MAXRHS;
constexpr int VP = 65;  // LDS pitch of a staged 64x64 block

// inv(L_kk) of the chunk at (c0, c0) into V, row-major: V[i*VP + j] = inv(i,j),
// zero above the diagonal and beyond nb. 256 threads, coalesced loads.
__device__ __forceinline__ void stage_inv(double* V, const double* Lj, int64_t ld, int c0,
                                          int nb, int tid) {
  const int row = tid & 63, cg = tid >> 6;
  const int rr = min(row, nb - 1);
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int col = min(cg + 4 * q, nb - 1);
    v[q] = Lj[(int64_t)(c0 + col) * ld + c0 + rr];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int col = cg + 4 * q;
    double e = 0.0;
    if (row < nb && col < nb) e = row < col ? v[q] : (row == col ? 1.0 / v[q] : 0.0);
    V[col * VP + row] = e;  // stored (row, col), row < col, is inv(col, row)
  }
}

// W[i*VP + j] = inv(L)(c0+64+i, c0+j): the off-diagonal block of the inverse
// of a two-chunk step's diagonal block, stored transposed in its unused upper
// block (row c0+j, column c0+64+i), zero outside nbB x 64
__device__ __forceinline__ void stage_w(double* W, const double* Lj, int64_t ld, int c0, int nbB,
                                        int tid) {
  const int row = tid & 63, cg = tid >> 6;
  const int ii = min(row, nbB - 1);
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = Lj[(int64_t)(c0 + 64 + ii) * ld + c0 + cg + 4 * q];
#pragma unroll
  for (int q = 0; q < 16; ++q) W[row * VP + cg + 4 * q] = row < nbB ? v[q] : 0.0;
}

// After the factorization (and k_tile_inverse), for every two-chunk solve
// step with a second chunk (64 < nb <= 128): the off-diagonal block of the
// inverse of its diagonal block, W = -inv(L_BB) L_BA inv(L_AA), into the
// step's unused upper block (W(i, j) at row c0+j, column c0+64+i). Two LDS
// blocks: L_BA and inv(L_AA) for the first product, then inv(L_BB) (held in
// registers until then) and M = L_BA inv(L_AA) for the second.
__global__ __launch_bounds__(256) void k_pair_inverse(const DiagTile* __restrict__ tiles,
                                                      double* __restrict__ L) {
  const DiagTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t ld = t.ld;
  double* D = L + t.diag;  // (c0, c0)
  const int nbB = t.nb - 64;
  __shared__ double V0[64 * VP];  // inv(L_AA), then M
  __shared__ double B[64 * VP];   // L_BA, then inv(L_BB)
  const int row = tid & 63, cg = tid >> 6;
  const int rr = min(row, nbB - 1);
  double v1[16];  // this thread's entries of inv(L_BB), as stage_inv reads them
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int col = min(cg + 4 * q, nbB - 1);
    v1[q] = D[(int64_t)(64 + col) * ld + 64 + rr];
  }
  stage_inv(V0, D, ld, 0, 64, tid);
  {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = D[(int64_t)(cg + 4 * q) * ld + 64 + rr];
#pragma unroll
    for (int q = 0; q < 16; ++q) B[row * VP + cg + 4 * q] = row < nbB ? v[q] : 0.0;
  }
  __syncthreads();
  // two 64x64 products, each thread a 4x4 block of outputs: M = L_BA
  // inv(L_AA) (kept in registers until V0 may be overwritten), then W =
  // -inv(L_BB) M
  const int ti = tid >> 4, tj = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
#pragma unroll 4
  for (int k = 0; k < 64; ++k) {
    double bv[4], vv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bv[r] = B[(4 * ti + r) * VP + k];
#pragma unroll
    for (int c = 0; c < 4; ++c) vv[c] = V0[k * VP + 4 * tj + c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += bv[r] * vv[c];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      V0[(4 * ti + r) * VP + 4 * tj + c] = acc[r][c];
      acc[r][c] = 0.0;
    }
#pragma unroll
  for (int q = 0; q < 16; ++q) {  // inv(L_BB) as stage_inv lays it out
    const int col = cg + 4 * q;
    double e = 0.0;
    if (row < nbB && col < nbB) e = row < col ? v1[q] : (row == col ? 1.0 / v1[q] : 0.0);
    B[col * VP + row] = e;
  }
  __syncthreads();
  const int kend = min(4 * ti + 4, nbB);  // inv(L_BB) is 0 above the diagonal
  for (int k = 0; k < kend; ++k) {
    double bv[4], vv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bv[r] = B[(4 * ti + r) * VP + k];
#pragma unroll
    for (int c = 0; c < 4; ++c) vv[c] = V0[k * VP + 4 * tj + c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += bv[r] * vv[c];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (4 * ti + r < nbB)
#pragma unroll
      for (int c = 0; c < 4; ++c) D[(int64_t)(64 + 4 * ti + r) * ld + 4 * tj + c] = -acc[r][c];
}

// Chained solve launches: all steps of a level in one launch. A workgroup
// takes the next tile in plan order by ticket when it starts, so every
// earlier tile is held by a running or finished workgroup and the earliest
// unfinished tile never waits: the launch cannot deadlock, whatever the
// number of resident workgroups. A tile waits until the counter of its step
// has the number of signals the plan counted (one from each earlier tile
// that writes into the step's columns; agent-scope acquire after the wait,
// release before each signal, since the tiles run on different XCDs with
// their own L2), and then signals the counters of the steps it writes into.
// A wait that exceeds CHAIN_SPIN_LIMIT sleeps sets *err and goes on (a plan
// error: the result is then wrong but the launch still ends).
constexpr int CHAIN_SPIN_LIMIT = 1 << 22;
constexpr int CHAIN_STEP = 128;  // columns of a solve step

__device__ __forceinline__ int chain_tile(const ChainArgs& ca) {
  if (!ca.tick) return (int)blockIdx.x;
  __shared__ int s_ticket;
  if (threadIdx.x == 0) s_ticket = atomicAdd(ca.tick, 1);
  __syncthreads();
  return s_ticket;
}

__device__ __forceinline__ void chain_wait(const ChainArgs& ca, int slot) {
  if (threadIdx.x == 0) {
    const int need = ca.need[slot];
    for (int spins = 0;
         __hip_atomic_load(ca.cnt + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need;
         ++spins) {
      if (spins >= CHAIN_SPIN_LIMIT) {
        atomicOr(ca.err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// every thread calls it (a workgroup barrier: all of the tile's writes done)
__device__ __forceinline__ void chain_signal(const ChainArgs& ca, int slot0, int s_lo, int s_hi) {
  __syncthreads();
  if (threadIdx.x == 0 && s_lo <= s_hi) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (int st = s_lo; st <= s_hi; ++st)
      __hip_atomic_fetch_add(ca.cnt + slot0 + st, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// forward step over one or two 64-column chunks of a supernode (nb <= 128),
// split by chunk over the workgroups (flags bit 1: the second chunk). With
// inv(L_DD) = [V0 0; W V1] (the stored inverses of the chunks' diagonal
// tiles and the off-diagonal block formed after the factorization), a
// workgroup of the first chunk forms x_A = V0 y_A, one of the second x_B =
// W y_A + V1 y_B, redundantly (x stored into z by the half's writer, flags
// bit 0), then y(rows r0..r1 of the supernode) -= L(rows, its chunk) x_chunk
// in blocks of 64 rows (the next block's entries loaded during the current
// one): wave g sums columns 16g..16g+15 of a row, the four partial sums meet
// in LDS; plainly for own rows of a one-chunk step, else with atomics (the
// other chunk's workgroups and other supernodes add too)
__global__ __launch_bounds__(256) void k_fwd_step(const SolveTile* __restrict__ tiles,
                                                  const int32_t* __restrict__ gl,
                                                  const double* __restrict__ L,
                                                  double* __restrict__ y, double* __restrict__ z,
                                                  int nrhs, int64_t ldy, ChainArgs ca) {
  const SolveTile t = tiles[chain_tile(ca)];
  const bool chained = ca.tick && t.cslot >= 0;
  const int tid = threadIdx.x, row = tid & 63, cg = tid >> 6;
  const double* Lj = L + t.off;
  const int64_t ld = t.ld;
  const int nbA = min(t.nb, 64), nbB = t.nb - nbA;
  const int half = (t.flags >> 1) & 1;
  const int cc = t.c0 + 64 * half;          // first column of this workgroup's chunk
  const int nbc = half ? nbB : nbA;         // its width
  __shared__ double V0[64 * VP];  // this chunk's inverse
  __shared__ double W[64 * VP];   // second chunk: the off-diagonal inverse block; then the partial sums
  // y of the step's columns [r][128] and x of the chunk [r][64], sized by
  // nrhs at launch
  extern __shared__ double fwd_dyn[];
  double* const ys = fwd_dyn;
  double* const xs = fwd_dyn + 128 * nrhs;
  // this thread's 16 entries of its row of a 64-row block (and the row's
  // index in the full vector), loaded ahead
  double l[16];
  int gq;
  auto load_rows = [&](int q0) {
    const int q = q0 + row;
    const int qq = min(q, t.ld - 1);
    gq = gl[t.gl + min(q, t.r1 - 1)];
#pragma unroll
    for (int c = 0; c < 16; ++c) l[c] = Lj[(int64_t)(cc + min(16 * cg + c, nbc - 1)) * ld + qq];
  };
  load_rows(t.r0);
  stage_inv(V0, Lj, ld, cc, nbc, tid);
  if (half) stage_w(W, Lj, ld, t.c0, nbB, tid);
  // the step's right-hand side is final once every earlier step's rows are in
  if (chained) chain_wait(ca, t.cslot + t.c0 / CHAIN_STEP);
  for (int e = tid; e < 128 * nrhs; e += 256) {
    const int i = e & 127, r = e >> 7;
    ys[r * 128 + i] = i < t.nb ? y[(int64_t)r * ldy + t.f + t.c0 + i] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * nrhs; e += 256) {
    const int i = e & 63, r = e >> 6;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
    for (int j = 0; j < 64; j += 2) {
      a0 += V0[i * VP + j] * ys[r * 128 + 64 * half + j];
      a1 += V0[i * VP + j + 1] * ys[r * 128 + 64 * half + j + 1];
    }
    if (half) {
#pragma unroll 8
      for (int j = 0; j < 64; j += 2) {
        a0 += W[i * VP + j] * ys[r * 128 + j];
        a1 += W[i * VP + j + 1] * ys[r * 128 + j + 1];
      }
    }
    xs[r * 64 + i] = a0 + a1;
  }
  __syncthreads();
  if (t.flags & 1)
    for (int e = tid; e < 64 * nrhs; e += 256) {
      const int i = e & 63, r = e >> 6;
      if (i < nbc) z[(int64_t)r * ldy + t.f + cc + i] = xs[r * 64 + i];
    }
  double* part = W;  // [cg][r][row], 4 * nrhs * 64 <= 64 * VP doubles
  for (int q0 = t.r0; q0 < t.r1; q0 += 64) {
    const int q = q0 + row, gqb = gq;
    double lb[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) lb[c] = l[c];
    if (q0 + 64 < t.r1) load_rows(q0 + 64);
    for (int r = 0; r < nrhs; ++r) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int c = 0; c < 16; c += 2) {
        a0 += lb[c] * xs[r * 64 + 16 * cg + c];  // xs is 0 beyond the chunk
        a1 += lb[c + 1] * xs[r * 64 + 16 * cg + c + 1];
      }
      part[(cg * nrhs + r) * 64 + row] = a0 + a1;
    }
    __syncthreads();
    if (q < t.r1)
      for (int r = cg; r < nrhs; r += 4) {
        const double acc = (part[(0 * nrhs + r) * 64 + row] + part[(1 * nrhs + r) * 64 + row]) +
                           (part[(2 * nrhs + r) * 64 + row] + part[(3 * nrhs + r) * 64 + row]);
        if (q < t.w && nbB == 0 && !ca.tick)
          y[(int64_t)r * ldy + gqb] -= acc;
        else
          atomicAdd(&y[(int64_t)r * ldy + gqb], -acc);
      }
    __syncthreads();  // the block's partial sums are read before the next block's
  }
  if (chained && t.r0 < t.w) {
    // the later steps of the supernode whose columns these rows are
    const int s_lo = max(t.r0 / CHAIN_STEP, t.c0 / CHAIN_STEP + 1);
    chain_signal(ca, t.cslot, s_lo, (min(t.r1, t.w) - 1) / CHAIN_STEP);
  }
}

// backward, ancestor rows: z(chunk columns) -= L(rows r0..r1, chunk)^T x(glbind rows),
// 64-row blocks staged in LDS (the next block's loads in flight), added atomically
__global__ __launch_bounds__(256) void k_bwd_below(const SolveTile* __restrict__ tiles,
                                                   const int32_t* __restrict__ gl,
                                                   const double* __restrict__ L,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ z, int nrhs,
                                                   int64_t ldy) {
  const SolveTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x, row = tid & 63, cg = tid >> 6;
  const double* Lj = L + t.off;
  const int64_t ld = t.ld;
  __shared__ double Lb[64][VP];      // Lb[row][col] = L(q0 + row, c0 + col)
  __shared__ double xr[MAXRHS][64];  // x of the block's rows
  double acc[MAXRHS / 4];
#pragma unroll
  for (int s = 0; s < MAXRHS / 4; ++s) acc[s] = 0.0;
  double v[16], xv[MAXRHS / 4];
  auto fetch = [&](int q0) {
    const int nrow = min(64, t.r1 - q0);
    const int qq = q0 + min(row, nrow - 1);
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = Lj[(int64_t)(t.c0 + min(cg + 4 * s, t.nb - 1)) * ld + qq];
    const int gq = gl[t.gl + qq];
#pragma unroll
    for (int s = 0; s < MAXRHS / 4; ++s) {
      const int r = cg + 4 * s;
      xv[s] = r < nrhs ? x[(int64_t)r * ldy + gq] : 0.0;
    }
  };
  fetch(t.r0);
  for (int q0 = t.r0; q0 < t.r1; q0 += 64) {
    const int nrow = min(64, t.r1 - q0);
#pragma unroll
    for (int s = 0; s < 16; ++s) Lb[row][cg + 4 * s] = (row < nrow && cg + 4 * s < t.nb) ? v[s] : 0.0;
#pragma unroll
    for (int s = 0; s < MAXRHS / 4; ++s) xr[cg + 4 * s][row] = row < nrow ? xv[s] : 0.0;
    __syncthreads();
    if (q0 + 64 < t.r1) fetch(q0 + 64);
#pragma unroll
    for (int s = 0; s < MAXRHS / 4; ++s) {
      const int r = cg + 4 * s;
      if (r < nrhs) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
        for (int i = 0; i < 64; i += 2) {
          a0 += Lb[i][row] * xr[r][i];
          a1 += Lb[i + 1][row] * xr[r][i + 1];
        }
        acc[s] += a0 + a1;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < MAXRHS / 4; ++s) {
    const int r = cg + 4 * s;
    if (r < nrhs && row < t.nb) atomicAdd(&z[(int64_t)r * ldy + t.f + t.c0 + row], -acc[s]);
  }
}

// backward step over one or two 64-column chunks (nb <= 128), split by
// chunk over the workgroups (flags bit 1: the second chunk): with
// inv(L_DD)^T = [V0^T W^T; 0 V1^T], a workgroup of the first chunk forms x_A
// = V0^T z_A + W^T z_B, one of the second x_B = V1^T z_B, redundantly (x
// stored by the half's writer, flags bit 0), then z(columns r0..r1) -=
// L(its chunk's rows, r0..r1)^T x_chunk for one earlier 64-column chunk,
// with atomics when the step has two chunks
__global__ __launch_bounds__(256) void k_bwd_step(const SolveTile* __restrict__ tiles,
                                                  const double* __restrict__ L,
                                                  double* __restrict__ z, double* __restrict__ x,
                                                  int nrhs, int64_t ldy, ChainArgs ca) {
  const SolveTile t = tiles[chain_tile(ca)];
  const bool chained = ca.tick && t.cslot >= 0;
  const int tid = threadIdx.x, row = tid & 63, cg = tid >> 6;
  const double* Lj = L + t.off;
  const int64_t ld = t.ld;
  const bool push = t.r1 > t.r0;
  const int nbA = min(t.nb, 64), nbB = t.nb - nbA;
  const int half = (t.flags >> 1) & 1;
  const int cc = t.c0 + 64 * half;
  const int nbc = half ? nbB : nbA;
  __shared__ double V[64 * VP];
  __shared__ double W[64 * VP];  // first chunk of a two-chunk step: the off-diagonal block
  __shared__ double Lb[64][VP];  // Lb[i][c] = L(cc + i, r0 + c)
  __shared__ double zs[MAXRHS][128];
  __shared__ double xs[MAXRHS][64];
  if (push) {
    double v[16];
    const int ii = min(row, nbc - 1);
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = Lj[(int64_t)(t.r0 + cg + 4 * s) * ld + cc + ii];
#pragma unroll
    for (int s = 0; s < 16; ++s) Lb[row][cg + 4 * s] = row < nbc ? v[s] : 0.0;
  }
  stage_inv(V, Lj, ld, cc, nbc, tid);
  if (!half && nbB > 0) stage_w(W, Lj, ld, t.c0, nbB, tid);
  // the step's columns are final once every later step has pushed into them
  if (chained) chain_wait(ca, t.cslot + t.c0 / CHAIN_STEP);
  for (int e = tid; e < 128 * nrhs; e += 256) {
    const int i = e & 127, r = e >> 7;
    zs[r][i] = i < t.nb ? z[(int64_t)r * ldy + t.f + t.c0 + i] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * nrhs; e += 256) {
    const int i = e & 63, r = e >> 6;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
    for (int m = 0; m < 64; m += 2) {
      a0 += V[m * VP + i] * zs[r][64 * half + m];
      a1 += V[(m + 1) * VP + i] * zs[r][64 * half + m + 1];
    }
    if (!half && nbB > 0) {
#pragma unroll 8
      for (int m = 0; m < 64; m += 2) {
        a0 += W[m * VP + i] * zs[r][64 + m];
        a1 += W[(m + 1) * VP + i] * zs[r][64 + m + 1];
      }
    }
    xs[r][i] = a0 + a1;
  }
  __syncthreads();
  if (t.flags & 1)
    for (int e = tid; e < 64 * nrhs; e += 256) {
      const int i = e & 63, r = e >> 6;
      if (i < nbc) x[(int64_t)r * ldy + t.f + cc + i] = xs[r][i];
    }
  if (push)
    for (int e = tid; e < 64 * nrhs; e += 256) {
      const int c = e & 63, r = e >> 6;
      double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
      for (int i = 0; i < 64; i += 2) {
        a0 += Lb[i][c] * xs[r][i];
        a1 += Lb[i + 1][c] * xs[r][i + 1];
      }
      double* p = &z[(int64_t)r * ldy + t.f + t.r0 + c];
      if (nbB > 0 || ca.tick)
        atomicAdd(p, -(a0 + a1));
      else
        *p -= a0 + a1;
    }
  if (chained && push) chain_signal(ca, t.cslot, t.r0 / CHAIN_STEP, t.r0 / CHAIN_STEP);
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
// r[:, k] = b[:, k] - A x[:, k] (b may be null: r = -A x) for up to MAXRHS
// columns: one thread per row reads the row's entries once and sums every
// column, entries in CSR order
__global__ __launch_bounds__(256) void k_residual(int64_t n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const int64_t* __restrict__ src,
                                                  const double* __restrict__ vals,
                                                  const double* __restrict__ x, int64_t ldx,
                                                  const double* __restrict__ b, int64_t ldb,
                                                  double* __restrict__ r, int64_t ldr, int nrhs) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double acc[MAXRHS];
#pragma unroll
  for (int q = 0; q < MAXRHS; ++q) acc[q] = 0.0;
  const int64_t e1 = rp[row + 1];
  for (int64_t e = rp[row]; e < e1; ++e) {
    const double a = vals[src[e]];
    const int64_t c = ci[e];
#pragma unroll
    for (int q = 0; q < MAXRHS; ++q)
      if (q < nrhs) acc[q] += a * x[q * ldx + c];
  }
#pragma unroll
  for (int q = 0; q < MAXRHS; ++q)
    if (q < nrhs) r[q * ldr + row] = (b ? b[q * ldb + row] : 0.0) - acc[q];
}

// out[k] = sum_i x[i + k*ldx] * y[i + k*ldy]: one workgroup per column, the
// terms summed in a fixed order (repeated calls give the same bits)
__global__ void k_dot_cols(const double* __restrict__ x, int64_t ldx, const double* __restrict__ y,
                           int64_t ldy, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.y;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += x[k * ldx + i] * y[k * ldy + i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

// y[:, k] = a[k] * x[:, k] + b[k] * y[:, k]
__global__ void k_axpby_cols(double* __restrict__ y, int64_t ldy, const double* __restrict__ x,
                             int64_t ldx, int64_t n, int nrhs, ColCoef a, ColCoef b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t row = i % n, k = i / n;
  y[k * ldy + row] = a.v[k] * x[k * ldx + row] + b.v[k] * y[k * ldy + row];
}

// largest m over a 256-thread workgroup, to thread 0 (m >= 0 everywhere)
__device__ __forceinline__ double block_max256(double m) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// out[k] = max(out[k], max_i |v[i + k*ld]|) via the ordering of non-negative
// doubles as unsigned integers; one atomic per workgroup
__global__ __launch_bounds__(256) void k_absmax(const double* __restrict__ v, int64_t n,
                                                int64_t ld, int nrhs,
                                                unsigned long long* __restrict__ out) {
  const int k = blockIdx.y;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(v[k * ld + i]));
  m = block_max256(m);
  if (threadIdx.x == 0) atomicMax(out + k, (unsigned long long)__double_as_longlong(m));
}

// infinity norm of A: max over rows of sum |a_ij|; one atomic per workgroup
__global__ __launch_bounds__(256) void k_anorm(int64_t n, const int64_t* __restrict__ rp,
                                               const int64_t* __restrict__ src,
                                               const double* __restrict__ vals,
                                               unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s += fabs(vals[src[e]]);
    m = fmax(m, s);
  }
  m = block_max256(m);
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
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
void launch_init_status(int* status, int count, int* counters, int ncounters, hipStream_t st) {
  hipLaunchKernelGGL(k_init_status, dim3(grid_for(std::max(count, ncounters), 256)), dim3(256), 0,
                     st, status, count, counters, ncounters);
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
template <int NBB, bool PRE>
static void launch_panel_n(const PanelTile* tiles, int64_t count, double* L, int* status,
                           int* counters, int mode, const double* thr,
                           const unsigned long long* amax, double ufix, unsigned long long* smax,
                           unsigned int* nfixed, const UpdTile* utiles, const UpdSeg* usegs,
                           int64_t ucount, float* Ls, hipStream_t st) {
  const int np = (int)count;
  const dim3 b(256);
  if (mode == 0)
    hipLaunchKernelGGL((k_panel<0, NBB, PRE>), dim3((unsigned)(count + ucount)), b, 0, st, tiles,
                       L, status, counters, thr, amax, ufix, smax, nfixed, utiles, usegs, np, Ls);
  else if (mode == 1)
    hipLaunchKernelGGL((k_panel<1, NBB, PRE>), dim3((unsigned)(count + ucount)), b, 0, st, tiles,
                       L, status, counters, thr, amax, ufix, smax, nfixed, utiles, usegs, np, Ls);
  else
    hipLaunchKernelGGL((k_panel<2, NBB, PRE>), dim3((unsigned)count), b, 0, st, tiles, L, status,
                       counters, thr, amax, ufix, smax, nfixed, utiles, usegs, np, Ls);
}
void launch_panel(const PanelTile* tiles, int64_t count, double* L, int* status, int* counters,
                  int precision, int nbb, bool pre, const double* thr,
                  const unsigned long long* amax, double ufix, unsigned long long* smax,
                  unsigned int* nfixed, const UpdTile* utiles, const UpdSeg* usegs,
                  int64_t ucount, hipStream_t st, float* Ls, int64_t wave_min) {
  if (count <= 0) return;
  if (precision == 2 || nbb < 4) ucount = 0;  // (the plan fuses into 64-column launches only)
  if (precision == 0 && nbb <= 1 && !pre && count >= wave_min) {
    // many small column blocks (as in a batch's merged launches): one
    // wavefront per group member
    hipLaunchKernelGGL(k_panel_w, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, st, tiles, L,
                       status, counters, (int)count);
    return;
  }
#define RLB_PANEL_N(N, P)                                                                       \
  launch_panel_n<N, P>(tiles, count, L, status, counters, precision, thr, amax, ufix, smax, nfixed, \
                       utiles, usegs, ucount, Ls, st)
  if (nbb <= 1) {
    if (pre) RLB_PANEL_N(1, true);
    else RLB_PANEL_N(1, false);
  } else if (nbb == 2) {
    if (pre) RLB_PANEL_N(2, true);
    else RLB_PANEL_N(2, false);
  } else {
    if (pre) RLB_PANEL_N(4, true);
    else RLB_PANEL_N(4, false);
  }
#undef RLB_PANEL_N
}
void launch_tile_inverse(const DiagTile* tiles, int64_t count, int nbb, double* L,
                         hipStream_t st) {
  if (count <= 0) return;
  const dim3 g((unsigned)count), b(256);
  if (nbb <= 1)
    hipLaunchKernelGGL(k_tile_inverse_w, dim3((unsigned)((count + 3) / 4)), b, 0, st, tiles, L,
                       (int)count);
  else if (nbb == 2)
    hipLaunchKernelGGL(k_tile_inverse<2>, g, b, 0, st, tiles, L);
  else
    hipLaunchKernelGGL(k_tile_inverse<4>, g, b, 0, st, tiles, L);
}
void launch_update(const UpdTile* tiles, const UpdSeg* segs, int64_t count, double* L,
                   int precision, const unsigned long long* smax, int variant, hipStream_t st,
                   int64_t nwave, const float* Ls, int64_t wave_min) {
  if (count <= 0) return;
  if (variant == UPD_TALL) {
    // 128x64 target tiles, FP64 (the other forms run the same work from its
    // 64x64 tiling)
    hipLaunchKernelGGL(k_update_tall, dim3((unsigned)count), dim3(512), 0, st, tiles, segs, L);
    return;
  }
  if (variant == UPD_BIG) {
    // 128x128 target tiles: FP64 or FP32 operands (the 16-bit forms run the
    // same work from its 64x64 tiling)
    if (precision == 1)
      hipLaunchKernelGGL(k_update_big<float>, dim3((unsigned)count), dim3(256), 0, st, tiles, segs,
                         L, Ls);
    else
      hipLaunchKernelGGL(k_update_big<double>, dim3((unsigned)count), dim3(256), 0, st, tiles,
                         segs, L, (const double*)L);
    return;
  }
  const bool shortk = variant == UPD_SHORT;
  const bool win = variant == UPD_TILE_WIN;
  const int xcd = variant == UPD_TILE_XCD ? 1 : 0;
  if (precision == 0 && nwave >= wave_min) {
    // the last nwave tiles are narrow: one wavefront each (a launch of its
    // own pays off for many of them, as in the merged launches of a batch)
    const int64_t nw = std::min(nwave, count);
    hipLaunchKernelGGL(k_update_w, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, st,
                       tiles + (count - nw), segs, L, (int)nw);
    count -= nw;
    if (count <= 0) return;
  }
  const dim3 g((unsigned)count), b(256);
  if (shortk && precision <= 1) {
    if (precision == 1)
      hipLaunchKernelGGL(k_update_short<float>, g, b, 0, st, tiles, segs, L, Ls);
    else
      hipLaunchKernelGGL(k_update_short<double>, g, b, 0, st, tiles, segs, L, (const double*)L);
  } else if (precision == 1)
    // (the FP32 form stays with the dense kernel: its 32-deep chunks already
    // halve the rounds, and the windows measured slower there)
    hipLaunchKernelGGL(k_update<float>, g, b, 0, st, tiles, segs, L, Ls, (int)count, xcd);
  else if (precision == 2)
    hipLaunchKernelGGL(k_update16<2>, g, b, 0, st, tiles, segs, L, smax);
  else if (precision == 3)
    hipLaunchKernelGGL(k_update16<3>, g, b, 0, st, tiles, segs, L, smax);
  else if (win)
    hipLaunchKernelGGL(k_update_win<double>, g, b, 0, st, tiles, segs, L, (const double*)L,
                       (int)count, 0);
  else if (variant == UPD_TILE_PACK)
    hipLaunchKernelGGL(k_update_pack, g, b, 0, st, tiles, segs, L);
  else
    hipLaunchKernelGGL(k_update<double>, g, b, 0, st, tiles, segs, L, (const double*)L,
                       (int)count, xcd);
}
void launch_part_reduce(const PartReduce* recs, int64_t count, double* L, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_part_reduce, dim3((unsigned)count), dim3(256), 0, st, recs, L);
}
void launch_assemble(const AsmCol* cols, int64_t count, const int32_t* rows, double* L,
                     hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, st, cols, rows,
                     L, (int)count);
}
// pivot thresholds of the reduced-precision forms: thr[j] = u * A_jj, and the
// largest diagonal entry (bit pattern; all positive on an SPD input)
__global__ void k_pivthr(const double* __restrict__ vals, const int64_t* __restrict__ dsrc,
                         int64_t n, double u, double* __restrict__ thr,
                         unsigned long long* __restrict__ amax) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double a = vals[dsrc[j]];
  thr[j] = u * a;
  if (a > 0.0) atomicMax(amax, (unsigned long long)__double_as_longlong(a));
}
void launch_pivthr(const double* vals, const int64_t* dsrc, int64_t n, double u, double* thr,
                   unsigned long long* amax, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pivthr, dim3(grid_for(n, 256, INT32_MAX)), dim3(256), 0, st, vals, dsrc,
                     n, u, thr, amax);
}
void launch_pair_inverse(const DiagTile* tiles, int64_t count, double* L, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_pair_inverse, dim3((unsigned)count), dim3(256), 0, st, tiles, L);
}
void launch_fwd_step(const SolveTile* tiles, int64_t count, const int32_t* gl, const double* L,
                     double* y, double* z, int nrhs, int64_t ldy, hipStream_t st, ChainArgs ca) {
  if (count <= 0) return;
  const size_t dyn = sizeof(double) * (128 + 64) * (size_t)nrhs;
  hipLaunchKernelGGL(k_fwd_step, dim3((unsigned)count), dim3(256), dyn, st, tiles, gl, L, y, z,
                     nrhs, ldy, ca);
}
void launch_bwd_below(const SolveTile* tiles, int64_t count, const int32_t* gl, const double* L,
                      const double* x, double* z, int nrhs, int64_t ldy, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_bwd_below, dim3((unsigned)count), dim3(256), 0, st, tiles, gl, L, x, z,
                     nrhs, ldy);
}
void launch_bwd_step(const SolveTile* tiles, int64_t count, const double* L, double* z, double* x,
                     int nrhs, int64_t ldy, hipStream_t st, ChainArgs ca) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_bwd_step, dim3((unsigned)count), dim3(256), 0, st, tiles, L, z, x, nrhs,
                     ldy, ca);
}
__global__ void k_zero_i32(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
void launch_zero_i32(int* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, (int)n);
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
  if (n <= 0) return;
  for (int c0 = 0; c0 < nrhs; c0 += MAXRHS) {
    const int nr = std::min(MAXRHS, nrhs - c0);
    hipLaunchKernelGGL(k_residual, dim3(grid_for(n, 256, INT32_MAX)), dim3(256), 0, st, n, rp, ci,
                       src, vals, x + c0 * ldx, ldx, b ? b + c0 * ldb : nullptr, ldb, r + c0 * ldr,
                       ldr, nr);
  }
}
void launch_absmax(const double* v, int64_t n, int64_t ld, int nrhs, unsigned long long* out,
                   hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(n, 256, 128), nrhs), dim3(256), 0, st, v, n, ld,
                     nrhs, out);
}
void launch_anorm(int64_t n, const int64_t* rp, const int64_t* src, const double* vals,
                  unsigned long long* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_anorm, dim3(grid_for(n, 256, 256)), dim3(256), 0, st, n, rp, src, vals,
                     out);
}
void launch_dot_cols(const double* x, int64_t ldx, const double* y, int64_t ldy, int64_t n,
                     int nrhs, double* out, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_dot_cols, dim3(1, nrhs), dim3(256), 0, st, x, ldx, y, ldy, n, out);
}
void launch_axpby_cols(double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, int nrhs,
                       const ColCoef& a, const ColCoef& b, hipStream_t st) {
  int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_axpby_cols, dim3(grid_for(tot, 256, INT32_MAX)), dim3(256), 0, st, y, ldy,
                     x, ldx, n, nrhs, a, b);
}
void launch_axpy(double* x, int64_t ldx, const double* d, int64_t ldd, int64_t n, int nrhs,
                 hipStream_t st) {
  int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(tot, 256, INT32_MAX)), dim3(256), 0, st, x, ldx, d,
                     ldd, n, nrhs);
}

}  // namespace rlb
