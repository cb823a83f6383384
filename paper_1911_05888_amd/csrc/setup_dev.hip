// Device part of the setup (K7): the element diagonal blocks A_EE of a
// smoothed level and their explicit inverses, written straight into the
// smoother's symmetric tile layout.  Section 3 precomputes a factorisation of
// every diagonal block; here each block is equilibrated with
// D = diag(|A_jj|^{-1/2}) and inverted in FP64 by Gauss-Jordan elimination
// with partial pivoting (row exchanges, columns unscrambled at the end), then
// inv(A) = D inv(D A D) D.
//
// The blocks themselves come from the element operator the smoother
// evaluates: for one colour (no two of its elements coupled), x = e_j on
// every element of the colour and zero elsewhere gives, for each such E,
// (b - A x)_E = -A_EE e_j with b = 0, i.e. column j of A_EE.  The caller runs
// the colour residual n_b times; the kernels here place the unit vectors and
// collect the columns.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ldgs_internal.hpp"

namespace ldgs {

namespace {

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : 1; }

// x_E[j] = 1 and x_E[j-1] = 0 (the previous unit vector) for the listed elements
__global__ void k_set_unit(int cnt, const int* __restrict__ elems, int nb, int j, double* __restrict__ x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    double* xe = x + (size_t)elems[i] * nb;
    if (j > 0) xe[j - 1] = 0.0;
    if (j < nb) xe[j] = 1.0;
  }
}

// column j of every block, stored as row j: A[i][j][row] = -r[i][row].  The
// blocks are thus kept transposed; only the symmetric part of the inverse is
// used, and that of inv(A^T) = inv(A)^T is the same.
__global__ void k_take_column(int cnt, int nb, int j, const double* __restrict__ r, double* __restrict__ A) {
  const int64_t n = (int64_t)cnt * nb;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / nb, row = t - i * nb;
    A[(i * nb + j) * nb + row] = -r[t];
  }
}

// Gauss-Jordan layout: the block's NB rows over the work-group, each row cut
// into S segments of CW consecutive columns held in registers by one thread.
template <int NB>
struct Gj {
  static constexpr int S0 = 256 / NB;
  static constexpr int CW = (NB + S0 - 1) / S0;      // columns per thread
  static constexpr int S = (NB + CW - 1) / CW;       // segments per row
  static constexpr int NT = NB * S;                  // active threads
  static_assert(NT <= 256, "block too large for one work-group");
};

// In-place inverse of nblk row-major NB x NB blocks (FP64).  nsing counts the
// blocks whose equilibrated 1-norm condition estimate exceeds 1e14 (or whose
// diagonal has a zero); their output is not usable.
template <int NB>
__global__ __launch_bounds__(256) void k_block_inverse(int nblk, double* __restrict__ A, int* __restrict__ nsing) {
  using C = Gj<NB>;
  __shared__ double colv[NB];      // column k of the current matrix
  __shared__ double rowk[NB];      // the pivot row, scaled
  __shared__ double swp[2][NB];    // the two rows of an exchange
  __shared__ double dsc[NB];       // equilibration
  __shared__ double csum[2][NB];   // column sums of |D A D| and of its inverse
  __shared__ int piv[NB];
  __shared__ int dest[NB];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int i = tid / C::S, sg = tid - i * C::S;
  const bool act = tid < C::NT;
  const int c0 = sg * C::CW;
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    double* Ab = A + (size_t)blk * NB * NB;
    double a[C::CW];
#pragma unroll
    for (int c = 0; c < C::CW; ++c) a[c] = (act && c0 + c < NB) ? Ab[(size_t)i * NB + c0 + c] : 0.0;
    if (tid == 0) bad = 0;
    if (tid < NB) {
      csum[0][tid] = 0.0;
      csum[1][tid] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < C::CW; ++c)
      if (act && c0 + c == i) dsc[i] = fabs(a[c]) > 0.0 ? 1.0 / sqrt(fabs(a[c])) : 0.0;
    __syncthreads();
    if (tid < NB && dsc[tid] == 0.0) bad = 1;
#pragma unroll
    for (int c = 0; c < C::CW; ++c)
      if (act && c0 + c < NB) {
        a[c] *= dsc[i] * dsc[c0 + c];
        atomicAdd(&csum[0][c0 + c], fabs(a[c]));
      }
    for (int k = 0; k < NB; ++k) {
      const int sk = k / C::CW;
      if (act && sg == sk) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < C::CW; ++c)
          if (c0 + c == k) v = a[c];
        colv[i] = v;
      }
      __syncthreads();
      // pivot row: largest |value| in column k among rows k..NB-1 (the
      // smallest row index on ties)
      if (tid < 64) {
        double best = -1.0;
        int bi = k;
        for (int r = k + tid; r < NB; r += 64) {
          const double v = fabs(colv[r]);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (tid == 0) piv[k] = bi;
      }
      __syncthreads();
      const int p = piv[k];
      const double pv = colv[p];
      if (p != k) {
        if (act && i == k)
#pragma unroll
          for (int c = 0; c < C::CW; ++c)
            if (c0 + c < NB) swp[0][c0 + c] = a[c];
        if (act && i == p)
#pragma unroll
          for (int c = 0; c < C::CW; ++c)
            if (c0 + c < NB) swp[1][c0 + c] = a[c];
        __syncthreads();
        if (act && i == k)
#pragma unroll
          for (int c = 0; c < C::CW; ++c)
            if (c0 + c < NB) a[c] = swp[1][c0 + c];
        if (act && i == p)
#pragma unroll
          for (int c = 0; c < C::CW; ++c)
            if (c0 + c < NB) a[c] = swp[0][c0 + c];
      }
      // column-k value of row i after the exchange
      const double mi = act ? ((i == p) ? colv[k] : colv[i]) : 0.0;
      const double ip = 1.0 / pv;
      if (act && i == k)
#pragma unroll
        for (int c = 0; c < C::CW; ++c)
          if (c0 + c < NB) {
            const double v = (c0 + c == k) ? ip : a[c] * ip;
            a[c] = v;
            rowk[c0 + c] = v;
          }
      __syncthreads();
      if (act && i != k)
#pragma unroll
        for (int c = 0; c < C::CW; ++c)
          if (c0 + c < NB) a[c] = (c0 + c == k) ? -mi * ip : a[c] - mi * rowk[c0 + c];
    }
    // undo the row exchanges on the columns, in reverse order
    if (tid == 0) {
      int at[NB];
      for (int j = 0; j < NB; ++j) at[j] = j;
      for (int k = NB - 1; k >= 0; --k) {
        const int t = at[k];
        at[k] = at[piv[k]];
        at[piv[k]] = t;
      }
      for (int j = 0; j < NB; ++j) dest[at[j]] = j;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C::CW; ++c)
      if (act && c0 + c < NB) {
        const int j = dest[c0 + c];
        atomicAdd(&csum[1][j], fabs(a[c]));
        Ab[(size_t)i * NB + j] = a[c] * dsc[i] * dsc[j];
      }
    __syncthreads();
    if (tid == 0) {
      double n0 = 0.0, n1 = 0.0;
      for (int j = 0; j < NB; ++j) {
        n0 = fmax(n0, csum[0][j]);
        n1 = fmax(n1, csum[1][j]);
      }
      if (bad || !(n0 * n1 < 1e14)) atomicAdd(nsing, 1);
    }
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ T cvt(double v);
template <>
__device__ __forceinline__ double cvt<double>(double v) { return v; }
template <>
__device__ __forceinline__ float cvt<float>(double v) { return (float)v; }
// bfloat16 by round-to-nearest-even of the FP32 value
template <>
__device__ __forceinline__ uint16_t cvt<uint16_t>(double v) {
  const float f = (float)v;
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// The symmetric part (A^-1 + A^-T) / 2 of each full inverse (row-major
// nb x nb) into the smoother's tile layout (SymTiles in ldgs_internal.hpp):
// thread = (block, tile, lane block (r, cb)), 4 entries each.
template <typename T>
__global__ void k_arrange_sym(int cnt, int nb, const double* __restrict__ inv, T* __restrict__ out, int64_t stride) {
  constexpr SymTiles L = sym_tiles(16, (int)sizeof(T));   // LB, EL, H depend on the width only
  const int TR = (nb + 15) / 16;
  const int ntile = TR * (TR + 1) / 2;
  const int64_t total = (int64_t)cnt * ntile * 64;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / (ntile * 64);
    const int rem = (int)(t - e * ntile * 64);
    const int tl = rem / 64, lb = rem - tl * 64;
    const int r = lb / 4, cb = lb % 4;
    // tile number tl -> (ti, tj), tj >= ti, and its offset
    int ti = 0, tj = 0, off = 0;
    for (int q = 0; q < tl; ++q) {
      off += (ti == tj ? SYM_DBLOCKS : 64) * 4;
      if (++tj == TR) tj = ++ti;
    }
    const bool diag = ti == tj;
    if (diag && cb < r / 4) continue;
    const int nblk = diag ? SYM_DBLOCKS : 64;
    const int slot = diag ? sym_dslot(r, cb) : 4 * r + cb;
    const double* M = inv + (size_t)e * nb * nb;
    T* o = out + (size_t)e * stride + off;
    const int row = 16 * ti + r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * tj + 4 * cb + v;
      const double s = (row < nb && col < nb) ? 0.5 * (M[(size_t)row * nb + col] + M[(size_t)col * nb + row]) : 0.0;
      const int h = v / L.EL, u = v % L.EL;
      o[((size_t)h * nblk + slot) * L.EL + u] = cvt<T>(s);
    }
  }
}

inline unsigned grid_for(int64_t n, int b, int64_t cap) {
  int64_t g = (n + b - 1) / b;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

int launch_set_unit(void* stream, int64_t cnt, const int* elems, int nb, int j, double* x) {
  if (cnt <= 0) return 0;
  hipLaunchKernelGGL(k_set_unit, dim3(grid_for(cnt, 256, 4096)), dim3(256), 0, (hipStream_t)stream, (int)cnt, elems,
                     nb, j, x);
  return ok();
}

int launch_take_column(void* stream, int64_t cnt, int nb, int j, const double* r, double* A) {
  if (cnt <= 0) return 0;
  hipLaunchKernelGGL(k_take_column, dim3(grid_for(cnt * nb, 256, 16384)), dim3(256), 0, (hipStream_t)stream,
                     (int)cnt, nb, j, r, A);
  return ok();
}

int launch_block_inverse(void* stream, int64_t nblk, int nb, double* A, int* nsing) {
  if (nblk <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const unsigned g = grid_for(nblk, 1, 65536);
  switch (nb) {
#define LDGS_GJ(NBV) \
  case NBV: hipLaunchKernelGGL((k_block_inverse<NBV>), dim3(g), dim3(256), 0, st, (int)nblk, A, nsing); break;
    LDGS_GJ(12) LDGS_GJ(27) LDGS_GJ(32) LDGS_GJ(48) LDGS_GJ(108)
#undef LDGS_GJ
    default: return 2;
  }
  return ok();
}

int launch_arrange_sym(void* stream, int64_t cnt, int nb, const double* inv, void* out, int bytes, int64_t stride) {
  if (cnt <= 0) return 0;
  const int TR = (nb + 15) / 16;
  const int64_t n = cnt * (int64_t)(TR * (TR + 1) / 2) * 64;
  const dim3 g(grid_for(n, 256, 65536)), b(256);
  hipStream_t st = (hipStream_t)stream;
  if (bytes == 8) hipLaunchKernelGGL((k_arrange_sym<double>), g, b, 0, st, (int)cnt, nb, inv, (double*)out, stride);
  else if (bytes == 4) hipLaunchKernelGGL((k_arrange_sym<float>), g, b, 0, st, (int)cnt, nb, inv, (float*)out, stride);
  else if (bytes == 2)
    hipLaunchKernelGGL((k_arrange_sym<uint16_t>), g, b, 0, st, (int)cnt, nb, inv, (uint16_t*)out, stride);
  else return 2;
  return ok();
}

}  // namespace ldgs
