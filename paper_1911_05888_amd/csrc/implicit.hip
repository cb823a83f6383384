// Kernels of the V-cycle on implicitly defined meshes, where every level is
// held as explicit element blocks (block-sparse rows, nb x nb blocks stored
// column-major): the multicoloured block Gauss-Seidel pass of section 3,
// x_E += A_EE^{-1} (b_E - sum_F A_EF x_F) for the elements of one colour,
// the residual b - A x, and the transfers (injection of section 3 and its
// transpose).
//
// The pass streams the row's blocks from HBM once: one wavefront per element,
// the block columns split between the two halves of the wavefront (nb <= 32)
// so that every load instruction reads two whole columns (2 nb contiguous
// values), each lane accumulating one row; the halves are summed with one
// cross-half shuffle.  The row's blocks are the dominant bytes (about seven
// blocks of nb^2 values per element for the viscous-stress stencil); the
// neighbours' x vectors are staged in LDS with coalesced loads and read back
// as broadcasts.
#include <hip/hip_runtime.h>

#include "implicit.hpp"

namespace ldgs {
namespace {

template <int NB>
struct RowMap {
  static constexpr int H = NB <= 32 ? 2 : 1;        // column interleave
  static constexpr int NC = (NB + H - 1) / H;       // columns per lane
};

// sum_F A_EF s_F x_F for row entry r of element E (valid in lanes r < NB of
// every half); s_F = (alpha, beta)-type column scaling when ds != nullptr.
// The x vectors of up to KS blocks of the row are staged in LDS (coalesced
// loads of whole vectors, the scaling applied there), then the blocks are
// streamed two at a time with all their loads issued before the
// multiply-adds; x is read back from LDS as broadcasts.
constexpr int KS = 8;

template <typename T, int NB>
__device__ __forceinline__ void block_terms(const T* __restrict__ B, const T* __restrict__ xs, int half, int r,
                                            T& acc) {
  using RM = RowMap<NB>;
  T a[RM::NC];
#pragma unroll
  for (int cc = 0; cc < RM::NC; ++cc) {
    const int c = RM::H * cc + half;
    a[cc] = c < NB ? B[c * NB + r] : (T)0;
  }
#pragma unroll
  for (int cc = 0; cc < RM::NC; ++cc) {
    const int c = RM::H * cc + half;
    if (c < NB) acc += a[cc] * xs[c];
  }
}

template <typename T, int NB>
__device__ __forceinline__ T block_row(const int* __restrict__ rowptr, const int* __restrict__ cols,
                                       const T* __restrict__ blk, const T* __restrict__ x, int E, int lane,
                                       const double* __restrict__ ds, T (*xs)[NB]) {
  using RM = RowMap<NB>;
  constexpr int NVEL = 2 * NB / 3;
  const int half = RM::H == 2 ? (lane >> 5) : 0;
  const int r = RM::H == 2 ? (lane & 31) : lane;
  const int rr = r < NB ? r : NB - 1;        // idle lanes read a valid row and discard it
  T acc = (T)0, acc2 = (T)0;
  const int k0 = rowptr[E], k1 = rowptr[E + 1];
  for (int kb = k0; kb < k1; kb += KS) {
    const int kn = min(KS, k1 - kb);
    for (int t = lane; t < kn * NB; t += 64) {
      const int jb = t / NB, c = t - jb * NB;
      const int F = cols[kb + jb];
      T v = x[(size_t)F * NB + c];
      if (ds) v *= (T)ds[2 * F + (c < NVEL ? 0 : 1)];
      xs[jb][c] = v;
    }
    __syncthreads();
    int jb = 0;
    for (; jb + 1 < kn; jb += 2) {
      block_terms<T, NB>(blk + (size_t)(kb + jb) * NB * NB, xs[jb], half, rr, acc);
      block_terms<T, NB>(blk + (size_t)(kb + jb + 1) * NB * NB, xs[jb + 1], half, rr, acc2);
    }
    if (jb < kn) block_terms<T, NB>(blk + (size_t)(kb + jb) * NB * NB, xs[jb], half, rr, acc);
    __syncthreads();
  }
  acc += acc2;
  if constexpr (RM::H == 2) acc += __shfl_xor(acc, 32);
  return acc;
}

template <typename T, int NB>
__global__ __launch_bounds__(64) void k_bsr_colour(int nelem, const int* __restrict__ elems,
                                                   const int* __restrict__ rowptr, const int* __restrict__ cols,
                                                   const T* __restrict__ blk, const T* __restrict__ inv,
                                                   const T* __restrict__ b, T* __restrict__ x) {
  using RM = RowMap<NB>;
  const int idx = blockIdx.x;
  if (idx >= nelem) return;
  const int lane = threadIdx.x;
  const int E = elems[idx];
  __shared__ T rv[NB];
  __shared__ T xs[KS][NB];
  const T ax = block_row<T, NB>(rowptr, cols, blk, x, E, lane, nullptr, xs);
  if (lane < NB) rv[lane] = b[(size_t)E * NB + lane] - ax;
  __syncthreads();
  const int half = RM::H == 2 ? (lane >> 5) : 0;
  const int r = RM::H == 2 ? (lane & 31) : lane;
  T y = (T)0;
  if (r < NB) {
    const T* Ai = inv + (size_t)E * NB * NB;
#pragma unroll
    for (int cc = 0; cc < RM::NC; ++cc) {
      const int c = RM::H * cc + half;
      if (c < NB) y += Ai[c * NB + r] * rv[c];
    }
  }
  if constexpr (RM::H == 2) y += __shfl_xor(y, 32);
  if (lane < NB) x[(size_t)E * NB + lane] += y;
}

// r = b - S A S x (b null: r = S A S x), S = diag of the per-element pairs ds
// (velocity, pressure) or the identity
template <typename T, int NB>
__global__ __launch_bounds__(64) void k_bsr_residual(int ne, const int* __restrict__ rowptr,
                                                     const int* __restrict__ cols, const T* __restrict__ blk,
                                                     const T* __restrict__ b, const T* __restrict__ x,
                                                     T* __restrict__ out, const double* __restrict__ ds) {
  constexpr int NVEL = 2 * NB / 3;
  const int E = blockIdx.x;
  if (E >= ne) return;
  const int lane = threadIdx.x;
  __shared__ T xs[KS][NB];
  T ax = block_row<T, NB>(rowptr, cols, blk, x, E, lane, ds, xs);
  if (lane < NB) {
    if (ds) ax *= (T)ds[2 * E + (lane < NVEL ? 0 : 1)];
    out[(size_t)E * NB + lane] = b ? b[(size_t)E * NB + lane] - ax : ax;
  }
}

// b_c[C, f, a] = sum_{children g of C} sum_b I_g[b][a] r[g, f, b]
template <typename T, int NQ>
__global__ __launch_bounds__(256) void k_bsr_restrict(int nc, const int* __restrict__ kid_ptr,
                                                      const int* __restrict__ kids, const T* __restrict__ I,
                                                      const T* __restrict__ r, T* __restrict__ bc) {
  constexpr int NB = 3 * NQ;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nc * NB) return;
  const int C = (int)(t / NB), row = (int)(t % NB);
  const int f = row / NQ, a = row % NQ;
  T s = (T)0;
  for (int k = kid_ptr[C]; k < kid_ptr[C + 1]; ++k) {
    const int g = kids[k];
    const T* Ig = I + (size_t)g * NQ * NQ;
    const T* rg = r + (size_t)g * NB + f * NQ;
#pragma unroll
    for (int bb = 0; bb < NQ; ++bb) s += Ig[bb * NQ + a] * rg[bb];
  }
  bc[t] = s;
}

// x[g, f, a] += sum_b I_g[a][b] xc[parent(g), f, b]
template <typename T, int NQ>
__global__ __launch_bounds__(256) void k_bsr_prolong(int nf, const int* __restrict__ parent, const T* __restrict__ I,
                                                     const T* __restrict__ xc, T* __restrict__ x) {
  constexpr int NB = 3 * NQ;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nf * NB) return;
  const int g = (int)(t / NB), row = (int)(t % NB);
  const int f = row / NQ, a = row % NQ;
  const T* Ig = I + (size_t)g * NQ * NQ + a * NQ;
  const T* xp = xc + (size_t)parent[g] * NB + f * NQ;
  T s = (T)0;
#pragma unroll
  for (int bb = 0; bb < NQ; ++bb) s += Ig[bb] * xp[bb];
  x[t] += s;
}

template <class F>
int by_nb(int nb, F&& f) {
  switch (nb) {
    case 12: return f(std::integral_constant<int, 12>{});
    case 27: return f(std::integral_constant<int, 27>{});
    case 48: return f(std::integral_constant<int, 48>{});
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

template <typename T>
int launch_bsr_colour(void* st, int nb, int64_t nelem, const int* elems, const int* rowptr, const int* cols,
                      const T* blk, const T* inv, const T* b, T* x) {
  if (nelem <= 0) return 0;
  return by_nb(nb, [&](auto N) {
    constexpr int NB = decltype(N)::value;
    hipLaunchKernelGGL((k_bsr_colour<T, NB>), dim3((unsigned)nelem), dim3(64), 0, (hipStream_t)st, (int)nelem, elems,
                       rowptr, cols, blk, inv, b, x);
    return (int)hipGetLastError();
  });
}

template <typename T>
int launch_bsr_residual(void* st, int nb, int64_t ne, const int* rowptr, const int* cols, const T* blk, const T* b,
                        const T* x, T* out, const double* ds) {
  if (ne <= 0) return 0;
  return by_nb(nb, [&](auto N) {
    constexpr int NB = decltype(N)::value;
    hipLaunchKernelGGL((k_bsr_residual<T, NB>), dim3((unsigned)ne), dim3(64), 0, (hipStream_t)st, (int)ne, rowptr,
                       cols, blk, b, x, out, ds);
    return (int)hipGetLastError();
  });
}

template <typename T>
int launch_bsr_restrict(void* st, int nb, int64_t nc, const int* kid_ptr, const int* kids, const T* I, const T* r,
                        T* bc) {
  if (nc <= 0) return 0;
  return by_nb(nb, [&](auto N) {
    constexpr int NQ = decltype(N)::value / 3;
    const int64_t nt = nc * (3 * NQ);
    hipLaunchKernelGGL((k_bsr_restrict<T, NQ>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, (hipStream_t)st,
                       (int)nc, kid_ptr, kids, I, r, bc);
    return (int)hipGetLastError();
  });
}

template <typename T>
int launch_bsr_prolong(void* st, int nb, int64_t nf, const int* parent, const T* I, const T* xc, T* x) {
  if (nf <= 0) return 0;
  return by_nb(nb, [&](auto N) {
    constexpr int NQ = decltype(N)::value / 3;
    const int64_t nt = nf * (3 * NQ);
    hipLaunchKernelGGL((k_bsr_prolong<T, NQ>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, (hipStream_t)st,
                       (int)nf, parent, I, xc, x);
    return (int)hipGetLastError();
  });
}

#define LDGS_INST(T)                                                                                             \
  template int launch_bsr_colour<T>(void*, int, int64_t, const int*, const int*, const int*, const T*, const T*,  \
                                    const T*, T*);                                                               \
  template int launch_bsr_residual<T>(void*, int, int64_t, const int*, const int*, const T*, const T*, const T*, \
                                      T*, const double*);                                                        \
  template int launch_bsr_restrict<T>(void*, int, int64_t, const int*, const int*, const T*, const T*, T*);      \
  template int launch_bsr_prolong<T>(void*, int, int64_t, const int*, const T*, const T*, T*);
LDGS_INST(double)
LDGS_INST(float)
#undef LDGS_INST

}  // namespace ldgs
