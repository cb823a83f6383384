// Learned post-smoothing correction on gfx950: inference (one wavefront per
// tile of 16 elements, bf16 MFMA 16x16x32 for the patch layer, 16x16x16 for
// the hidden and output layers), training-crop extraction, and the training
// forward/backward pass with weight gradients on the same MFMA shapes.
//
// MFMA operand layouts used (lane l, r = l % 16, g = l / 16):
//   16x16x32 bf16: A[r][8g + j], B[8g + j][r], j < 8
//   16x16x16 bf16: A[r][4g + j], B[4g + j][r], j < 4
//   result D[4g + j][r], j < 4 (both shapes)
#include <hip/hip_runtime.h>

#include <mutex>

#include <cmath>
#include <type_traits>

#include "learned_internal.hpp"

namespace ldgs {

namespace {

template <int B, int E>
struct Pw { static constexpr int v = B * Pw<B, E - 1>::v; };
template <int B>
struct Pw<B, 0> { static constexpr int v = 1; };

template <int D, int P>
struct NetSz {
  static constexpr int M = P + 1, NQ = Pw<M, D>::v, NB = (D + 1) * NQ, NVEL = D * NQ;
  static constexpr int CH = NB + 1, CHP = (CH + 7) / 8 * 8, NOFF = Pw<3, D>::v;
  static constexpr int K1 = NOFF * CHP, K1P = (K1 + 31) / 32 * 32, NOUT = (NB + 15) / 16 * 16, H = NET_H;
  static constexpr int oW1 = 0, ob1 = H * K1P, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H;
  static constexpr int ob3 = oW3 + NOUT * H, total = ob3 + NOUT;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
struct alignas(16) U8 { uint16_t v[8]; };
struct alignas(8) U4 { uint16_t v[4]; };

// float -> bfloat16, round to nearest, ties to even
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mma32(const U8& a, const U8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}
__device__ __forceinline__ f32x4 mma16(const U4& a, const U4& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c, 0,
                                                   0, 0);
}

// element of patch offset o (base 3, axis 0 fastest, digit 1 = centre) around
// coordinates c on the n^D grid; -1 outside a non-periodic wall
template <int D>
__device__ __forceinline__ int patch_elem(const int* c, int o, int n, int lgn, int permask) {
  int e = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int v = c[k] + o % 3 - 1;
    o /= 3;
    if (v < 0 || v >= n) {
      if (!((permask >> k) & 1)) return -1;
      v = (v + n) & (n - 1);
    }
    e |= v << (k * lgn);
  }
  return e;
}

__device__ __forceinline__ double field_scale(const double* sums, int f, double cnt) {
  const double s = sums[f] > 0.0 ? sqrt(sums[f] / cnt) : 1.0;
  return s;
}

// ---------------------------------------------------------------------------
constexpr int RBLK = 256;

template <typename T>
__global__ __launch_bounds__(RBLK) void k_field_sumsq(int64_t ne, int nb, int nvel, const T* __restrict__ r,
                                                      const double* __restrict__ dscale, double* __restrict__ part) {
  __shared__ double su[RBLK], sp[RBLK];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RBLK + threadIdx.x; i < ne * nb; i += (int64_t)gridDim.x * RBLK) {
    const int64_t e = i / nb;
    const int c = (int)(i - e * nb);
    double v = (double)r[i];
    if (dscale) v /= dscale[2 * e + (c >= nvel ? 1 : 0)];
    if (c < nvel) a += v * v;
    else b += v * v;
  }
  su[threadIdx.x] = a;
  sp[threadIdx.x] = b;
  __syncthreads();
  for (int st = RBLK / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      su[threadIdx.x] += su[threadIdx.x + st];
      sp[threadIdx.x] += sp[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = su[0];
    part[2 * blockIdx.x + 1] = sp[0];
  }
}

__global__ __launch_bounds__(RBLK) void k_sum_pairs(int nblk, const double* __restrict__ part, double* __restrict__ sums) {
  __shared__ double su[RBLK], sp[RBLK];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += RBLK) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  su[threadIdx.x] = a;
  sp[threadIdx.x] = b;
  __syncthreads();
  for (int st = RBLK / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      su[threadIdx.x] += su[threadIdx.x + st];
      sp[threadIdx.x] += sp[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[0] = su[0];
    sums[1] = sp[0];
  }
}

// Minimal-residual step length of the correction: partial sums of r . q and
// q . q (q = A dx) per block, FP64 accumulation in a fixed order.
template <typename T>
__global__ __launch_bounds__(RBLK) void k_dot2(int64_t n, const T* __restrict__ r, const T* __restrict__ q,
                                               double* __restrict__ part) {
  __shared__ double sa[RBLK], sb[RBLK];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RBLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * RBLK) {
    const double qv = (double)q[i];
    a += (double)r[i] * qv;
    b += qv * qv;
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int st = RBLK / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sa[threadIdx.x] += sa[threadIdx.x + st];
      sb[threadIdx.x] += sb[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa[0];
    part[2 * blockIdx.x + 1] = sb[0];
  }
}

// out = base + w dx with w = sums[0] / sums[1] (0 when sums[1] is 0), or
// w = 1 when sums is null (the full step); w is also stored in sums[2]
__global__ __launch_bounds__(256) void k_minres_update(int64_t n, double* __restrict__ sums,
                                                       const double* __restrict__ base, const double* __restrict__ dx,
                                                       double* __restrict__ out) {
  if (!sums) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
      out[i] = base[i] + dx[i];
    return;
  }
  const double w = sums[1] > 0.0 ? sums[0] / sums[1] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) sums[2] = w;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = base[i] + w * dx[i];
}

// ---------------------------------------------------------------------------
// inference: out = base + dx for the 16 elements E0 .. E0 + 15
// ---------------------------------------------------------------------------
struct ApplyArgs {
  int n, lgn, permask;
  const double* dscale;
  const float* logmu;
  const double* sums;
  double cnt_u, cnt_p, c_u, c_p;
  NetDev net;
  const double* base;
  double* out;
};

template <typename Tin, int D, int P>
__global__ __launch_bounds__(64) void k_net_apply(ApplyArgs a, const Tin* __restrict__ r) {
  using S = NetSz<D, P>;
  __shared__ uint16_t h1s[16][16], h2s[16][16];
  const int l = threadIdx.x, row = l & 15, grp = l >> 4;
  const int NE = 1 << (D * a.lgn);
  const int E0 = blockIdx.x * 16;
  const int E = E0 + row;
  const bool valid = E < NE;
  int c[D];
#pragma unroll
  for (int k = 0; k < D; ++k) c[k] = (E >> (k * a.lgn)) & (a.n - 1);
  const double su = field_scale(a.sums, 0, a.cnt_u), sp = field_scale(a.sums, 1, a.cnt_p);
  const double isu = 1.0 / su, isp = 1.0 / sp;
  const uint16_t* W1 = a.net.wbf + S::oW1;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < S::K1P / 32; ++kc) {
    const int k = kc * 32 + grp * 8;
    const int o = k / S::CHP, ch0 = k - o * S::CHP;
    const int F = (valid && o < S::NOFF) ? patch_elem<D>(c, o, a.n, a.lgn, a.permask) : -1;
    U8 ua;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int ch = ch0 + j;
      float v = 0.f;
      if (F >= 0) {
        if (ch < S::NB) {
          double rv = (double)r[(size_t)F * S::NB + ch];
          if (a.dscale) rv /= a.dscale[2 * F + (ch >= S::NVEL ? 1 : 0)];
          v = (float)(rv * (ch < S::NVEL ? isu : isp));
        } else if (ch == S::NB) {
          v = a.logmu[F];
        }
      }
      ua.v[j] = f2bf(v);
    }
    const U8 ub = *reinterpret_cast<const U8*>(W1 + row * S::K1P + k);
    acc = mma32(ua, ub, acc);
  }
  const float* mw = a.net.master;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float h = acc[j] + mw[S::ob1 + row];
    h1s[4 * grp + j][row] = f2bf(h > 0.f ? h : 0.f);
  }
  __syncthreads();
  U4 xa, wb;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    xa.v[j] = h1s[row][4 * grp + j];
    wb.v[j] = a.net.wbf[S::oW2 + row * 16 + 4 * grp + j];
  }
  f32x4 acc2 = mma16(xa, wb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float h = acc2[j] + mw[S::ob2 + row];
    h2s[4 * grp + j][row] = f2bf(h > 0.f ? h : 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) xa.v[j] = h2s[row][4 * grp + j];
  for (int t = 0; t < S::NOUT / 16; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) wb.v[j] = a.net.wbf[S::oW3 + (t * 16 + row) * 16 + 4 * grp + j];
    const f32x4 y = mma16(xa, wb, f32x4{0.f, 0.f, 0.f, 0.f});
    const int oc = t * 16 + row;
    if (oc < S::NB) {
      const double sc = oc < S::NVEL ? su * a.c_u : sp * a.c_p;
      const float bb = mw[S::ob3 + oc];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int Ej = E0 + 4 * grp + j;
        if (Ej < NE) {
          const size_t idx = (size_t)Ej * S::NB + oc;
          a.out[idx] = (a.base ? a.base[idx] : 0.0) + (double)(y[j] + bb) * sc;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// training crops
// ---------------------------------------------------------------------------
struct CropArgs {
  int n, lgn, permask, C, ncrop;
  const int* origins;
  const double* r;
  const double* e;
  const float* logmu;
  const double* sums;
  double cnt_u, cnt_p;
  uint16_t* feat;
  uint16_t* targ;
};

template <int D, int P>
__global__ void k_crop_feat(CropArgs a) {
  using S = NetSz<D, P>;
  const int M = a.C + 2;
  int Md = 1;
  for (int k = 0; k < D; ++k) Md *= M;
  const int64_t total = (int64_t)a.ncrop * Md * S::CHP;
  const double isu = 1.0 / field_scale(a.sums, 0, a.cnt_u), isp = 1.0 / field_scale(a.sums, 1, a.cnt_p);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(i % S::CHP);
    const int64_t q = i / S::CHP;
    int t = (int)(q % Md);
    const int cr = (int)(q / Md);
    int F = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int v = a.origins[cr * D + k] - 1 + t % M;
      t /= M;
      if (v < 0 || v >= a.n) {
        if (!((a.permask >> k) & 1)) ok = false;
        v = (v + a.n) & (a.n - 1);
      }
      F |= v << (k * a.lgn);
    }
    float val = 0.f;
    if (ok) {
      if (ch < S::NB) val = (float)(a.r[(size_t)F * S::NB + ch] * (ch < S::NVEL ? isu : isp));
      else if (ch == S::NB) val = a.logmu[F];
    }
    a.feat[i] = f2bf(val);
  }
}

template <int D, int P>
__global__ void k_crop_targ(CropArgs a) {
  using S = NetSz<D, P>;
  int Cd = 1;
  for (int k = 0; k < D; ++k) Cd *= a.C;
  const int64_t total = (int64_t)a.ncrop * Cd * S::NB;
  const double isu = 1.0 / field_scale(a.sums, 0, a.cnt_u), isp = 1.0 / field_scale(a.sums, 1, a.cnt_p);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(i % S::NB);
    const int64_t q = i / S::NB;
    int t = (int)(q % Cd);
    const int cr = (int)(q / Cd);
    int F = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int v = (a.origins[cr * D + k] + t % a.C) & (a.n - 1);
      t /= a.C;
      F |= v << (k * a.lgn);
    }
    a.targ[i] = f2bf((float)(a.e[(size_t)F * S::NB + ch] * (ch < S::NVEL ? isu : isp)));
  }
}

// ---------------------------------------------------------------------------
// training: forward, loss and backward for TPW tiles of 16 crop elements
// ---------------------------------------------------------------------------
struct TrainArgs {
  int C, lgC, nbatch;
  const int* batch;
  const uint16_t* feat;
  const uint16_t* targ;
  float c_u, c_p, inv_count;
  NetDev net;
  float* grad;
  double* loss;
};

constexpr int TPW = 4;

template <int D, int P>
__global__ __launch_bounds__(64) void k_train_grad(TrainArgs a) {
  using S = NetSz<D, P>;
  __shared__ uint16_t h1s[TPW][16][16], h2s[TPW][16][16], da1s[TPW][16][16], da2s[TPW][16][16];
  __shared__ uint16_t dys[TPW][16][S::NOUT];
  const int l = threadIdx.x, row = l & 15, grp = l >> 4;
  const int M = a.C + 2;
  int Md = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) Md *= M;
  const int lgCd = D * a.lgC;
  const int ntiles = (a.nbatch << lgCd) / 16;
  const float* mw = a.net.master;
  const uint16_t* wbf = a.net.wbf;
  // linear offset of patch offset o inside a crop with halo
  auto lin = [&](int o) {
    int s = 0, m = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      s += (o % 3 - 1) * m;
      o /= 3;
      m *= M;
    }
    return s;
  };
  // crop id and halo-grid index of crop element g
  auto locate = [&](int g, int& cr, int& hc) {
    const int b = g >> lgCd;
    const int q = g & ((1 << lgCd) - 1);
    cr = a.batch[b];
    hc = 0;
    int m = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      hc += (((q >> (k * a.lgC)) & (a.C - 1)) + 1) * m;
      m *= M;
    }
  };
  const int nvalid = min(TPW, ntiles - (int)blockIdx.x * TPW);
  int ecr[TPW][4], ehc[TPW][4];
  double lsum = 0.0;
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    const int tile = blockIdx.x * TPW + ti;
    if (ti >= nvalid) continue;
    int cr, hc;
    locate(tile * 16 + row, cr, hc);
#pragma unroll
    for (int j = 0; j < 4; ++j) locate(tile * 16 + 4 * grp + j, ecr[ti][j], ehc[ti][j]);
    const uint16_t* fb = a.feat + (size_t)cr * Md * S::CHP;
    // layer 1
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < S::K1P / 32; ++kc) {
      const int k = kc * 32 + grp * 8;
      const int o = k / S::CHP, ch0 = k - o * S::CHP;
      U8 ua;
      if (o < S::NOFF) {
        ua = *reinterpret_cast<const U8*>(fb + (size_t)(hc + lin(o)) * S::CHP + ch0);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) ua.v[j] = 0;
      }
      const U8 ub = *reinterpret_cast<const U8*>(wbf + S::oW1 + row * S::K1P + k);
      acc = mma32(ua, ub, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float h = acc[j] + mw[S::ob1 + row];
      h1s[ti][4 * grp + j][row] = f2bf(h > 0.f ? h : 0.f);
    }
    __syncthreads();
    U4 xa, wb;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      xa.v[j] = h1s[ti][row][4 * grp + j];
      wb.v[j] = wbf[S::oW2 + row * 16 + 4 * grp + j];
    }
    const f32x4 acc2 = mma16(xa, wb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float h = acc2[j] + mw[S::ob2 + row];
      h2s[ti][4 * grp + j][row] = f2bf(h > 0.f ? h : 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) xa.v[j] = h2s[ti][row][4 * grp + j];
    for (int t = 0; t < S::NOUT / 16; ++t) {
#pragma unroll
      for (int j = 0; j < 4; ++j) wb.v[j] = wbf[S::oW3 + (t * 16 + row) * 16 + 4 * grp + j];
      const f32x4 y = mma16(xa, wb, f32x4{0.f, 0.f, 0.f, 0.f});
      const int oc = t * 16 + row;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint16_t dyb = 0;
        if (oc < S::NB) {
          const int g = tile * 16 + 4 * grp + j;
          const int b = g >> lgCd, q = g & ((1 << lgCd) - 1);
          const float tv = bf2f(a.targ[((size_t)a.batch[b] << lgCd) * S::NB + (size_t)q * S::NB + oc]) /
                           (oc < S::NVEL ? a.c_u : a.c_p);
          const float diff = (y[j] + mw[S::ob3 + oc]) - tv;
          lsum += (double)diff * (double)diff;
          dyb = f2bf(2.f * diff * a.inv_count);
        }
        dys[ti][4 * grp + j][oc] = dyb;
      }
    }
    __syncthreads();
    // dh2 = dy W3, masked by h2 > 0
    f32x4 d2 = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < S::NOUT / 16; ++kt) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        xa.v[j] = dys[ti][row][16 * kt + 4 * grp + j];
        wb.v[j] = wbf[S::oW3 + (16 * kt + 4 * grp + j) * 16 + row];
      }
      d2 = mma16(xa, wb, d2);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool on = h2s[ti][4 * grp + j][row] != 0;
      da2s[ti][4 * grp + j][row] = on ? f2bf(d2[j]) : (uint16_t)0;
    }
    __syncthreads();
    // dh1 = da2 W2, masked by h1 > 0
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      xa.v[j] = da2s[ti][row][4 * grp + j];
      wb.v[j] = wbf[S::oW2 + (4 * grp + j) * 16 + row];
    }
    const f32x4 d1 = mma16(xa, wb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool on = h1s[ti][4 * grp + j][row] != 0;
      da1s[ti][4 * grp + j][row] = on ? f2bf(d1[j]) : (uint16_t)0;
    }
    __syncthreads();
  }
  // ---- weight gradients, summed over the work-group's tiles ----
  float* g = a.grad;
  for (int t = 0; t < S::NOUT / 16; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti) {
      if (ti >= nvalid) continue;
      U4 xa, wb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        xa.v[j] = dys[ti][4 * grp + j][16 * t + row];
        wb.v[j] = h2s[ti][4 * grp + j][row];
      }
      acc = mma16(xa, wb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&g[S::oW3 + (16 * t + 4 * grp + j) * 16 + row], acc[j]);
  }
  for (int oc = l; oc < S::NOUT; oc += 64) {
    float s = 0.f;
    for (int ti = 0; ti < nvalid; ++ti)
      for (int e = 0; e < 16; ++e) s += bf2f(dys[ti][e][oc]);
    atomicAdd(&g[S::ob3 + oc], s);
  }
  {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti) {
      if (ti >= nvalid) continue;
      U4 xa, wb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        xa.v[j] = da2s[ti][4 * grp + j][row];
        wb.v[j] = h1s[ti][4 * grp + j][row];
      }
      acc = mma16(xa, wb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&g[S::oW2 + (4 * grp + j) * 16 + row], acc[j]);
  }
  if (l < 16) {
    float s2 = 0.f, s1 = 0.f;
    for (int ti = 0; ti < nvalid; ++ti)
      for (int e = 0; e < 16; ++e) {
        s2 += bf2f(da2s[ti][e][l]);
        s1 += bf2f(da1s[ti][e][l]);
      }
    atomicAdd(&g[S::ob2 + l], s2);
    atomicAdd(&g[S::ob1 + l], s1);
  }
  U4 da[TPW];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
    for (int j = 0; j < 4; ++j) da[ti].v[j] = ti < nvalid ? da1s[ti][4 * grp + j][row] : (uint16_t)0;
  for (int kt = 0; kt < S::K1P / 16; ++kt) {
    const int f = 16 * kt + row;
    const int o = f / S::CHP, ch = f - o * S::CHP;
    const int off = (o < S::NOFF) ? lin(o) : 0;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti) {
      if (ti >= nvalid) continue;
      U4 xb;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        xb.v[j] = (o < S::NOFF)
                      ? a.feat[((size_t)ecr[ti][j] * Md + (size_t)(ehc[ti][j] + off)) * S::CHP + ch]
                      : (uint16_t)0;
      acc = mma16(da[ti], xb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&g[S::oW1 + (4 * grp + j) * S::K1P + f], acc[j]);
  }
  // summed squared error
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
  if (l == 0) atomicAdd(a.loss, lsum);
}

__global__ void k_adam(int64_t n, float* __restrict__ w, uint16_t* __restrict__ wbf, const float* __restrict__ gr,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
  w[i] = wi;
  wbf[i] = f2bf(wi);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ s, uint16_t* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = f2bf(s[i]);
}

template <class F>
int net_dispatch(int d, int p, F&& f) {
  using std::integral_constant;
  if (d == 2 && p == 1) f(integral_constant<int, 2>{}, integral_constant<int, 1>{});
  else if (d == 2 && p == 2) f(integral_constant<int, 2>{}, integral_constant<int, 2>{});
  else if (d == 2 && p == 3) f(integral_constant<int, 2>{}, integral_constant<int, 3>{});
  else if (d == 3 && p == 1) f(integral_constant<int, 3>{}, integral_constant<int, 1>{});
  else if (d == 3 && p == 2) f(integral_constant<int, 3>{}, integral_constant<int, 2>{});
  else return 2;
  return 0;
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : 1; }
inline unsigned blocks(int64_t n, int b, int64_t cap) {
  int64_t g = (n + b - 1) / b;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

NetShape net_shape(int d, int p) {
  NetShape s{};
  s.d = d;
  s.p = p;
  s.nq = 1;
  for (int k = 0; k < d; ++k) s.nq *= p + 1;
  s.nb = (d + 1) * s.nq;
  s.ch = s.nb + 1;
  s.chp = (s.ch + 7) / 8 * 8;
  s.noff = d == 2 ? 9 : 27;
  s.k1 = s.noff * s.chp;
  s.k1p = (s.k1 + 31) / 32 * 32;
  s.nout = (s.nb + 15) / 16 * 16;
  const int H = NET_H;
  s.oW1 = 0;
  s.ob1 = (int64_t)H * s.k1p;
  s.oW2 = s.ob1 + H;
  s.ob2 = s.oW2 + H * H;
  s.oW3 = s.ob2 + H;
  s.ob3 = s.oW3 + (int64_t)s.nout * H;
  s.total = s.ob3 + s.nout;
  s.flat_total = (int64_t)H * s.noff * s.ch + H + H * H + H + (int64_t)s.nb * H + s.nb;
  return s;
}

template <typename T>
int launch_field_sumsq(void* stream, int64_t ne, int nb, int nvel, const T* r, const double* dscale, double* part,
                       int nblk, double* sums) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL((k_field_sumsq<T>), dim3(nblk), dim3(RBLK), 0, st, ne, nb, nvel, r, dscale, part);
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(RBLK), 0, st, nblk, part, sums);
  return ok();
}

template <typename Tin>
int launch_net_apply(void* stream, int d, int p, int n, int lgn, int permask, const Tin* r, const double* dscale,
                     const float* logmu, const double* sums, double cnt_u, double cnt_p, double c_u, double c_p,
                     NetDev net, const double* base, double* out) {
  ApplyArgs a{n, lgn, permask, dscale, logmu, sums, cnt_u, cnt_p, c_u, c_p, net, base, out};
  int64_t NE = 1;
  for (int k = 0; k < d; ++k) NE *= n;
  const unsigned grid = (unsigned)((NE + 15) / 16);
  hipStream_t st = (hipStream_t)stream;
  if (net_dispatch(d, p, [&](auto Dc, auto Pc) {
        constexpr int D_ = decltype(Dc)::value, P_ = decltype(Pc)::value;
        hipLaunchKernelGGL((k_net_apply<Tin, D_, P_>), dim3(grid), dim3(64), 0, st, a, r);
      }))
    return 2;
  return ok();
}

template <typename T>
int launch_minres_sums(void* stream, int64_t n, const T* r, const T* q, double* part, int nblk, double* sums) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL((k_dot2<T>), dim3(nblk), dim3(RBLK), 0, st, n, r, q, part);
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(RBLK), 0, st, nblk, part, sums);
  return ok();
}

int launch_minres_update(void* stream, int64_t n, double* sums, const double* base, const double* dx, double* out) {
  hipLaunchKernelGGL(k_minres_update, dim3(blocks(n, 256, 4096)), dim3(256), 0, (hipStream_t)stream, n, sums, base, dx,
                     out);
  return ok();
}

int launch_collect_crops(void* stream, int d, int p, int n, int lgn, int permask, int C, int lgC, int ncrop,
                         const int* origins, const double* r, const double* e, const float* logmu,
                         const double* sums, double cnt_u, double cnt_p, uint16_t* feat, uint16_t* targ) {
  (void)lgC;
  CropArgs a{n, lgn, permask, C, ncrop, origins, r, e, logmu, sums, cnt_u, cnt_p, feat, targ};
  hipStream_t st = (hipStream_t)stream;
  if (net_dispatch(d, p, [&](auto Dc, auto Pc) {
        constexpr int D_ = decltype(Dc)::value, P_ = decltype(Pc)::value;
        hipLaunchKernelGGL((k_crop_feat<D_, P_>), dim3(2048), dim3(256), 0, st, a);
        hipLaunchKernelGGL((k_crop_targ<D_, P_>), dim3(2048), dim3(256), 0, st, a);
      }))
    return 2;
  return ok();
}

int launch_train_grad(void* stream, int d, int p, int C, int lgC, int nbatch, const int* batch,
                      const uint16_t* feat, const uint16_t* targ, double c_u, double c_p, double inv_count,
                      NetDev net, float* grad, double* loss) {
  TrainArgs a{C, lgC, nbatch, batch, feat, targ, (float)c_u, (float)c_p, (float)inv_count, net, grad, loss};
  int64_t Cd = 1;
  for (int k = 0; k < d; ++k) Cd *= C;
  const int64_t ntiles = (int64_t)nbatch * Cd / 16;
  const unsigned grid = (unsigned)((ntiles + TPW - 1) / TPW);
  hipStream_t st = (hipStream_t)stream;
  if (net_dispatch(d, p, [&](auto Dc, auto Pc) {
        constexpr int D_ = decltype(Dc)::value, P_ = decltype(Pc)::value;
        hipLaunchKernelGGL((k_train_grad<D_, P_>), dim3(grid), dim3(64), 0, st, a);
      }))
    return 2;
  return ok();
}

int launch_adam(void* stream, int64_t n, float* master, uint16_t* wbf, const float* grad, float* m, float* v, float lr,
                float beta1, float beta2, float eps, float bc1, float bc2) {
  hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256, 1 << 30)), dim3(256), 0, (hipStream_t)stream, n, master, wbf, grad, m,
                     v, lr, beta1, beta2, eps, bc1, bc2);
  return ok();
}

int launch_to_bf16(void* stream, int64_t n, const float* src, uint16_t* dst) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n, 256, 1 << 30)), dim3(256), 0, (hipStream_t)stream, n, src, dst);
  return ok();
}

// Fixed workspace of the training entry point that allocates nothing: one
// copy per GPU in device global memory, alive until the process ends.  On
// the host the symbol names a host-side stand-in, never device memory: host
// code uses only the address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) unsigned char scratch[LDGS_TRAIN_WORKSPACE_BYTES];

int train_workspace(void** ptr) {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static void* addr[MAXDEV] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return 1;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return 1;
    }
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return 0;
}

template int launch_field_sumsq<float>(void*, int64_t, int, int, const float*, const double*, double*, int, double*);
template int launch_field_sumsq<double>(void*, int64_t, int, int, const double*, const double*, double*, int, double*);
template int launch_minres_sums<float>(void*, int64_t, const float*, const float*, double*, int, double*);
template int launch_minres_sums<double>(void*, int64_t, const double*, const double*, double*, int, double*);
template int launch_net_apply<float>(void*, int, int, int, int, int, const float*, const double*, const float*,
                                     const double*, double, double, double, double, NetDev, const double*, double*);
template int launch_net_apply<double>(void*, int, int, int, int, int, const double*, const double*, const float*,
                                      const double*, double, double, double, double, NetDev, const double*, double*);

}  // namespace ldgs
