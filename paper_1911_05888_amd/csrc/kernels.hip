// HIP kernels of the LDG-Stokes V-cycle for gfx950 (CDNA4).
//
// One 64-lane work-group (one wavefront) owns one element.  It stages the x
// coefficients of the element and of the neighbours its residual depends on
// in LDS, evaluates (A x)_E matrix-free from the factored operator (G in
// closed-form 1D tensors, M_mu blocks, penalty face matrices), and in the
// smoother applies the element's precomputed inverse diagonal block, which is
// streamed from HBM in a lane-blocked layout (colour-major order, so that
// consecutive work-groups read consecutive memory) and prefetched into
// registers before the residual is evaluated.
//
// The operator action follows eq. (stokessystem) / eq. (viscousop) with M = I:
//   (A x)_{u_i} = sum_k G_k^T s_ik + Et u_i + (rho/delta) u_i - G_i^T p,
//   s_ik = M_mu (G_k u_i + gamma G_i u_k),
//   (A x)_p     = -sum_i G_i u_i - E p.
// G_k^T s receives, from each face normal to k, the one-sided flux
// h^-1 (wR s_R|lo + wL s_L|hi) (sigma-hat of eq. qstarflux): +e0 on the high
// element R and -e1 on the low element L.  For the neighbour E+e_k only the
// low-face trace of s is needed; it is formed with the trace-projected mass
// rows R_k = (e0^T)_k M_mu of that neighbour.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <type_traits>

#include "ldgs_internal.hpp"

namespace ldgs {

template <int B, int E>
struct Pow { static constexpr int v = B * Pow<B, E - 1>::v; };
template <int B>
struct Pow<B, 0> { static constexpr int v = 1; };

template <int D, int P, bool IF = false>
struct Sz {
  static constexpr int M = P + 1;
  static constexpr int NQ = Pow<M, D>::v;
  static constexpr int MT = Pow<M, D - 1>::v;
  static constexpr int NB = (D + 1) * NQ;
  // stencil slots: E, E-e_k, E+e_k, E+e_k-e_j (j != k); with interphase
  // faces (IF) also E-2e_k, E+2e_k, E-e_k-e_j, E+e_k+e_j (k < j)
  static constexpr int NBASE = 1 + 2 * D + D * (D - 1);
  static constexpr int NPAIR = D * (D - 1) / 2;
  static constexpr int NSLOT = IF ? NBASE + 2 * D + 2 * NPAIR : NBASE;
  // elements whose gradient is needed: E, E+e_k, and with IF E-e_k
  static constexpr int NFS = IF ? 1 + 2 * D : 1 + D;
};

constexpr int WG = 64;

// 1D tables in the arithmetic type of the kernel
template <typename T>
struct TabT {
  T K[MAXM * MAXM];
  T e0[MAXM];
  T e1[MAXM];
  T P[2][MAXM * MAXM];
};
template <typename T>
static TabT<T> tab_of(const Tab1D& t) {
  TabT<T> r{};
  for (int i = 0; i < MAXM * MAXM; ++i) {
    r.K[i] = (T)t.K[i];
    r.P[0][i] = (T)t.P[0][i];
    r.P[1][i] = (T)t.P[1][i];
  }
  for (int i = 0; i < MAXM; ++i) {
    r.e0[i] = (T)t.e0[i];
    r.e1[i] = (T)t.e1[i];
  }
  return r;
}

// tensor index helpers (axis 0 fastest); the axis is a run-time value, each
// case compiles to constant divisors
template <int M, int K>
__device__ __forceinline__ int compose_c(int t, int c) {
  constexpr int lo = Pow<M, K>::v;
  return t % lo + lo * c + lo * M * (t / lo);
}
template <int M>
__device__ __forceinline__ int compose(int t, int c, int k) {
  return k == 0 ? compose_c<M, 0>(t, c) : (k == 1 ? compose_c<M, 1>(t, c) : compose_c<M, 2>(t, c));
}
template <int M>
__device__ __forceinline__ int stride_of(int k) {
  return k == 0 ? 1 : (k == 1 ? M : M * M);
}
template <int M, int K>
__device__ __forceinline__ int digit_c(int a) { return (a / Pow<M, K>::v) % M; }
template <int M, int K>
__device__ __forceinline__ int tang_c(int a) {
  constexpr int lo = Pow<M, K>::v;
  return a % lo + lo * (a / (lo * M));
}

// coordinates of element e on an n^D grid, n = 2^lgn
template <int D>
__device__ __forceinline__ void coords_of(int e, int lgn, int* c) {
  const int mask = (1 << lgn) - 1;
#pragma unroll
  for (int j = 0; j < D; ++j) c[j] = (e >> (j * lgn)) & mask;
}
template <int D>
__device__ __forceinline__ int index_of(const int* c, int lgn) {
  int e = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) e |= c[j] << (j * lgn);
  return e;
}
// shift coordinate k by s; false if it leaves a non-periodic grid
__device__ __forceinline__ bool shift1(int* c, int k, int s, int n, bool per) {
  // n is a power of two: the mask wraps -1 to n - 1 and n to 0 (periodic);
  // without periodicity an outside neighbour is reported absent
  const int v = c[k] + s;
  c[k] = v & (n - 1);
  return per || (unsigned)v < (unsigned)n;
}
template <int D>
__device__ __forceinline__ int face_index(const int* c, int n, int nfk, int k, int f) {
  int e = 0, s = 1;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    e += ((j == k) ? f : c[j]) * s;
    s *= (j == k) ? nfk : n;
  }
  return e;
}

// Element idx of colour pcol under parity colouring with the elements of a
// colour in increasing order (colour bits b_k = c_k mod 2, c_k = 2 i_k + b_k,
// idx = sum_k i_k (n/2)^k); pcol < 0: the colour's element list.
template <int D>
__device__ __forceinline__ int colour_elem(int idx, int pcol, int lgn, const int* __restrict__ elems) {
  if (pcol < 0) return elems[idx];
  const int lgh = lgn - 1, hm = (1 << lgh) - 1;
  int E = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) E |= ((((idx >> (k * lgh)) & hm) << 1) | ((pcol >> k) & 1)) << (k * lgn);
  return E;
}

// face with both neighbours present (intraphase, or interphase on levels
// that have interphase faces)
template <bool IF>
__device__ __forceinline__ bool two_sided(unsigned char t) {
  if constexpr (IF) return t == F_INTRA || t == F_INTER;
  else return t == F_INTRA;
}
template <bool IF>
__device__ __forceinline__ bool is_inter(unsigned char t) {
  if constexpr (IF) return t == F_INTER;
  else return false;
}

// pair (i, k) of stress row pr: all D^2 pairs (i major), or with sym the
// D (D + 1) / 2 pairs i <= k in the order (0,0), (0,1), ..., (1,1), ...
template <int D>
__device__ __forceinline__ void stress_pair(int pr, bool sym, int& i, int& k) {
  if (!sym) {
    i = pr / D;
    k = pr % D;
  } else if constexpr (D == 2) {
    i = pr == 2 ? 1 : 0;
    k = pr == 0 ? 0 : 1;
  } else {
    i = pr < 3 ? 0 : (pr < 5 ? 1 : 2);
    k = pr < 3 ? pr : (pr < 5 ? pr - 2 : 2);
  }
}

// stencil slots (see Sz)
template <int D>
__device__ __forceinline__ int pair_of(int a, int b) {   // a != b
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return D == 2 ? 0 : (lo == 0 ? hi - 1 : 2);
}
template <int D>
struct Slot {
  static constexpr int NBASE = 1 + 2 * D + D * (D - 1), NPAIR = D * (D - 1) / 2;
  __device__ static int m(int k) { return 1 + k; }                                       // E - e_k
  __device__ static int p(int k) { return 1 + D + k; }                                   // E + e_k
  __device__ static int pm(int k, int j) { return 1 + 2 * D + k * (D - 1) + (j < k ? j : j - 1); }  // E+e_k-e_j
  __device__ static int mm2(int k) { return NBASE + k; }                                 // E - 2e_k
  __device__ static int pp2(int k) { return NBASE + D + k; }                             // E + 2e_k
  __device__ static int mm(int k, int j) { return NBASE + 2 * D + pair_of<D>(k, j); }     // E-e_k-e_j
  __device__ static int pp(int k, int j) { return NBASE + 2 * D + NPAIR + pair_of<D>(k, j); }  // E+e_k+e_j
};
// gradient element fi: E (0), E + e_j (1 + j), E - e_j (1 + D + j)
template <int D>
__device__ __forceinline__ int f_slot(int fi) {
  return fi == 0 ? 0 : (fi <= D ? Slot<D>::p(fi - 1) : Slot<D>::m(fi - 1 - D));
}
// slot of F - e_k and of F + e_k for gradient element fi
template <int D>
__device__ __forceinline__ int low_slot(int fi, int k) {
  if (fi == 0) return Slot<D>::m(k);
  if (fi <= D) {
    const int j = fi - 1;
    return k == j ? 0 : Slot<D>::pm(j, k);
  }
  const int j = fi - 1 - D;
  return k == j ? Slot<D>::mm2(j) : Slot<D>::mm(j, k);
}
template <int D>
__device__ __forceinline__ int high_slot(int fi, int k) {
  if (fi == 0) return Slot<D>::p(k);
  if (fi <= D) {
    const int j = fi - 1;
    return k == j ? Slot<D>::pp2(j) : Slot<D>::pp(j, k);
  }
  const int j = fi - 1 - D;
  return k == j ? 0 : Slot<D>::pm(k, j);
}

// Where the traces of p and of s_E are formed: in 3D with the gradient lines
// (p) and inline in the flux step (s), one barrier fewer (C3 125 -> 120 ms);
// in 2D in a step of their own, which measured faster there (the finest C2
// pass 27.7 -> 26.6 us)
template <int D>
constexpr bool FOLD_TRACES = D == 3;

// shared-memory work area of one element evaluation
// In 3D without interphase faces the slots E+e_a-e_b are read only for
// their component a (the line of G_b u_a at E+e_a reaches back into them):
// they are held compactly, one field each (xpm), which keeps the work area of
// the FP64 evaluation small enough for four work-groups per CU.
template <int D, bool IF>
constexpr bool COMPACT_PM = D == 3 && !IF;

template <typename T, int D, int P, bool IF = false>
struct Work {
  using S = Sz<D, P, IF>;
  static constexpr bool STAGE_M = (size_t)S::NQ * S::NQ * sizeof(T) <= 8192;
  static constexpr bool CPM = COMPACT_PM<D, IF>;
  static constexpr int NXS = CPM ? 1 + 2 * D : S::NSLOT;   // slots held whole
  alignas(16) T xs[NXS][S::NB];
  alignas(16) T xpm[CPM ? D * (D - 1) : 1][CPM ? S::NQ : 1];   // component a of E+e_a-e_b
  alignas(16) T th[2][D][S::MT * S::MT];          // penalty matrices of E's low/high faces
  alignas(16) T g[S::NFS][D * D][S::NQ];          // G_k u_i at E, E+e_k (and E-e_k) (needed components)
  alignas(16) T s0[D * D][S::NQ];                 // s_ik at E
  alignas(16) T trx[2][D][D + 1][S::MT];          // traces of x_E: [lo/hi][axis][field][t]
  alignas(16) T trn[2][D][D + 1][S::MT];          // [0]: x_{E-e_k}|hi, [1]: x_{E+e_k}|lo
  // s_E[i][k] lo/hi along k (only where a separate trace step forms it)
  alignas(16) T trs[FOLD_TRACES<D> ? 1 : 2][FOLD_TRACES<D> ? 1 : D][FOLD_TRACES<D> ? 1 : D][FOLD_TRACES<D> ? 1 : S::MT];
  alignas(16) T trr[D][D][S::MT];                 // s_{E+e_k}[i][k] at its low face along k
  alignas(16) T trrh[IF ? D : 1][IF ? D : 1][IF ? S::MT : 1];   // (IF) s_{E-e_k}[i][k] at its high face along k
  alignas(16) T flux[2][D][D + 1][S::MT];         // coefficients of e0 (lo) and e1 (hi) per axis/field
  // the 1D tables K, e0, e1 (TabT layout) for lookups whose index differs
  // between lanes (kernel-argument arrays indexed per lane become memory loads)
  alignas(16) T tabs[3 * MAXM * MAXM + 2 * MAXM];   // K, e0, e1, P[0], P[1]
  unsigned char ft[S::NFS][D][2];
  alignas(16) T fwl[S::NFS][D][2], fwr[S::NFS][D][2];
  // residual of the element, last before the viscosity data: the arrays before
  // it are free again once it is formed (scratch of the inverse product)
  alignas(16) T res[S::NB];
  // viscosity data, last: levels with constant viscosity do not allocate it
  alignas(16) T rr[D][S::MT * S::NQ];             // R_k = (e0^T)_k M_mu of E+e_k
  alignas(16) T rrh[IF ? D : 1][IF ? S::MT * S::NQ : 1];   // (IF) (e1^T)_k M_mu of E-e_k
  alignas(16) T mm[STAGE_M ? S::NQ * S::NQ : 1];   // M_mu of E
};

// LDS bytes of the evaluation (dynamic shared memory of the element kernels):
// the viscosity part only when the level's viscosity varies
template <typename T, int D, int P, bool IF>
constexpr size_t work_bytes(bool var_mu) {
  using W = Work<T, D, P, IF>;
  return var_mu ? sizeof(W) : offsetof(W, rr);
}

// Per-lane items of the trace step (where the traces are not folded), decoded
// at compile time: item u takes the trace of the line at `src` (offset in the
// work area, entries of T) with e1 (hi) or e0 along axis k (stride M^k) and
// stores it at `dst`.  Packed: src | dst << 12 | k << 24 | hi << 26.
template <typename T, int D, int P, bool IF>
struct TraceItems {
  using W = Work<T, D, P, IF>;
  using S = Sz<D, P, IF>;
  static constexpr int M = S::M, NQ = S::NQ, MT = S::MT, NB = S::NB;
  static constexpr int NX = 2 * MT, NN = 2 * MT, NTR = 2 * D * MT, PER_K = NX + NN + NTR, N = D * PER_K;
  struct Tab {
    unsigned w[N];
  };
  static constexpr int off(size_t member) { return (int)(member / sizeof(T)); }
  static constexpr Tab make() {
    Tab t{};
    for (int u = 0; u < N; ++u) {
      const int k = u / PER_K, r = u % PER_K, bm = r % MT;
      int lo = 1;
      for (int j = 0; j < k; ++j) lo *= M;
      const int base = bm % lo + lo * M * (bm / lo);   // line start: coordinate k = 0
      const bool isx = r < NX, isn = !isx && r < NX + NN;
      const int r2 = isx ? r : (isn ? r - NX : r - NX - NN);
      const int fs = (r2 / MT) % D;
      const int side = isx || isn ? r2 / MT : r2 / (MT * D);
      const int src = isx ? off(offsetof(W, xs)) + D * NQ + base
                          : (isn ? off(offsetof(W, xs)) + (side ? 1 + D + k : 1 + k) * NB + D * NQ + base
                                 : off(offsetof(W, s0)) + (fs * D + k) * NQ + base);
      const int dst = isx ? off(offsetof(W, trx)) + ((side * D + k) * (D + 1) + D) * MT + bm
                          : (isn ? off(offsetof(W, trn)) + ((side * D + k) * (D + 1) + D) * MT + bm
                                 : off(offsetof(W, trs)) + ((side * D + k) * D + fs) * MT + bm);
      const bool hi = isn ? side == 0 : side != 0;
      t.w[u] = (unsigned)src | ((unsigned)dst << 12) | ((unsigned)k << 24) | ((hi ? 1u : 0u) << 26);
    }
    return t;
  }
  static constexpr Tab tab = make();
  static_assert(sizeof(W) / sizeof(T) < 4096, "12-bit offsets");
};

// Per-lane items of the gradient-line step on levels without interphase faces
// where the traces are not folded, decoded at compile time (the order of the
// step's own decoding: axis k, then F = E, E+e_k, E+e_j, then the line t).
// a: offset of the line of F (uu) | offset of the line of F - e_k (ul) << 12 |
//    k << 24 | trace kind << 26 (1: F = E, 2: F = E + e_k) | slot of F << 28
// b: offset of the output line g_F (go) | face entry fi * D + k << 12 |
//    trace index (k (D + 1) + i) MT + t << 16
struct alignas(8) GradWord {
  unsigned a, b;
};
template <typename T, int D, int P>
struct GradItems {
  using W = Work<T, D, P, false>;
  using S = Sz<D, P, false>;
  static constexpr int M = S::M, NQ = S::NQ, MT = S::MT, NB = S::NB;
  static constexpr int PER_K = (3 * D - 1) * MT, N = D * PER_K;
  struct Tab {
    GradWord w[N];
  };
  static constexpr int off(size_t member) { return (int)(member / sizeof(T)); }
  static constexpr Tab make() {
    Tab tb{};
    for (int u = 0; u < N; ++u) {
      const int k = u / PER_K, r = u % PER_K, t = r % MT, q = r / MT;
      int fi = 0, i = 0;
      if (q < D) { fi = 0; i = q; }
      else if (q < 2 * D) { fi = 1 + k; i = q - D; }
      else { const int j0 = q - 2 * D; const int j = j0 < k ? j0 : j0 + 1; fi = 1 + j; i = j; }
      const int sF = fi == 0 ? 0 : 1 + D + (fi - 1);
      const int jj = fi - 1;
      const int sL = fi == 0 ? 1 + k : (k == jj ? 0 : 1 + 2 * D + jj * (D - 1) + (k < jj ? k : k - 1));
      int lo = 1;
      for (int j = 0; j < k; ++j) lo *= M;
      const int base = t % lo + lo * M * (t / lo);
      const int uu = off(offsetof(W, xs)) + sF * NB + i * NQ + base;
      const int ul = off(offsetof(W, xs)) + sL * NB + i * NQ + base;
      const int go = off(offsetof(W, g)) + (fi * D * D + i * D + k) * NQ + base;
      const int kind = fi == 0 ? 1 : (fi == 1 + k ? 2 : 0);
      const int tidx = (k * (D + 1) + i) * MT + t;
      tb.w[u].a = (unsigned)uu | ((unsigned)ul << 12) | ((unsigned)k << 24) | ((unsigned)kind << 26) | ((unsigned)sF << 28);
      tb.w[u].b = (unsigned)go | ((unsigned)(fi * D + k) << 12) | ((unsigned)tidx << 16);
    }
    return tb;
  }
  static constexpr Tab tab = make();
  static_assert(sizeof(W) / sizeof(T) < 4096 && 1 + 2 * D + D * (D - 1) <= 16 && D * (D + 1) * MT <= 256, "packing");
};

extern __shared__ __align__(16) unsigned char dyn_lds[];
template <typename T, int D, int P, bool IF>
__device__ __forceinline__ Work<T, D, P, IF>& work_lds() {
  return *reinterpret_cast<Work<T, D, P, IF>*>(dyn_lds);
}

// Registers of one element's evaluation between issuing its loads and
// staging them in LDS: the stencil (uniform), the raw loaded values, the face
// data (uniform).
template <typename T, int D, int P, int NT, bool IF = false>
struct ElemData {
  using S = Sz<D, P, IF>;
  static constexpr int XQ = (S::NB + NT - 1) / NT;
  static constexpr int MQ = Work<T, D, P, IF>::STAGE_M ? (S::NQ * S::NQ + NT - 1) / NT : 1;
  static constexpr int RQ = (S::MT * S::NQ + NT - 1) / NT;
  static constexpr int TQ = (S::MT * S::MT + NT - 1) / NT;
  int E;
  int se[S::NSLOT];              // element of each slot, -1 outside a wall
  int vmask;                     // bit sl set when slot sl exists
  T xr[S::NSLOT][XQ];
  T mr[MQ];
  T rv[D][RQ];
  T rvh[IF ? D : 1][RQ];
  T tr[D][2][TQ];
  T br[XQ];
  T tabv;                        // entry `lane` of the tables K, e0, e1, P
  unsigned char fty[S::NFS][D][2];
  T fwl[S::NFS][D][2], fwr[S::NFS][D][2];
  T dsv[S::NSLOT], dsp[S::NSLOT];
  unsigned titem;                // this lane's trace-step item (TraceItems), where the traces are not folded
  GradWord gitem;                // this lane's gradient-line item (GradItems), on the same levels without IF
};

// Computes the stencil and face data of E and issues every load of the
// element at once (addresses in bounds; masks are applied when staging).
template <typename T, int D, int P, int NT, bool IF, bool INT = false>
__device__ __forceinline__ void elem_issue(const DevLevel<T>& lev, const TabT<T>& tab, int E,
                                           const T* __restrict__ x, const T* __restrict__ b, int mode,
                                           ElemData<T, D, P, NT, IF>& d, int lane) {
  using S = Sz<D, P, IF>;
  using ED = ElemData<T, D, P, NT, IF>;
  constexpr int NQ = S::NQ, MT = S::MT, NB = S::NB, NFS = S::NFS, NSLOT = S::NSLOT;
  constexpr int XQ = ED::XQ, MQ = ED::MQ, RQ = ED::RQ, TQ = ED::TQ;
  const int n = lev.n, lgn = lev.lgn;
  d.E = E;
  constexpr int TABN = 3 * MAXM * MAXM + 2 * MAXM;
  static_assert(TABN <= 64, "one table entry per lane of the first wavefront");
  d.tabv = reinterpret_cast<const T*>(&tab)[lane < TABN ? lane : 0];
  if constexpr (!FOLD_TRACES<D>) {
    using TRI = TraceItems<T, D, P, IF>;
    static_assert(TRI::N <= 64, "one trace item per lane of the first wavefront");
    d.titem = TRI::tab.w[lane < TRI::N ? lane : 0];
    if constexpr (!IF) {
      using GRI = GradItems<T, D, P>;
      static_assert(GRI::N <= 64, "one gradient item per lane of the first wavefront");
      d.gitem = GRI::tab.w[lane < GRI::N ? lane : 0];
    }
  }
  int c[D];
  coords_of<D>(E, lgn, c);
  d.se[0] = E;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int cm[D], cp[D];
#pragma unroll
    for (int j = 0; j < D; ++j) cm[j] = cp[j] = c[j];
    // (INT: an interior element, whose stencil is complete)
    d.se[1 + k] = (shift1(cm, k, -1, n, lev.nf[k] == n) || INT) ? index_of<D>(cm, lgn) : -1;
    d.se[1 + D + k] = (shift1(cp, k, +1, n, lev.nf[k] == n) || INT) ? index_of<D>(cp, lgn) : -1;
#pragma unroll
    for (int q = 0; q < D - 1; ++q) {
      const int kk = q < k ? q : q + 1;
      int cq[D];
#pragma unroll
      for (int j = 0; j < D; ++j) cq[j] = c[j];
      const bool ok = shift1(cq, k, +1, n, lev.nf[k] == n) && shift1(cq, kk, -1, n, lev.nf[kk] == n);
      d.se[1 + 2 * D + k * (D - 1) + q] = (ok || INT) ? index_of<D>(cq, lgn) : -1;
    }
  }
  if constexpr (IF) {
    // two-step neighbours reached by the interphase liftings
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int cm[D], cp[D];
#pragma unroll
      for (int j = 0; j < D; ++j) cm[j] = cp[j] = c[j];
      const bool per = lev.nf[k] == n;
      const bool okm = shift1(cm, k, -1, n, per) && shift1(cm, k, -1, n, per);
      const bool okp = shift1(cp, k, +1, n, per) && shift1(cp, k, +1, n, per);
      d.se[Slot<D>::mm2(k)] = okm ? index_of<D>(cm, lgn) : -1;
      d.se[Slot<D>::pp2(k)] = okp ? index_of<D>(cp, lgn) : -1;
#pragma unroll
      for (int j = k + 1; j < D; ++j) {
        int cmm[D], cpp[D];
#pragma unroll
        for (int l = 0; l < D; ++l) cmm[l] = cpp[l] = c[l];
        const bool okmm = shift1(cmm, k, -1, n, per) && shift1(cmm, j, -1, n, lev.nf[j] == n);
        const bool okpp = shift1(cpp, k, +1, n, per) && shift1(cpp, j, +1, n, lev.nf[j] == n);
        d.se[Slot<D>::mm(k, j)] = okmm ? index_of<D>(cmm, lgn) : -1;
        d.se[Slot<D>::pp(k, j)] = okpp ? index_of<D>(cpp, lgn) : -1;
      }
    }
  }
  d.vmask = 0;
#pragma unroll
  for (int sl = 0; sl < NSLOT; ++sl) d.vmask |= (d.se[sl] >= 0 ? 1 : 0) << sl;
  if constexpr (INT) d.vmask = (1 << NSLOT) - 1;
#pragma unroll
  for (int sl = 0; sl < NSLOT; ++sl)
#pragma unroll
    for (int q = 0; q < XQ; ++q) {
      const int i = lane + q * NT;
      const int e = d.se[sl] >= 0 ? d.se[sl] : E;
      d.xr[sl][q] = x[(size_t)e * NB + (i < NB ? i : 0)];
    }
  {
    // issued whether or not the viscosity varies (a load under a branch makes
    // every later wait assume the branch skipped it): without viscosity data
    // the loads read x[0] and are discarded when staging
    const bool vm = lev.mmu != nullptr;
    const T* mb = vm ? lev.mmu : x;
    const T* rb = vm ? lev.rmu : x;
    if constexpr (Work<T, D, P, IF>::STAGE_M) {
#pragma unroll
      for (int q = 0; q < MQ; ++q) {
        const int t = lane + q * NT;
        d.mr[q] = mb[vm ? (size_t)E * NQ * NQ + (t < NQ * NQ ? t : 0) : 0];
      }
    }
    if constexpr (IF) {
      const T* rhb = vm ? lev.rmuh : x;
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
          const int t = lane + q * NT;
          const int e = d.se[1 + k];
          d.rvh[k][q] = rhb[vm ? ((size_t)(e >= 0 ? e : E) * D + k) * MT * NQ + (t < MT * NQ ? t : 0) : 0];
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int t = lane + q * NT;
        const int e = d.se[1 + D + k];
        d.rv[k][q] = rb[vm ? ((size_t)(e >= 0 ? e : E) * D + k) * MT * NQ + (t < MT * NQ ? t : 0) : 0];
      }
  }
  int fid0[D][2];
#pragma unroll
  for (int fi = 0; fi < NFS; ++fi) {
    int cF[D];
#pragma unroll
    for (int j = 0; j < D; ++j) cF[j] = c[j];
    bool valid = true;
    if (fi >= 1 && fi <= D) valid = shift1(cF, fi - 1, +1, n, lev.nf[fi - 1] == n);
    if (fi > D) valid = shift1(cF, fi - 1 - D, -1, n, lev.nf[fi - 1 - D] == n);
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const bool per = lev.nf[k] == n;
        int f = cF[k] + side;
        unsigned char ty = F_INTRA;
        if (!per && f == 0) ty = lev.stress ? (unsigned char)F_NONE : (unsigned char)F_DIR_LO;
        if (!per && f == n) ty = lev.stress ? (unsigned char)F_NONE : (unsigned char)F_DIR_HI;
        if (per) f &= n - 1;
        const int id = face_index<D>(cF, n, lev.nf[k], k, f);
        if constexpr (IF) {
          // interphase faces: type and lifting weights from the level's tables
          d.fty[fi][k][side] = valid ? lev.ftype[k][id] : (unsigned char)F_NONE;
          d.fwl[fi][k][side] = valid ? lev.fw[k][2 * id] : (T)0;
          d.fwr[fi][k][side] = valid ? lev.fw[k][2 * id + 1] : (T)0;
        } else if constexpr (INT) {
          // an interior element: every face of E and E+e_j is intraphase
          (void)valid;
          d.fty[fi][k][side] = F_INTRA;
          d.fwl[fi][k][side] = (T)0;
          d.fwr[fi][k][side] = (T)1;
        } else {
          // without interphase faces the type and the lifting weights follow
          // from the position: Dirichlet faces at the walls (weight 1 on their
          // element), intraphase faces elsewhere, (wL, wR) = (0, 1); stress
          // walls carry no face terms (type F_NONE, weights 0)
          d.fty[fi][k][side] = valid ? ty : (unsigned char)F_NONE;
          d.fwl[fi][k][side] = (valid && ty == F_DIR_HI) ? (T)1 : (T)0;
          d.fwr[fi][k][side] = (valid && ty != F_DIR_HI && ty != F_NONE) ? (T)1 : (T)0;
        }
        if (fi == 0) fid0[k][side] = id;
      }
  }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int q = 0; q < TQ; ++q) {
        const int t = lane + q * NT;
        d.tr[k][side][q] = lev.fT[k][(size_t)fid0[k][side] * MT * MT + (t < MT * MT ? t : 0)];
      }
#pragma unroll
  for (int q = 0; q < XQ; ++q) {
    const int i = lane + q * NT;
    d.br[q] = (mode == 0) ? b[(size_t)E * NB + (i < NB ? i : 0)] : (T)0;
  }
#pragma unroll
  for (int sl = 0; sl < NSLOT; ++sl) {
    d.dsv[sl] = (T)1;
    d.dsp[sl] = (T)1;
    if (lev.dscale) {
      const int e = d.se[sl] >= 0 ? d.se[sl] : E;
      d.dsv[sl] = lev.dscale[2 * e];
      d.dsp[sl] = lev.dscale[2 * e + 1];
    }
  }
}

// Writes the loaded element data to LDS (waits for the loads).
template <typename T, int D, int P, int NT, bool IF, bool INT = false>
__device__ __forceinline__ void elem_stage(const DevLevel<T>& lev, const ElemData<T, D, P, NT, IF>& d,
                                           Work<T, D, P, IF>& w, int lane) {
  if (lane < 3 * MAXM * MAXM + 2 * MAXM) w.tabs[lane] = d.tabv;
  using S = Sz<D, P, IF>;
  using ED = ElemData<T, D, P, NT, IF>;
  constexpr int NQ = S::NQ, MT = S::MT, NB = S::NB, NFS = S::NFS, NSLOT = S::NSLOT;
  constexpr int XQ = ED::XQ, MQ = ED::MQ, RQ = ED::RQ, TQ = ED::TQ;
  using W = Work<T, D, P, IF>;
#pragma unroll
  for (int sl = 0; sl < NSLOT; ++sl)
#pragma unroll
    for (int q = 0; q < XQ; ++q) {
      const int i = lane + q * NT;
      const T v = d.se[sl] >= 0 ? d.xr[sl][q] * (i >= D * NQ ? d.dsp[sl] : d.dsv[sl]) : (T)0;
      if constexpr (W::CPM) {
        if (sl < W::NXS) {
          if (i < NB) w.xs[sl < W::NXS ? sl : 0][i] = v;
        } else {
          // slot E+e_a-e_b keeps component a only
          const int pm = sl - W::NXS, a = pm / (D - 1);
          if (i >= a * NQ && i < (a + 1) * NQ) w.xpm[pm][i - a * NQ] = v;
        }
      } else {
        if (i < NB) w.xs[sl][i] = v;
      }
    }
  if (lev.mmu) {
    if constexpr (Work<T, D, P, IF>::STAGE_M) {
#pragma unroll
      for (int q = 0; q < MQ; ++q) {
        const int t = lane + q * NT;
        if (t < NQ * NQ) w.mm[t] = d.mr[q];
      }
    }
    if constexpr (IF) {
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
          const int t = lane + q * NT;
          if (t < MT * NQ) w.rrh[k][t] = d.se[1 + k] >= 0 ? d.rvh[k][q] : (T)0;
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const int t = lane + q * NT;
        if (t < MT * NQ) w.rr[k][t] = d.se[1 + D + k] >= 0 ? d.rv[k][q] : (T)0;
      }
  }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int q = 0; q < TQ; ++q) {
        const int t = lane + q * NT;
        if (t < MT * MT) w.th[side][k][t] = d.tr[k][side][q];
      }
  if (!INT && lane == 0) {
#pragma unroll
    for (int fi = 0; fi < NFS; ++fi)
#pragma unroll
      for (int k = 0; k < D; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          w.ft[fi][k][side] = d.fty[fi][k][side];
          w.fwl[fi][k][side] = d.fwl[fi][k][side];
          w.fwr[fi][k][side] = d.fwr[fi][k][side];
        }
  }
  __syncthreads();
}

// Phases 2-6 on the staged element: (A x)_E (mode 1) or b_E - (A x)_E
// (mode 0, b_E in bc) into w.res.  Operators of the diagonally scaled system
// D A D when lev.dscale is set (ds0v, ds0p: the element's scaling).
template <typename T, int D, int P, int NT, bool IF, bool INT = false>
__device__ __forceinline__ void elem_compute(const DevLevel<T>& lev, const TabT<T>& tab, int E, int vmask_in, int mode,
                                             const T* bc, T ds0v, T ds0p, unsigned titem, GradWord gitem,
                                             Work<T, D, P, IF>& w, int lane) {
  using S = Sz<D, P, IF>;
  constexpr int M = S::M, NQ = S::NQ, MT = S::MT, NB = S::NB;
  constexpr int XQ = ElemData<T, D, P, NT, IF>::XQ;
  using W = Work<T, D, P, IF>;
  const T hinv = lev.hinv;
  const T gam = (T)lev.gamma;
  // INT (an interior element): every stencil slot exists and every face of E
  // and E+e_j is intraphase with lifting weights (wL, wR) = (0, 1); the face
  // data are then constants instead of LDS reads
  const int vmask = INT ? (1 << S::NSLOT) - 1 : vmask_in;
  // ---- phase 2: gradient lines g_F = G_k u_i along axis k ----
  // per axis k: F = E (all i), F = E+e_k (all i), F = E+e_j (j != k, component
  // i = j); with interphase faces also F = E-e_k (all i), F = E-e_j (i = j).
  // With FOLD_TRACES further items: the traces of p along k (p_E at both
  // faces, p_{E-e_k} at its high face, p_{E+e_k} at its low face)
  //
  // One line: the traces of u_i along k at the faces of F, the lifted jumps,
  // and g_F = G_k u_i on the line (go), from the line of F (uu), of F - e_k
  // (ul) and, with interphase faces, of F + e_k (uh, read only when needed).
  auto line = [&](const T* uu, const T* ul, const T* uh, int st, unsigned char tlo, unsigned char thi, T wR, T wL,
                  T* go, T& trlo, T& trhi, T& trLhi) {
    T uv[M];
    trlo = 0;
    trhi = 0;
    trLhi = 0;
#pragma unroll
    for (int bb = 0; bb < M; ++bb) {
      uv[bb] = uu[bb * st];
      trlo += tab.e0[bb] * uv[bb];
      trhi += tab.e1[bb] * uv[bb];
      trLhi += tab.e1[bb] * ul[bb * st];
    }
    const T jlo = (tlo == F_NONE) ? (T)0 : wR * (trlo - (two_sided<IF>(tlo) ? trLhi : (T)0));
    // lifting of the high-face jump onto F (weight wL: Dirichlet, or an
    // interphase face lifting onto its low element)
    T jhi = (thi == F_DIR_HI) ? wL * trhi : (T)0;
    if constexpr (IF) {
      if (thi == F_INTRA || thi == F_INTER) {
        T trHlo = 0;
#pragma unroll
        for (int bb = 0; bb < M; ++bb) trHlo += tab.e0[bb] * uh[bb * st];
        jhi = wL * (trhi - trHlo);
      }
    }
#pragma unroll
    for (int ak = 0; ak < M; ++ak) {
      T v = tab.e0[ak] * jlo - tab.e1[ak] * jhi;
#pragma unroll
      for (int bb = 0; bb < M; ++bb) v += tab.K[ak * M + bb] * uv[bb];
      go[ak * st] = hinv * v;
    }
  };
  // the velocity traces along k that the fluxes need come out of these lines:
  // x_E at both faces (trx), x_{E-e_k} at its high face (trn[0]), x_{E+e_k}
  // at its low face (trn[1]); entries (k (D + 1) + i) MT + t
  T* const trx0 = &w.trx[0][0][0][0];
  T* const trx1 = &w.trx[1][0][0][0];
  T* const trn0 = &w.trn[0][0][0][0];
  T* const trn1 = &w.trn[1][0][0][0];
  if constexpr (!IF && !FOLD_TRACES<D>) {
    // each lane's item decoded at compile time (GradItems)
    if (lane < GradItems<T, D, P>::N) {
      const int sF = (int)(gitem.a >> 28), kind = (int)((gitem.a >> 26) & 3u), tidx = (int)((gitem.b >> 16) & 255u);
      if (!((vmask >> sF) & 1)) {
        if (kind == 2) trn1[tidx] = 0;   // no E + e_k: its traces read as zero
      } else {
        T* wb = reinterpret_cast<T*>(&w);
        const int k = (int)((gitem.a >> 24) & 3u), fk = (int)((gitem.b >> 12) & 15u);
        const unsigned char* ft = &w.ft[0][0][0];
        T trlo, trhi, trLhi;
        line(wb + (gitem.a & 0xfffu), wb + ((gitem.a >> 12) & 0xfffu), nullptr, stride_of<M>(k),
             INT ? (unsigned char)F_INTRA : ft[2 * fk], INT ? (unsigned char)F_INTRA : ft[2 * fk + 1],
             INT ? (T)1 : (&w.fwr[0][0][0])[2 * fk], INT ? (T)0 : (&w.fwl[0][0][0])[2 * fk + 1],
             wb + (gitem.b & 0xfffu), trlo, trhi, trLhi);
        if (kind == 1) {
          trx0[tidx] = trlo;
          trx1[tidx] = trhi;
          trn0[tidx] = trLhi;
        } else if (kind == 2) {
          trn1[tidx] = trlo;
        }
      }
    }
  } else {
    (void)gitem;
    constexpr int PER_K = (IF ? 5 * D - 2 : 3 * D - 1) * MT;
    constexpr int NPT = FOLD_TRACES<D> ? D * 4 * MT : 0;
    for (int u = lane; u < D * PER_K + NPT; u += NT) {
      if (u >= D * PER_K) {
        const int r = u - D * PER_K;
        const int t = r % MT, kind = (r / MT) % 4, k = r / (4 * MT);
        const int base = compose<M>(t, 0, k), st = stride_of<M>(k);
        const int sl = kind < 2 ? 0 : (kind == 2 ? Slot<D>::m(k) : Slot<D>::p(k));
        const bool hi = kind == 1 || kind == 2;   // trace at the element's high face (e1) or low face (e0)
        const T* src = &w.xs[sl][D * NQ + base];
        T v = 0;
#pragma unroll
        for (int bb = 0; bb < M; ++bb) v += w.tabs[MAXM * MAXM + (hi ? MAXM : 0) + bb] * src[bb * st];
        *(kind < 2 ? &w.trx[kind][k][D][t] : &w.trn[kind - 2][k][D][t]) = v;
        continue;
      }
      const int k = u / PER_K;
      const int r = u % PER_K;
      const int t = r % MT;
      const int q = r / MT;
      int fi, i;
      if (q < D) { fi = 0; i = q; }
      else if (q < 2 * D) { fi = 1 + k; i = q - D; }
      else if (q < 3 * D - 1) { const int j0 = q - 2 * D; const int j = j0 < k ? j0 : j0 + 1; fi = 1 + j; i = j; }
      else if (q < 4 * D - 1) { fi = 1 + D + k; i = q - (3 * D - 1); }
      else { const int j0 = q - (4 * D - 1); const int j = j0 < k ? j0 : j0 + 1; fi = 1 + D + j; i = j; }
      const int sF = f_slot<D>(fi);
      const int tidx = (k * (D + 1) + i) * MT + t;
      if (!((vmask >> sF) & 1)) {
        if (fi == 1 + k) trn1[tidx] = 0;   // no E + e_k: its traces read as zero
        continue;
      }
      const int base = compose<M>(t, 0, k), st = stride_of<M>(k);
      T trlo, trhi, trLhi;
      const int sL = low_slot<D>(fi, k);
      const T* ul;
      if constexpr (W::CPM) ul = sL < W::NXS ? &w.xs[sL < W::NXS ? sL : 0][i * NQ + base] : &w.xpm[sL - W::NXS][base];
      else ul = &w.xs[sL][i * NQ + base];
      line(&w.xs[sF][i * NQ + base], ul,
           IF ? &w.xs[IF ? high_slot<D>(fi, k) : 0][i * NQ + base] : nullptr, st,
           INT ? (unsigned char)F_INTRA : w.ft[fi][k][0], INT ? (unsigned char)F_INTRA : w.ft[fi][k][1],
           INT ? (T)1 : w.fwr[fi][k][0], INT ? (T)0 : w.fwl[fi][k][1], &w.g[fi][i * D + k][base], trlo, trhi, trLhi);
      if (fi == 0) {
        trx0[tidx] = trlo;
        trx1[tidx] = trhi;
        trn0[tidx] = trLhi;
      } else if (fi == 1 + k) {
        trn1[tidx] = trlo;
      }
    }
  }
  __syncthreads();
  // ---- phase 3: s_E = M_mu (g + gamma g^T) and the low-face traces of s at E+e_k ----
  {
    constexpr int NTRR = D * D * MT;
    // rows of s_E: with gamma = 1 s_E is symmetric and only the pairs i <= k
    // are formed (the other half is copied)
    const bool sym = lev.gamma != 0;
    const int NS0 = (sym ? D * (D + 1) / 2 : D * D) * NQ;
    for (int u = lane; u < NS0 + (IF ? 2 : 1) * NTRR; u += NT) {
      if (IF && u >= NS0 + NTRR) {
        // high-face traces of s at E - e_k (interphase liftings onto E)
        const int r = u - NS0 - NTRR;
        const int t = r % MT, i = (r / MT) % D, k = r / (MT * D);
        T v = 0;
        if ((vmask >> (1 + k)) & 1) {
          const int fi = 1 + D + k;
          const T* g1 = w.g[fi][i * D + k];
          const T* g2 = w.g[fi][k * D + i];
          if (lev.mmu) {
            const T* R = &w.rrh[IF ? k : 0][t * NQ];
#pragma unroll 8
            for (int bb = 0; bb < NQ; ++bb) v += R[bb] * (g1[bb] + gam * g2[bb]);
          } else {
            const int base = compose<M>(t, 0, k), st = stride_of<M>(k);
#pragma unroll
            for (int cc = 0; cc < M; ++cc) v += tab.e1[cc] * (g1[base + cc * st] + gam * g2[base + cc * st]);
            v *= lev.mu_const;
          }
        }
        w.trrh[IF ? k : 0][i][t] = v;
      } else if (lev.mmu && W::STAGE_M) {
        // variable viscosity, one code path for both kinds of row: s_E = M_mu
        // (g + gamma g^T) at node a of E, and the low-face trace of s at E+e_k
        // from its trace row (e0^T)_k M_mu
        const bool isS = u < NS0;
        const int a = u % NQ, pr = u / NQ;
        const int r = u - NS0;
        const int t = r % MT, ir = (r / MT) % D, kr = r / (MT * D);
        int si, sk;
        stress_pair<D>(pr, sym, si, sk);
        const int i = isS ? si : ir, k = isS ? sk : kr;
        const int fi = isS ? 0 : 1 + k;
        const bool valid = isS || ((vmask >> (1 + D + k)) & 1);
        const T* g1 = w.g[fi][i * D + k];
        const T* g2 = w.g[fi][k * D + i];
        const T* R = isS ? &w.mm[a * NQ] : &w.rr[k][t * NQ];   // M_mu symmetric: row a
        T v = 0;
#pragma unroll 8
        for (int bb = 0; bb < NQ; ++bb) v += R[bb] * (g1[bb] + gam * g2[bb]);
        v = valid ? v : (T)0;
        T* o = isS ? &w.s0[i * D + k][a] : &w.trr[k][i][t];
        *o = v;
        if (isS && sym && i != k) w.s0[k * D + i][a] = v;
      } else if (u < NS0) {
        const int a = u % NQ, pr = u / NQ;
        int i, k;
        stress_pair<D>(pr, sym, i, k);
        const T* g1 = w.g[0][i * D + k];
        const T* g2 = w.g[0][k * D + i];
        T v = 0;
        if (lev.mmu) {
          const T* Mm;
          if constexpr (W::STAGE_M) Mm = w.mm;
          else Mm = lev.mmu + (size_t)E * NQ * NQ;
#pragma unroll 8
          for (int bb = 0; bb < NQ; ++bb) v += Mm[a * NQ + bb] * (g1[bb] + gam * g2[bb]);   // M_mu symmetric
        } else {
          v = lev.mu_const * (g1[a] + gam * g2[a]);
        }
        w.s0[i * D + k][a] = v;
        if (sym && i != k) w.s0[k * D + i][a] = v;
      } else {
        const int r = u - NS0;
        const int t = r % MT, i = (r / MT) % D, k = r / (MT * D);
        T v = 0;
        if ((vmask >> (1 + D + k)) & 1) {
          const T* g1 = w.g[1 + k][i * D + k];
          const T* g2 = w.g[1 + k][k * D + i];
          if (lev.mmu) {
            const T* R = &w.rr[k][t * NQ];
#pragma unroll 8
            for (int bb = 0; bb < NQ; ++bb) v += R[bb] * (g1[bb] + gam * g2[bb]);
          } else {
            const int base = compose<M>(t, 0, k), st = stride_of<M>(k);
#pragma unroll
            for (int cc = 0; cc < M; ++cc) v += tab.e0[cc] * (g1[base + cc * st] + gam * g2[base + cc * st]);
            v *= lev.mu_const;
          }
        }
        w.trr[k][i][t] = v;
      }
    }
  }
  __syncthreads();
  // ---- phase 4 (without FOLD_TRACES): the remaining traces along each axis:
  // p_E at both faces, p_{E-e_k} at its high face and p_{E+e_k} at its low
  // face, s_E[i][k] at both faces; each lane's source, face and destination
  // come decoded from TraceItems ----
  if constexpr (!FOLD_TRACES<D>) {
    if (lane < TraceItems<T, D, P, IF>::N) {
      const T* src = reinterpret_cast<const T*>(&w) + (titem & 0xfffu);
      T* dst = reinterpret_cast<T*>(&w) + ((titem >> 12) & 0xfffu);
      const int st = stride_of<M>((int)((titem >> 24) & 3u));
      const T* e = &w.tabs[MAXM * MAXM + (int)((titem >> 26) & 1u) * MAXM];
      T v = 0;
#pragma unroll
      for (int bb = 0; bb < M; ++bb) v += e[bb] * src[bb * st];
      *dst = v;
    }
    __syncthreads();
  }
  // ---- phase 5: face fluxes, one code path for every kind of face and field
  // (the terms present are selected through their coefficients) ----
  for (int u = lane; u < D * 2 * (D + 1) * MT; u += NT) {
    const int tt = u % MT, f = (u / MT) % (D + 1), side = (u / (MT * (D + 1))) % 2, k = u / (2 * MT * (D + 1));
    const unsigned char ty = INT ? (unsigned char)F_INTRA : w.ft[0][k][side];
    const T wL = INT ? (T)0 : w.fwl[0][k][side], wR = INT ? (T)1 : w.fwr[0][k][side];
    const T* Th = &w.th[side][k][tt * MT];
    const bool vel = f < D, two = two_sided<IF>(ty), inter = is_inter<IF>(ty);
    const bool dir = ty == (side ? F_DIR_HI : F_DIR_LO), has = ty != F_NONE, intra = ty == F_INTRA;
    const int i = vel ? f : 0;
    const bool kk = vel && k == i;
    // penalty: Th applied to the face values of x_E (ca) and of the
    // neighbour (cb): u at Dirichlet and interphase faces, p at intraphase faces
    const T ca = vel ? ((dir || inter) ? (T)1 : (T)0) : (intra ? (T)-1 : (T)0);
    const T cb = vel ? (inter ? (T)-1 : (T)0) : (intra ? (T)1 : (T)0);
    const T* xa = w.trx[side][k][f];
    const T* xb = w.trn[side][k][f];
    T v = 0;
#pragma unroll
    for (int q = 0; q < MT; ++q) v += Th[q] * (ca * xa[q] + cb * xb[q]);
    // averages of s and p.  Low face (E is its high element R): wR s_E, the
    // interphase lifting onto E - e_k (wL, trrh), wR p_E, wL p_{E-e_k}; high
    // face (E is its low element L): wL s_E, wR s_{E+e_k}, wL p_E, wR p_{E+e_k}
    T cs, cr, cpx, cpn, sr;
    if (side == 0) {
      cs = (vel && has) ? wR : (T)0;
      cr = (IF && vel && two) ? wL : (T)0;
      cpx = (kk && has) ? -wR : (T)0;
      cpn = (IF && kk && two) ? -wL : (T)0;
      sr = IF ? w.trrh[IF ? k : 0][i][tt] : (T)0;
    } else {
      cs = vel ? -wL : (T)0;
      cr = (vel && two) ? -wR : (T)0;
      cpx = kk ? wL : (T)0;
      cpn = (kk && two) ? wR : (T)0;
      sr = w.trr[k][i][tt];
    }
    // s_E[i][k] at this face
    T se;
    if constexpr (FOLD_TRACES<D>) {
      const T* sv = &w.s0[i * D + k][compose<M>(tt, 0, k)];
      const int st = stride_of<M>(k);
      se = 0;
#pragma unroll
      for (int bb = 0; bb < M; ++bb) se += w.tabs[MAXM * MAXM + (side ? MAXM : 0) + bb] * sv[bb * st];
    } else {
      se = w.trs[side][k][i][tt];
    }
    v += cs * se + cr * sr + cpx * w.trx[side][k][D][tt] + cpn * w.trn[side][k][D][tt];
    w.flux[side][k][f][tt] = hinv * v;
  }
  __syncthreads();
  // ---- phase 6: assemble (A x)_E and the residual, one code path for the
  // rows of u (div s, grad p, rho/delta u) and of p (div u) ----
#pragma unroll
  for (int q = 0; q < XQ; ++q) {
    const int t = lane + q * NT;
    if (t >= NB) break;
    const int f = t / NQ, a = t % NQ;
    const bool vel = f < D;
    const int i = vel ? f : 0;
    T acc = vel ? lev.rho_delta * w.xs[0][t] : (T)0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int ak = k == 0 ? digit_c<M, 0>(a) : (k == 1 ? digit_c<M, 1>(a) : digit_c<M, 2>(a));
      const int tt = k == 0 ? tang_c<M, 0>(a) : (k == 1 ? tang_c<M, 1>(a) : tang_c<M, 2>(a));
      const int base = compose<M>(tt, 0, k), st = stride_of<M>(k);
      const T* sv = &w.s0[i * D + k][base];
      const T* pv = &w.xs[0][D * NQ + base];
      T vol = 0, pvol = 0;
#pragma unroll
      for (int bb = 0; bb < M; ++bb) {
        vol += w.tabs[bb * M + ak] * sv[bb * st];
        pvol += w.tabs[bb * M + ak] * pv[bb * st];
      }
      const T cv = vel ? hinv : (T)0, cp = (vel && k == i) ? -hinv : (T)0, cg = vel ? (T)0 : (T)-1;
      acc += cv * vol + cp * pvol + cg * w.g[0][k * D + k][a] + w.tabs[MAXM * MAXM + ak] * w.flux[0][k][f][tt] +
             w.tabs[MAXM * MAXM + MAXM + ak] * w.flux[1][k][f][tt];
    }
    if (lev.dscale) acc *= (f == D ? ds0p : ds0v);
    w.res[t] = (mode == 0) ? bc[q] - acc : acc;
  }
  __syncthreads();
}

// Work-groups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b mod 8).  Give each XCD a contiguous range of the launch's elements so
// that neighbours in a stencil are read through the same L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G / NXCD, r = G % NXCD;
  const int x = b % NXCD, j = b / NXCD;
  return x * q + (x < r ? x : r) + j;
}

struct NoHook {
  __device__ void operator()() const {}
};

template <typename T, int D, int P, int NT, bool IF, bool INT, class Hook>
__device__ __forceinline__ void element_operator_v(const DevLevel<T>& lev, const TabT<T>& tab, int E,
                                                   const T* __restrict__ x, const T* __restrict__ b, int mode,
                                                   Work<T, D, P, IF>& w, Hook& after_loads) {
  ElemData<T, D, P, NT, IF> d;
  const int lane = threadIdx.x;
  elem_issue<T, D, P, NT, IF, INT>(lev, tab, E, x, b, mode, d, lane);
  after_loads();
  elem_stage<T, D, P, NT, IF, INT>(lev, d, w, lane);
  elem_compute<T, D, P, NT, IF, INT>(lev, tab, E, d.vmask, mode, d.br, d.dsv[0], d.dsp[0], d.titem, d.gitem, w,
                                     lane);
}

// Element E is interior when along every axis the grid is periodic or
// 1 <= c_k <= n - 3: its stencil is complete and every face of E and of
// E+e_j is an intraphase face.
template <typename T, int D>
__device__ __forceinline__ bool interior_elem(const DevLevel<T>& lev, int E) {
  int c[D];
  coords_of<D>(E, lev.lgn, c);
  bool in = true;
#pragma unroll
  for (int k = 0; k < D; ++k) in = in && (lev.nf[k] == lev.n || (c[k] >= 1 && c[k] <= lev.n - 3));
  return in;
}

// Evaluates (A x)_E (mode 1) or b_E - (A x)_E (mode 0) into w.res.
// `after_loads` runs once the element's loads are issued and before they are
// waited for: loads it issues then overlap the evaluation.  Levels without
// interphase faces evaluate interior elements with the face data as constants.
template <typename T, int D, int P, int NT, bool IF, class Hook = NoHook>
__device__ __forceinline__ void element_operator(const DevLevel<T>& lev, const TabT<T>& tab, int E,
                                                 const T* __restrict__ x, const T* __restrict__ b,
                                                 int mode, Work<T, D, P, IF>& w, Hook after_loads = Hook()) {
  if constexpr (!IF) {
    if (interior_elem<T, D>(lev, E)) {
      element_operator_v<T, D, P, NT, IF, true>(lev, tab, E, x, b, mode, w, after_loads);
      return;
    }
  }
  element_operator_v<T, D, P, NT, IF, false>(lev, tab, E, x, b, mode, w, after_loads);
}

// Raw words of one lane's load of the inverse (sym_tiles: LB bytes) and entry
// u of them in the arithmetic type
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename TI>
using InvWord = std::conditional_t<sizeof(TI) == 2, u32x2, u32x4>;

template <typename T, typename TI>
__device__ __forceinline__ T inv_entry(const InvWord<TI>& raw, int u) {
  if constexpr (sizeof(TI) == 8) {
    const unsigned long long bits = (unsigned long long)raw[2 * u] | ((unsigned long long)raw[2 * u + 1] << 32);
    return (T)__longlong_as_double((long long)bits);
  } else if constexpr (sizeof(TI) == 4) {
    return (T)__uint_as_float(raw[u]);
  } else {
    const unsigned int word = raw[u >> 1];
    const unsigned int bits = (u & 1) ? (word & 0xffff0000u) : (word << 16);
    return (T)__uint_as_float(bits);
  }
}

template <typename T>
__device__ __forceinline__ T shfl_xor64(T v, int m) {
  return __shfl_xor(v, m, 64);
}

// ---------------------------------------------------------------------------
// Smoother: one colour pass.  x_E += Ainv_E (b - A x)_E for the listed elements.
// Ainv_E is symmetric and stored as its upper 16 x 16 tiles (sym_tiles); the
// first wave forms the product: for tile (i, j) lane (row, 4 columns) adds
// T r_j to its row of y_i and, off the diagonal, T^T r_i to its columns of y_j;
// the partial sums are reduced across lanes.  The first tiles are requested
// before the residual is evaluated.
// ---------------------------------------------------------------------------
// Tiles of the element's inverse requested ahead of the product (32 registers
// of words) and the product itself: the first wavefront forms y = Ainv res
// from the stored upper tiles; y = part[0] + part[1] on return (after a
// work-group barrier).
template <typename TI, int NB>
struct SymProd {
  static constexpr SymTiles LY = sym_tiles(NB, (int)sizeof(TI));
  static constexpr int TR = LY.TR, NTILE = LY.NTILE, H = LY.H, EL = LY.EL;
  static constexpr int ESTRIDE = sym_tile_off(TR, NTILE);   // entries per element
  using Word = InvWord<TI>;
  static constexpr int PFMAX = 32 / (H * (int)(sizeof(Word) / 4));
  static constexpr int PF = NTILE < PFMAX ? NTILE : PFMAX;
};

// tile row of tile t (tiles numbered row by row over the upper triangle)
constexpr int sym_tile_row(int TR, int t) {
  int i = 0;
  while (t >= TR - i) { t -= TR - i; ++i; }
  return i;
}

// word of lane l's load h of tile t (diag: a diagonal tile, whose lanes below
// the diagonal read the first stored block and discard it)
template <typename TI, int NB>
__device__ __forceinline__ int sym_word(int t, bool diag, int h, int l) {
  using SP = SymProd<TI, NB>;
  const int r = l >> 2, cb = l & 3;
  const int slot = diag ? (cb >= (r >> 2) ? sym_dslot(r, cb) : 0) : l;
  return sym_tile_off(SP::TR, t) / SP::EL + h * (diag ? SYM_DBLOCKS : 64) + slot;
}

// every lane issues the loads (lanes 64.. repeat the first wavefront's
// addresses): a load under a branch would make the waits of the evaluation
// that follows assume it was skipped, and wait for these tiles too
template <typename TI, int NB>
__device__ __forceinline__ void sym_prefetch(const InvWord<TI>* __restrict__ Ai,
                                             InvWord<TI> (&pre)[SymProd<TI, NB>::PF][SymProd<TI, NB>::H], int lane) {
  using SP = SymProd<TI, NB>;
  const int l = lane & 63;
#pragma unroll
  for (int t = 0; t < SP::PF; ++t) {
    const int i = sym_tile_row(SP::TR, t);
    const bool diag = t == i * SP::TR - i * (i - 1) / 2;
#pragma unroll
    for (int h = 0; h < SP::H; ++h) pre[t][h] = __builtin_nontemporal_load(&Ai[sym_word<TI, NB>(t, diag, h, l)]);
  }
}

// red: LDS scratch of 256 TR entries (not overlapping res or part), for the
// column sums of the transposed contributions
template <typename T, typename TI, int NB, int NT>
__device__ __forceinline__ void sym_product(const InvWord<TI>* __restrict__ Ai,
                                            const InvWord<TI> (&pre)[SymProd<TI, NB>::PF][SymProd<TI, NB>::H],
                                            const T* res, T (*part)[16 * SymProd<TI, NB>::TR], T* red, int lane) {
  using SP = SymProd<TI, NB>;
  constexpr int TR = SP::TR, PF = SP::PF, H = SP::H, EL = SP::EL;
  using Word = typename SP::Word;
  if (lane < 64) {
    const int l = lane;
    const int row = l >> 2, c4 = (l & 3) * 4;
    T dir[TR], trn[TR][4];
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      dir[i] = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) trn[i][v] = 0;
    }
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const T ri = (16 * i + row < NB) ? res[16 * i + row] : (T)0;
#pragma unroll
      for (int j = i; j < TR; ++j) {
        const int t = i * TR - i * (i - 1) / 2 + (j - i);
        const bool diag = j == i;
        Word raw[H];
#pragma unroll
        for (int h = 0; h < H; ++h)
          raw[h] = (t < PF) ? pre[t < PF ? t : 0][h] : __builtin_nontemporal_load(&Ai[sym_word<TI, NB>(t, diag, h, l)]);
        // a diagonal tile: blocks left of the diagonal block are not stored
        // (their entries come from the mirrored blocks right of it)
        const bool keep = !diag || (l & 3) >= (row >> 2);
        T a[4], rj[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          a[v] = keep ? inv_entry<T, TI>(raw[v / EL], v % EL) : (T)0;
          const int cj = 16 * j + c4 + v;
          rj[v] = cj < NB ? res[cj] : (T)0;
        }
        dir[i] += a[0] * rj[0] + a[1] * rj[1] + a[2] * rj[2] + a[3] * rj[3];
        if (!diag || (l & 3) > (row >> 2)) {
#pragma unroll
          for (int v = 0; v < 4; ++v) trn[j][v] += a[v] * ri;
        }
      }
    }
    // dir: sum over the 4 lanes of a row (cross-lane); trn: the 16 rows'
    // partial column sums go through LDS (red[row][column])
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      dir[i] += shfl_xor64(dir[i], 1);
      dir[i] += shfl_xor64(dir[i], 2);
    }
    if ((l & 3) == 0) {
#pragma unroll
      for (int i = 0; i < TR; ++i) part[0][16 * i + row] = dir[i];
    }
#pragma unroll
    for (int j = 0; j < TR; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[row * 16 * TR + 16 * j + c4 + v] = trn[j][v];
  }
  __syncthreads();
  for (int col = lane; col < 16 * TR; col += NT) {
    T sum = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) sum += red[r * 16 * TR + col];
    part[1][col] = sum;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Smoother: one colour pass.  x_E += Ainv_E (b - A x)_E for the listed elements.
// Ainv_E is symmetric and stored as its upper 16 x 16 tiles (sym_tiles); the
// first wave forms the product: for tile (i, j) lane (row, 4 columns) adds
// T r_j to its row of y_i and, off the diagonal, T^T r_i to its columns of y_j;
// the partial sums are reduced across lanes.  The first tiles are requested
// before the residual is evaluated.
// ---------------------------------------------------------------------------
template <typename T, typename TI, int D, int P, int NT, bool IF>
__global__ __launch_bounds__(NT) void k_smooth_colour(DevLevel<T> lev, TabT<T> tab, const int* __restrict__ elems,
                                                      int pcol, const TI* __restrict__ inv, const T* __restrict__ b,
                                                      T* __restrict__ x, int inv_shared) {
  using S = Sz<D, P>;
  constexpr int NB = S::NB;
  using SP = SymProd<TI, NB>;
  Work<T, D, P, IF>& w = work_lds<T, D, P, IF>();
  __shared__ T part[2][16 * SP::TR];
  const int lane = threadIdx.x;
  const int idx = xcd_remap(blockIdx.x, gridDim.x);
  const int E = colour_elem<D>(idx, pcol, lev.lgn, elems);
  // inv_shared: one inverse for every element of the level (read through the caches)
  const auto* Ai = reinterpret_cast<const typename SP::Word*>(inv + (inv_shared ? (size_t)0 : (size_t)idx * SP::ESTRIDE));
  typename SP::Word pre[SP::PF][SP::H];
  element_operator<T, D, P, NT, IF>(lev, tab, E, x, b, 0, w, [&]() { sym_prefetch<TI, NB>(Ai, pre, lane); });
  // the evaluation's arrays before res are free again: column-sum scratch
  using W = Work<T, D, P, IF>;
  static_assert(offsetof(W, res) >= 256 * SP::TR * sizeof(T), "LDS scratch");
  sym_product<T, TI, NB, NT>(Ai, pre, w.res, part, reinterpret_cast<T*>(&w), lane);
  for (int r = lane; r < NB; r += NT) x[(size_t)E * NB + r] += part[0][r] + part[1][r];
}


// The product of one wavefront with the stored upper tiles, streamed column
// by column of tiles (j outer, i <= j inner), so that the transposed sums of
// a tile column are complete when the column ends and leave the registers:
// live are the row sums of every tile row, the row values r_i met so far and
// one column's transposed sums.  Tile requests run WIN tiles ahead of their
// use in a ring of registers; a scheduling barrier after each request keeps
// the later requests behind it (otherwise every tile of a large block is
// hoisted to the start: for n_b = 108 in FP64 that took over 400 registers
// and left one wavefront per SIMD).  The transposed sums of a column are
// summed over the lanes that share bits 0-1 and 4-5 of the lane index (bits
// 2-3 cross-lane, then bits 4-5 through LDS: red holds 64 TR entries).
// y = part[0] + part[1] on return.
// tile number and kind of the s-th tile in column order, as a table decoded
// at compile time (indexed with unrolled loop counters, its entries fold into
// immediates)
template <int TR>
struct ColOrder {
  struct Tab {
    int tile[TR * (TR + 1) / 2];
    bool diag[TR * (TR + 1) / 2];
  };
  static constexpr Tab make() {
    Tab tb{};
    int s = 0;
    for (int j = 0; j < TR; ++j)
      for (int i = 0; i <= j; ++i, ++s) {
        tb.tile[s] = i * TR - i * (i - 1) / 2 + (j - i);
        tb.diag[s] = i == j;
      }
    return tb;
  }
  static constexpr Tab tab = make();
};
// tiles in flight per wavefront in the streamed product: 64 registers of requests
template <typename TI, int NB>
constexpr int stream_window() {
  using SP = SymProd<TI, NB>;
  constexpr int regs = SP::H * (int)sizeof(typename SP::Word) / 4;
  return 64 / regs < 1 ? 1 : 64 / regs;
}
template <typename T, typename TI, int NB, int WIN>
__device__ __forceinline__ void sym_product_stream(const InvWord<TI>* __restrict__ Ai, const T* __restrict__ rsrc,
                                                   T* res, T (*part)[16 * SymProd<TI, NB>::TR], T* red, int lane) {
  using SP = SymProd<TI, NB>;
  constexpr int TR = SP::TR, NTILE = SP::NTILE, H = SP::H, EL = SP::EL;
  using Word = typename SP::Word;
  const int l = lane;
  const int row = l >> 2, c4 = (l & 3) * 4;
  auto request = [&](int s, Word (&w)[H]) {
    const int t = ColOrder<TR>::tab.tile[s];
    const bool diag = ColOrder<TR>::tab.diag[s];
#pragma unroll
    for (int h = 0; h < H; ++h) w[h] = __builtin_nontemporal_load(&Ai[sym_word<TI, NB>(t, diag, h, l)]);
  };
  Word ring[WIN][H];
#pragma unroll
  for (int s = 0; s < WIN && s < NTILE; ++s) request(s, ring[s]);
  // the residual after the first requests, so that they are in flight meanwhile
  for (int q = lane; q < NB; q += 64) res[q] = rsrc[q];
  __syncthreads();
  T dir[TR], ri[TR];
#pragma unroll
  for (int i = 0; i < TR; ++i) dir[i] = 0;
#pragma unroll
  for (int j = 0; j < TR; ++j) {
    ri[j] = (16 * j + row < NB) ? res[16 * j + row] : (T)0;
    T rj[4], trn[4] = {0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) rj[v] = (16 * j + c4 + v < NB) ? res[16 * j + c4 + v] : (T)0;
#pragma unroll
    for (int i = 0; i <= j; ++i) {
      const int s = j * (j + 1) / 2 + i;
      const bool diag = j == i;
      Word raw[H];
#pragma unroll
      for (int h = 0; h < H; ++h) raw[h] = ring[s % WIN][h];
      if (s + WIN < NTILE) request(s + WIN, ring[s % WIN]);
      __builtin_amdgcn_sched_barrier(0);
      // a diagonal tile: blocks left of the diagonal block are not stored
      const bool keep = !diag || (l & 3) >= (row >> 2);
      T a[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) a[v] = keep ? inv_entry<T, TI>(raw[v / EL], v % EL) : (T)0;
      dir[i] += a[0] * rj[0] + a[1] * rj[1] + a[2] * rj[2] + a[3] * rj[3];
      if (!diag || (l & 3) > (row >> 2)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) trn[v] += a[v] * ri[i];
      }
    }
    // column j done: its transposed sums over the rows of the lane's group
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      trn[v] += shfl_xor64(trn[v], 4);
      trn[v] += shfl_xor64(trn[v], 8);
    }
    if (((l >> 2) & 3) == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(l >> 4) * 16 * TR + 16 * j + c4 + v] = trn[v];
    }
  }
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    dir[i] += shfl_xor64(dir[i], 1);
    dir[i] += shfl_xor64(dir[i], 2);
  }
  if ((l & 3) == 0) {
#pragma unroll
    for (int i = 0; i < TR; ++i) part[0][16 * i + row] = dir[i];
  }
  __syncthreads();
  for (int col = lane; col < 16 * TR; col += 64)
    part[1][col] = red[col] + red[16 * TR + col] + red[32 * TR + col] + red[48 * TR + col];
  __syncthreads();
}

// First colour pass from x = 0: the residual is b, so x_E = Ainv_E b_E with
// no operator evaluation; the work-groups also set every other element of
// the level to zero (zl: those elements, nzero of them; work-group idx takes
// entries idx, idx + cnt, ...).  Same results as zeroing x and running the
// colour pass.
template <typename T, typename TI, int D, int P, int NT>
__global__ __launch_bounds__(NT) void k_first_colour(int lgn, const int* __restrict__ elems, int pcol,
                                                     const TI* __restrict__ inv, const T* __restrict__ b,
                                                     T* __restrict__ x, const int* __restrict__ zl, int nzero) {
  using S = Sz<D, P>;
  constexpr int NB = S::NB;
  using SP = SymProd<TI, NB>;
  __shared__ alignas(16) T res[NB];
  __shared__ T part[2][16 * SP::TR];
  __shared__ T red[(NT == 64 ? 64 : 256) * SP::TR];
  const int lane = threadIdx.x;
  const int idx = xcd_remap(blockIdx.x, gridDim.x);
  const int E = colour_elem<D>(idx, pcol, lgn, elems);
  const auto* Ai = reinterpret_cast<const typename SP::Word*>(inv + (size_t)idx * SP::ESTRIDE);
  if constexpr (NT == 64) {
    // one wavefront per element: the streamed product (as in the split pass)
    for (int m = idx; m < nzero; m += (int)gridDim.x) {
      const size_t z = (size_t)zl[m] * NB;
      for (int t = lane; t < NB; t += NT) x[z + t] = (T)0;
    }
    sym_product_stream<T, TI, NB, stream_window<TI, NB>()>(Ai, b + (size_t)E * NB, res, part, red, lane);
  } else {
    typename SP::Word pre[SP::PF][SP::H];
    sym_prefetch<TI, NB>(Ai, pre, lane);
    for (int t = lane; t < NB; t += NT) res[t] = b[(size_t)E * NB + t];
    for (int m = idx; m < nzero; m += (int)gridDim.x) {
      const size_t z = (size_t)zl[m] * NB;
      for (int t = lane; t < NB; t += NT) x[z + t] = (T)0;
    }
    __syncthreads();
    sym_product<T, TI, NB, NT>(Ai, pre, res, part, red, lane);
  }
  for (int r = lane; r < NB; r += NT) x[(size_t)E * NB + r] = part[0][r] + part[1][r];
}

// Second half of a colour pass split into residual and product: x_E += Ainv_E
// r[idx] for the listed elements, with the per-element inverses of the tile
// layout.  One wavefront per element: the evaluation of the residual (an
// LDS-bound kernel of its own) no longer holds the inverse's stream back, and
// many elements' tiles are in flight per CU.
template <typename T, typename TI, int D, int P>
__global__ __launch_bounds__(64) void k_apply_inverse(int lgn, const int* __restrict__ elems, int pcol, int ibase,
                                                      const TI* __restrict__ inv, const T* __restrict__ r,
                                                      T* __restrict__ x) {
  using S = Sz<D, P>;
  constexpr int NB = S::NB;
  using SP = SymProd<TI, NB>;
  constexpr int WIN = stream_window<TI, NB>();
  __shared__ alignas(16) T res[NB];
  __shared__ T part[2][16 * SP::TR];
  __shared__ T red[64 * SP::TR];
  const int lane = threadIdx.x;
  const int idx = ibase + xcd_remap(blockIdx.x, gridDim.x);
  const int E = colour_elem<D>(idx, pcol, lgn, elems);
  const auto* Ai = reinterpret_cast<const typename SP::Word*>(inv + (size_t)idx * SP::ESTRIDE);
  sym_product_stream<T, TI, NB, WIN>(Ai, r + (size_t)idx * NB, res, part, red, lane);
  for (int q = lane; q < NB; q += 64) x[(size_t)E * NB + q] += part[0][q] + part[1][q];
}

template <typename T, int D, int P, int NT, bool IF>
__global__ __launch_bounds__(NT) void k_residual(DevLevel<T> lev, TabT<T> tab, const T* __restrict__ b,
                                                 const T* __restrict__ x, T* __restrict__ out, int mode) {
  using S = Sz<D, P>;
  Work<T, D, P, IF>& w = work_lds<T, D, P, IF>();
  const int E = xcd_remap(blockIdx.x, gridDim.x);
  element_operator<T, D, P, NT, IF>(lev, tab, E, x, b, mode, w);
  for (int t = threadIdx.x; t < S::NB; t += NT) out[(size_t)E * S::NB + t] = w.res[t];
}

// Residual of the listed elements into a compact buffer: r[idx] = (b - A x)_E,
// E = elems[idx] (the first half of a colour pass with a shared inverse).
template <typename T, int D, int P, int NT, bool IF>
__global__ __launch_bounds__(NT) void k_colour_residual(DevLevel<T> lev, TabT<T> tab, const int* __restrict__ elems,
                                                        int pcol, int ibase, const T* __restrict__ b,
                                                        const T* __restrict__ x, T* __restrict__ r) {
  using S = Sz<D, P, IF>;
  Work<T, D, P, IF>& w = work_lds<T, D, P, IF>();
  const int idx = ibase + xcd_remap(blockIdx.x, gridDim.x);
  element_operator<T, D, P, NT, IF>(lev, tab, colour_elem<D>(idx, pcol, lev.lgn, elems), x, b, 0, w);
  for (int t = threadIdx.x; t < S::NB; t += NT) r[(size_t)idx * S::NB + t] = w.res[t];
}

// x_E += Ainv r[idx] for the listed elements, Ainv shared by every element of
// the level (translation-invariant operator: constant coefficients, periodic
// grid).  A dense product Ainv [NB x NB] * R [NB x n] on vector ALUs (n is one
// colour, tens of thousands of columns; the work is bound by streaming R and x).
// Ainv is given k-major and zero-padded to RS rows (a[k * NB + row], k < RS);
// it is staged in LDS when it fits in 64 KB, else read through the caches.
// A work-group of 256 threads has G = 256 / NB element groups of NB threads
// (one output row each); a thread accumulates Q elements of its group, so a
// tile holds TE = G * Q elements.  R tiles are staged in LDS with row stride
// RS (16-byte aligned) and read as 16-byte broadcasts.
constexpr int SU_THREADS = 256;
template <typename T, int NB, int Q_>
struct SuCfg {
  static constexpr int V = 16 / sizeof(T);                    // entries per 16-byte read
  static constexpr int RS = (NB + V - 1) / V * V;
  static constexpr int G = SU_THREADS / NB;
  static constexpr int Q = Q_;
  static constexpr int TE = G * Q;
  // A in LDS only while it leaves room for several work-groups per CU
  static constexpr bool A_LDS = (size_t)RS * NB * sizeof(T) <= 32768;
  static constexpr int A_SZ = A_LDS ? RS * NB : 1;
};

// first: first pass from x = 0 (r is b, read at the listed elements; x_E is
// assigned; the nzero elements zl of the other colours are set to zero)
template <typename T, int NB, int Q>
__global__ __launch_bounds__(SU_THREADS) void k_shared_update(int nelems, const T* __restrict__ ainv,
                                                              const T* __restrict__ r, const int* __restrict__ elems,
                                                              T* __restrict__ x, int first, const int* __restrict__ zl,
                                                              int nzero) {
  using C = SuCfg<T, NB, Q>;
  using V4 = std::conditional_t<sizeof(T) == 8, double2, float4>;
  __shared__ alignas(16) T As[C::A_SZ];
  __shared__ alignas(16) T Rs[C::TE * C::RS];
  __shared__ int Eo[C::TE];   // x offset of each staged element (-1 past the end)
  const int tid = threadIdx.x;
  if constexpr (C::A_LDS)
    for (int i = tid; i < C::RS * NB; i += SU_THREADS) As[i] = ainv[i];
  const T* A = C::A_LDS ? As : ainv;
  const int g = tid / NB, row = tid - g * NB;
  const bool active = g < C::G;
  const int ntile = (nelems + C::TE - 1) / C::TE;
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int base = tile * C::TE;
    const int cnt = min(C::TE, nelems - base);
    __syncthreads();
    // (a tile can hold more elements than the work-group has threads:
    // 21 groups x 16 = 336 for NB = 12)
    for (int i = tid; i < C::TE; i += SU_THREADS) Eo[i] = i < cnt ? elems[base + i] * NB : -1;
    __syncthreads();
    // all loads of the tile issued before any is stored (unrolled; masked
    // loads read r[0] and are discarded)
    constexpr int TOT = C::TE * C::RS, ITER = (TOT + SU_THREADS - 1) / SU_THREADS;
    T v[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int i = tid + SU_THREADS * it;
      const int e = i / C::RS, k = i - e * C::RS;
      const bool ok = i < TOT && e < cnt && k < NB;
      v[it] = r[ok ? (first ? (size_t)Eo[e] + k : (size_t)(base + e) * NB + k) : 0];
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int i = tid + SU_THREADS * it;
      const int e = i / C::RS, k = i - e * C::RS;
      if (i < TOT) Rs[i] = (e < cnt && k < NB) ? v[it] : T(0);
    }
    __syncthreads();
    if (active) {
      T acc[C::Q];
#pragma unroll
      for (int q = 0; q < C::Q; ++q) acc[q] = 0;
      const T* Rg = Rs + g * C::Q * C::RS;
#pragma unroll 2
      for (int k = 0; k < C::RS; k += C::V) {
        T a[C::V];
#pragma unroll
        for (int j = 0; j < C::V; ++j) a[j] = A[(k + j) * NB + row];
#pragma unroll
        for (int q = 0; q < C::Q; ++q) {
          const V4 rv = *reinterpret_cast<const V4*>(Rg + q * C::RS + k);
          if constexpr (C::V == 4)
            acc[q] += a[0] * rv.x + a[1] * rv.y + a[2] * rv.z + a[3] * rv.w;
          else
            acc[q] += a[0] * rv.x + a[1] * rv.y;
        }
      }
#pragma unroll
      for (int q = 0; q < C::Q; ++q) {
        const int e = g * C::Q + q;
        if (e < cnt) {
          T* xe = &x[(size_t)Eo[e] + row];
          *xe = first ? acc[q] : *xe + acc[q];
        }
      }
    }
  }
  for (int64_t i = (int64_t)blockIdx.x * SU_THREADS + tid; i < (int64_t)nzero * NB; i += (int64_t)gridDim.x * SU_THREADS)
    x[(size_t)zl[i / NB] * NB + i % NB] = T(0);
}

// The same update on the matrix cores (FP32 MFMA 16x16x4) for large colours:
// X_c += Ainv [NB x NB] R_c [NB x n] is a dense product.  Ainv is padded to
// KP = roundup(NB, 16); each of the 4 wavefronts keeps the A operands of its
// 16-row tiles for the whole launch in registers (lane l holds A[16 t + l % 16]
// [4 s + l / 16] for k-step s).  A work-group stages 32 elements of R in LDS
// (B[k][n] = R[n][k]; lane l reads B[l / 16][l % 16] of a 16-element block),
// and lane l receives rows 4 (l / 16) .. + 3 of column l % 16 of each 16 x 16
// output tile.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// one 16 x 16 x 4 matrix-core step in the arithmetic type: A 16 x 4 (lane
// i + 16 k holds A[i][k]) and B 4 x 16 (lane j + 16 k holds B[k][j]) in both;
// the accumulator 16 x 16, lane j + 16 q holding four entries of column j:
// rows 4 q .. 4 q + 3 in FP32, rows q, q + 4, q + 8, q + 12 in FP64 (row()
// gives the row of entry v)
template <typename T>
struct MfmaStep;
template <>
struct MfmaStep<float> {
  using Acc = f32x4;
  static __device__ __forceinline__ Acc run(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};
template <>
struct MfmaStep<double> {
  using Acc = f64x4;
  static __device__ __forceinline__ Acc run(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
};
template <int NB>
struct MfmaSu {
  static constexpr int KP = (NB + 15) / 16 * 16;
  static constexpr int KS = KP / 4;                  // k-steps of 4
  static constexpr int MTILES = KP / 16;             // 16-row tiles of the output
  static constexpr int WAVES = 4;
  static constexpr int MPW = (MTILES + WAVES - 1) / WAVES;   // row tiles per wavefront
  static constexpr int NSUB = 2;                     // 16-element blocks per work-group tile
  static constexpr int TN = 16 * NSUB;
  static constexpr int LDR = KP + 1;                 // LDS stride of one staged element
};

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_shared_update_mfma(int nelems, const T* __restrict__ ainv,
                                                           const T* __restrict__ r,
                                                           const int* __restrict__ elems, T* __restrict__ x,
                                                           int first, const int* __restrict__ zl, int nzero) {
  using C = MfmaSu<NB>;
  using M = MfmaStep<T>;
  __shared__ T Rs[C::TN * C::LDR];
  __shared__ int Eo[C::TN];   // x offset of each staged element (-1 past the end)
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int lr = l & 15, lg = l >> 4;
  T a[C::MPW][C::KS];
#pragma unroll
  for (int mi = 0; mi < C::MPW; ++mi) {
    const int m = 16 * (wv + C::WAVES * mi) + lr;
#pragma unroll
    for (int ks = 0; ks < C::KS; ++ks) {
      const int k = 4 * ks + lg;
      a[mi][ks] = (m < NB && k < NB) ? ainv[k * NB + m] : (T)0;
    }
  }
  const int ntiles = (nelems + C::TN - 1) / C::TN;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * C::TN;
    const int cnt = min(C::TN, nelems - base);
    __syncthreads();
    if (tid < C::TN) Eo[tid] = tid < cnt ? elems[base + tid] * NB : -1;
    __syncthreads();
    // all loads of the tile issued before any is stored (unrolled; masked
    // loads read r[0] and are discarded)
    constexpr int TOT = C::TN * C::KP, ITER = (TOT + 255) / 256;
    T v[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int i = tid + 256 * it;
      const int e = i / C::KP, k = i - e * C::KP;
      const bool ok = i < TOT && e < cnt && k < NB;
      const size_t src = ok ? (first ? (size_t)Eo[e] + k : (size_t)(base + e) * NB + k) : 0;
      v[it] = r[src];
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int i = tid + 256 * it;
      const int e = i / C::KP, k = i - e * C::KP;
      if (i < TOT) Rs[e * C::LDR + k] = (e < cnt && k < NB) ? v[it] : (T)0;
    }
    int eoff[C::NSUB];
#pragma unroll
    for (int sb = 0; sb < C::NSUB; ++sb) eoff[sb] = Eo[16 * sb + lr];
    __syncthreads();
#pragma unroll
    for (int sb = 0; sb < C::NSUB; ++sb) {
      typename M::Acc acc[C::MPW];
#pragma unroll
      for (int mi = 0; mi < C::MPW; ++mi) acc[mi] = typename M::Acc{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < C::KS; ++ks) {
        const T bv = Rs[(16 * sb + lr) * C::LDR + 4 * ks + lg];
#pragma unroll
        for (int mi = 0; mi < C::MPW; ++mi)
          acc[mi] = M::run(a[mi][ks], bv, acc[mi]);
      }
      if (eoff[sb] >= 0) {
#pragma unroll
        for (int mi = 0; mi < C::MPW; ++mi)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = 16 * (wv + C::WAVES * mi) + M::row(lg, i);
            if (m < NB) {
              T* xm = x + (size_t)eoff[sb] + m;
              *xm = first ? acc[mi][i] : *xm + acc[mi][i];
            }
          }
      }
    }
  }
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < (int64_t)nzero * NB; i += (int64_t)gridDim.x * 256)
    x[(size_t)zl[i / NB] * NB + i % NB] = (T)0;
}

// product of 1D injection entries, (P_o)[af][ac] for child offset bits o, from
// a copy of the two 1D tables P[0], P[1] (MAXM x MAXM each) in LDS (indices
// differ between lanes: kernel-argument arrays would become memory loads)
template <typename T, int D, int M>
__device__ __forceinline__ T pfull_lds(const T* Pt, int o, int af, int ac) {
  T v = 1;
  int fa = af, ca = ac;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    v *= Pt[((o >> k) & 1) * MAXM * MAXM + (fa % M) * M + (ca % M)];
    fa /= M;
    ca /= M;
  }
  return v;
}

// r_c = I^T (b - A x): one work-group per coarse element, looping over children.
template <typename T, int D, int P, int NT, bool IF>
__global__ __launch_bounds__(NT) void k_residual_restrict(DevLevel<T> lev, TabT<T> tab, const T* __restrict__ b,
                                                          const T* __restrict__ x, T* __restrict__ rc) {
  using S = Sz<D, P>;
  constexpr int M = S::M, NQ = S::NQ, NB = S::NB;
  constexpr int PER = (NB + NT - 1) / NT;
  Work<T, D, P, IF>& w = work_lds<T, D, P, IF>();
  const int lgc = lev.lgn - 1;
  const int C = xcd_remap(blockIdx.x, gridDim.x);
  int cc[D];
  coords_of<D>(C, lgc, cc);
  T acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = 0;
  for (int o = 0; o < (1 << D); ++o) {
    int cf[D];
#pragma unroll
    for (int j = 0; j < D; ++j) cf[j] = 2 * cc[j] + ((o >> j) & 1);
    const int E = index_of<D>(cf, lev.lgn);
    element_operator<T, D, P, NT, IF>(lev, tab, E, x, b, 0, w);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < NB) {
        const int f = t / NQ, ac = t % NQ;
        T s = 0;
        for (int af = 0; af < NQ; ++af) s += pfull_lds<T, D, M>(w.tabs + MAXM * MAXM + 2 * MAXM, o, af, ac) * w.res[f * NQ + af];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = threadIdx.x + q * NT;
    if (t < NB) rc[(size_t)C * NB + t] = acc[q];
  }
}


// sum over the coarse (or fine) coefficient digits of prod_k fac[k][digit_k] v[.]:
// one tensor-product row of the injection applied to one field block
template <typename T, int D, int M>
__device__ __forceinline__ T tensor_row(const T (&fac)[D][M], const T* v) {
  T s = 0;
  if constexpr (D == 2) {
#pragma unroll
    for (int c1 = 0; c1 < M; ++c1) {
      const T w1 = fac[1][c1];
#pragma unroll
      for (int c0 = 0; c0 < M; ++c0) s += w1 * fac[0][c0] * v[c0 + M * c1];
    }
  } else {
#pragma unroll
    for (int c2 = 0; c2 < M; ++c2)
#pragma unroll
      for (int c1 = 0; c1 < M; ++c1) {
        const T w21 = fac[2][c2] * fac[1][c1];
#pragma unroll
        for (int c0 = 0; c0 < M; ++c0) s += w21 * fac[0][c0] * v[c0 + M * c1 + M * M * c2];
      }
  }
  return s;
}

// r_c = I^T r, one work-group per coarse element: the 2^d children's
// residuals are staged in LDS (coalesced reads, each value read once), then
// every coarse coefficient is the tensor-product column of the injection
// applied to each child's field block.
template <typename T, int D, int P>
__global__ __launch_bounds__(128) void k_restrict_elem(int lgn, TabT<T> tab, const T* __restrict__ r,
                                                       T* __restrict__ rc) {
  using S = Sz<D, P>;
  constexpr int M = S::M, NQ = S::NQ, NB = S::NB, NCH = 1 << D;
  __shared__ T Pt[2 * MAXM * MAXM];
  __shared__ T rs[NCH][NB];
  const int C = (int)blockIdx.x;
  if (threadIdx.x < 2 * MAXM * MAXM) Pt[threadIdx.x] = (&tab.P[0][0])[threadIdx.x];
  int cc[D];
  coords_of<D>(C, lgn - 1, cc);
  for (int t = threadIdx.x; t < NCH * NB; t += 128) {
    const int o = t / NB, q = t - o * NB;
    int cf[D];
#pragma unroll
    for (int j = 0; j < D; ++j) cf[j] = 2 * cc[j] + ((o >> j) & 1);
    rs[o][q] = r[(size_t)index_of<D>(cf, lgn) * NB + q];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NB; q += 128) {
    const int f = q / NQ, ac = q - f * NQ;
    T acc = 0;
#pragma unroll
    for (int o = 0; o < NCH; ++o) {
      T fac[D][M];
      int ca = ac;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int bit = (o >> k) & 1, ck = ca % M;
        ca /= M;
#pragma unroll
        for (int m = 0; m < M; ++m) fac[k][m] = Pt[bit * MAXM * MAXM + m * M + ck];
      }
      acc += tensor_row<T, D, M>(fac, &rs[o][f * NQ]);
    }
    rc[(size_t)C * NB + q] = acc;
  }
}

// x += I x_c, one work-group per coarse element: its coefficients staged in
// LDS, every fine coefficient of its 2^d children the tensor-product row of
// the injection applied to one coarse field block.
template <typename T, int D, int P>
__global__ __launch_bounds__(256) void k_prolong_elem(int lgn, TabT<T> tab, const T* __restrict__ xc,
                                                      T* __restrict__ x) {
  using S = Sz<D, P>;
  constexpr int M = S::M, NQ = S::NQ, NB = S::NB, NCH = 1 << D;
  __shared__ T Pt[2 * MAXM * MAXM];
  __shared__ T xs[NB];
  const int C = (int)blockIdx.x;
  if (threadIdx.x < 2 * MAXM * MAXM) Pt[threadIdx.x] = (&tab.P[0][0])[threadIdx.x];
  for (int q = threadIdx.x; q < NB; q += 256) xs[q] = xc[(size_t)C * NB + q];
  __syncthreads();
  int cc[D];
  coords_of<D>(C, lgn - 1, cc);
  for (int t = threadIdx.x; t < NCH * NB; t += 256) {
    const int o = t / NB, q = t - o * NB;
    const int f = q / NQ, af = q - f * NQ;
    T fac[D][M];
    int cf[D];
    int fa = af;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int bit = (o >> k) & 1, fk = fa % M;
      fa /= M;
      cf[k] = 2 * cc[k] + bit;
#pragma unroll
      for (int m = 0; m < M; ++m) fac[k][m] = Pt[bit * MAXM * MAXM + fk * M + m];
    }
    x[(size_t)index_of<D>(cf, lgn) * NB + q] += tensor_row<T, D, M>(fac, &xs[f * NQ]);
  }
}


// y = z + sign * M x with M row-major FP64 (N x N), one wavefront per row;
// z may be null.  Used by the bottom solve (pseudo-inverse and refinement).
template <typename Tin, typename Tout>
__global__ void k_dense_mv(int64_t N, const double* __restrict__ A, const Tin* __restrict__ x,
                           const double* __restrict__ z, double sign, Tout* __restrict__ y) {
  int64_t row = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < N; j += WG) s += A[row * N + j] * (double)x[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, WG);
  if (threadIdx.x == 0) y[row] = (Tout)((z ? z[row] : 0.0) + sign * s);
}

// ---------------------------------------------------------------------------
// vector helpers
// ---------------------------------------------------------------------------
__global__ void k_cast_d2f(int64_t n, const double* a, float* b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_cast_f2d_add(int64_t n, const float* a, double* b, int add) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = add ? b[i] + (double)a[i] : (double)a[i];
}
__global__ void k_axpby(int64_t n, double a, const double* x, double bcoef, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + bcoef * y[i];
}
__global__ void k_axpy(int64_t n, double a, const double* x, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}
__global__ void k_scale_copy(int64_t n, double a, const double* x, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}
template <typename T>
__global__ void k_fill(int64_t n, T v, T* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
__global__ void k_f2bf16(int64_t n, const float* a, uint16_t* b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    // round to nearest even
    unsigned int u = __float_as_uint(a[i]);
    unsigned int lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    b[i] = (uint16_t)(u >> 16);
  }
}

template <typename Tin, typename Tout>
__global__ void k_scale_cast(int64_t ne, int nb, int nvel, const double* dscale, const Tin* in, Tout* out, int invert,
                             int add) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne * nb) return;
  double v = (double)in[t];
  if (dscale) {
    int64_t e = t / nb;
    double s = dscale[2 * e + ((t % nb) >= nvel ? 1 : 0)];
    v = invert ? v / s : v * s;
  }
  out[t] = add ? (Tout)((double)out[t] + v) : (Tout)v;
}

constexpr int RB = 256;
__global__ __launch_bounds__(RB) void k_dot_partial(int64_t n, const double* x, const double* y, double* out) {
  __shared__ double sm[RB];
  const double* yy = y ? y : x;
  const int64_t gs = (int64_t)gridDim.x * RB;
  int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
  // four independent strided partial sums: four loads in flight per thread
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (; i + 3 * gs < n; i += 4 * gs) {
    s0 += x[i] * yy[i];
    s1 += x[i + gs] * yy[i + gs];
    s2 += x[i + 2 * gs] * yy[i + 2 * gs];
    s3 += x[i + 3 * gs] * yy[i + 3 * gs];
  }
  for (; i < n; i += gs) s0 += x[i] * yy[i];
  const double s = (s0 + s1) + (s2 + s3);
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = RB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}
// y += a x, and the block partial sums of y . z (z null: y . y) for the updated
// y, summed exactly as k_dot_partial sums x . y (the same strides, pairing and
// tree), so that a fused update + inner product equals the two launches
__global__ __launch_bounds__(RB) void k_axpy_dot_partial(int64_t n, double a, const double* __restrict__ x,
                                                         double* __restrict__ y, const double* __restrict__ z,
                                                         double* __restrict__ out) {
  __shared__ double sm[RB];
  const int64_t gs = (int64_t)gridDim.x * RB;
  int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (; i + 3 * gs < n; i += 4 * gs) {
    double y0 = y[i], y1 = y[i + gs], y2 = y[i + 2 * gs], y3 = y[i + 3 * gs];
    y0 += a * x[i];
    y1 += a * x[i + gs];
    y2 += a * x[i + 2 * gs];
    y3 += a * x[i + 3 * gs];
    y[i] = y0;
    y[i + gs] = y1;
    y[i + 2 * gs] = y2;
    y[i + 3 * gs] = y3;
    s0 += y0 * (z ? z[i] : y0);
    s1 += y1 * (z ? z[i + gs] : y1);
    s2 += y2 * (z ? z[i + 2 * gs] : y2);
    s3 += y3 * (z ? z[i + 3 * gs] : y3);
  }
  for (; i < n; i += gs) {
    double y0 = y[i];
    y0 += a * x[i];
    y[i] = y0;
    s0 += y0 * (z ? z[i] : y0);
  }
  const double s = (s0 + s1) + (s2 + s3);
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = RB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}
__global__ __launch_bounds__(RB) void k_strided_sum_partial(int64_t ne, int nb, int off, const double* x, double* out) {
  __shared__ double sm[RB];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < ne; e += (int64_t)gridDim.x * RB) s += x[e * nb + off];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = RB / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}
__global__ void k_strided_add(int64_t ne, int nb, int off, double v, double* x) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) x[e * nb + off] += v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int hip_ok() { return hipGetLastError() == hipSuccess ? 0 : 1; }
static inline unsigned grid1(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// runs f(D, P) for the supported (dimension, degree) pairs; 2 if unsupported
template <class F>
static int dispatch(int dim, int p, F&& f) {
  using std::integral_constant;
  if (dim == 2 && p == 1) f(integral_constant<int, 2>{}, integral_constant<int, 1>{});
  else if (dim == 2 && p == 2) f(integral_constant<int, 2>{}, integral_constant<int, 2>{});
  else if (dim == 2 && p == 3) f(integral_constant<int, 2>{}, integral_constant<int, 3>{});
  else if (dim == 3 && p == 1) f(integral_constant<int, 3>{}, integral_constant<int, 1>{});
  else if (dim == 3 && p == 2) f(integral_constant<int, 3>{}, integral_constant<int, 2>{});
  else return 2;
  return 0;
}

// threads per work-group for the element kernels: one wavefront per element
// when the launch has enough elements to fill the chip, several wavefronts
// per element on small (coarse) grids, where the latency of one element's
// evaluation sets the time of the launch
constexpr int NT_SMALL = 128;
// levels with interphase faces use the extended stencil (2D only)
template <class F>
static int dispatch_if(int iface, int dim, F&& f) {
  if (!iface) {
    f(std::false_type{});
    return 0;
  }
  if (dim != 2) return 2;
  f(std::true_type{});
  return 0;
}
// Work-groups whose LDS block exceeds this also run two wavefronts per element
// on large grids: LDS then limits the work-groups per CU, and one wavefront
// each would leave the SIMDs idle (3D, FP64).
constexpr size_t LDS_WIDE = 12288;
// 3D elements have 2-3x the work items per phase of 2D ones: four wavefronts
// per element on small (latency-bound) grids and in FP64 (measured: the FP64
// 64^3 residual 2.57 -> 2.03 ms); two for large FP32 launches (four were slower
// there: the colour residual 164 -> 174 us)
constexpr int NT_WIDE3 = 256;
template <int D = 2, int TBYTES = 4, class F>
static void dispatch_nt(int64_t nelems, int small_grid, size_t lds_bytes, F&& f) {
  if (nelems >= small_grid && lds_bytes <= LDS_WIDE) f(std::integral_constant<int, WG>{});
  else if constexpr (D == 3) {
    if (TBYTES == 8 || nelems < small_grid) f(std::integral_constant<int, NT_WIDE3>{});
    else f(std::integral_constant<int, NT_SMALL>{});
  } else {
    f(std::integral_constant<int, NT_SMALL>{});
  }
}

template <typename T>
int launch_smooth_colour(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab, const int* elems, int pcol,
                         int64_t nelems, const void* inv, int inv_kind, const T* b, T* x, bool inv_shared) {
  if (nelems <= 0) return 0;
  const unsigned grid = (unsigned)nelems;
  bool bad = false;   // no kernel for this level (interphase faces in 3D)
  hipStream_t st = (hipStream_t)c.stream;
  const TabT<T> tt = tab_of<T>(tab);
  if constexpr (sizeof(T) == 8) {
    if (inv_kind != 0) return 2;
    if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; if (dispatch_if(lev.iface, D_, [&](auto Ic) { constexpr bool IF_ = decltype(Ic)::value; if constexpr (!IF_ || D_ == 2) dispatch_nt<D_, (int)sizeof(T)>(nelems, c.small_grid, work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr), [&](auto Nc) { constexpr int NT_ = decltype(Nc)::value; hipLaunchKernelGGL((k_smooth_colour<T, double, D_, P_, NT_, IF_>), dim3(grid), dim3(NT_), (work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr)), st,
                                                  lev, tt, elems, pcol, (const double*)inv, b, x, (int)inv_shared); }); })) bad = true; })) return 2;
  } else {
    if (inv_kind == 1) {
      if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; if (dispatch_if(lev.iface, D_, [&](auto Ic) { constexpr bool IF_ = decltype(Ic)::value; if constexpr (!IF_ || D_ == 2) dispatch_nt<D_, (int)sizeof(T)>(nelems, c.small_grid, work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr), [&](auto Nc) { constexpr int NT_ = decltype(Nc)::value; hipLaunchKernelGGL((k_smooth_colour<T, float, D_, P_, NT_, IF_>), dim3(grid), dim3(NT_), (work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr)), st,
                                                    lev, tt, elems, pcol, (const float*)inv, b, x, (int)inv_shared); }); })) bad = true; })) return 2;
    } else if (inv_kind == 2) {
      if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; if (dispatch_if(lev.iface, D_, [&](auto Ic) { constexpr bool IF_ = decltype(Ic)::value; if constexpr (!IF_ || D_ == 2) dispatch_nt<D_, (int)sizeof(T)>(nelems, c.small_grid, work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr), [&](auto Nc) { constexpr int NT_ = decltype(Nc)::value; hipLaunchKernelGGL((k_smooth_colour<T, uint16_t, D_, P_, NT_, IF_>), dim3(grid), dim3(NT_), (work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr)), st,
                                                    lev, tt, elems, pcol, (const uint16_t*)inv, b, x, (int)inv_shared); }); })) bad = true; })) return 2;
    } else {
      return 2;
    }
  }
  if (bad) return 2;
  return hip_ok();
}

template <typename T>
int launch_residual(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab, const T* b, const T* x, T* out,
                    int mode) {
  int64_t NE = 1;
  for (int j = 0; j < c.dim; ++j) NE *= lev.n;
  bool bad = false;   // no kernel for this level (interphase faces in 3D)
  hipStream_t st = (hipStream_t)c.stream;
  const TabT<T> tt = tab_of<T>(tab);
  if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; if (dispatch_if(lev.iface, D_, [&](auto Ic) { constexpr bool IF_ = decltype(Ic)::value; if constexpr (!IF_ || D_ == 2) dispatch_nt<D_, (int)sizeof(T)>(NE, c.small_grid, work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr), [&](auto Nc) { constexpr int NT_ = decltype(Nc)::value; hipLaunchKernelGGL((k_residual<T, D_, P_, NT_, IF_>), dim3((unsigned)NE), dim3(NT_), (work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr)), st,
                                                lev, tt, b, x, out, mode); }); })) bad = true; })) return 2;
  if (bad) return 2;
  return hip_ok();
}

template <typename T>
int launch_colour_residual(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab, const int* elems, int pcol,
                           int64_t nelems, const T* b, const T* x, T* r, int64_t ibase) {
  if (nelems <= 0) return 0;
  bool bad = false;
  hipStream_t st = (hipStream_t)c.stream;
  const TabT<T> tt = tab_of<T>(tab);
  if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; if (dispatch_if(lev.iface, D_, [&](auto Ic) { constexpr bool IF_ = decltype(Ic)::value; if constexpr (!IF_ || D_ == 2) dispatch_nt<D_, (int)sizeof(T)>(nelems, c.small_grid, work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr), [&](auto Nc) { constexpr int NT_ = decltype(Nc)::value; hipLaunchKernelGGL((k_colour_residual<T, D_, P_, NT_, IF_>), dim3((unsigned)nelems), dim3(NT_), (work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr)), st,
                                                lev, tt, elems, pcol, (int)ibase, b, x, r); }); })) bad = true; })) return 2;
  if (bad) return 2;
  return hip_ok();
}

template <typename T, int NB, int Q>
static void shared_update_q(hipStream_t st, int64_t nelems, const T* ainv, const T* r, const int* elems, T* x,
                            int first, const int* zl, int64_t nzero) {
  using C = SuCfg<T, NB, Q>;
  int64_t g = (nelems + C::TE - 1) / C::TE;
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL((k_shared_update<T, NB, Q>), dim3((unsigned)g), dim3(SU_THREADS), 0, st, (int)nelems, ainv, r,
                     elems, x, first, zl, (int)nzero);
}
// large colours (at least mfma_min elements; 0: never): the matrix cores in
// the arithmetic type, FP32 or FP64 (blocks up to 128), else 16 elements per
// thread from 8192 elements;
// small colours: 4 elements per thread (more work-groups, shorter chains:
// small launches are latency bound)
template <typename T, int NB>
static void shared_update_nb(hipStream_t st, int64_t nelems, const T* ainv, const T* r, const int* elems, T* x,
                             int first, const int* zl, int64_t nzero, int64_t mfma_min) {
  if constexpr (NB <= 128) {
    if (mfma_min > 0 && nelems >= mfma_min) {
      int64_t g = (nelems + MfmaSu<NB>::TN - 1) / MfmaSu<NB>::TN;
      if (g > 1024) g = 1024;
      hipLaunchKernelGGL((k_shared_update_mfma<T, NB>), dim3((unsigned)g), dim3(256), 0, st, (int)nelems, ainv, r,
                         elems, x, first, zl, (int)nzero);
      return;
    }
  }
  if (nelems >= 8192) shared_update_q<T, NB, 16>(st, nelems, ainv, r, elems, x, first, zl, nzero);
  else shared_update_q<T, NB, 4>(st, nelems, ainv, r, elems, x, first, zl, nzero);
}

template <typename T>
int launch_shared_update(void* stream, int64_t nelems, int nb, const T* ainv, const T* r, const int* elems, T* x,
                         int first, const int* zl, int64_t nzero, int64_t mfma_min) {
  if (nelems <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  switch (nb) {
#define LDGS_SU(NBV) \
  case NBV: shared_update_nb<T, NBV>(st, nelems, ainv, r, elems, x, first, zl, nzero, mfma_min); break;
    LDGS_SU(12) LDGS_SU(27) LDGS_SU(48) LDGS_SU(32) LDGS_SU(108) LDGS_SU(256)
#undef LDGS_SU
    default: return 2;
  }
  return hip_ok();
}

template <typename T>
int launch_first_colour(const LaunchCfg& c, int lgn, const int* elems, int pcol, int64_t nelems, const void* inv,
                        int inv_kind, const T* b, T* x, const int* zl, int64_t nzero) {
  if (nelems <= 0) return 0;
  hipStream_t st = (hipStream_t)c.stream;
  auto go = [&](auto tag) {
    using TI = decltype(tag);
    return dispatch(c.dim, c.p, [&](auto Dc, auto Pc) {
      constexpr int D_ = decltype(Dc)::value;
      constexpr int P_ = decltype(Pc)::value;
      dispatch_nt(nelems, c.small_grid, 0, [&](auto Nc) {
        constexpr int NT_ = decltype(Nc)::value;
        hipLaunchKernelGGL((k_first_colour<T, TI, D_, P_, NT_>), dim3((unsigned)nelems), dim3(NT_), 0, st, lgn, elems,
                           pcol, (const TI*)inv, b, x, zl, (int)nzero);
      });
    });
  };
  bool bad;
  if constexpr (sizeof(T) == 8) {
    if (inv_kind != 0) return 2;
    bad = go(double{});
  } else {
    if (inv_kind == 1) bad = go(float{});
    else if (inv_kind == 2) bad = go(uint16_t{});
    else return 2;
  }
  if (bad) return 2;
  return hip_ok();
}

template <typename T>
int launch_apply_inverse(const LaunchCfg& c, int lgn, const int* elems, int pcol, int64_t nelems, const void* inv,
                         int inv_kind, const T* r, T* x, int64_t ibase) {
  if (nelems <= 0) return 0;
  hipStream_t st = (hipStream_t)c.stream;
  auto go = [&](auto tag) {
    using TI = decltype(tag);
    return dispatch(c.dim, c.p, [&](auto Dc, auto Pc) {
      constexpr int D_ = decltype(Dc)::value;
      constexpr int P_ = decltype(Pc)::value;
      hipLaunchKernelGGL((k_apply_inverse<T, TI, D_, P_>), dim3((unsigned)nelems), dim3(64), 0, st, lgn, elems, pcol,
                         (int)ibase, (const TI*)inv, r, x);
    });
  };
  bool bad;
  if constexpr (sizeof(T) == 8) {
    if (inv_kind != 0) return 2;
    bad = go(double{});
  } else {
    if (inv_kind == 1) bad = go(float{});
    else if (inv_kind == 2) bad = go(uint16_t{});
    else return 2;
  }
  if (bad) return 2;
  return hip_ok();
}

int shared_inverse_rows(int nb, int bytes) {
  const int v = 16 / bytes;
  return (nb + v - 1) / v * v;
}

template <typename T>
int launch_residual_restrict(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab, const T* b, const T* x,
                             T* rc, T* rfine) {
  int64_t NC = 1;
  for (int j = 0; j < c.dim; ++j) NC *= lev.n / 2;
  bool bad = false;   // no kernel for this level (interphase faces in 3D)
  hipStream_t st = (hipStream_t)c.stream;
  const TabT<T> tt = tab_of<T>(tab);
  if (rfine && (NC < c.small_grid || c.dim == 3)) {
    // small grids, and every 3D grid: every fine element's residual in
    // parallel, then I^T r (at 128^3 Q_2 FP64: 15.0 + 0.4 ms against 18.8 ms
    // for the fused form, whose work-groups evaluate their 8 children one
    // after another)
    const int r1 = launch_residual<T>(c, lev, tab, b, x, rfine, 0);
    if (r1 != 0) return r1;
    if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) {
          constexpr int D_ = decltype(Dc)::value;
          constexpr int P_ = decltype(Pc)::value;
          hipLaunchKernelGGL((k_restrict_elem<T, D_, P_>), dim3((unsigned)NC), dim3(128), 0, st, lev.lgn, tt,
                             (const T*)rfine, rc);
        }))
      return 2;
    return hip_ok();
  }
  if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; if (dispatch_if(lev.iface, D_, [&](auto Ic) { constexpr bool IF_ = decltype(Ic)::value; if constexpr (!IF_ || D_ == 2) dispatch_nt<2>(NC, c.small_grid, work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr), [&](auto Nc) { constexpr int NT_ = decltype(Nc)::value; hipLaunchKernelGGL((k_residual_restrict<T, D_, P_, NT_, IF_>), dim3((unsigned)NC), dim3(NT_), (work_bytes<T, D_, P_, IF_>(lev.mmu != nullptr)), st,
                                                lev, tt, b, x, rc); }); })) bad = true; })) return 2;
  if (bad) return 2;
  return hip_ok();
}

template <typename T>
int launch_prolong_add(const LaunchCfg& c, int n_fine, const Tab1D& tab, const T* xc, T* x) {
  int64_t NE = 1;
  for (int j = 0; j < c.dim; ++j) NE *= n_fine;
  int64_t nb = (int64_t)(c.dim + 1);
  for (int j = 0; j < c.dim; ++j) nb *= (c.p + 1);
  int64_t total = NE * nb;
  hipStream_t st = (hipStream_t)c.stream;
  const TabT<T> tt = tab_of<T>(tab);
  (void)total;
  int lgf = 0;
  while ((1 << lgf) < n_fine) ++lgf;
  const unsigned ncoarse = (unsigned)(NE >> c.dim);
  if (dispatch(c.dim, c.p, [&](auto Dc, auto Pc) { constexpr int D_ = decltype(Dc)::value; constexpr int P_ = decltype(Pc)::value; hipLaunchKernelGGL((k_prolong_elem<T, D_, P_>), dim3(ncoarse), dim3(256), 0, st,
                                                lgf, tt, xc, x); })) return 2;
  return hip_ok();
}

template <typename Tin, typename Tout>
int launch_dense_mv(void* stream, int64_t N, const double* M, const Tin* x, const double* z, double sign, Tout* y) {
  hipLaunchKernelGGL((k_dense_mv<Tin, Tout>), dim3((unsigned)N), dim3(WG), 0, (hipStream_t)stream, N, M, x, z, sign, y);
  return hip_ok();
}

int launch_cast_d2f(void* stream, int64_t n, const double* a, float* b) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, a, b);
  return hip_ok();
}
int launch_cast_f2d_add(void* stream, int64_t n, const float* a, double* b, int add) {
  hipLaunchKernelGGL(k_cast_f2d_add, dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, a, b, add);
  return hip_ok();
}
int launch_axpy(void* stream, int64_t n, double alpha, const double* x, double* y) {
  hipLaunchKernelGGL(k_axpy, dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, alpha, x, y);
  return hip_ok();
}
int launch_axpby(void* stream, int64_t n, double a, const double* x, double b, double* y) {
  hipLaunchKernelGGL(k_axpby, dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, a, x, b, y);
  return hip_ok();
}
int launch_scale_copy(void* stream, int64_t n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, a, x, y);
  return hip_ok();
}
template <typename T>
int launch_fill(void* stream, int64_t n, T v, T* y) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, v, y);
  return hip_ok();
}
int launch_dot_partial(void* stream, int64_t n, const double* x, const double* y, double* out, int nblk) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblk), dim3(RB), 0, (hipStream_t)stream, n, x, y, out);
  return hip_ok();
}
int launch_axpy_dot_partial(void* stream, int64_t n, double a, const double* x, double* y, const double* z,
                            double* out, int nblk) {
  hipLaunchKernelGGL(k_axpy_dot_partial, dim3(nblk), dim3(RB), 0, (hipStream_t)stream, n, a, x, y, z, out);
  return hip_ok();
}
int launch_strided_sum_partial(void* stream, int64_t nelem, int nb, int off, const double* x, double* out, int nblk) {
  hipLaunchKernelGGL(k_strided_sum_partial, dim3(nblk), dim3(RB), 0, (hipStream_t)stream, nelem, nb, off, x, out);
  return hip_ok();
}
// Rigid rotation mode r of the kernel with stress walls: entry t = (E, field
// f, coefficient q) is m_a(E) at (f = b, q = 0), h / (2 sqrt 3) at (f = b, q =
// M^a), -m_b(E) at (f = a, q = 0), -h / (2 sqrt 3) at (f = a, q = M^b), zero
// elsewhere; m_k(E) = (c_k(E) + 1/2) h - 1/2.  OP 0: partial sums of v . r per
// block (out[block]); OP 1: v += alpha r.
template <int OP>
__global__ __launch_bounds__(256) void k_rotation(int64_t N, int d, int M, int nb, int nq, int lgn, double h, int a,
                                                  int b, double alpha, const double* __restrict__ vin,
                                                  double* __restrict__ vout, double* __restrict__ out) {
  __shared__ double sm[256];
  const double lin = h / (2.0 * sqrt(3.0));
  int Ma = 1, Mb = 1;
  for (int j = 0; j < a; ++j) Ma *= M;
  for (int j = 0; j < b; ++j) Mb *= M;
  const int n = 1 << lgn;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N; t += (int64_t)gridDim.x * 256) {
    const int64_t E = t / nb;
    const int r = (int)(t - E * nb), f = r / nq, q = r - f * nq;
    double val = 0.0;
    if (f == b || f == a) {
      const int ax = f == b ? a : b;
      const double sg = f == b ? 1.0 : -1.0;
      const int c = (int)((E >> (ax * lgn)) & (n - 1));
      if (q == 0) val = sg * ((c + 0.5) * h - 0.5);
      else if (q == (f == b ? Ma : Mb)) val = sg * lin;
    }
    if (OP == 0) acc += vin[t] * val;
    else if (val != 0.0) vout[t] += alpha * val;
  }
  if (OP == 0) {
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
  }
}

int launch_rotation_dot_partial(void* stream, int d, int p, int lgn, double h, int a, int b, const double* v,
                                double* out, int nblk) {
  const int M = p + 1;
  int nq = 1;
  for (int j = 0; j < d; ++j) nq *= M;
  const int nb = (d + 1) * nq;
  const int64_t N = ((int64_t)1 << (d * lgn)) * nb;
  hipLaunchKernelGGL(k_rotation<0>, dim3(nblk), dim3(256), 0, (hipStream_t)stream, N, d, M, nb, nq, lgn, h, a, b, 0.0,
                     v, nullptr, out);
  return hip_ok();
}

int launch_rotation_axpy(void* stream, int d, int p, int lgn, double h, int a, int b, double alpha, double* v) {
  const int M = p + 1;
  int nq = 1;
  for (int j = 0; j < d; ++j) nq *= M;
  const int nb = (d + 1) * nq;
  const int64_t N = ((int64_t)1 << (d * lgn)) * nb;
  hipLaunchKernelGGL(k_rotation<1>, dim3(grid1(N, 256)), dim3(256), 0, (hipStream_t)stream, N, d, M, nb, nq, lgn, h, a,
                     b, alpha, nullptr, v, nullptr);
  return hip_ok();
}

int launch_strided_add(void* stream, int64_t nelem, int nb, int off, double v, double* x) {
  hipLaunchKernelGGL(k_strided_add, dim3(grid1(nelem, 256)), dim3(256), 0, (hipStream_t)stream, nelem, nb, off, v, x);
  return hip_ok();
}
int launch_f2bf16(void* stream, int64_t n, const float* a, uint16_t* b) {
  hipLaunchKernelGGL(k_f2bf16, dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, n, a, b);
  return hip_ok();
}

template <typename Tin, typename Tout>
int launch_scale_cast(void* stream, int64_t ne, int nb, int nvel, const double* dscale, const Tin* in, Tout* out,
                      int invert, int add) {
  int64_t n = ne * nb;
  hipLaunchKernelGGL((k_scale_cast<Tin, Tout>), dim3(grid1(n, 256)), dim3(256), 0, (hipStream_t)stream, ne, nb, nvel,
                     dscale, in, out, invert, add);
  return hip_ok();
}

// explicit instantiations
template int launch_scale_cast<double, double>(void*, int64_t, int, int, const double*, const double*, double*, int, int);
template int launch_scale_cast<double, float>(void*, int64_t, int, int, const double*, const double*, float*, int, int);
template int launch_scale_cast<float, double>(void*, int64_t, int, int, const double*, const float*, double*, int, int);
template int launch_smooth_colour<double>(const LaunchCfg&, const DevLevel<double>&, const Tab1D&, const int*, int, int64_t,
                                          const void*, int, const double*, double*, bool);
template int launch_smooth_colour<float>(const LaunchCfg&, const DevLevel<float>&, const Tab1D&, const int*, int, int64_t,
                                         const void*, int, const float*, float*, bool);
template int launch_residual<double>(const LaunchCfg&, const DevLevel<double>&, const Tab1D&, const double*,
                                     const double*, double*, int);
template int launch_residual<float>(const LaunchCfg&, const DevLevel<float>&, const Tab1D&, const float*, const float*,
                                    float*, int);
template int launch_residual_restrict<double>(const LaunchCfg&, const DevLevel<double>&, const Tab1D&, const double*,
                                              const double*, double*, double*);
template int launch_residual_restrict<float>(const LaunchCfg&, const DevLevel<float>&, const Tab1D&, const float*,
                                             const float*, float*, float*);
template int launch_colour_residual<double>(const LaunchCfg&, const DevLevel<double>&, const Tab1D&, const int*, int,
                                            int64_t, const double*, const double*, double*, int64_t);
template int launch_colour_residual<float>(const LaunchCfg&, const DevLevel<float>&, const Tab1D&, const int*, int,
                                           int64_t, const float*, const float*, float*, int64_t);
template int launch_shared_update<double>(void*, int64_t, int, const double*, const double*, const int*, double*,
                                          int, const int*, int64_t, int64_t);
template int launch_shared_update<float>(void*, int64_t, int, const float*, const float*, const int*, float*, int,
                                         const int*, int64_t, int64_t);
template int launch_first_colour<double>(const LaunchCfg&, int, const int*, int, int64_t, const void*, int,
                                         const double*, double*, const int*, int64_t);
template int launch_apply_inverse<double>(const LaunchCfg&, int, const int*, int, int64_t, const void*, int,
                                          const double*, double*, int64_t);
template int launch_apply_inverse<float>(const LaunchCfg&, int, const int*, int, int64_t, const void*, int,
                                         const float*, float*, int64_t);
template int launch_first_colour<float>(const LaunchCfg&, int, const int*, int, int64_t, const void*, int,
                                        const float*, float*, const int*, int64_t);
template int launch_prolong_add<double>(const LaunchCfg&, int, const Tab1D&, const double*, double*);
template int launch_prolong_add<float>(const LaunchCfg&, int, const Tab1D&, const float*, float*);
template int launch_dense_mv<double, double>(void*, int64_t, const double*, const double*, const double*, double, double*);
template int launch_dense_mv<double, float>(void*, int64_t, const double*, const double*, const double*, double, float*);
template int launch_fill<double>(void*, int64_t, double, double*);
template int launch_fill<float>(void*, int64_t, float, float*);

}  // namespace ldgs
