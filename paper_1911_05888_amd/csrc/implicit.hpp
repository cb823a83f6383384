// Implicitly defined meshes (2D): a circle cuts the cells of the background
// Cartesian grid; the operator of every level is held as explicit element
// blocks (block-sparse rows), since cut and merged elements have no tensor-
// product structure.  Host setup in implicit.cpp, kernels in implicit.hip.
#pragma once

#include <cstdint>
#include <memory>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/ldgs.h"

namespace ldgs {

// Allocator whose resize leaves new entries uninitialised: the operator
// arrays (gigabytes on fine grids) are written by parallel loops, and a
// zero fill first would touch every page from one thread.
template <class T>
struct UninitAlloc : std::allocator<T> {
  UninitAlloc() = default;
  template <class U>
  UninitAlloc(const UninitAlloc<U>&) noexcept {}
  template <class U>
  struct rebind {
    using other = UninitAlloc<U>;
  };
  template <class U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new ((void*)p) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
using BigVec = std::vector<double, UninitAlloc<double>>;

// Square block-sparse matrix with nq x nq blocks (row-major within a block);
// rows keep their columns sorted.
struct SBM {
  int nq = 0;
  int64_t NE = 0;
  std::vector<std::vector<int>> col;
  std::vector<std::vector<double>> val;
  void init(int64_t ne, int q);
  double* at(int64_t r, int c);              // inserts a zero block if absent
  const double* get(int64_t r, int c) const;  // nullptr if absent
};

// One level of the implicit hierarchy.
struct ImpLevel {
  int n = 0;                        // background cells per axis
  int64_t NE = 0;
  std::vector<int> host;            // host cell index i0 + n i1
  std::vector<int> phase;
  std::vector<unsigned char> full;  // basis needs no orthonormalisation
  std::vector<double> L;            // [NE][nq*nq] Cholesky factor of the raw mass (row-major)
  std::vector<double> area;
  // scalar operator components (Algorithm 2 carries them level to level)
  SBM M, Mmu, G[2], Et, E;
  SBM Mrho, Emu, Erho;              // unsteady: rho-weighted mass, the two pressure-penalty limits
  // Stokes operator, element-major nb x nb blocks, column-major in a block
  std::vector<int> rowptr, cols;
  BigVec blk;
  BigVec inv;                       // [NE][nb*nb] column-major
  std::vector<double> dscale;       // [NE][2] (alpha, beta) or empty
  int ncol = 0;
  std::vector<int> colour;
  std::vector<std::vector<int>> elems;
  // injection to the next coarser level: parent and the nq x nq block
  // I[a][b] (fine a, coarse b) of every element of this level
  std::vector<int> parent;
  std::vector<double> Iblk;
  // children of every element of this level (as the coarse side)
  std::vector<int> kid_ptr, kids;
};

// Fine-mesh geometry kept for the right-hand side.
struct ImpElemRule {
  std::vector<double> X, w;         // X: [Q][2]
};
struct ImpFace {
  int kind = 0;                     // 0 intraphase, 1 interphase, 2 wall
  int minus = -1, plus = -1;
  std::vector<double> X, w, nrm;    // X, nrm: [Q][2]
};

struct ImpHier {
  int p = 2, m = 3, nq = 9, nb = 27;
  double cx = 0.5, cy = 0.5, r = 0.3;
  int n_cut = 0, n_merged = 0;
  std::vector<ImpLevel> lv;
  std::vector<ImpElemRule> rules;   // fine elements
  std::vector<ImpFace> faces;       // fine faces
  std::vector<double> kernel;       // fine kernel vector (constant pressure), unit norm
  // bottom
  int64_t Nc = 0;
  std::vector<double> pinv, Ac, eig;
};

// Builds every level on the host (throws std::runtime_error on failure).
void imp_build(const ldgs_problem& P, ImpHier& H);
// Element basis (orthonormalised over the element) at points X (Q x 2):
// out [Q][nq]; deriv_axis -1 for values.
void imp_basis(const ImpHier& H, const ImpLevel& L, int64_t e, int Q, const double* X, int deriv_axis,
               double* out);
// Right-hand side of eq. (stokessystem) on the fine implicit mesh.
void imp_rhs(const ldgs_problem& P, const ImpHier& H, const ldgs_rhs_data& data, double* b);

// Kernel launchers (implicit.hip); stream is a hipStream_t, the result a
// hipError_t.  nb in {12, 27, 48}.
// colour pass: x_E += inv_E (b_E - sum_F A_EF x_F) for E in elems[0..nelem)
template <typename T>
int launch_bsr_colour(void* st, int nb, int64_t nelem, const int* elems, const int* rowptr, const int* cols,
                      const T* blk, const T* inv, const T* b, T* x);
// out = b - S A S x (b null: out = S A S x); ds: per-element (velocity,
// pressure) factors of S, or null for S = I
template <typename T>
int launch_bsr_residual(void* st, int nb, int64_t ne, const int* rowptr, const int* cols, const T* blk, const T* b,
                        const T* x, T* out, const double* ds);
// bc = I^T r (coarse elements nc, children lists kid_ptr / kids)
template <typename T>
int launch_bsr_restrict(void* st, int nb, int64_t nc, const int* kid_ptr, const int* kids, const T* I, const T* r,
                        T* bc);
// x += I xc (fine elements nf, parent of each)
template <typename T>
int launch_bsr_prolong(void* st, int nb, int64_t nf, const int* parent, const T* I, const T* xc, T* x);

}  // namespace ldgs
