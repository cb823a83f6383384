// Host-side structures of the LDG-Stokes library: the 1D basis tables, the
// per-level operator data, the context.  See ldgs_internal.hpp for the
// operator representation shared with the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldgs.h"
#include "ldgs_internal.hpp"

namespace ldgs {

// Orthonormal shifted Legendre basis l_m(xi) = sqrt(2m+1) P_m(2 xi - 1) on
// [0,1] with closed-form traces and derivative matrix, Gauss rules and the
// 1D injection matrices.
struct Basis {
  int p = 0, m = 0;
  std::vector<double> e0, e1, K;   // K[r*m + c] = int l_c' l_r
  std::vector<double> P[2];        // P[o][f*m + c]
  void init(int p);
  static double leg(int mm, double xi);                      // l_mm(xi)
  static void gauss(int q, std::vector<double>& x, std::vector<double>& w);  // on [0,1]
  Tab1D tab() const;
};

struct FaceSet {
  int nfk = 0;                       // faces per grid line along the axis (n or n+1)
  int64_t count = 0;                 // total faces normal to the axis
  std::vector<unsigned char> type;   // FaceType
  std::vector<double> w;             // [count][2] = (wL, wR)
  std::vector<double> T;             // [count][MT*MT]
  std::vector<double> Tmu, Trho;     // unsteady: the two pressure-penalty parts
};

struct Level {
  int n = 0;
  double h = 0;
  int64_t NE = 0;
  bool mu_is_const = false;
  double mu_c = 1.0;
  std::vector<double> mmu;           // [NE][NQ*NQ] when !mu_is_const
  FaceSet faces[3];
  double rho_delta = 0.0;
  std::vector<double> dscale;        // [NE][2] (alpha, beta) or empty
  std::vector<int> chi;              // phase per element (1 or 2)
  // smoother data (smoothed levels)
  int ncol = 0;
  std::vector<int> colour;           // per element
  std::vector<std::vector<int>> elems;   // per colour, element ids
  bool uniform = false;              // every diagonal block is the same matrix (one inverse for the level)
};

struct Geometry {
  int d = 2, p = 1, m = 2, nq = 4, mt = 2, nb = 12;
  void set(int dim, int deg);
};

// face-adjacent elements: (L, R) of face number f (position along the axis)
// with tangential coordinates taken from c (c[axis] ignored); -1 if absent
void face_elements(const Level& L, int d, int axis, int f, const int* c, int64_t* eL, int64_t* eR);
int64_t face_id(const Level& L, int d, int axis, const int* c, int f);

// host operator kernels (setup and validation only)
void host_apply(const Level& L, const Geometry& g, const Basis& B, int gamma, const double* x, double* y);
void host_grad(const Level& L, const Geometry& g, const Basis& B, int k, const double* u, double* out);
void host_gradT(const Level& L, const Geometry& g, const Basis& B, int k, const double* s, double* out);
void host_mmu(const Level& L, const Geometry& g, const double* u, double* out);
void host_diag_block(const Level& L, const Geometry& g, const Basis& B, int gamma, int64_t E, double* A);

// dense symmetric eigen-decomposition A = V diag(lam) V^T (A row-major n x n,
// overwritten by V with eigenvectors in columns)
void sym_eigen(int n, std::vector<double>& A, std::vector<double>& lam);
// explicit inverse of the Jacobi-equilibrated LU; returns false if singular
bool block_inverse(int n, const double* A, double* inv, double rcond_min);

}  // namespace ldgs
