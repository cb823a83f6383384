// Internal declarations shared by the host setup (C++) and the HIP kernels.
//
// Operator representation on every level (uniform Cartesian grid, width h,
// orthonormal tensor Legendre basis so that M = I):
//  * discrete gradient G_k (eq. geqn): volume part h^-1 K along axis k and,
//    per face normal to k with low element L and high element R, a lifting of
//    the jump u_R|lo - u_L|hi onto L with weight wL and onto R with weight wR,
//    along the face trace vectors e1 (L) and e0 (R).  Intraphase faces have
//    (wL, wR) = (0, 1) (flux u-hat = u^-), Dirichlet faces lift onto their one
//    element with weight 1 (outside value 0), interphase faces carry the
//    viscosity-upwinded lambda of eq. (viscosityupwind).
//  * mu-weighted mass M_mu: one dense symmetric block per element (or one
//    constant).
//  * penalties: per face a tangential matrix That (face mass weighted by
//    tau), applied to the jump (intraphase faces: pressure penalty E;
//    interphase faces: velocity penalty E-tilde) or to the one trace
//    (Dirichlet faces: velocity penalty).
//  * unsteady term rho/delta (constant rho), optional per-element diagonal
//    scaling (alpha on velocity, beta on pressure).
#pragma once

#include <cstdint>
#include <cstddef>

namespace ldgs {

enum FaceType : unsigned char {
  F_NONE = 0,     // no face terms (not used by the built-in boundary types)
  F_INTRA = 1,    // intraphase, both neighbours present (periodic wrap included)
  F_INTER = 2,    // interphase, both neighbours present
  F_DIR_LO = 3,   // Dirichlet boundary at x_k = 0 (only R present)
  F_DIR_HI = 4    // Dirichlet boundary at x_k = 1 (only L present)
};

constexpr int MAXM = 4;  // p <= 3

// 1D tables of the orthonormal Legendre basis on [0,1]:
// K[r*M+c] = int l_c' l_r, e0[m] = l_m(0), e1[m] = l_m(1),
// P[o][f*M+c] = 2^{-1/2} int l_f(xi) l_c((xi+o)/2) (injection, child o).
struct Tab1D {
  int M;
  double K[MAXM * MAXM];
  double e0[MAXM];
  double e1[MAXM];
  double P[2][MAXM * MAXM];
};

// Symmetric tile layout of one element's inverse block for the smoother's
// matrix-vector product.  The diagonal block of the (symmetric) LDG operator
// is symmetric, so is its inverse: only the tiles on and above the diagonal
// are stored, and of a diagonal tile only the lane blocks that reach its upper
// triangle.  The block, zero-padded to 16 TR rows and columns
// (TR = ceil(nb / 16)), is cut into 16 x 16 tiles; tile (i, j), i <= j, has
// number t = i TR - i (i - 1) / 2 + (j - i), NTILE = TR (TR + 1) / 2 tiles.
// Lane block (r, cb) of a tile is row r < 16, columns 4 cb .. 4 cb + 3 (the
// block of lane l = 4 r + cb).  An off-diagonal tile stores all 64 blocks at
// slot 4 r + cb; a diagonal tile stores the 40 blocks with cb >= r / 4, at slot
// sym_dslot(r, cb), with their true entries (those of the block on the
// diagonal that lie below it included).  Read back: every stored entry (r, c)
// of tile (i, j) gives A[16i + r][16j + c]; off the diagonal, and in a
// diagonal tile for blocks with cb > r / 4, also A[16j + c][16i + r].
// One load reads LB = min(16, 4 * bytes) bytes (EL = LB / bytes entries) of a
// block; H = 4 * bytes / LB loads cover it.  Entry v = h EL + u of slot s of a
// tile with nblk stored blocks is at entry (h nblk + s) EL + u of the tile,
// tiles follow one another in the order t (sym_tile_off), so each load of the
// stored lanes reads consecutive words.  Element stride: sym_tile_off(NTILE).
struct SymTiles {
  int TR, NTILE, LB, EL, H;
};
constexpr SymTiles sym_tiles(int nb, int bytes) {
  SymTiles L{(nb + 15) / 16, 0, 4 * bytes < 16 ? 4 * bytes : 16, 0, 0};
  L.NTILE = L.TR * (L.TR + 1) / 2;
  L.EL = L.LB / bytes;
  L.H = 4 * bytes / L.LB;
  return L;
}
constexpr int SYM_DBLOCKS = 40;   // stored blocks of a diagonal tile
// slot of block (r, cb), cb >= r / 4, of a diagonal tile
constexpr int sym_dslot(int r, int cb) {
  const int g = r / 4;
  const int base = g == 0 ? 0 : (g == 1 ? 16 : (g == 2 ? 28 : 36));
  return base + (r % 4) * (4 - g) + (cb - g);
}
// entry offset of tile t (tiles in the order t) for TR tile rows
constexpr int sym_tile_off(int TR, int t) {
  int off = 0, i = 0, j = 0;
  for (int q = 0; q < t; ++q) {
    off += (i == j ? SYM_DBLOCKS : 64) * 4;
    if (++j == TR) j = ++i;
  }
  return off;
}

// Device view of one level's operator, element type T.
template <typename T>
struct DevLevel {
  int n;                 // elements per axis
  int lgn;               // log2(n)
  int nf[3];             // faces per grid line along each axis (n or n+1)
  T hinv;                // 1 / h
  const unsigned char* ftype[3];   // [faces]
  const T* fw[3];                  // [faces][2] = (wL, wR)
  const T* fT[3];                  // [faces][MT*MT] penalty matrices
  const T* mmu;                    // [NE][NQ*NQ] or nullptr (then mu_const)
  const T* rmu;                    // [NE][D][MT*NQ] low-face trace rows (e0^T)_k M_mu, with mmu
  const T* rmuh;                   // [NE][D][MT*NQ] high-face trace rows (e1^T)_k M_mu (levels with interphase faces)
  int iface;                       // level has interphase faces: extended stencil, face data from the tables
  int stress;                      // the walls are stress walls (no face terms), not Dirichlet
  T mu_const;
  T rho_delta;                     // rho / delta (0: steady)
  const T* dscale;                 // [NE][2] (alpha, beta) or nullptr
  int gamma;
};

// Launchers (defined in kernels.hip).  All are stream-ordered, asynchronous.
// Every kernel handles one element per 64-thread work-group.
struct LaunchCfg {
  int dim, p;
  void* stream;
  // launches with at least this many elements run one wavefront per element,
  // smaller ones two (the context's setting; tests lower it to reach the
  // one-wavefront kernels on grids the oracle assembles quickly)
  int small_grid = 4096;
};

// elems: the colour's elements; pcol >= 0 instead: parity colour pcol with
// its elements in increasing order, computed from the launch index;
// inv_shared: inv holds one inverse (tile layout) for every element
template <typename T>
int launch_smooth_colour(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab,
                         const int* elems, int pcol, int64_t nelems, const void* inv, int inv_kind,
                         const T* b, T* x, bool inv_shared = false);
template <typename T>
int launch_residual(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab,
                    const T* b, const T* x, T* out, int mode);   // mode 0: b - A x, 1: A x
template <typename T>
// rc = I^T (b - A x); rfine (fine-level size, may be null): scratch for the
// split form used when the coarse grid has fewer than small_grid elements
int launch_residual_restrict(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab,
                             const T* b, const T* x, T* rc, T* rfine);
// colour pass with an inverse shared by all elements: residuals of the listed
// elements into r (compact, [nelems][nb]), then x_E += Ainv r (Ainv k-major,
// a[k nb + row], zero-padded to shared_inverse_rows(nb, sizeof(T)) rows)
int shared_inverse_rows(int nb, int bytes);
// ibase: the launch covers positions ibase .. ibase + nelems - 1 of the
// listed elements (elems, or the parity colour pcol), r indexed by position
template <typename T>
int launch_colour_residual(const LaunchCfg& c, const DevLevel<T>& lev, const Tab1D& tab, const int* elems, int pcol,
                           int64_t nelems, const T* b, const T* x, T* r, int64_t ibase = 0);
// first != 0: the first pass from x = 0 (r is then b, read at the listed
// elements; x_E is assigned and the nzero elements zl are set to zero);
// FP32 products of colours of at least mfma_min elements (0: none) on the
// matrix cores
template <typename T>
int launch_shared_update(void* stream, int64_t nelems, int nb, const T* ainv, const T* r, const int* elems, T* x,
                         int first, const int* zl, int64_t nzero, int64_t mfma_min);
// first colour pass from x = 0 with per-element inverses: x_E = Ainv_E b_E for
// the listed elements (same element / inverse conventions as
// launch_smooth_colour), and the nzero elements zl set to zero
template <typename T>
int launch_first_colour(const LaunchCfg& c, int lgn, const int* elems, int pcol, int64_t nelems, const void* inv,
                        int inv_kind, const T* b, T* x, const int* zl, int64_t nzero);
// x_E += Ainv_E r[idx] for the listed elements (per-element inverses, same
// conventions as launch_smooth_colour; r compact as from launch_colour_residual;
// positions ibase .. ibase + nelems - 1, inv and r indexed by position)
template <typename T>
int launch_apply_inverse(const LaunchCfg& c, int lgn, const int* elems, int pcol, int64_t nelems, const void* inv,
                         int inv_kind, const T* r, T* x, int64_t ibase = 0);
template <typename T>
int launch_prolong_add(const LaunchCfg& c, int n_fine, const Tab1D& tab, const T* xc, T* x);
// y = z + sign * M x, M dense row-major FP64 N x N, z optional
template <typename Tin, typename Tout>
int launch_dense_mv(void* stream, int64_t N, const double* M, const Tin* x, const double* z, double sign, Tout* y);

// vector helpers
int launch_cast_d2f(void* stream, int64_t n, const double* a, float* b);
int launch_cast_f2d_add(void* stream, int64_t n, const float* a, double* b, int add);
int launch_axpy(void* stream, int64_t n, double alpha, const double* x, double* y);   // y += a x
int launch_axpby(void* stream, int64_t n, double a, const double* x, double b, double* y); // y = a x + b y
int launch_scale_copy(void* stream, int64_t n, double a, const double* x, double* y); // y = a x
template <typename T>
int launch_fill(void* stream, int64_t n, T v, T* y);
// partial sums: out[blk] for blk < nblk (<= 1024 blocks)
int launch_dot_partial(void* stream, int64_t n, const double* x, const double* y, double* out, int nblk);
// y += a x, then partial sums of y . z (z null: y . y) as launch_dot_partial(y, z)
int launch_axpy_dot_partial(void* stream, int64_t n, double a, const double* x, double* y, const double* z,
                            double* out, int nblk);
// partial sums of the coefficient at offset `off` of every element (stride nb)
int launch_strided_sum_partial(void* stream, int64_t nelem, int nb, int off, const double* x,
                               double* out, int nblk);
int launch_strided_add(void* stream, int64_t nelem, int nb, int off, double v, double* x);
// rigid rotation (x_a - 1/2) e_b - (x_b - 1/2) e_a on the n^d grid (n = 2^lgn,
// width h), as coefficients without the common factor h^{d/2}: partial sums
// of <v, r> (out: nblk doubles), and v += alpha r
int launch_rotation_dot_partial(void* stream, int d, int p, int lgn, double h, int a, int b, const double* v,
                                double* out, int nblk);
int launch_rotation_axpy(void* stream, int d, int p, int lgn, double h, int a, int b, double alpha, double* v);

// Device setup of per-element inverses (setup_dev.hip): unit vectors e_j on
// the listed elements (j = nb only clears entry nb - 1), column j of each
// block from a colour residual r = -A x, in-place FP64 inverses of row-major
// nb x nb blocks (nsing counts singular ones), and the symmetric part of each
// inverse into the tile layout of SymTiles (bytes 8, 4 or 2 per entry).
int launch_set_unit(void* stream, int64_t cnt, const int* elems, int nb, int j, double* x);
int launch_take_column(void* stream, int64_t cnt, int nb, int j, const double* r, double* A);
int launch_block_inverse(void* stream, int64_t nblk, int nb, double* A, int* nsing);
int launch_arrange_sym(void* stream, int64_t cnt, int nb, const double* inv, void* out, int bytes, int64_t stride);

// bf16 <-> float helpers used by the BF16-block path
int launch_f2bf16(void* stream, int64_t n, const float* a, uint16_t* b);

// out[e][i] (+)= in[e][i] * s, s = dscale[2e + (i >= nvel)] (or its inverse);
// dscale may be null (s = 1).  Converts between element types.
template <typename Tin, typename Tout>
int launch_scale_cast(void* stream, int64_t ne, int nb, int nvel, const double* dscale, const Tin* in, Tout* out,
                      int invert, int add);

}  // namespace ldgs
