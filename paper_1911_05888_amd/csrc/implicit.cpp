// Host setup of implicitly defined meshes (2D, a circle cutting the
// background grid; section 5 "Curved domain geometry", section 3 "Mesh
// hierarchy", appendix A "Specification of penalty parameters"):
//
// * quadrature on cut cells by dimension reduction (the high-order method the
//   paper cites, restated): a height axis along which phi is monotone on the
//   box (else the box is halved), the base interval split at the roots of
//   phi on the two bounding lines, q Gauss points per piece, and at each
//   base point the height line split at its root of phi; the root is a
//   point of the interface rule with weight w |grad phi| / |d_k phi|;
// * a piece of a cell below a quarter of the cell merges into the
//   neighbouring piece of its phase across the cell face it shares most of,
//   large pieces preferred (faces tried -x, +x, -y, +y, first of equals);
// * every element's basis is Q_p on its host cell, orthonormalised over the
//   element by the Cholesky factor of its raw mass matrix (whole cells keep
//   the cell basis);
// * fine operators (M, M_mu, G_k, the velocity and pressure penalties) by
//   quadrature, coarse ones by Algorithm 2 with the injection of nested
//   elements (coarse element = the fine elements of one phase whose host
//   cells share a parent; the injection is exact polynomial re-expansion,
//   I = L_f^T S^T L_c^{-T} with S the coarse raw basis written in the fine
//   raw basis);
// * the Stokes operator of eq. (stokessystem) as explicit element blocks,
//   (alpha, beta) scaling, greedy colours, equilibrated-LU block inverses
//   and the eigendecomposition pseudo-inverse at the bottom.
#include "implicit.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>

#include "build.hpp"
#include "host.hpp"

namespace ldgs {

void SBM::init(int64_t ne, int q) {
  NE = ne;
  nq = q;
  col.assign(ne, {});
  val.assign(ne, {});
}

double* SBM::at(int64_t r, int c) {
  auto& cr = col[r];
  auto it = std::lower_bound(cr.begin(), cr.end(), c);
  const size_t k = it - cr.begin();
  const size_t bs = (size_t)nq * nq;
  if (it == cr.end() || *it != c) {
    cr.insert(it, c);
    val[r].insert(val[r].begin() + k * bs, bs, 0.0);
  }
  return val[r].data() + k * bs;
}

const double* SBM::get(int64_t r, int c) const {
  const auto& cr = col[r];
  auto it = std::lower_bound(cr.begin(), cr.end(), c);
  if (it == cr.end() || *it != c) return nullptr;
  return val[r].data() + (size_t)(it - cr.begin()) * nq * nq;
}

namespace {

constexpr int NSAMP = 32;
constexpr double FRAC_MIN = 0.25;

[[noreturn]] void fail(const std::string& m) { throw std::runtime_error(m); }

struct Circle {
  double c[2], r;
  double phi(const double* x) const {
    const double a = x[0] - c[0], b = x[1] - c[1];
    return std::sqrt(a * a + b * b) - r;
  }
  void grad(const double* x, double* g) const {
    const double a = x[0] - c[0], b = x[1] - c[1];
    const double s = std::sqrt(a * a + b * b);
    g[0] = a / s;
    g[1] = b / s;
  }
  // exact minimum and maximum of phi over the box [lo, hi]
  void range(const double* lo, const double* hi, double& mn, double& mx) const {
    double dn = 0.0, df = 0.0;
    for (int k = 0; k < 2; ++k) {
      const double near = std::min(std::max(c[k], lo[k]), hi[k]) - c[k];
      const double far = (std::fabs(lo[k] - c[k]) > std::fabs(hi[k] - c[k]) ? lo[k] : hi[k]) - c[k];
      dn += near * near;
      df += far * far;
    }
    mn = std::sqrt(dn) - r;
    mx = std::sqrt(df) - r;
  }
};

// a root of f in [a, b] with f(a) f(b) < 0: bisection with secant steps kept
// inside the bracket, to |b - a| <= 1e-16 + 1e-15 |x|
template <class F>
double bracket_root(F f, double a, double b, double fa, double fb) {
  for (int it = 0; it < 200; ++it) {
    double x = b - fb * (b - a) / (fb - fa);
    const double lo = std::min(a, b), hi = std::max(a, b);
    if (!(x > lo && x < hi)) x = 0.5 * (a + b);
    // alternate with bisection so that the bracket always shrinks
    if (it % 2) x = 0.5 * (a + b);
    const double fx = f(x);
    if (fx == 0.0) return x;
    if ((fx < 0.0) == (fa < 0.0)) {
      a = x;
      fa = fx;
    } else {
      b = x;
      fb = fx;
    }
    if (std::fabs(b - a) <= 1e-16 + 1e-15 * std::fabs(x)) return std::fabs(fa) < std::fabs(fb) ? a : b;
  }
  return 0.5 * (a + b);
}

template <class F>
void line_roots(F f, double a, double b, std::vector<double>& out) {
  const double step = (b - a) / NSAMP;
  double s0 = a, v0 = f(a);
  for (int i = 0; i < NSAMP; ++i) {
    const double s1 = (i + 1 == NSAMP) ? b : a + (i + 1) * step;
    const double v1 = f(s1);
    if (v0 == 0.0) {
      if (i > 0) out.push_back(s0);
    } else if (v0 * v1 < 0.0) {
      out.push_back(bracket_root(f, s0, s1, v0, v1));
    }
    s0 = s1;
    v0 = v1;
  }
}

struct Rule {
  std::vector<double> X, w;   // X [Q][2]
  void add(double x0, double x1, double wt) {
    X.push_back(x0);
    X.push_back(x1);
    w.push_back(wt);
  }
  void append(const Rule& o) {
    X.insert(X.end(), o.X.begin(), o.X.end());
    w.insert(w.end(), o.w.begin(), o.w.end());
  }
  double sum() const {
    double s = 0.0;
    for (double v : w) s += v;
    return s;
  }
};

struct BoxRules {
  Rule vol[2];
  Rule surf;
  std::vector<double> nrm;
};

inline void put(int k, double tb, double th, double* x) {
  x[k] = th;
  x[1 - k] = tb;
}

void cut_box(const Circle& ls, const double* lo, const double* hi, int q, const std::vector<double>& gx,
             const std::vector<double>& gw, BoxRules& out) {
  double cen[2] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])}, gc[2];
  ls.grad(cen, gc);
  const int k = std::fabs(gc[1]) > std::fabs(gc[0]) ? 1 : 0;
  bool pos = true, neg = true;
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double x[2] = {lo[0] + (hi[0] - lo[0]) * i / 8.0, lo[1] + (hi[1] - lo[1]) * j / 8.0}, g[2];
      ls.grad(x, g);
      pos = pos && g[k] > 0.0;
      neg = neg && g[k] < 0.0;
    }
  if (!pos && !neg) {
    const int ax = (hi[1] - lo[1]) > (hi[0] - lo[0]) ? 1 : 0;
    const double mid = 0.5 * (lo[ax] + hi[ax]);
    double hi1[2] = {hi[0], hi[1]}, lo2[2] = {lo[0], lo[1]};
    hi1[ax] = mid;
    lo2[ax] = mid;
    cut_box(ls, lo, hi1, q, gx, gw, out);
    cut_box(ls, lo2, hi, q, gx, gw, out);
    return;
  }
  const int j = 1 - k;
  std::vector<double> brk = {lo[j], hi[j]};
  for (double side : {lo[k], hi[k]}) {
    auto f = [&](double t) {
      double x[2];
      put(k, t, side, x);
      return ls.phi(x);
    };
    line_roots(f, lo[j], hi[j], brk);
  }
  std::sort(brk.begin(), brk.end());
  brk.erase(std::unique(brk.begin(), brk.end()), brk.end());
  for (size_t s = 0; s + 1 < brk.size(); ++s) {
    const double a = brk[s], b = brk[s + 1];
    if (!(b - a > 0.0)) continue;
    for (int i = 0; i < q; ++i) {
      const double t = a + (b - a) * gx[i], wb = (b - a) * gw[i];
      auto f = [&](double sh) {
        double x[2];
        put(k, t, sh, x);
        return ls.phi(x);
      };
      const double fa = f(lo[k]), fb = f(hi[k]);
      double cuts[3] = {lo[k], hi[k], 0.0};
      int nc = 2;
      if (fa * fb < 0.0) {
        const double rt = bracket_root(f, lo[k], hi[k], fa, fb);
        cuts[1] = rt;
        cuts[2] = hi[k];
        nc = 3;
        double xr[2], g[2];
        put(k, t, rt, xr);
        ls.grad(xr, g);
        const double gn = std::sqrt(g[0] * g[0] + g[1] * g[1]);
        out.surf.add(xr[0], xr[1], wb * gn / std::fabs(g[k]));
        out.nrm.push_back(g[0] / gn);
        out.nrm.push_back(g[1] / gn);
      }
      for (int c = 0; c + 1 < nc; ++c) {
        const double c0 = cuts[c], c1 = cuts[c + 1];
        if (!(c1 - c0 > 0.0)) continue;
        const int chi = f(0.5 * (c0 + c1)) < 0.0 ? 0 : 1;
        for (int r = 0; r < q; ++r) {
          double x[2];
          put(k, t, c0 + (c1 - c0) * gx[r], x);
          out.vol[chi].add(x[0], x[1], wb * (c1 - c0) * gw[r]);
        }
      }
    }
  }
}

// per-phase rules of the segment {x_axis = val, a <= x_other <= b}
void segment(const Circle& ls, int axis, double val, double a, double b, int q, const std::vector<double>& gx,
             const std::vector<double>& gw, Rule out[2]) {
  auto f = [&](double t) {
    double x[2];
    put(axis, t, val, x);
    return ls.phi(x);
  };
  std::vector<double> brk = {a, b};
  line_roots(f, a, b, brk);
  std::sort(brk.begin(), brk.end());
  brk.erase(std::unique(brk.begin(), brk.end()), brk.end());
  for (size_t s = 0; s + 1 < brk.size(); ++s) {
    const double c0 = brk[s], c1 = brk[s + 1];
    if (!(c1 - c0 > 0.0)) continue;
    const int chi = f(0.5 * (c0 + c1)) < 0.0 ? 0 : 1;
    for (int i = 0; i < q; ++i) {
      double x[2];
      put(axis, c0 + (c1 - c0) * gx[i], val, x);
      out[chi].add(x[0], x[1], (c1 - c0) * gw[i]);
    }
  }
}

// l_0..l_p and their derivatives at xi (orthonormal shifted Legendre)
void leg_all(int p, double xi, double* v, double* dv) {
  const double t = 2.0 * xi - 1.0;
  double P[8], dP[8];
  P[0] = 1.0;
  dP[0] = 0.0;
  if (p >= 1) {
    P[1] = t;
    dP[1] = 1.0;
  }
  for (int m = 1; m < p; ++m) {
    P[m + 1] = ((2.0 * m + 1.0) * t * P[m] - m * P[m - 1]) / (m + 1.0);
    dP[m + 1] = dP[m - 1] + (2.0 * m + 1.0) * P[m];
  }
  for (int m = 0; m <= p; ++m) {
    const double s = std::sqrt(2.0 * m + 1.0);
    v[m] = s * P[m];
    dv[m] = 2.0 * s * dP[m];
  }
}

// raw basis (h-scaled tensor Legendre on the host box) at Q points; deriv -1
// for values, else d/dx_deriv
void raw_basis(int p, double h, const double* lo, int Q, const double* X, int deriv, double* out) {
  const int m = p + 1, nq = m * m;
  double v0[8], d0[8], v1[8], d1[8];
  for (int q = 0; q < Q; ++q) {
    leg_all(p, (X[2 * q] - lo[0]) / h, v0, d0);
    leg_all(p, (X[2 * q + 1] - lo[1]) / h, v1, d1);
    for (int a1 = 0; a1 < m; ++a1)
      for (int a0 = 0; a0 < m; ++a0) {
        double val;
        if (deriv == 0) val = d0[a0] * v1[a1] / h;
        else if (deriv == 1) val = v0[a0] * d1[a1] / h;
        else val = v0[a0] * v1[a1];
        out[(size_t)q * nq + a0 + m * a1] = val / h;
      }
  }
}

// Lower-triangular L with positive diagonal and L L^T = Z^T Z, from a
// Householder QR of Z (rows x n, row-major, overwritten): L = R^T.  (The
// Cholesky factor of Z^T Z, computed without forming Z^T Z, whose condition
// number is the square of Z's.)
void qr_lower(int rows, int n, std::vector<double>& Z, double* L) {
  if (rows < n) fail("too few samples for the element basis");
  for (int k = 0; k < n; ++k) {
    double nrm = 0.0;
    for (int i = k; i < rows; ++i) nrm += Z[(size_t)i * n + k] * Z[(size_t)i * n + k];
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0)) fail("element basis is rank deficient on the element");
    const double a = Z[(size_t)k * n + k];
    const double alpha = a > 0.0 ? -nrm : nrm;
    // v = x - alpha e_k, stored in place below the diagonal (v_k separately)
    const double vk = a - alpha;
    double vnorm2 = vk * vk;
    for (int i = k + 1; i < rows; ++i) vnorm2 += Z[(size_t)i * n + k] * Z[(size_t)i * n + k];
    Z[(size_t)k * n + k] = alpha;
    if (vnorm2 > 0.0)
      for (int j = k + 1; j < n; ++j) {
        double s = vk * Z[(size_t)k * n + j];
        for (int i = k + 1; i < rows; ++i) s += Z[(size_t)i * n + k] * Z[(size_t)i * n + j];
        const double f = 2.0 * s / vnorm2;
        Z[(size_t)k * n + j] -= f * vk;
        for (int i = k + 1; i < rows; ++i) Z[(size_t)i * n + j] -= f * Z[(size_t)i * n + k];
      }
  }
  for (int i = 0; i < n; ++i) {
    const double sg = Z[(size_t)i * n + i] < 0.0 ? -1.0 : 1.0;
    for (int j = 0; j < n; ++j) L[j * n + i] = j >= i ? sg * Z[(size_t)i * n + j] : 0.0;
  }
}

// inverse of a lower-triangular matrix (row-major)
void tri_inverse(int n, const double* L, double* X) {
  for (int i = 0; i < n * n; ++i) X[i] = 0.0;
  for (int c = 0; c < n; ++c) {
    X[c * n + c] = 1.0 / L[c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s -= L[i * n + k] * X[k * n + c];
      X[i * n + c] = s / L[i * n + i];
    }
  }
}

// inverse of a general n x n matrix (row-major) by Gauss-Jordan with partial pivoting
void gj_inverse(int n, const double* A, double* X) {
  std::vector<double> W(A, A + n * n);
  for (int i = 0; i < n * n; ++i) X[i] = 0.0;
  for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(W[r * n + c]) > std::fabs(W[pr * n + c])) pr = r;
    if (W[pr * n + c] == 0.0) fail("singular mass block");
    if (pr != c)
      for (int k = 0; k < n; ++k) {
        std::swap(W[pr * n + k], W[c * n + k]);
        std::swap(X[pr * n + k], X[c * n + k]);
      }
    const double d = 1.0 / W[c * n + c];
    for (int k = 0; k < n; ++k) {
      W[c * n + k] *= d;
      X[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r)
      if (r != c && W[r * n + c] != 0.0) {
        const double f = W[r * n + c];
        for (int k = 0; k < n; ++k) {
          W[r * n + k] -= f * W[c * n + k];
          X[r * n + k] -= f * X[c * n + k];
        }
      }
  }
}

// C (+)= op(A) * B for n x n row-major blocks; ta: A transposed
inline void gemm(int n, const double* A, bool ta, const double* B, double* C, double alpha = 1.0) {
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double a = alpha * (ta ? A[k * n + i] : A[i * n + k]);
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
}

// face block sum_q w coef Trow[q][a] Tcol[q][b] added into out (scaled by s)
void face_block(int nq, int Q, const double* w, const double* coef, const double* Tr, const double* Tc, double s,
                double* out) {
  for (int q = 0; q < Q; ++q) {
    const double cw = s * w[q] * coef[q];
    if (cw == 0.0) continue;
    for (int a = 0; a < nq; ++a) {
      const double ta = cw * Tr[(size_t)q * nq + a];
      for (int b = 0; b < nq; ++b) out[a * nq + b] += ta * Tc[(size_t)q * nq + b];
    }
  }
}

struct Fine {
  int n;
  double h;
  std::vector<Rule> piece;            // [2 * cell + (chi - 1)], empty if absent
  std::vector<unsigned char> cut;     // per cell
  std::vector<BoxRules> surf;         // per cut cell (indexed through surf_of)
  std::vector<int> surf_of;           // cell -> index into surf, -1
  std::vector<int> elem_of;           // [2 * cell + (chi - 1)] -> element, -1
};

// per-phase rules of the grid edge x_axis = m h, x_other in [io h, (io+1) h]
void edge_rules(const Circle& ls, const Fine& F, int axis, int mpos, int io, int q_full, int q_cut,
                const std::vector<double>& gf, const std::vector<double>& wf, const std::vector<double>& gc,
                const std::vector<double>& wc, Rule out[2]) {
  const double h = F.h, a = io * h, b = (io + 1) * h;
  double lo[2], hi[2];
  lo[axis] = hi[axis] = mpos * h;
  lo[1 - axis] = a;
  hi[1 - axis] = b;
  double mn, mx;
  ls.range(lo, hi, mn, mx);
  if (mn < 0.0 && 0.0 < mx) {
    segment(ls, axis, mpos * h, a, b, q_cut, gc, wc, out);
    return;
  }
  const int chi = mx <= 0.0 ? 0 : 1;
  for (int i = 0; i < q_full; ++i) {
    double x[2];
    put(axis, a + h * gf[i], mpos * h, x);
    out[chi].add(x[0], x[1], wf[i] * h);
  }
}

double lam_of(double mm, double mp) { return mm < mp ? 0.0 : (mm == mp ? 0.5 : 1.0); }

}  // namespace

void imp_basis(const ImpHier& H, const ImpLevel& L, int64_t e, int Q, const double* X, int deriv, double* out) {
  const int nq = H.nq;
  const double h = 1.0 / L.n;
  const int hc = L.host[e];
  const double lo[2] = {(hc % L.n) * h, (hc / L.n) * h};
  std::vector<double> R((size_t)Q * nq);
  raw_basis(H.p, h, lo, Q, X, deriv, R.data());
  if (L.full[e]) {
    std::memcpy(out, R.data(), R.size() * sizeof(double));
    return;
  }
  // psi = L^{-1} phi: forward substitution per point
  const double* Lf = L.L.data() + (size_t)e * nq * nq;
  for (int q = 0; q < Q; ++q) {
    const double* r = R.data() + (size_t)q * nq;
    double* o = out + (size_t)q * nq;
    for (int a = 0; a < nq; ++a) {
      double s = r[a];
      for (int b = 0; b < a; ++b) s -= Lf[a * nq + b] * o[b];
      o[a] = s / Lf[a * nq + a];
    }
  }
}

namespace {

// Algorithm 2 with the injection of level F (fine) into C (coarse)
void coarsen_ops(const ImpHier& H, const ImpLevel& F, ImpLevel& C) {
  const int nq = H.nq;
  const size_t bs = (size_t)nq * nq;
  const int64_t NC = C.NE;
  auto triple = [&](auto rowfn, double scale, SBM& out) {
    out.init(NC, nq);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < NC; ++c) {
      std::map<int, std::vector<double>> acc;
      std::vector<double> T(bs), X(bs);
      for (int k = C.kid_ptr[c]; k < C.kid_ptr[c + 1]; ++k) {
        const int f = C.kids[k];
        const double* If = F.Iblk.data() + (size_t)f * bs;
        rowfn(f, [&](int g, const double* Xfg) {
          std::fill(T.begin(), T.end(), 0.0);
          gemm(nq, If, true, Xfg, T.data());               // I_f^T X_fg
          auto& dst = acc[F.parent[g]];
          if (dst.empty()) dst.assign(bs, 0.0);
          gemm(nq, T.data(), false, F.Iblk.data() + (size_t)g * bs, dst.data(), scale);
        });
      }
      for (auto& kv : acc) {
        out.col[c].push_back(kv.first);
        out.val[c].insert(out.val[c].end(), kv.second.begin(), kv.second.end());
      }
    }
  };
  auto rows_of = [&](const SBM& A) {
    return [&A, nq](int f, auto emit) {
      for (size_t k = 0; k < A.col[f].size(); ++k) emit(A.col[f][k], A.val[f].data() + k * nq * nq);
    };
  };
  triple(rows_of(F.M), 1.0, C.M);
  triple(rows_of(F.Mmu), 1.0, C.Mmu);
  triple(rows_of(F.Et), 0.5, C.Et);
  if (F.Mrho.NE > 0) {
    // Algorithm 3: M_rho, the two pressure-penalty limits with factors 2 and
    // 1/2, blended per element pair by eq. (Etimedep) (Frobenius norms)
    triple(rows_of(F.Mrho), 1.0, C.Mrho);
    triple(rows_of(F.Emu), 2.0, C.Emu);
    triple(rows_of(F.Erho), 0.5, C.Erho);
    C.E.init(NC, nq);
    for (int64_t c = 0; c < NC; ++c) {
      std::vector<int> cols = C.Emu.col[c];
      cols.insert(cols.end(), C.Erho.col[c].begin(), C.Erho.col[c].end());
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      for (int f : cols) {
        const double* a = C.Emu.get(c, f);
        const double* b = C.Erho.get(c, f);
        double na = 0.0, nb = 0.0;
        for (size_t i = 0; i < bs; ++i) {
          if (a) na += a[i] * a[i];
          if (b) nb += b[i] * b[i];
        }
        na = std::sqrt(na);
        nb = std::sqrt(nb);
        if (na + nb == 0.0) continue;
        const double wa = (nb / (na + nb)) * (nb / (na + nb)), wb = (na / (na + nb)) * (na / (na + nb));
        double* o = C.E.at(c, f);
        for (size_t i = 0; i < bs; ++i) o[i] = (a ? wa * a[i] : 0.0) + (b ? wb * b[i] : 0.0);
      }
    }
  } else {
    triple(rows_of(F.E), 2.0, C.E);
  }
  std::vector<double> M2inv((size_t)NC * bs);
  for (int64_t c = 0; c < NC; ++c) {
    const double* m2 = C.M.get(c, (int)c);
    if (!m2) fail("coarse mass block missing");
    gj_inverse(nq, m2, M2inv.data() + c * bs);
  }
  for (int k = 0; k < 2; ++k) {
    SBM T;
    const SBM& Gk = F.G[k];
    triple(
        [&](int f, auto emit) {
          const double* Mf = F.M.get(f, f);
          std::vector<double> MG(bs);
          for (size_t j = 0; j < Gk.col[f].size(); ++j) {
            std::fill(MG.begin(), MG.end(), 0.0);
            gemm(nq, Mf, false, Gk.val[f].data() + j * bs, MG.data());
            emit(Gk.col[f][j], MG.data());
          }
        },
        1.0, T);
    C.G[k].init(NC, nq);
    for (int64_t c = 0; c < NC; ++c) {
      C.G[k].col[c] = T.col[c];
      C.G[k].val[c].assign(T.val[c].size(), 0.0);
      for (size_t j = 0; j < T.col[c].size(); ++j)
        gemm(nq, M2inv.data() + c * bs, false, T.val[c].data() + j * bs, C.G[k].val[c].data() + j * bs);
    }
  }
}

// transpose index of a block-sparse matrix: for column e, (row, slot) pairs
std::vector<std::vector<std::pair<int, int>>> transpose_index(const SBM& A) {
  std::vector<std::vector<std::pair<int, int>>> t(A.NE);
  for (int64_t r = 0; r < A.NE; ++r)
    for (size_t k = 0; k < A.col[r].size(); ++k) t[A.col[r][k]].push_back({(int)r, (int)k});
  return t;
}

// eq. (stokessystem) with eq. (viscousop) as element blocks, (alpha, beta)
// scaled when requested; colours, inverses
void compose(const ldgs_problem& P, const ImpHier& H, ImpLevel& L) {
  const int nq = H.nq, nb = H.nb;
  const size_t bs = (size_t)nq * nq;
  const int64_t NE = L.NE;
  const double gamma = P.form == LDGS_VISCOUS_STRESS ? 1.0 : 0.0;
  auto tG0 = transpose_index(L.G[0]);
  auto tG1 = transpose_index(L.G[1]);
  const decltype(tG0)* tG[2] = {&tG0, &tG1};
  if (P.diag_scaling) {
    L.dscale.resize(NE * 2);
    for (int64_t e = 0; e < NE; ++e) {
      const double mu = L.Mmu.get(e, (int)e)[0];
      L.dscale[2 * e] = 1.0 / std::sqrt(mu);
      L.dscale[2 * e + 1] = std::sqrt(mu);
    }
  }
  // block structure of every row: the union of the columns its terms reach
  L.rowptr.assign(NE + 1, 0);
  std::vector<std::vector<int>> rcols(NE);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t e = 0; e < NE; ++e) {
    std::vector<int>& c = rcols[e];
    for (int j = 0; j < 2; ++j)
      for (auto [hrow, slot] : (*tG[j])[e]) {
        (void)slot;
        c.push_back(hrow);
        for (int i = 0; i < 2; ++i) c.insert(c.end(), L.G[i].col[hrow].begin(), L.G[i].col[hrow].end());
      }
    c.insert(c.end(), L.Et.col[e].begin(), L.Et.col[e].end());
    c.insert(c.end(), L.E.col[e].begin(), L.E.col[e].end());
    for (int i = 0; i < 2; ++i) c.insert(c.end(), L.G[i].col[e].begin(), L.G[i].col[e].end());
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
  }
  for (int64_t e = 0; e < NE; ++e) L.rowptr[e + 1] = L.rowptr[e] + (int)rcols[e].size();
  L.cols.resize(L.rowptr[NE]);
  for (int64_t e = 0; e < NE; ++e) std::copy(rcols[e].begin(), rcols[e].end(), L.cols.begin() + L.rowptr[e]);
  rcols.clear();
  rcols.shrink_to_fit();
  L.blk.resize((size_t)L.rowptr[NE] * nb * nb);        // every entry written below
#pragma omp parallel
  {
    std::vector<double> T(bs), U(bs), R;
#pragma omp for schedule(dynamic, 256)
    for (int64_t e = 0; e < NE; ++e) {
      const int k0 = L.rowptr[e], nk = L.rowptr[e + 1] - k0;
      R.assign((size_t)nk * nb * nb, 0.0);       // the row's blocks, row-major
      auto addsub = [&](int c, int bi, int bj, const double* S, double s) {
        const int k = (int)(std::lower_bound(L.cols.begin() + k0, L.cols.begin() + k0 + nk, c) - (L.cols.begin() + k0));
        double* B = R.data() + (size_t)k * nb * nb;
        for (int a = 0; a < nq; ++a)
          for (int b = 0; b < nq; ++b) B[(size_t)(bi * nq + a) * nb + bj * nq + b] += s * S[a * nq + b];
      };
      // scalar blocks of row e: P_ij = G_j^T Mmu G_i (i, j < 2), Et, E, G_j^T M, M G_i
      for (int j = 0; j < 2; ++j)
        for (auto [hrow, slot] : (*tG[j])[e]) {
          const double* Gje = L.G[j].val[hrow].data() + (size_t)slot * bs;   // G_j[h][e]
          const double* Mh = L.Mmu.get(hrow, hrow);
          std::fill(T.begin(), T.end(), 0.0);
          gemm(nq, Gje, true, Mh, T.data());                                 // G_j[h][e]^T Mmu_h
          for (int i = 0; i < 2; ++i)
            for (size_t k = 0; k < L.G[i].col[hrow].size(); ++k) {
              const int f = L.G[i].col[hrow][k];
              std::fill(U.begin(), U.end(), 0.0);
              gemm(nq, T.data(), false, L.G[i].val[hrow].data() + k * bs, U.data());   // P_ij(e, f)
              if (i == j) {
                addsub(f, 0, 0, U.data(), 1.0);
                addsub(f, 1, 1, U.data(), 1.0);
              }
              if (gamma != 0.0) addsub(f, i, j, U.data(), gamma);
            }
          // -(G_j^T M)(e, h)
          std::fill(U.begin(), U.end(), 0.0);
          gemm(nq, Gje, true, L.M.get(hrow, hrow), U.data());
          addsub(hrow, j, 2, U.data(), -1.0);
        }
      for (size_t k = 0; k < L.Et.col[e].size(); ++k) {
        addsub(L.Et.col[e][k], 0, 0, L.Et.val[e].data() + k * bs, 1.0);
        addsub(L.Et.col[e][k], 1, 1, L.Et.val[e].data() + k * bs, 1.0);
      }
      const double* Me = L.M.get(e, (int)e);
      for (int i = 0; i < 2; ++i)
        for (size_t k = 0; k < L.G[i].col[e].size(); ++k) {
          std::fill(U.begin(), U.end(), 0.0);
          gemm(nq, Me, false, L.G[i].val[e].data() + k * bs, U.data());       // (M G_i)(e, f)
          addsub(L.G[i].col[e][k], 2, i, U.data(), -1.0);
        }
      for (size_t k = 0; k < L.E.col[e].size(); ++k) addsub(L.E.col[e][k], 2, 2, L.E.val[e].data() + k * bs, -1.0);
      if (P.delta > 0.0) {
        // eq. (timedep2): M_rho / delta on every velocity component
        const double* Mr = L.Mrho.get(e, (int)e);
        addsub((int)e, 0, 0, Mr, 1.0 / P.delta);
        addsub((int)e, 1, 1, Mr, 1.0 / P.delta);
      }
      for (int k = 0; k < nk; ++k) {
        const int f = L.cols[k0 + k];
        const double* B = R.data() + (size_t)k * nb * nb;
        double* O = L.blk.data() + (size_t)(k0 + k) * nb * nb;      // column-major
        for (int r = 0; r < nb; ++r) {
          const double sr = P.diag_scaling ? L.dscale[2 * e + (r < 2 * nq ? 0 : 1)] : 1.0;
          for (int c = 0; c < nb; ++c) {
            const double sc = P.diag_scaling ? L.dscale[2 * f + (c < 2 * nq ? 0 : 1)] : 1.0;
            O[(size_t)c * nb + r] = B[r * nb + c] * sr * sc;
          }
        }
      }
    }
  }
}

void colour_and_invert(ImpLevel& L, int nb) {
  const int64_t NE = L.NE;
  std::vector<std::vector<int>> nbr(NE);
  for (int64_t e = 0; e < NE; ++e)
    for (int k = L.rowptr[e]; k < L.rowptr[e + 1]; ++k) {
      if (L.cols[k] == e) continue;
      // a block of the structure whose entries all vanish couples nothing
      const double* B = L.blk.data() + (size_t)k * nb * nb;
      bool any = false;
      for (size_t i = 0; i < (size_t)nb * nb && !any; ++i) any = B[i] != 0.0;
      if (!any) continue;
      nbr[e].push_back(L.cols[k]);
      nbr[L.cols[k]].push_back((int)e);
    }
  L.colour.assign(NE, -1);
  L.ncol = 0;
  for (int64_t e = 0; e < NE; ++e) {
    std::vector<char> used(L.ncol + 1, 0);
    for (int f : nbr[e])
      if (L.colour[f] >= 0 && L.colour[f] <= L.ncol) used[L.colour[f]] = 1;
    int c = 0;
    while (used[c]) ++c;
    L.colour[e] = c;
    L.ncol = std::max(L.ncol, c + 1);
  }
  // verified against the stored blocks: no block couples two elements of one
  // colour (the colour pass updates a colour's elements simultaneously)
  for (int64_t e = 0; e < NE; ++e)
    for (int f : nbr[e])
      if (L.colour[f] == L.colour[e]) fail("colouring couples two elements of one colour");
  L.elems.assign(L.ncol, {});
  for (int64_t e = 0; e < NE; ++e) L.elems[L.colour[e]].push_back((int)e);
  L.inv.resize((size_t)NE * nb * nb);                  // every block written below
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 256) reduction(&& : ok)
  for (int64_t e = 0; e < NE; ++e) {
    const double* D = nullptr;
    for (int k = L.rowptr[e]; k < L.rowptr[e + 1]; ++k)
      if (L.cols[k] == e) D = L.blk.data() + (size_t)k * nb * nb;
    std::vector<double> A((size_t)nb * nb), X((size_t)nb * nb);
    if (!D) {
      ok = false;
      continue;
    }
    for (int r = 0; r < nb; ++r)
      for (int c = 0; c < nb; ++c) A[r * nb + c] = D[(size_t)c * nb + r];
    if (!block_inverse(nb, A.data(), X.data(), 1e-14)) {
      ok = false;
      continue;
    }
    double* I = L.inv.data() + (size_t)e * nb * nb;
    for (int r = 0; r < nb; ++r)
      for (int c = 0; c < nb; ++c) I[(size_t)c * nb + r] = X[r * nb + c];
  }
  if (!ok) fail("singular element block");
}

}  // namespace

void imp_build(const ldgs_problem& P, ImpHier& H) {
  if (P.dim != 2) fail("implicitly defined meshes are two-dimensional");
  if (P.bc[0] != LDGS_DIRICHLET || P.bc[1] != LDGS_DIRICHLET) fail("implicitly defined meshes: Dirichlet walls only");
  H.p = P.degree;
  H.m = H.p + 1;
  H.nq = H.m * H.m;
  H.nb = 3 * H.nq;
  H.r = P.levelset_params[0];
  H.cx = P.levelset_centre[0];
  H.cy = P.levelset_centre[1];
  if (!(H.r > 0.0)) fail("circle radius must be positive");
  const Circle ls{{H.cx, H.cy}, H.r};
  // a curved domain (the disk alone): phase 2 is not part of the domain
  const int nphase = P.levelset_kind == LDGS_LEVELSET_DISK ? 1 : 2;
  // LDGS_SETUP_TIMING=1: wall time of each phase on stderr
  const bool timing = std::getenv("LDGS_SETUP_TIMING") && std::atoi(std::getenv("LDGS_SETUP_TIMING"));
  auto tmark = std::chrono::steady_clock::now();
  auto phase = [&](const char* what) {
    if (!timing) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[ldgs implicit] %-26s %8.3f s\n", what, std::chrono::duration<double>(now - tmark).count());
    tmark = now;
  };
  const int n = P.n, p = H.p, m = H.m, nq = H.nq;
  const int q_full = p + 2, q_cut = P.q_cut > 0 ? P.q_cut : 8;
  const double h = 1.0 / n;
  std::vector<double> gf, wf, gc, wc;
  Basis::gauss(q_full, gf, wf);
  Basis::gauss(q_cut, gc, wc);
  // ---------------------------------------------------------------- pieces
  Fine F;
  F.n = n;
  F.h = h;
  const int64_t NCELL = (int64_t)n * n;
  F.piece.assign(2 * NCELL, Rule{});
  F.cut.assign(NCELL, 0);
  F.surf_of.assign(NCELL, -1);
  for (int i1 = 0; i1 < n; ++i1)
    for (int i0 = 0; i0 < n; ++i0) {
      const int64_t c = i0 + (int64_t)n * i1;
      const double lo[2] = {i0 * h, i1 * h}, hi[2] = {(i0 + 1) * h, (i1 + 1) * h};
      double mn, mx;
      ls.range(lo, hi, mn, mx);
      if (mn < 0.0 && 0.0 < mx) {
        BoxRules br;
        cut_box(ls, lo, hi, q_cut, gc, wc, br);
        for (int chi = 0; chi < nphase; ++chi)
          if (!br.vol[chi].w.empty() && br.vol[chi].sum() > 0.0) F.piece[2 * c + chi] = br.vol[chi];
        F.cut[c] = 1;
        F.surf_of[c] = (int)F.surf.size();
        F.surf.push_back(std::move(br));
      } else {
        const int chi = mx <= 0.0 ? 0 : 1;
        if (chi >= nphase) continue;      // outside a curved domain
        Rule& R = F.piece[2 * c + chi];
        for (int b = 0; b < q_full; ++b)
          for (int a = 0; a < q_full; ++a) R.add((i0 + gf[a]) * h, (i1 + gf[b]) * h, wf[a] * wf[b] * h * h);
      }
    }
  H.n_cut = (int)F.surf.size();
  phase("cells and quadrature");
  // --------------------------------------------------------------- merging
  auto exists = [&](int64_t key) { return !F.piece[key].w.empty(); };
  std::vector<double> frac(2 * NCELL, 0.0);
  for (int64_t k = 0; k < 2 * NCELL; ++k)
    if (exists(k)) frac[k] = F.piece[k].sum() / (h * h);
  std::vector<int64_t> target(2 * NCELL, -1);
  const int DIRS[4][2] = {{0, -1}, {0, 1}, {1, -1}, {1, 1}};
  for (int64_t key = 0; key < 2 * NCELL; ++key) {
    if (!exists(key) || frac[key] >= FRAC_MIN) continue;
    const int64_t c = key / 2;
    const int chi = (int)(key % 2);
    const int i0 = (int)(c % n), i1 = (int)(c / n);
    int64_t best = -1;
    bool best_large = false;
    double best_len = 0.0;
    for (auto& dir : DIRS) {
      const int axis = dir[0], step = dir[1];
      int j[2] = {i0, i1};
      j[axis] += step;
      if (j[0] < 0 || j[0] >= n || j[1] < 0 || j[1] >= n) continue;
      const int64_t c2 = j[0] + (int64_t)n * j[1];
      if (!exists(2 * c2 + chi)) continue;
      const int ij[2] = {i0, i1};
      Rule er[2];
      edge_rules(ls, F, axis, ij[axis] + (step > 0 ? 1 : 0), ij[1 - axis], q_full, q_cut, gf, wf, gc, wc, er);
      const double len = er[chi].sum();
      if (!(len > 0.0)) continue;
      const bool large = frac[2 * c2 + chi] >= FRAC_MIN;
      // lengths within a relative 1e-12 count as equal (mirror-symmetric
      // ties of the circle): the first face in the order above wins
      if (best < 0 || large > best_large || (large == best_large && len > best_len * (1.0 + 1e-12))) {
        best = 2 * c2 + chi;
        best_large = large;
        best_len = len;
      }
    }
    if (best < 0) fail("a small cut piece has no neighbour of its phase to merge with");
    target[key] = best;
  }
  std::vector<int64_t> root(2 * NCELL, -1);
  for (int64_t key = 0; key < 2 * NCELL; ++key) {
    if (!exists(key)) continue;
    int64_t k = key;
    int guard = 0;
    while (target[k] >= 0) {
      k = target[k];
      if (++guard > 64) fail("merging cycle");
    }
    root[key] = k;
    if (target[key] >= 0) ++H.n_merged;
  }
  phase("merging");
  // elements: roots in (cell, phase) order; members in (cell, phase) order
  F.elem_of.assign(2 * NCELL, -1);
  std::vector<int64_t> roots;
  for (int64_t key = 0; key < 2 * NCELL; ++key)
    if (exists(key) && root[key] == key) roots.push_back(key);
  std::vector<int> rid(2 * NCELL, -1);
  for (size_t i = 0; i < roots.size(); ++i) rid[roots[i]] = (int)i;
  const int64_t NE = (int64_t)roots.size();
  H.lv.clear();
  H.lv.emplace_back();
  ImpLevel& L0 = H.lv[0];
  L0.n = n;
  L0.NE = NE;
  L0.host.resize(NE);
  L0.phase.resize(NE);
  L0.full.assign(NE, 1);
  L0.area.assign(NE, 0.0);
  H.rules.assign(NE, ImpElemRule{});
  std::vector<int> nmem(NE, 0);
  for (int64_t key = 0; key < 2 * NCELL; ++key) {
    if (!exists(key)) continue;
    const int e = rid[root[key]];
    F.elem_of[key] = e;
    H.rules[e].X.insert(H.rules[e].X.end(), F.piece[key].X.begin(), F.piece[key].X.end());
    H.rules[e].w.insert(H.rules[e].w.end(), F.piece[key].w.begin(), F.piece[key].w.end());
    ++nmem[e];
  }
  for (int64_t e = 0; e < NE; ++e) {
    const int64_t key = roots[e];
    L0.host[e] = (int)(key / 2);
    L0.phase[e] = (int)(key % 2) + 1;
    L0.full[e] = (nmem[e] == 1 && !F.cut[key / 2]) ? 1 : 0;
    for (double v : H.rules[e].w) L0.area[e] += v;
  }
  // orthonormalisation factors
  L0.L.assign((size_t)NE * nq * nq, 0.0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < NE; ++e) {
    double* Le = L0.L.data() + (size_t)e * nq * nq;
    if (L0.full[e]) {
      for (int a = 0; a < nq; ++a) Le[a * nq + a] = 1.0;
      continue;
    }
    const int Q = (int)H.rules[e].w.size();
    const double lo[2] = {(L0.host[e] % n) * h, (L0.host[e] / n) * h};
    std::vector<double> R((size_t)Q * nq);
    raw_basis(p, h, lo, Q, H.rules[e].X.data(), -1, R.data());
    for (int q = 0; q < Q; ++q) {
      const double sw = std::sqrt(H.rules[e].w[q]);
      for (int a = 0; a < nq; ++a) R[(size_t)q * nq + a] *= sw;
    }
    qr_lower(Q, nq, R, Le);
  }
  phase("elements and bases");
  // ----------------------------------------------------------------- faces
  H.faces.clear();
  for (int axis = 0; axis < 2; ++axis)
    for (int mp = 0; mp <= n; ++mp)
      for (int io = 0; io < n; ++io) {
        Rule er[2];
        edge_rules(ls, F, axis, mp, io, q_full, q_cut, gf, wf, gc, wc, er);
        for (int chi = 0; chi < nphase; ++chi) {
          if (er[chi].w.empty()) continue;
          int64_t lo_c = -1, hi_c = -1;
          int ij[2];
          if (mp > 0) {
            ij[axis] = mp - 1;
            ij[1 - axis] = io;
            lo_c = ij[0] + (int64_t)n * ij[1];
          }
          if (mp < n) {
            ij[axis] = mp;
            ij[1 - axis] = io;
            hi_c = ij[0] + (int64_t)n * ij[1];
          }
          ImpFace f;
          f.X = er[chi].X;
          f.w = er[chi].w;
          f.nrm.assign(2 * f.w.size(), 0.0);
          auto elem = [&](int64_t cell) {
            const int e = F.elem_of[2 * cell + chi];
            if (e < 0) fail("edge piece without an element");
            return e;
          };
          if (lo_c < 0) {
            for (size_t q = 0; q < f.w.size(); ++q) f.nrm[2 * q + axis] = -1.0;
            f.kind = 2;
            f.minus = elem(hi_c);
          } else if (hi_c < 0) {
            for (size_t q = 0; q < f.w.size(); ++q) f.nrm[2 * q + axis] = 1.0;
            f.kind = 2;
            f.minus = elem(lo_c);
          } else {
            const int e1 = elem(lo_c), e2 = elem(hi_c);
            if (e1 == e2) continue;
            for (size_t q = 0; q < f.w.size(); ++q) f.nrm[2 * q + axis] = 1.0;
            f.kind = 0;
            f.minus = e1;
            f.plus = e2;
          }
          H.faces.push_back(std::move(f));
        }
      }
  for (int64_t c = 0; c < NCELL; ++c) {
    if (!F.cut[c]) continue;
    const BoxRules& br = F.surf[F.surf_of[c]];
    if (br.surf.w.empty()) continue;
    ImpFace f;
    f.minus = F.elem_of[2 * c];
    if (nphase == 1) {
      // the boundary of a curved domain: a Dirichlet wall of the inside element
      f.kind = 2;
      f.plus = -1;
      if (f.minus < 0) fail("boundary piece without an element");
    } else {
      f.kind = 1;
      f.plus = F.elem_of[2 * c + 1];
      if (f.minus < 0 || f.plus < 0) fail("interface piece without two elements");
    }
    f.X = br.surf.X;
    f.w = br.surf.w;
    f.nrm = br.nrm;
    H.faces.push_back(std::move(f));
  }
  phase("faces");
  // ------------------------------------------------------ fine operators
  const size_t bs = (size_t)nq * nq;
  L0.M.init(NE, nq);
  L0.Mmu.init(NE, nq);
  L0.G[0].init(NE, nq);
  L0.G[1].init(NE, nq);
  L0.Et.init(NE, nq);
  L0.E.init(NE, nq);
  const bool unsteady = P.delta > 0.0;
  if (unsteady) {
    L0.Mrho.init(NE, nq);
    L0.Emu.init(NE, nq);
    L0.Erho.init(NE, nq);
    for (int64_t e = 0; e < NE; ++e) L0.Mrho.at(e, (int)e);
  }
  for (int64_t e = 0; e < NE; ++e) {
    L0.M.at(e, (int)e);
    L0.Mmu.at(e, (int)e);
    L0.G[0].at(e, (int)e);
    L0.G[1].at(e, (int)e);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < NE; ++e) {
    const int Q = (int)H.rules[e].w.size();
    const double* X = H.rules[e].X.data();
    const double* w = H.rules[e].w.data();
    std::vector<double> B((size_t)Q * nq), D0((size_t)Q * nq), D1((size_t)Q * nq), mu(Q);
    std::vector<int> ph(Q, L0.phase[e]);
    imp_basis(H, L0, e, Q, X, -1, B.data());
    imp_basis(H, L0, e, Q, X, 0, D0.data());
    imp_basis(H, L0, e, Q, X, 1, D1.data());
    eval_field(P.mu, 2, Q, X, ph.data(), mu.data());
    std::vector<double> rho(unsteady ? Q : 0);
    if (unsteady) eval_field(P.rho, 2, Q, X, ph.data(), rho.data());
    double* Mr = unsteady ? L0.Mrho.val[e].data() : nullptr;
    double* Me = L0.M.val[e].data();
    double* Mm = L0.Mmu.val[e].data();
    double* G0 = L0.G[0].val[e].data();
    double* G1 = L0.G[1].val[e].data();
    for (int q = 0; q < Q; ++q)
      for (int a = 0; a < nq; ++a) {
        const double ba = w[q] * B[(size_t)q * nq + a];
        for (int b = 0; b < nq; ++b) {
          Me[a * nq + b] += ba * B[(size_t)q * nq + b];
          Mm[a * nq + b] += ba * mu[q] * B[(size_t)q * nq + b];
          if (Mr) Mr[a * nq + b] += ba * rho[q] * B[(size_t)q * nq + b];
          G0[a * nq + b] += ba * D0[(size_t)q * nq + b];
          G1[a * nq + b] += ba * D1[(size_t)q * nq + b];
        }
      }
  }
  const double Cb = P.tau_u_bdry_C > 0 ? P.tau_u_bdry_C : 10.0;
  const double Ci = P.tau_u_inter_C > 0 ? P.tau_u_inter_C : 8.0;
  const double C0 = P.tau_u_intra_C;
  const double tau = P.tau;
  // face blocks computed in parallel into per-face lists (matrix, row,
  // column, block), then added into the operators in face order
  struct FaceOut {
    std::vector<int> key;        // (matrix, row, column) triples; matrices G_0, G_1, Et, E, Emu, Erho
    std::vector<double> val;
  };
  const int64_t NF = (int64_t)H.faces.size();
  const int64_t CHUNK = 16384;
  std::vector<FaceOut> fout((size_t)std::min(NF, CHUNK));
  SBM* mats[6] = {&L0.G[0], &L0.G[1], &L0.Et, &L0.E, &L0.Emu, &L0.Erho};
  for (int64_t f0 = 0; f0 < NF; f0 += CHUNK) {
  const int64_t f1 = std::min(NF, f0 + CHUNK);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t fi = f0; fi < f1; ++fi) {
    const ImpFace& f = H.faces[fi];
    FaceOut& fo = fout[fi - f0];
    fo.key.clear();
    fo.val.clear();
    auto slot = [&](int mat, int r, int c) {
      fo.key.push_back(mat);
      fo.key.push_back(r);
      fo.key.push_back(c);
      fo.val.resize(fo.val.size() + bs, 0.0);
      return fo.val.data() + fo.val.size() - bs;
    };
    const int Q = (int)f.w.size();
    std::vector<double> Tm((size_t)Q * nq), Tp((size_t)Q * nq), mum(Q), mup(Q), coef(Q);
    std::vector<int> phm(Q, L0.phase[f.minus]), php(Q, f.plus >= 0 ? L0.phase[f.plus] : 0);
    imp_basis(H, L0, f.minus, Q, f.X.data(), -1, Tm.data());
    eval_field(P.mu, 2, Q, f.X.data(), phm.data(), mum.data());
    if (f.plus >= 0) {
      imp_basis(H, L0, f.plus, Q, f.X.data(), -1, Tp.data());
      eval_field(P.mu, 2, Q, f.X.data(), php.data(), mup.data());
    }
    const int mi = f.minus, pl = f.plus;
    auto jump = [&](int mat, const std::vector<double>& t) {
      face_block(nq, Q, f.w.data(), t.data(), Tm.data(), Tm.data(), 1.0, slot(mat, mi, mi));
      face_block(nq, Q, f.w.data(), t.data(), Tp.data(), Tp.data(), 1.0, slot(mat, pl, pl));
      face_block(nq, Q, f.w.data(), t.data(), Tm.data(), Tp.data(), -1.0, slot(mat, mi, pl));
      face_block(nq, Q, f.w.data(), t.data(), Tp.data(), Tm.data(), -1.0, slot(mat, pl, mi));
    };
    for (int k = 0; k < 2; ++k) {
      std::vector<double> nk(Q);
      bool any = false;
      for (int q = 0; q < Q; ++q) {
        nk[q] = f.nrm[2 * q + k];
        any = any || nk[q] != 0.0;
      }
      if (!any) continue;
      if (f.kind == 0) {
        face_block(nq, Q, f.w.data(), nk.data(), Tp.data(), Tp.data(), 1.0, slot(k, pl, pl));
        face_block(nq, Q, f.w.data(), nk.data(), Tp.data(), Tm.data(), -1.0, slot(k, pl, mi));
      } else if (f.kind == 1) {
        std::vector<double> cm(Q), cp(Q);
        for (int q = 0; q < Q; ++q) {
          const double lam = lam_of(mum[q], mup[q]);
          cm[q] = (1.0 - lam) * nk[q];
          cp[q] = lam * nk[q];
        }
        face_block(nq, Q, f.w.data(), cm.data(), Tm.data(), Tp.data(), 1.0, slot(k, mi, pl));
        face_block(nq, Q, f.w.data(), cm.data(), Tm.data(), Tm.data(), -1.0, slot(k, mi, mi));
        face_block(nq, Q, f.w.data(), cp.data(), Tp.data(), Tp.data(), 1.0, slot(k, pl, pl));
        face_block(nq, Q, f.w.data(), cp.data(), Tp.data(), Tm.data(), -1.0, slot(k, pl, mi));
      } else {
        face_block(nq, Q, f.w.data(), nk.data(), Tm.data(), Tm.data(), -1.0, slot(k, mi, mi));
      }
    }
    if (f.kind == 2) {
      for (int q = 0; q < Q; ++q) coef[q] = Cb * p * mum[q] * n;
      face_block(nq, Q, f.w.data(), coef.data(), Tm.data(), Tm.data(), 1.0, slot(2, mi, mi));
    } else if (f.kind == 1) {
      for (int q = 0; q < Q; ++q) coef[q] = Ci * p * std::min(mum[q], mup[q]) * n;
      jump(2, coef);
    } else {
      if (C0 > 0.0) {
        for (int q = 0; q < Q; ++q) coef[q] = C0 * p * mum[q] * n;
        jump(2, coef);
      }
      if (!unsteady) {
        for (int q = 0; q < Q; ++q) coef[q] = tau * h / mum[q];
        jump(3, coef);
      } else {
        // eq. (taugeneral) on the fine level, and its two limits for Algorithm 3
        std::vector<double> rhom(Q);
        eval_field(P.rho, 2, Q, f.X.data(), phm.data(), rhom.data());
        for (int q = 0; q < Q; ++q)
          coef[q] = 1.0 / (h * rhom[q] / (P.tau0 * P.delta) + mum[q] / (tau * h));
        jump(3, coef);
        for (int q = 0; q < Q; ++q) coef[q] = tau * h / mum[q];
        jump(4, coef);
        for (int q = 0; q < Q; ++q) coef[q] = P.tau0 * P.delta / (h * rhom[q]);
        jump(5, coef);
      }
    }
  }
  for (int64_t fi = f0; fi < f1; ++fi) {
    const FaceOut& fo = fout[fi - f0];
    for (size_t t = 0; t * 3 < fo.key.size(); ++t) {
      double* d = mats[fo.key[3 * t]]->at(fo.key[3 * t + 1], fo.key[3 * t + 2]);
      const double* v = fo.val.data() + t * bs;
      for (size_t i = 0; i < bs; ++i) d[i] += v[i];
    }
  }
  }
  (void)bs;
  (void)m;
  phase("fine operators");
  compose(P, H, L0);
  phase("fine Stokes blocks");
  // ------------------------------------------------------- coarse levels
  const int coarsest = P.coarsest_n > 0 ? P.coarsest_n : 4;
  Basis B1;
  B1.init(p);
  while (H.lv.back().n > coarsest) {
    const size_t li = H.lv.size() - 1;
    H.lv.emplace_back();
    ImpLevel& Fl = H.lv[li];
    ImpLevel& C = H.lv[li + 1];
    const int nc = Fl.n / 2;
    C.n = nc;
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int64_t f = 0; f < Fl.NE; ++f) {
      const int hc = Fl.host[f];
      const int pc = (hc % Fl.n) / 2 + nc * ((hc / Fl.n) / 2);
      groups[{pc, Fl.phase[f]}].push_back((int)f);
    }
    C.NE = (int64_t)groups.size();
    C.host.resize(C.NE);
    C.phase.resize(C.NE);
    C.full.assign(C.NE, 0);
    C.area.assign(C.NE, 0.0);
    C.kid_ptr.assign(C.NE + 1, 0);
    Fl.parent.assign(Fl.NE, -1);
    int64_t cid = 0;
    for (auto& kv : groups) {
      C.host[cid] = kv.first.first;
      C.phase[cid] = kv.first.second;
      bool all_full = kv.second.size() == 4;
      for (int f : kv.second) {
        Fl.parent[f] = (int)cid;
        C.kids.push_back(f);
        all_full = all_full && Fl.full[f];
        C.area[cid] += Fl.area[f];
      }
      C.full[cid] = all_full ? 1 : 0;
      C.kid_ptr[cid + 1] = (int)C.kids.size();
      ++cid;
    }
    // injection: S2 (coarse raw in fine raw) per child offset, raw coarse
    // mass, Cholesky factor, I = L_f^T S2^T L_c^{-T}
    C.L.assign((size_t)C.NE * nq * nq, 0.0);
    Fl.Iblk.assign((size_t)Fl.NE * nq * nq, 0.0);
    auto S2 = [&](int f, std::vector<double>& S) {
      const int hc = Fl.host[f];
      const int o0 = (hc % Fl.n) % 2, o1 = (hc / Fl.n) % 2;
      for (int a1 = 0; a1 < m; ++a1)
        for (int a0 = 0; a0 < m; ++a0)
          for (int b1 = 0; b1 < m; ++b1)
            for (int b0 = 0; b0 < m; ++b0)
              S[(a0 + m * a1) * nq + b0 + m * b1] = B1.P[o0][b0 * m + a0] * B1.P[o1][b1 * m + a1];
    };
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < C.NE; ++c) {
      std::vector<double> S(bs), T(bs), Linv(bs);
      double* Lc = C.L.data() + (size_t)c * bs;
      if (C.full[c]) {
        for (int a = 0; a < nq; ++a) Lc[a * nq + a] = 1.0;
      } else {
        // raw coarse mass = sum_f (S L_f)(S L_f)^T = Z^T Z with Z the stack of
        // the blocks (S L_f)^T
        const int nk = C.kid_ptr[c + 1] - C.kid_ptr[c];
        std::vector<double> Z((size_t)nk * nq * nq);
        for (int k = C.kid_ptr[c]; k < C.kid_ptr[c + 1]; ++k) {
          const int f = C.kids[k];
          S2(f, S);
          const double* L = Fl.L.data() + (size_t)f * bs;
          std::fill(T.begin(), T.end(), 0.0);
          gemm(nq, S.data(), false, L, T.data());     // T = S L_f
          double* Zk = Z.data() + (size_t)(k - C.kid_ptr[c]) * bs;
          for (int a = 0; a < nq; ++a)
            for (int b = 0; b < nq; ++b) Zk[a * nq + b] = T[b * nq + a];
        }
        qr_lower(nk * nq, nq, Z, Lc);
      }
      tri_inverse(nq, Lc, Linv.data());
      for (int k = C.kid_ptr[c]; k < C.kid_ptr[c + 1]; ++k) {
        const int f = C.kids[k];
        S2(f, S);
        const double* L = Fl.L.data() + (size_t)f * bs;
        // I = L_f^T S^T Linv^T: I[a][b] = sum_j (S L_f)[j][a] Linv[b][j]
        std::fill(T.begin(), T.end(), 0.0);
        gemm(nq, S.data(), false, L, T.data());   // T = S L_f
        double* I = Fl.Iblk.data() + (size_t)f * bs;
        for (int a = 0; a < nq; ++a)
          for (int b = 0; b < nq; ++b) {
            double s = 0.0;
            for (int j = 0; j < nq; ++j) s += T[j * nq + a] * Linv[b * nq + j];
            I[a * nq + b] = s;
          }
      }
    }
    coarsen_ops(H, Fl, C);
    compose(P, H, C);
    phase("coarse level");
  }
  for (size_t l = 0; l + 1 < H.lv.size(); ++l) colour_and_invert(H.lv[l], H.nb);
  phase("colours and inverses");
  // ----------------------------------------------------------- bottom
  {
    const ImpLevel& Bt = H.lv.back();
    const int nb = H.nb;
    const int64_t N = Bt.NE * nb;
    if (N > 20000) fail("coarsest implicit level too large for the dense bottom solver");
    H.Nc = N;
    H.Ac.assign(N * N, 0.0);
    for (int64_t e = 0; e < Bt.NE; ++e)
      for (int k = Bt.rowptr[e]; k < Bt.rowptr[e + 1]; ++k) {
        const int f = Bt.cols[k];
        const double* B = Bt.blk.data() + (size_t)k * nb * nb;
        for (int r = 0; r < nb; ++r)
          for (int c = 0; c < nb; ++c) H.Ac[(e * nb + r) * N + f * nb + c] = B[(size_t)c * nb + r];
      }
    std::vector<double> dg(N), Bd(N * N), lam;
    for (int64_t i = 0; i < N; ++i) dg[i] = 1.0 / std::sqrt(std::fabs(H.Ac[i * N + i]));
    for (int64_t i = 0; i < N; ++i)
      for (int64_t j = 0; j < N; ++j)
        Bd[i * N + j] = 0.5 * (dg[i] * H.Ac[i * N + j] * dg[j] + dg[j] * H.Ac[j * N + i] * dg[i]);
    sym_eigen((int)N, Bd, lam);
    std::vector<int64_t> order(N);
    for (int64_t i = 0; i < N; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return std::fabs(lam[a]) < std::fabs(lam[b]); });
    double lmax = 0.0;
    for (double v : lam) lmax = std::max(lmax, std::fabs(v));
    const int k0 = 1;
    if (std::fabs(lam[order[k0]]) <= 1e-8 * lmax) fail("coarsest operator has more near-zero eigenvalues than the kernel");
    std::vector<double> inv(N, 0.0);
    for (int64_t i = k0; i < N; ++i) inv[order[i]] = 1.0 / lam[order[i]];
    H.pinv.assign(N * N, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
      for (int64_t k = 0; k < N; ++k) {
        const double vik = Bd[i * N + k] * inv[k];
        if (vik == 0.0) continue;
        for (int64_t j = 0; j < N; ++j) H.pinv[i * N + j] += vik * Bd[j * N + k];
      }
    for (int64_t i = 0; i < N; ++i)
      for (int64_t j = 0; j < N; ++j) H.pinv[i * N + j] *= dg[i] * dg[j];
    H.eig = lam;
  }
  phase("bottom");
  // fine kernel: the constant pressure, sqrt(|E|) on the first pressure function
  const ImpLevel& Lf0 = H.lv[0];   // (the level vector has grown since L0 was taken)
  H.kernel.assign((size_t)Lf0.NE * H.nb, 0.0);
  double s = 0.0;
  for (int64_t e = 0; e < Lf0.NE; ++e) s += Lf0.area[e];
  for (int64_t e = 0; e < Lf0.NE; ++e) H.kernel[(size_t)e * H.nb + 2 * nq] = std::sqrt(Lf0.area[e] / s);
}

void imp_rhs(const ldgs_problem& P, const ImpHier& H, const ldgs_rhs_data& data, double* b) {
  const ImpLevel& L = H.lv[0];
  const int nq = H.nq, nb = H.nb;
  const int64_t NE = L.NE;
  const double h = 1.0 / L.n;
  const double gamma = P.form == LDGS_VISCOUS_STRESS ? 1.0 : 0.0;
  const double Cb = P.tau_u_bdry_C > 0 ? P.tau_u_bdry_C : 10.0;
  const double Ci = P.tau_u_inter_C > 0 ? P.tau_u_inter_C : 8.0;
  const int p = H.p;
  // per-field coefficient vectors [NE][nq]
  std::vector<double> Pf[2], Jg[2][2], Jh[2], pen[2], Pfd(NE * nq, 0.0), Jgn(NE * nq, 0.0);
  for (int i = 0; i < 2; ++i) {
    Pf[i].assign(NE * nq, 0.0);
    Jh[i].assign(NE * nq, 0.0);
    pen[i].assign(NE * nq, 0.0);
    for (int k = 0; k < 2; ++k) Jg[i][k].assign(NE * nq, 0.0);
  }
  auto call = [&](ldgs_eval_fn fn, int Q, const double* X, const int* ph, const double* nrm, int ncomp,
                  std::vector<double>& out) {
    out.assign((size_t)Q * ncomp, 0.0);
    if (fn) fn(Q, X, ph, nrm, out.data(), data.user);
  };
  for (int64_t e = 0; e < NE; ++e) {
    const ImpElemRule& R = H.rules[e];
    const int Q = (int)R.w.size();
    std::vector<double> B((size_t)Q * nq), f, fd;
    std::vector<int> ph(Q, L.phase[e]);
    imp_basis(H, L, e, Q, R.X.data(), -1, B.data());
    call(data.f, Q, R.X.data(), ph.data(), nullptr, 2, f);
    call(data.f_div, Q, R.X.data(), ph.data(), nullptr, 1, fd);
    for (int q = 0; q < Q; ++q)
      for (int a = 0; a < nq; ++a) {
        const double bw = R.w[q] * B[(size_t)q * nq + a];
        Pf[0][e * nq + a] += bw * f[2 * q];
        Pf[1][e * nq + a] += bw * f[2 * q + 1];
        Pfd[e * nq + a] += bw * fd[q];
      }
  }
  for (const ImpFace& F : H.faces) {
    if (F.kind == 0) continue;
    const int Q = (int)F.w.size();
    const int mi = F.minus, pl = F.plus;
    std::vector<double> Tm((size_t)Q * nq), Tp((size_t)Q * nq), mum(Q), mup(Q);
    std::vector<int> phm(Q, L.phase[mi]), php(Q, pl >= 0 ? L.phase[pl] : 0);
    imp_basis(H, L, mi, Q, F.X.data(), -1, Tm.data());
    eval_field(P.mu, 2, Q, F.X.data(), phm.data(), mum.data());
    if (pl >= 0) {
      imp_basis(H, L, pl, Q, F.X.data(), -1, Tp.data());
      eval_field(P.mu, 2, Q, F.X.data(), php.data(), mup.data());
    }
    auto addm = [&](std::vector<double>& v, int e, const std::vector<double>& T, int q, double c) {
      for (int a = 0; a < nq; ++a) v[e * nq + a] += c * T[(size_t)q * nq + a];
    };
    if (F.kind == 2) {
      std::vector<double> g;
      call(data.g_dirichlet, Q, F.X.data(), phm.data(), F.nrm.data(), 2, g);
      for (int q = 0; q < Q; ++q) {
        const double w = F.w[q], tau = Cb * p * mum[q] / h;
        double gn = 0.0;
        for (int i = 0; i < 2; ++i) {
          for (int k = 0; k < 2; ++k) addm(Jg[i][k], mi, Tm, q, w * g[2 * q + i] * F.nrm[2 * q + k]);
          addm(pen[i], mi, Tm, q, w * tau * g[2 * q + i]);
          gn += g[2 * q + i] * F.nrm[2 * q + i];
        }
        addm(Jgn, mi, Tm, q, w * gn);
      }
    } else {
      std::vector<double> g, hj;
      call(data.g_jump, Q, F.X.data(), phm.data(), F.nrm.data(), 2, g);
      call(data.h_jump, Q, F.X.data(), phm.data(), F.nrm.data(), 2, hj);
      for (int q = 0; q < Q; ++q) {
        const double w = F.w[q], lam = lam_of(mum[q], mup[q]);
        const double tau = Ci * p * std::min(mum[q], mup[q]) / h;
        double gn = 0.0;
        for (int i = 0; i < 2; ++i) {
          for (int k = 0; k < 2; ++k) {
            addm(Jg[i][k], mi, Tm, q, w * (1 - lam) * g[2 * q + i] * F.nrm[2 * q + k]);
            addm(Jg[i][k], pl, Tp, q, w * lam * g[2 * q + i] * F.nrm[2 * q + k]);
          }
          addm(Jh[i], mi, Tm, q, w * lam * hj[2 * q + i]);
          addm(Jh[i], pl, Tp, q, w * (1 - lam) * hj[2 * q + i]);
          addm(pen[i], mi, Tm, q, w * tau * g[2 * q + i]);
          addm(pen[i], pl, Tp, q, -w * tau * g[2 * q + i]);
          gn += g[2 * q + i] * F.nrm[2 * q + i];
        }
        addm(Jgn, mi, Tm, q, w * (1 - lam) * gn);
        addm(Jgn, pl, Tp, q, w * lam * gn);
      }
    }
  }
  // b_u,i = Pf_i + Jh_i + pen_i - sum_j G_j^T Mmu (Jg_ij + gamma Jg_ji); b_p = Pfd + Jgn
  const size_t bs = (size_t)nq * nq;
  auto tG0 = transpose_index(L.G[0]);
  auto tG1 = transpose_index(L.G[1]);
  const decltype(tG0)* tG[2] = {&tG0, &tG1};
  for (int64_t e = 0; e < NE; ++e)
    for (int a = 0; a < nq; ++a) {
      for (int i = 0; i < 2; ++i) b[e * nb + i * nq + a] = Pf[i][e * nq + a] + Jh[i][e * nq + a] + pen[i][e * nq + a];
      b[e * nb + 2 * nq + a] = Pfd[e * nq + a] + Jgn[e * nq + a];
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      // y = Mmu (Jg_ij + gamma Jg_ji) per element; then b_i -= G_j^T y
      std::vector<double> y(NE * nq, 0.0);
      for (int64_t e = 0; e < NE; ++e) {
        const double* Mm = L.Mmu.get(e, (int)e);
        for (int a = 0; a < nq; ++a) {
          double s = 0.0;
          for (int c = 0; c < nq; ++c) s += Mm[a * nq + c] * (Jg[i][j][e * nq + c] + gamma * Jg[j][i][e * nq + c]);
          y[e * nq + a] = s;
        }
      }
      for (int64_t e = 0; e < NE; ++e)
        for (auto [hrow, slot] : (*tG[j])[e]) {
          const double* Gb = L.G[j].val[hrow].data() + (size_t)slot * bs;   // G_j[h][e]
          for (int a = 0; a < nq; ++a) {
            double s = 0.0;
            for (int c = 0; c < nq; ++c) s += Gb[c * nq + a] * y[hrow * nq + c];
            b[e * nb + i * nq + a] -= s;
          }
        }
    }
}

}  // namespace ldgs
