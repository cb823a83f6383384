// Host setup of the LDG-Stokes hierarchy: basis tables, fine-grid operator
// data, operator coarsening (Algorithms 2 and 3 of the paper), element blocks
// and their factorised inverses, and host versions of the operator used to
// assemble the bottom matrix and the right-hand side.
//
// The fine-grid operator is built from closed-form 1D factors of the
// orthonormal Legendre basis (traces e0, e1 and the derivative matrix K);
// only the coefficient-weighted face and element masses use quadrature.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "host.hpp"

namespace ldgs {

// ---------------------------------------------------------------------------
// 1D basis
// ---------------------------------------------------------------------------
double Basis::leg(int mm, double xi) {
  double x = 2.0 * xi - 1.0;
  double p0 = 1.0, p1 = x;
  if (mm == 0) return 1.0;
  for (int k = 1; k < mm; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return std::sqrt(2.0 * mm + 1.0) * p1;
}

void Basis::gauss(int q, std::vector<double>& xs, std::vector<double>& ws) {
  // roots of the Legendre polynomial P_q by Newton's method, mapped to [0,1]
  xs.assign(q, 0.0);
  ws.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < q; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      double pq = (q == 0) ? 1.0 : p1;
      double pqm1 = (q == 1) ? 1.0 : p0;
      if (q == 1) { pq = z; pqm1 = 1.0; }
      dp = q * (z * pq - pqm1) / (z * z - 1.0);
      double dz = pq / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < q; ++k) {
      double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    double pq = (q == 1) ? z : p1, pqm1 = (q == 1) ? 1.0 : p0;
    dp = q * (z * pq - pqm1) / (z * z - 1.0);
    xs[q - 1 - i] = 0.5 * (z + 1.0);
    ws[q - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   // 2/((1-z^2)P'^2) halved for [0,1]
  }
}

void Basis::init(int deg) {
  p = deg;
  m = deg + 1;
  e0.assign(m, 0.0);
  e1.assign(m, 0.0);
  K.assign(m * m, 0.0);
  for (int a = 0; a < m; ++a) {
    e1[a] = std::sqrt(2.0 * a + 1.0);
    e0[a] = (a % 2 ? -1.0 : 1.0) * e1[a];
  }
  // int_0^1 l_c' l_r = 2 sqrt((2c+1)(2r+1)) when c > r and c + r is odd
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c)
      if (c > r && (c + r) % 2 == 1) K[r * m + c] = 2.0 * std::sqrt((2.0 * c + 1.0) * (2.0 * r + 1.0));
  std::vector<double> gx, gw;
  gauss(m + 1, gx, gw);
  for (int o = 0; o < 2; ++o) {
    P[o].assign(m * m, 0.0);
    for (int f = 0; f < m; ++f)
      for (int c = 0; c < m; ++c) {
        double s = 0.0;
        for (size_t q = 0; q < gx.size(); ++q) s += gw[q] * leg(f, gx[q]) * leg(c, 0.5 * (gx[q] + o));
        P[o][f * m + c] = s / std::sqrt(2.0);
      }
  }
}

Tab1D Basis::tab() const {
  Tab1D t;
  std::memset(&t, 0, sizeof(t));
  t.M = m;
  for (int i = 0; i < m * m; ++i) {
    t.K[i] = K[i];
    t.P[0][i] = P[0][i];
    t.P[1][i] = P[1][i];
  }
  for (int i = 0; i < m; ++i) {
    t.e0[i] = e0[i];
    t.e1[i] = e1[i];
  }
  return t;
}

void Geometry::set(int dim, int deg) {
  d = dim;
  p = deg;
  m = deg + 1;
  nq = 1;
  for (int j = 0; j < d; ++j) nq *= m;
  mt = nq / m;
  nb = (d + 1) * nq;
}

// ---------------------------------------------------------------------------
// tensor index helpers (axis 0 fastest)
// ---------------------------------------------------------------------------
static inline int ipow(int b, int e) {
  int v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}
static inline int digit(int a, int k, int m) { return (a / ipow(m, k)) % m; }
static inline int tang(int a, int k, int m) { return a % ipow(m, k) + ipow(m, k) * (a / ipow(m, k + 1)); }
static inline int compose(int t, int c, int k, int m) {
  return t % ipow(m, k) + ipow(m, k) * c + ipow(m, k + 1) * (t / ipow(m, k));
}

static inline void coords(int64_t E, int n, int d, int* c) {
  for (int j = 0; j < d; ++j) {
    c[j] = (int)(E % n);
    E /= n;
  }
}
static inline int64_t eindex(const int* c, int n, int d) {
  int64_t e = 0, s = 1;
  for (int j = 0; j < d; ++j) {
    e += c[j] * s;
    s *= n;
  }
  return e;
}

int64_t face_id(const Level& L, int d, int axis, const int* c, int f) {
  int64_t e = 0, s = 1;
  for (int j = 0; j < d; ++j) {
    int v = (j == axis) ? f : c[j];
    e += (int64_t)v * s;
    s *= (j == axis) ? L.faces[axis].nfk : L.n;
  }
  return e;
}

void face_elements(const Level& L, int d, int axis, int f, const int* c, int64_t* eL, int64_t* eR) {
  int cc[3] = {c[0], d > 1 ? c[1] : 0, d > 2 ? c[2] : 0};
  const bool per = L.faces[axis].nfk == L.n;
  *eL = -1;
  *eR = -1;
  if (f < L.n) {
    cc[axis] = f;
    *eR = eindex(cc, L.n, d);
  }
  if (f >= 1) {
    cc[axis] = f - 1;
    *eL = eindex(cc, L.n, d);
  } else if (per) {
    cc[axis] = L.n - 1;
    *eL = eindex(cc, L.n, d);
  }
}

// iterate the faces normal to `axis`: fn(face_id, f, c)
template <class F>
static void for_faces(const Level& L, int d, int axis, F fn) {
  const FaceSet& fs = L.faces[axis];
  for (int64_t id = 0; id < fs.count; ++id) {
    int c[3] = {0, 0, 0};
    int64_t r = id;
    int f = 0;
    for (int j = 0; j < d; ++j) {
      int ext = (j == axis) ? fs.nfk : L.n;
      int v = (int)(r % ext);
      r /= ext;
      if (j == axis) f = v;
      else c[j] = v;
    }
    fn(id, f, c);
  }
}

// trace of an element coefficient block along axis k with vector e -> mt values
static void trace(const double* u, int k, const double* e, int m, int mt, double* out) {
  for (int t = 0; t < mt; ++t) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += e[c] * u[compose(t, c, k, m)];
    out[t] = s;
  }
}
// out += scale * e (x)_k phi
static void expand_add(double* out, int k, const double* e, const double* phi, double scale, int m, int mt) {
  for (int t = 0; t < mt; ++t)
    for (int c = 0; c < m; ++c) out[compose(t, c, k, m)] += scale * e[c] * phi[t];
}

// ---------------------------------------------------------------------------
// host operator (face loops; used for the bottom matrix, the RHS and checks)
// ---------------------------------------------------------------------------
void host_grad(const Level& L, const Geometry& g, const Basis& B, int k, const double* u, double* out) {
  const int m = g.m, nq = g.nq, mt = g.mt;
  const double hinv = 1.0 / L.h;
  std::fill(out, out + L.NE * nq, 0.0);
  for (int64_t E = 0; E < L.NE; ++E) {
    const double* ue = u + E * nq;
    double* oe = out + E * nq;
    for (int a = 0; a < nq; ++a) {
      int ak = digit(a, k, m), t = tang(a, k, m);
      double s = 0.0;
      for (int b = 0; b < m; ++b) s += B.K[ak * m + b] * ue[compose(t, b, k, m)];
      oe[a] += hinv * s;
    }
  }
  std::vector<double> jl(mt), tr(mt);
  for_faces(L, g.d, k, [&](int64_t id, int f, const int* c) {
    unsigned char ty = L.faces[k].type[id];
    if (ty == F_NONE) return;
    int64_t eL, eR;
    face_elements(L, g.d, k, f, c, &eL, &eR);
    std::fill(jl.begin(), jl.end(), 0.0);
    if (eR >= 0) {
      trace(u + eR * nq, k, B.e0.data(), m, mt, tr.data());
      for (int t = 0; t < mt; ++t) jl[t] += tr[t];
    }
    if (eL >= 0) {
      trace(u + eL * nq, k, B.e1.data(), m, mt, tr.data());
      for (int t = 0; t < mt; ++t) jl[t] -= tr[t];
    }
    double wL = L.faces[k].w[2 * id], wR = L.faces[k].w[2 * id + 1];
    if (eR >= 0 && wR != 0.0) expand_add(out + eR * nq, k, B.e0.data(), jl.data(), hinv * wR, m, mt);
    if (eL >= 0 && wL != 0.0) expand_add(out + eL * nq, k, B.e1.data(), jl.data(), hinv * wL, m, mt);
  });
}

void host_gradT(const Level& L, const Geometry& g, const Basis& B, int k, const double* s, double* out) {
  const int m = g.m, nq = g.nq, mt = g.mt;
  const double hinv = 1.0 / L.h;
  std::fill(out, out + L.NE * nq, 0.0);
  for (int64_t E = 0; E < L.NE; ++E) {
    const double* se = s + E * nq;
    double* oe = out + E * nq;
    for (int a = 0; a < nq; ++a) {
      int ak = digit(a, k, m), t = tang(a, k, m);
      double v = 0.0;
      for (int b = 0; b < m; ++b) v += B.K[b * m + ak] * se[compose(t, b, k, m)];
      oe[a] += hinv * v;
    }
  }
  std::vector<double> phi(mt), tr(mt);
  for_faces(L, g.d, k, [&](int64_t id, int f, const int* c) {
    unsigned char ty = L.faces[k].type[id];
    if (ty == F_NONE) return;
    int64_t eL, eR;
    face_elements(L, g.d, k, f, c, &eL, &eR);
    double wL = L.faces[k].w[2 * id], wR = L.faces[k].w[2 * id + 1];
    std::fill(phi.begin(), phi.end(), 0.0);
    if (eR >= 0) {
      trace(s + eR * nq, k, B.e0.data(), m, mt, tr.data());
      for (int t = 0; t < mt; ++t) phi[t] += hinv * wR * tr[t];
    }
    if (eL >= 0) {
      trace(s + eL * nq, k, B.e1.data(), m, mt, tr.data());
      for (int t = 0; t < mt; ++t) phi[t] += hinv * wL * tr[t];
    }
    if (eR >= 0) expand_add(out + eR * nq, k, B.e0.data(), phi.data(), 1.0, m, mt);
    if (eL >= 0) expand_add(out + eL * nq, k, B.e1.data(), phi.data(), -1.0, m, mt);
  });
}

void host_mmu(const Level& L, const Geometry& g, const double* u, double* out) {
  const int nq = g.nq;
  for (int64_t E = 0; E < L.NE; ++E) {
    if (L.mu_is_const) {
      for (int a = 0; a < nq; ++a) out[E * nq + a] = L.mu_c * u[E * nq + a];
    } else {
      const double* M = L.mmu.data() + E * nq * nq;
      for (int a = 0; a < nq; ++a) {
        double s = 0.0;
        for (int b = 0; b < nq; ++b) s += M[a * nq + b] * u[E * nq + b];
        out[E * nq + a] = s;
      }
    }
  }
}

// penalty terms on one scalar field: `velocity` selects Dirichlet and
// interphase faces (E-tilde), otherwise intraphase faces (E)
static void host_penalty(const Level& L, const Geometry& g, const Basis& B, bool velocity, const double* u,
                         double* out) {
  const int m = g.m, nq = g.nq, mt = g.mt;
  const double hinv = 1.0 / L.h;
  std::vector<double> j(mt), tr(mt), v(mt);
  for (int k = 0; k < g.d; ++k) {
    for_faces(L, g.d, k, [&](int64_t id, int f, const int* c) {
      unsigned char ty = L.faces[k].type[id];
      bool use = velocity ? (ty == F_INTER || ty == F_DIR_LO || ty == F_DIR_HI) : (ty == F_INTRA);
      if (!use) return;
      int64_t eL, eR;
      face_elements(L, g.d, k, f, c, &eL, &eR);
      std::fill(j.begin(), j.end(), 0.0);
      if (eL >= 0 && ty != F_DIR_LO) {
        trace(u + eL * nq, k, B.e1.data(), m, mt, tr.data());
        for (int t = 0; t < mt; ++t) j[t] += tr[t];
      }
      if (eR >= 0 && ty != F_DIR_HI) {
        trace(u + eR * nq, k, B.e0.data(), m, mt, tr.data());
        // jump u_L|hi - u_R|lo; for a low Dirichlet face only the trace counts
        for (int t = 0; t < mt; ++t) j[t] += (ty == F_DIR_LO) ? tr[t] : -tr[t];
      }
      const double* T = L.faces[k].T.data() + id * mt * mt;
      for (int t = 0; t < mt; ++t) {
        double s = 0.0;
        for (int q = 0; q < mt; ++q) s += T[t * mt + q] * j[q];
        v[t] = hinv * s;
      }
      if (ty == F_DIR_LO) expand_add(out + eR * nq, k, B.e0.data(), v.data(), 1.0, m, mt);
      else if (ty == F_DIR_HI) expand_add(out + eL * nq, k, B.e1.data(), v.data(), 1.0, m, mt);
      else {
        expand_add(out + eL * nq, k, B.e1.data(), v.data(), 1.0, m, mt);
        expand_add(out + eR * nq, k, B.e0.data(), v.data(), -1.0, m, mt);
      }
    });
  }
}

void host_apply(const Level& L, const Geometry& g, const Basis& B, int gamma, const double* x, double* y) {
  const int d = g.d, nq = g.nq, nb = g.nb;
  const int64_t S = L.NE * nq;
  // gather fields (unscaled values; scaling applied around)
  std::vector<double> xs(L.NE * nb);
  for (int64_t E = 0; E < L.NE; ++E)
    for (int i = 0; i < nb; ++i) {
      double v = x[E * nb + i];
      if (!L.dscale.empty()) v *= L.dscale[2 * E + (i >= d * nq ? 1 : 0)];
      xs[E * nb + i] = v;
    }
  std::vector<std::vector<double>> u(d + 1, std::vector<double>(S));
  for (int64_t E = 0; E < L.NE; ++E)
    for (int f = 0; f <= d; ++f)
      for (int a = 0; a < nq; ++a) u[f][E * nq + a] = xs[E * nb + f * nq + a];
  std::vector<std::vector<double>> gr(d * d, std::vector<double>(S));
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) host_grad(L, g, B, k, u[i].data(), gr[i * d + k].data());
  std::vector<std::vector<double>> out(d + 1, std::vector<double>(S, 0.0));
  std::vector<double> tau(S), s(S), tmp(S);
  for (int i = 0; i < d; ++i) {
    for (int k = 0; k < d; ++k) {
      for (int64_t q = 0; q < S; ++q) tau[q] = gr[i * d + k][q] + gamma * gr[k * d + i][q];
      host_mmu(L, g, tau.data(), s.data());
      host_gradT(L, g, B, k, s.data(), tmp.data());
      for (int64_t q = 0; q < S; ++q) out[i][q] += tmp[q];
    }
    host_penalty(L, g, B, true, u[i].data(), out[i].data());
    for (int64_t q = 0; q < S; ++q) out[i][q] += L.rho_delta * u[i][q];
    host_gradT(L, g, B, i, u[d].data(), tmp.data());
    for (int64_t q = 0; q < S; ++q) out[i][q] -= tmp[q];
  }
  for (int i = 0; i < d; ++i)
    for (int64_t q = 0; q < S; ++q) out[d][q] -= gr[i * d + i][q];
  std::vector<double> pe(S, 0.0);
  host_penalty(L, g, B, false, u[d].data(), pe.data());
  for (int64_t q = 0; q < S; ++q) out[d][q] -= pe[q];
  for (int64_t E = 0; E < L.NE; ++E)
    for (int f = 0; f <= d; ++f)
      for (int a = 0; a < nq; ++a) {
        double v = out[f][E * nq + a];
        if (!L.dscale.empty()) v *= L.dscale[2 * E + (f == d ? 1 : 0)];
        y[E * nb + f * nq + a] = v;
      }
}

// ---------------------------------------------------------------------------
// diagonal element block A_EE (row-major nb x nb), scaled when dscale is set
// ---------------------------------------------------------------------------
// dense (p+1)^d matrix of a 1D m x m matrix acting on axis k
static void kron_axis(const double* mat1d, int k, int m, int nq, double* out) {
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b) {
      out[a * nq + b] = (tang(a, k, m) == tang(b, k, m)) ? mat1d[digit(a, k, m) * m + digit(b, k, m)] : 0.0;
    }
}
// dense matrix (v w^T)_k (x) T (T on the tangential axes)
static void face_block(const double* v, const double* w, const double* T, int k, int m, int nq, int mt, double scale,
                       double* out) {
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b)
      out[a * nq + b] += scale * v[digit(a, k, m)] * w[digit(b, k, m)] * T[tang(a, k, m) * mt + tang(b, k, m)];
}

static void matmul_tn(const double* A, const double* B, const double* C, int n, double scale, double* out) {
  // out += scale * A^T B C   (n x n row-major)
  std::vector<double> tmp(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double aki = A[k * n + i];
      if (aki == 0.0) continue;
      for (int j = 0; j < n; ++j) tmp[i * n + j] += aki * B[k * n + j];
    }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double t = tmp[i * n + k];
      if (t == 0.0) continue;
      for (int j = 0; j < n; ++j) out[i * n + j] += scale * t * C[k * n + j];
    }
}

void host_diag_block(const Level& L, const Geometry& g, const Basis& B, int gamma, int64_t E, double* A) {
  const int d = g.d, m = g.m, nq = g.nq, mt = g.mt, nb = g.nb;
  const double hinv = 1.0 / L.h;
  std::fill(A, A + nb * nb, 0.0);
  int c[3] = {0, 0, 0};
  coords(E, L.n, d, c);
  std::vector<double> Ident(nq * nq, 0.0);
  for (int a = 0; a < nq; ++a) Ident[a * nq + a] = 1.0;
  auto mmu_of = [&](int64_t e) -> const double* {
    if (L.mu_is_const) return nullptr;
    return L.mmu.data() + e * nq * nq;
  };
  std::vector<double> Mc(nq * nq);
  auto mat_of = [&](int64_t e) -> const double* {
    const double* p = mmu_of(e);
    if (p) return p;
    for (int i = 0; i < nq * nq; ++i) Mc[i] = L.mu_c * Ident[i];
    return Mc.data();
  };
  // G_k(E,E), G_k(E+e_k,E), G_k(E-e_k,E) and the faces
  std::vector<std::vector<double>> Gd(d, std::vector<double>(nq * nq)), Gr(d), Gl(d);
  std::vector<int64_t> nR(d, -1), nL(d, -1);
  std::vector<double> mat1(m * m);
  int64_t flo[3], fhi[3];
  for (int k = 0; k < d; ++k) {
    const FaceSet& fs = L.faces[k];
    const bool per = fs.nfk == L.n;
    flo[k] = face_id(L, d, k, c, c[k]);
    fhi[k] = face_id(L, d, k, c, per ? (c[k] + 1) % L.n : c[k] + 1);
    double wR_lo = fs.w[2 * flo[k] + 1], wL_lo = fs.w[2 * flo[k]];
    double wL_hi = fs.w[2 * fhi[k]], wR_hi = fs.w[2 * fhi[k] + 1];
    unsigned char tlo = fs.type[flo[k]], thi = fs.type[fhi[k]];
    if (tlo == F_NONE) wR_lo = wL_lo = 0.0;
    if (thi == F_NONE) wR_hi = wL_hi = 0.0;
    for (int r = 0; r < m; ++r)
      for (int q = 0; q < m; ++q)
        mat1[r * m + q] = hinv * (B.K[r * m + q] + wR_lo * B.e0[r] * B.e0[q] - wL_hi * B.e1[r] * B.e1[q]);
    kron_axis(mat1.data(), k, m, nq, Gd[k].data());
    if (thi == F_INTRA || thi == F_INTER) {
      int64_t eL, eR;
      face_elements(L, d, k, (int)(per ? (c[k] + 1) % L.n : c[k] + 1), c, &eL, &eR);
      nR[k] = eR;
      Gr[k].assign(nq * nq, 0.0);
      for (int r = 0; r < m; ++r)
        for (int q = 0; q < m; ++q) mat1[r * m + q] = -hinv * wR_hi * B.e0[r] * B.e1[q];
      kron_axis(mat1.data(), k, m, nq, Gr[k].data());
    }
    if (tlo == F_INTRA || tlo == F_INTER) {
      int64_t eL, eR;
      face_elements(L, d, k, c[k], c, &eL, &eR);
      nL[k] = eL;
      Gl[k].assign(nq * nq, 0.0);
      for (int r = 0; r < m; ++r)
        for (int q = 0; q < m; ++q) mat1[r * m + q] = hinv * wL_lo * B.e1[r] * B.e0[q];
      kron_axis(mat1.data(), k, m, nq, Gl[k].data());
    }
  }
  // velocity-velocity blocks
  std::vector<double> lap(nq * nq, 0.0), blk(nq * nq);
  for (int k = 0; k < d; ++k) {
    matmul_tn(Gd[k].data(), mat_of(E), Gd[k].data(), nq, 1.0, lap.data());
    if (nR[k] >= 0) matmul_tn(Gr[k].data(), mat_of(nR[k]), Gr[k].data(), nq, 1.0, lap.data());
    if (nL[k] >= 0) matmul_tn(Gl[k].data(), mat_of(nL[k]), Gl[k].data(), nq, 1.0, lap.data());
  }
  // velocity penalty (Dirichlet / interphase faces of E) and rho/delta
  std::vector<double> pen(nq * nq, 0.0), ppen(nq * nq, 0.0);
  for (int k = 0; k < d; ++k) {
    const FaceSet& fs = L.faces[k];
    unsigned char tlo = fs.type[flo[k]], thi = fs.type[fhi[k]];
    const double* Tlo = fs.T.data() + flo[k] * mt * mt;
    const double* Thi = fs.T.data() + fhi[k] * mt * mt;
    if (tlo == F_DIR_LO || tlo == F_INTER) face_block(B.e0.data(), B.e0.data(), Tlo, k, m, nq, mt, hinv, pen.data());
    if (thi == F_DIR_HI || thi == F_INTER) face_block(B.e1.data(), B.e1.data(), Thi, k, m, nq, mt, hinv, pen.data());
    if (tlo == F_INTRA) face_block(B.e0.data(), B.e0.data(), Tlo, k, m, nq, mt, hinv, ppen.data());
    if (thi == F_INTRA) face_block(B.e1.data(), B.e1.data(), Thi, k, m, nq, mt, hinv, ppen.data());
  }
  for (int i = 0; i < d; ++i)
    for (int ip = 0; ip < d; ++ip) {
      std::fill(blk.begin(), blk.end(), 0.0);
      if (i == ip) {
        for (int q = 0; q < nq * nq; ++q) blk[q] = lap[q] + pen[q] + L.rho_delta * Ident[q];
        if (gamma) {
          matmul_tn(Gd[i].data(), mat_of(E), Gd[i].data(), nq, 1.0, blk.data());
          if (nR[i] >= 0) matmul_tn(Gr[i].data(), mat_of(nR[i]), Gr[i].data(), nq, 1.0, blk.data());
          if (nL[i] >= 0) matmul_tn(Gl[i].data(), mat_of(nL[i]), Gl[i].data(), nq, 1.0, blk.data());
        }
      } else if (gamma) {
        // gamma G_{i'}(E,E)^T M_E G_i(E,E)
        matmul_tn(Gd[ip].data(), mat_of(E), Gd[i].data(), nq, 1.0, blk.data());
      }
      for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b) A[(i * nq + a) * nb + ip * nq + b] = blk[a * nq + b];
    }
  // velocity-pressure and pressure-velocity: -G_i^T, -G_i
  for (int i = 0; i < d; ++i)
    for (int a = 0; a < nq; ++a)
      for (int b = 0; b < nq; ++b) {
        A[(i * nq + a) * nb + d * nq + b] = -Gd[i][b * nq + a];
        A[(d * nq + a) * nb + i * nq + b] = -Gd[i][a * nq + b];
      }
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b) A[(d * nq + a) * nb + d * nq + b] = -ppen[a * nq + b];
  if (!L.dscale.empty()) {
    for (int r = 0; r < nb; ++r)
      for (int q = 0; q < nb; ++q)
        A[r * nb + q] *= L.dscale[2 * E + (r >= d * nq ? 1 : 0)] * L.dscale[2 * E + (q >= d * nq ? 1 : 0)];
  }
}

// ---------------------------------------------------------------------------
// explicit inverse of the Jacobi-equilibrated LU with partial pivoting
// ---------------------------------------------------------------------------
bool block_inverse(int n, const double* A, double* inv, double rcond_min) {
  std::vector<double> Dg(n), S(n * n), X(n * n, 0.0);
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) {
    double a = std::fabs(A[i * n + i]);
    if (!(a > 0.0)) return false;
    Dg[i] = 1.0 / std::sqrt(a);
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = Dg[i] * A[i * n + j] * Dg[j];
  double norm1 = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(S[i * n + j]);
    norm1 = std::max(norm1, s);
  }
  // LU with partial pivoting, in place
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(S[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(S[i * n + k]) > best) { best = std::fabs(S[i * n + k]); p = i; }
    if (best == 0.0) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(S[k * n + j], S[p * n + j]);
    double dinv = 1.0 / S[k * n + k];
    for (int i = k + 1; i < n; ++i) {
      double l = S[i * n + k] * dinv;
      S[i * n + k] = l;
      if (l != 0.0)
        for (int j = k + 1; j < n; ++j) S[i * n + j] -= l * S[k * n + j];
    }
  }
  // solve for the identity: P S = L U  =>  S^{-1} = U^{-1} L^{-1} P
  for (int col = 0; col < n; ++col) {
    std::vector<double> b(n, 0.0);
    b[col] = 1.0;
    for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i) {
      double s = b[i];
      for (int j = 0; j < i; ++j) s -= S[i * n + j] * b[j];
      b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = b[i];
      for (int j = i + 1; j < n; ++j) s -= S[i * n + j] * b[j];
      b[i] = s / S[i * n + i];
    }
    for (int i = 0; i < n; ++i) X[i * n + col] = b[i];
  }
  double ninv = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(X[i * n + j]);
    ninv = std::max(ninv, s);
  }
  if (!(1.0 / (norm1 * ninv) >= rcond_min)) return false;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = Dg[i] * X[i * n + j] * Dg[j];
  return true;
}

}  // namespace ldgs
