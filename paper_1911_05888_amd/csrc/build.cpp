// Construction of the level hierarchy on the host: fine-grid coefficient data
// (mu-weighted masses, penalty face matrices, lifting weights), operator
// coarsening down to the bottom grid (Algorithms 2 and 3 of the paper), the
// diagonal (alpha, beta) scaling and the multicolour ordering.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "build.hpp"

namespace ldgs {

static inline int ipow(int b, int e) {
  int v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}
static inline int digit(int a, int k, int m) { return (a / ipow(m, k)) % m; }

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

// ---------------------------------------------------------------------------
// coefficient fields
// ---------------------------------------------------------------------------
void eval_field(const ldgs_field& f, int d, int64_t n, const double* x, const int* phase, double* out) {
  switch (f.kind) {
    case LDGS_FIELD_CONST:
      for (int64_t i = 0; i < n; ++i) out[i] = f.params[0];
      break;
    case LDGS_FIELD_SINSIN:
      for (int64_t i = 0; i < n; ++i) {
        double s = 1.0;
        for (int j = 0; j < d; ++j) s *= std::sin(2.0 * M_PI * f.params[2] * x[i * d + j]);
        out[i] = f.params[0] + f.params[1] * s;
      }
      break;
    case LDGS_FIELD_LOGNORMAL_RFF: {
      int64_t K = f.nparams / (d + 1);
      const double* kv = f.params;
      const double* ph = f.params + K * d;
      const double sc = std::sqrt(2.0 / (double)K);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        double g = 0.0;
        for (int64_t q = 0; q < K; ++q) {
          double a = ph[q];
          for (int j = 0; j < d; ++j) a += kv[q * d + j] * x[i * d + j];
          g += std::cos(a);
        }
        out[i] = std::pow(10.0, sc * g);
      }
      break;
    }
    case LDGS_FIELD_PHASE_CONST:
      for (int64_t i = 0; i < n; ++i) out[i] = f.params[phase[i] - 1];
      break;
    case LDGS_FIELD_CALLBACK:
      f.fn(n, x, phase, nullptr, out, f.user);
      break;
    default:
      throw std::invalid_argument("unknown field kind");
  }
}

static bool field_is_const(const ldgs_field& f) { return f.kind == LDGS_FIELD_CONST; }

// The log-normal field 10^g, g = sqrt(2/K) sum_m cos(k_m . x + phi_m), at the
// points x = h (c + xi_q) of a tensor point set: anchors c (integer grid
// coordinates of an element or a face, from anchor(a, c)) times local
// offsets xi_q.  With e^{i k_m . x} = prod_j e^{i k_mj h c_j} e^{i k_m . h xi_q}
// the cosines factor into per-axis tables and one table per offset, so a
// point costs K multiply-adds instead of K cosines:
//   g(a, q) = sqrt(2/K) sum_m Re(z_m(a) w_m(q)),  z_m(a) = prod_j T_j[c_j][m],
//   w_m(q) = e^{i (k_m . h xi_q + phi_m)}.
// out[a * nq + q] = 10^g.  cmax: largest grid coordinate (n for faces).
template <class Anchor>
static void rff_tensor_points(const ldgs_field& f, int d, double h, int cmax, int64_t nanchor, Anchor anchor,
                              int nq, const double* xi, double* out) {
  const int64_t K = f.nparams / (d + 1);
  const double* kv = f.params;
  const double* ph = f.params + K * d;
  const double sc = std::sqrt(2.0 / (double)K);
  const int nc = cmax + 1;
  std::vector<double> Tr((size_t)d * nc * K), Ti((size_t)d * nc * K);
  for (int j = 0; j < d; ++j)
    for (int c = 0; c < nc; ++c)
      for (int64_t m = 0; m < K; ++m) {
        const double a = kv[m * d + j] * h * c;
        Tr[((size_t)j * nc + c) * K + m] = std::cos(a);
        Ti[((size_t)j * nc + c) * K + m] = std::sin(a);
      }
  std::vector<double> Wr((size_t)nq * K), Wi((size_t)nq * K);
  for (int q = 0; q < nq; ++q)
    for (int64_t m = 0; m < K; ++m) {
      double a = ph[m];
      for (int j = 0; j < d; ++j) a += kv[m * d + j] * h * xi[q * d + j];
      Wr[(size_t)q * K + m] = std::cos(a);
      Wi[(size_t)q * K + m] = std::sin(a);
    }
#pragma omp parallel
  {
    std::vector<double> zr(K), zi(K);
#pragma omp for schedule(static)
    for (int64_t a = 0; a < nanchor; ++a) {
      int c[3] = {0, 0, 0};
      anchor(a, c);
      for (int64_t m = 0; m < K; ++m) {
        double r = Tr[(size_t)c[0] * K + m], i = Ti[(size_t)c[0] * K + m];
        for (int j = 1; j < d; ++j) {
          const double tr = Tr[((size_t)j * nc + c[j]) * K + m], ti = Ti[((size_t)j * nc + c[j]) * K + m];
          const double nr = r * tr - i * ti;
          i = r * ti + i * tr;
          r = nr;
        }
        zr[m] = r;
        zi[m] = i;
      }
      for (int q = 0; q < nq; ++q) {
        const double* wr = &Wr[(size_t)q * K];
        const double* wi = &Wi[(size_t)q * K];
        double g = 0.0;
#pragma omp simd reduction(+ : g)
        for (int64_t m = 0; m < K; ++m) g += zr[m] * wr[m] - zi[m] * wi[m];
        out[(size_t)a * nq + q] = std::pow(10.0, sc * g);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// fine grid
// ---------------------------------------------------------------------------
static int phase_of_centre(const ldgs_problem& P, const double* xc) {
  if (P.levelset_kind != LDGS_LEVELSET_BOX) return 1;
  for (int j = 0; j < P.dim; ++j)
    if (!(xc[j] > P.levelset_params[0] && xc[j] < P.levelset_params[1])) return 2;
  return 1;
}

static void tangential_basis(const Basis& B, int d, int q, std::vector<double>& pts, std::vector<double>& wts,
                             std::vector<double>& Bt) {
  // (d-1)-dimensional tensor Gauss rule with the tangential basis values
  std::vector<double> gx, gw;
  Basis::gauss(q, gx, gw);
  const int m = B.m;
  int nt = ipow(q, d - 1), mt = ipow(m, d - 1);
  pts.assign(nt * std::max(d - 1, 1), 0.0);
  wts.assign(nt, 1.0);
  Bt.assign(nt * mt, 1.0);
  for (int i = 0; i < nt; ++i) {
    for (int j = 0; j < d - 1; ++j) {
      int qi = (i / ipow(q, j)) % q;
      pts[i * (d - 1) + j] = gx[qi];
      wts[i] *= gw[qi];
    }
    for (int t = 0; t < mt; ++t) {
      double v = 1.0;
      for (int j = 0; j < d - 1; ++j) v *= Basis::leg(digit(t, j, m), pts[i * (d - 1) + j]);
      Bt[i * mt + t] = v;
    }
  }
}

void build_fine_level(const ldgs_problem& P, const Geometry& g, const Basis& B, Level& L) {
  const int d = g.d, m = g.m, nq = g.nq, mt = g.mt, n = P.n;
  const int p = P.degree;
  L.n = n;
  L.h = 1.0 / n;
  L.NE = 1;
  for (int j = 0; j < d; ++j) L.NE *= n;
  const double h = L.h;
  // phases
  L.chi.assign(L.NE, 1);
  for (int64_t E = 0; E < L.NE; ++E) {
    int c[3];
    coords(E, n, d, c);
    double xc[3];
    for (int j = 0; j < d; ++j) xc[j] = (c[j] + 0.5) * h;
    L.chi[E] = phase_of_centre(P, xc);
  }
  // mu-weighted element masses, q = p + 2 Gauss points per axis
  const int q = p + 2;
  std::vector<double> gx, gw;
  Basis::gauss(q, gx, gw);
  const int nv = ipow(q, d);
  std::vector<double> Bv(nv * nq), wv(nv), xi(nv * d);
  for (int i = 0; i < nv; ++i) {
    wv[i] = 1.0;
    for (int j = 0; j < d; ++j) {
      int qi = (i / ipow(q, j)) % q;
      xi[i * d + j] = gx[qi];
      wv[i] *= gw[qi];
    }
    for (int a = 0; a < nq; ++a) {
      double v = 1.0;
      for (int j = 0; j < d; ++j) v *= Basis::leg(digit(a, j, m), xi[i * d + j]);
      Bv[i * nq + a] = v;
    }
  }
  if (field_is_const(P.mu)) {
    L.mu_is_const = true;
    L.mu_c = P.mu.params[0];
  } else {
    L.mu_is_const = false;
    L.mmu.assign((size_t)L.NE * nq * nq, 0.0);
    std::vector<double> mu((size_t)L.NE * nv);
    if (P.mu.kind == LDGS_FIELD_LOGNORMAL_RFF) {
      rff_tensor_points(P.mu, d, h, n, L.NE, [&](int64_t E, int* c) { coords(E, n, d, c); }, nv, xi.data(), mu.data());
    } else {
      std::vector<double> X((size_t)L.NE * nv * d);
      std::vector<int> ph((size_t)L.NE * nv);
      for (int64_t E = 0; E < L.NE; ++E) {
        int c[3];
        coords(E, n, d, c);
        for (int i = 0; i < nv; ++i) {
          for (int j = 0; j < d; ++j) X[((size_t)E * nv + i) * d + j] = (c[j] + xi[i * d + j]) * h;
          ph[(size_t)E * nv + i] = L.chi[E];
        }
      }
      eval_field(P.mu, d, L.NE * nv, X.data(), ph.data(), mu.data());
    }
#pragma omp parallel for schedule(static)
    for (int64_t E = 0; E < L.NE; ++E) {
      double* M = L.mmu.data() + (size_t)E * nq * nq;
      for (int i = 0; i < nv; ++i) {
        double wm = wv[i] * mu[(size_t)E * nv + i];
        const double* bi = &Bv[i * nq];
        for (int a = 0; a < nq; ++a)
          for (int b = 0; b < nq; ++b) M[a * nq + b] += wm * bi[a] * bi[b];
      }
    }
  }
  // faces
  std::vector<double> tp, tw, Bt;
  tangential_basis(B, d, q, tp, tw, Bt);
  const int nt = (int)tw.size();
  const bool unsteady = P.delta > 0.0;
  const double rho_c = unsteady ? P.rho.params[0] : 0.0;
  L.rho_delta = unsteady ? rho_c / P.delta : 0.0;
  for (int k = 0; k < d; ++k) {
    FaceSet& fs = L.faces[k];
    const bool per = P.bc[k] == LDGS_PERIODIC;
    fs.nfk = per ? n : n + 1;
    fs.count = fs.nfk;
    for (int j = 0; j < d; ++j)
      if (j != k) fs.count *= n;
    fs.type.assign(fs.count, F_NONE);
    fs.w.assign(2 * fs.count, 0.0);
    fs.T.assign((size_t)fs.count * mt * mt, 0.0);
    if (unsteady) {
      fs.Tmu.assign((size_t)fs.count * mt * mt, 0.0);
      fs.Trho.assign((size_t)fs.count * mt * mt, 0.0);
    }
    // all face quadrature points of this axis, with the phase of each side
    auto face_coords = [&](int64_t id, int* c) {
      int64_t r = id;
      for (int j = 0; j < d; ++j) {
        const int ext = (j == k) ? fs.nfk : n;
        c[j] = (int)(r % ext);
        r /= ext;
      }
    };
    std::vector<int64_t> EL(fs.count), ER(fs.count);
    for (int64_t id = 0; id < fs.count; ++id) {
      int c[3] = {0, 0, 0};
      face_coords(id, c);
      const int f = c[k];
      face_elements(L, d, k, f, c, &EL[id], &ER[id]);
    }
    std::vector<double> muL((size_t)fs.count * nt), muR;
    if (P.mu.kind == LDGS_FIELD_LOGNORMAL_RFF) {
      // one value per point (the field does not depend on the phase); face
      // points have offset 0 along the normal axis
      std::vector<double> xf((size_t)nt * d, 0.0);
      for (int i = 0; i < nt; ++i) {
        int jj = 0;
        for (int j = 0; j < d; ++j) xf[(size_t)i * d + j] = (j == k) ? 0.0 : tp[i * (d - 1) + jj++];
      }
      rff_tensor_points(P.mu, d, h, n, fs.count, face_coords, nt, xf.data(), muL.data());
      muR = muL;
    } else {
      std::vector<double> X((size_t)fs.count * nt * d);
      std::vector<int> phL((size_t)fs.count * nt), phR((size_t)fs.count * nt);
      for (int64_t id = 0; id < fs.count; ++id) {
        int c[3] = {0, 0, 0};
        face_coords(id, c);
        const int f = c[k];
        for (int i = 0; i < nt; ++i) {
          int jj = 0;
          for (int j = 0; j < d; ++j) {
            double v;
            if (j == k) v = f * h;
            else v = (c[j] + tp[i * (d - 1) + jj++]) * h;
            X[((size_t)id * nt + i) * d + j] = v;
          }
          phL[(size_t)id * nt + i] = EL[id] >= 0 ? L.chi[EL[id]] : L.chi[ER[id]];
          phR[(size_t)id * nt + i] = ER[id] >= 0 ? L.chi[ER[id]] : L.chi[EL[id]];
        }
      }
      muR.resize((size_t)fs.count * nt);
      eval_field(P.mu, d, fs.count * nt, X.data(), phL.data(), muL.data());
      eval_field(P.mu, d, fs.count * nt, X.data(), phR.data(), muR.data());
    }
    const double tb = P.tau_u_bdry_C * p / h;
    const double ti = P.tau_u_inter_C * p / h;
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < fs.count; ++id) {
      std::vector<double> tau(nt), tmu(nt), trho(nt);
      unsigned char ty;
      double wL = 0.0, wR = 0.0;
      if ((EL[id] < 0 || ER[id] < 0) && P.bc[k] == LDGS_STRESS) {
        // stress wall: u-hat = u- (no lift), sigma-hat = h n (data only), no
        // velocity or pressure penalty: no operator terms
        ty = F_NONE;
        for (int i = 0; i < nt; ++i) tau[i] = 0.0;
      } else if (EL[id] < 0) {
        ty = F_DIR_LO;
        wR = 1.0;
        for (int i = 0; i < nt; ++i) tau[i] = tb * muR[(size_t)id * nt + i];
      } else if (ER[id] < 0) {
        ty = F_DIR_HI;
        wL = 1.0;
        for (int i = 0; i < nt; ++i) tau[i] = tb * muL[(size_t)id * nt + i];
      } else if (L.chi[EL[id]] != L.chi[ER[id]]) {
        ty = F_INTER;
        // minus side = lower phase index; lambda of eq. (viscosityupwind)
        const bool minusL = L.chi[EL[id]] < L.chi[ER[id]];
        double mum = minusL ? muL[(size_t)id * nt] : muR[(size_t)id * nt];
        double mup = minusL ? muR[(size_t)id * nt] : muL[(size_t)id * nt];
        double lam = (mum < mup) ? 0.0 : (mum > mup ? 1.0 : 0.5);
        if (minusL) { wL = 1.0 - lam; wR = lam; }
        else { wL = lam; wR = 1.0 - lam; }
        for (int i = 0; i < nt; ++i)
          tau[i] = ti * std::min(muL[(size_t)id * nt + i], muR[(size_t)id * nt + i]);
      } else {
        ty = F_INTRA;
        wR = 1.0;
        for (int i = 0; i < nt; ++i) {
          double mu = muL[(size_t)id * nt + i];
          tmu[i] = P.tau * h / mu;
          if (unsteady) {
            trho[i] = P.tau0 * P.delta / (h * rho_c);
            tau[i] = 1.0 / (h * rho_c / (P.tau0 * P.delta) + mu / (P.tau * h));
          } else {
            tau[i] = tmu[i];
          }
        }
      }
      fs.type[id] = ty;
      fs.w[2 * id] = wL;
      fs.w[2 * id + 1] = wR;
      double* T = fs.T.data() + (size_t)id * mt * mt;
      for (int i = 0; i < nt; ++i)
        for (int a = 0; a < mt; ++a)
          for (int b = 0; b < mt; ++b) T[a * mt + b] += tw[i] * tau[i] * Bt[i * mt + a] * Bt[i * mt + b];
      if (unsteady && ty == F_INTRA) {
        double* Tm = fs.Tmu.data() + (size_t)id * mt * mt;
        double* Tr = fs.Trho.data() + (size_t)id * mt * mt;
        for (int i = 0; i < nt; ++i)
          for (int a = 0; a < mt; ++a)
            for (int b = 0; b < mt; ++b) {
              Tm[a * mt + b] += tw[i] * tmu[i] * Bt[i * mt + a] * Bt[i * mt + b];
              Tr[a * mt + b] += tw[i] * trho[i] * Bt[i * mt + a] * Bt[i * mt + b];
            }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// coarsening
// ---------------------------------------------------------------------------
// dense injection block of child offset bits o over the axes in `axes`
static void injection_dense(const Basis& B, int o, const int* axes, int na, std::vector<double>& Pm) {
  const int m = B.m;
  int sz = ipow(m, na);
  Pm.assign(sz * sz, 0.0);
  for (int af = 0; af < sz; ++af)
    for (int ac = 0; ac < sz; ++ac) {
      double v = 1.0;
      for (int j = 0; j < na; ++j) {
        int bit = (o >> axes[j]) & 1;
        v *= B.P[bit][digit(af, j, m) * m + digit(ac, j, m)];
      }
      Pm[af * sz + ac] = v;
    }
}

// out += P^T A P (all sz x sz)
static void ptap_add(const std::vector<double>& Pm, const double* A, int sz, double scale, double* out) {
  std::vector<double> AP(sz * sz, 0.0);
  for (int i = 0; i < sz; ++i)
    for (int k = 0; k < sz; ++k) {
      double a = A[i * sz + k];
      if (a == 0.0) continue;
      for (int j = 0; j < sz; ++j) AP[i * sz + j] += a * Pm[k * sz + j];
    }
  for (int k = 0; k < sz; ++k)
    for (int i = 0; i < sz; ++i) {
      double p = Pm[k * sz + i];
      if (p == 0.0) continue;
      for (int j = 0; j < sz; ++j) out[i * sz + j] += scale * p * AP[k * sz + j];
    }
}

static double frob(const double* A, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += A[i] * A[i];
  return std::sqrt(s);
}

void coarsen_level(const ldgs_problem& P, const Geometry& g, const Basis& B, const Level& F, Level& C) {
  const int d = g.d, nq = g.nq, mt = g.mt;
  C.n = F.n / 2;
  C.h = 2.0 * F.h;
  C.NE = 1;
  for (int j = 0; j < d; ++j) C.NE *= C.n;
  C.rho_delta = F.rho_delta;
  C.mu_is_const = F.mu_is_const;
  C.mu_c = F.mu_c;
  // phases: all children must agree (agglomeration within one phase only)
  C.chi.assign(C.NE, 1);
  for (int64_t Ec = 0; Ec < C.NE; ++Ec) {
    int cc[3];
    coords(Ec, C.n, d, cc);
    int ch = -1;
    for (int o = 0; o < (1 << d); ++o) {
      int cf[3];
      for (int j = 0; j < d; ++j) cf[j] = 2 * cc[j] + ((o >> j) & 1);
      int v = F.chi[eindex(cf, F.n, d)];
      if (ch < 0) ch = v;
      else if (ch != v) throw std::runtime_error("interface not aligned with the coarse grid");
    }
    C.chi[Ec] = ch;
  }
  // M_mu,2h = I^T M_mu,h I
  int all_axes[3] = {0, 1, 2};
  std::vector<std::vector<double>> Pfull(1 << d);
  for (int o = 0; o < (1 << d); ++o) injection_dense(B, o, all_axes, d, Pfull[o]);
  if (!F.mu_is_const) {
    C.mmu.assign((size_t)C.NE * nq * nq, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t Ec = 0; Ec < C.NE; ++Ec) {
      int cc[3];
      coords(Ec, C.n, d, cc);
      for (int o = 0; o < (1 << d); ++o) {
        int cf[3];
        for (int j = 0; j < d; ++j) cf[j] = 2 * cc[j] + ((o >> j) & 1);
        int64_t Ef = eindex(cf, F.n, d);
        ptap_add(Pfull[o], F.mmu.data() + (size_t)Ef * nq * nq, nq, 1.0, C.mmu.data() + (size_t)Ec * nq * nq);
      }
    }
  }
  // faces: coarse face = 2^{d-1} fine faces at twice the position
  const bool unsteady = !F.faces[0].Tmu.empty();
  for (int k = 0; k < d; ++k) {
    const FaceSet& ff = F.faces[k];
    FaceSet& cf = C.faces[k];
    const bool per = ff.nfk == F.n;
    cf.nfk = per ? C.n : C.n + 1;
    cf.count = cf.nfk;
    for (int j = 0; j < d; ++j)
      if (j != k) cf.count *= C.n;
    cf.type.assign(cf.count, F_NONE);
    cf.w.assign(2 * cf.count, 0.0);
    cf.T.assign((size_t)cf.count * mt * mt, 0.0);
    if (unsteady) {
      cf.Tmu.assign((size_t)cf.count * mt * mt, 0.0);
      cf.Trho.assign((size_t)cf.count * mt * mt, 0.0);
    }
    int taxes[2], na = 0;
    for (int j = 0; j < d; ++j)
      if (j != k) taxes[na++] = j;
    std::vector<std::vector<double>> Pt(1 << d);
    for (int o = 0; o < (1 << d); ++o) injection_dense(B, o, taxes, na, Pt[o]);
    bool bad = false;
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < cf.count; ++id) {
      int c[3] = {0, 0, 0};
      int64_t r = id;
      int fpos = 0;
      for (int j = 0; j < d; ++j) {
        int ext = (j == k) ? cf.nfk : C.n;
        int v = (int)(r % ext);
        r /= ext;
        if (j == k) fpos = v;
        else c[j] = v;
      }
      unsigned char ty = 255;
      double wL = 0, wR = 0;
      double* T = cf.T.data() + (size_t)id * mt * mt;
      for (int o = 0; o < (1 << d); ++o) {
        if ((o >> k) & 1) continue;   // tangential children only
        int fc[3];
        for (int j = 0; j < d; ++j) fc[j] = (j == k) ? 0 : 2 * c[j] + ((o >> j) & 1);
        int64_t fid = face_id(F, d, k, fc, 2 * fpos);
        unsigned char t2 = ff.type[fid];
        if (ty == 255) {
          ty = t2;
          wL = ff.w[2 * fid];
          wR = ff.w[2 * fid + 1];
        } else if (ty != t2 || wL != ff.w[2 * fid] || wR != ff.w[2 * fid + 1]) {
          bad = true;
        }
        // E_2h = 2 I^T E I on intraphase faces; E-tilde_2h = 1/2 I^T E-tilde I elsewhere
        double fac = (t2 == F_INTRA) ? 2.0 : 0.5;
        ptap_add(Pt[o], ff.T.data() + (size_t)fid * mt * mt, mt, fac, T);
        if (unsteady && t2 == F_INTRA) {
          ptap_add(Pt[o], ff.Tmu.data() + (size_t)fid * mt * mt, mt, 2.0, cf.Tmu.data() + (size_t)id * mt * mt);
          ptap_add(Pt[o], ff.Trho.data() + (size_t)fid * mt * mt, mt, 0.5, cf.Trho.data() + (size_t)id * mt * mt);
        }
      }
      cf.type[id] = ty;
      cf.w[2 * id] = wL;
      cf.w[2 * id + 1] = wR;
      if (unsteady && ty == F_INTRA) {
        // eq. (Etimedep): Frobenius-weighted blend of the two coarsened parts
        const double* Tm = cf.Tmu.data() + (size_t)id * mt * mt;
        const double* Tr = cf.Trho.data() + (size_t)id * mt * mt;
        double nm = frob(Tm, mt * mt), nr = frob(Tr, mt * mt);
        for (int i = 0; i < mt * mt; ++i)
          T[i] = (nm + nr > 0.0) ? (nr / (nm + nr)) * (nr / (nm + nr)) * Tm[i] + (nm / (nm + nr)) * (nm / (nm + nr)) * Tr[i]
                                 : 0.0;
      }
    }
    if (bad) throw std::runtime_error("face types differ within a coarse face");
  }
}

void set_scaling(Level& L, const Geometry& g) {
  const int nq = g.nq;
  L.dscale.assign(2 * L.NE, 1.0);
  for (int64_t E = 0; E < L.NE; ++E) {
    double mu = L.mu_is_const ? L.mu_c : L.mmu[(size_t)E * nq * nq];
    L.dscale[2 * E] = 1.0 / std::sqrt(mu);
    L.dscale[2 * E + 1] = std::sqrt(mu);
  }
}

// ---------------------------------------------------------------------------
// colouring
// ---------------------------------------------------------------------------
int colour_count(int scheme, int d) {
  switch (scheme) {
    case LDGS_COLOR_RED_BLACK: return 2;
    case LDGS_COLOR_PARITY: return 1 << d;
    case LDGS_COLOR_MOD3: return d == 2 ? 9 : 27;
  }
  return 0;
}

static int colour_of(int scheme, const int* c, int d) {
  int v = 0;
  if (scheme == LDGS_COLOR_RED_BLACK) {
    for (int j = 0; j < d; ++j) v += c[j];
    return v % 2;
  }
  if (scheme == LDGS_COLOR_PARITY) {
    for (int j = 0; j < d; ++j) v += (c[j] % 2) << j;
    return v;
  }
  int s = 1;
  for (int j = 0; j < d; ++j) {
    v += (c[j] % 3) * s;
    s *= 3;
  }
  return v;
}

// Elements X whose gradient component G_k u depends on u_E (axis k given,
// or any axis when k < 0): X = E, or X shares a face normal to k with E and
// the lifting weight on X's side of that face is nonzero.  Face neighbours
// are also collected in adj when requested.
static void lift_set(const Level& L, int d, int64_t E, int kk, std::vector<int64_t>& out,
                     std::vector<int64_t>* adj) {
  out.clear();
  out.push_back(E);
  int c[3];
  coords(E, L.n, d, c);
  for (int k = 0; k < d; ++k) {
    const FaceSet& fs = L.faces[k];
    const bool per = fs.nfk == L.n;
    int flo = c[k], fhi = per ? (c[k] + 1) % L.n : c[k] + 1;
    int64_t idlo = face_id(L, d, k, c, flo), idhi = face_id(L, d, k, c, fhi);
    int64_t eL, eR;
    face_elements(L, d, k, flo, c, &eL, &eR);
    if (eL >= 0 && (fs.type[idlo] == F_INTRA || fs.type[idlo] == F_INTER)) {
      if (adj) adj->push_back(eL);
      if ((kk < 0 || kk == k) && fs.w[2 * idlo] != 0.0) out.push_back(eL);   // L side weight of E's low face
    }
    face_elements(L, d, k, fhi, c, &eL, &eR);
    if (eR >= 0 && (fs.type[idhi] == F_INTRA || fs.type[idhi] == F_INTER)) {
      if (adj) adj->push_back(eR);
      if ((kk < 0 || kk == k) && fs.w[2 * idhi + 1] != 0.0) out.push_back(eR);
    }
  }
}

// Block (E, F) of the operator is nonzero when E and F share a face (pressure
// penalty, G and G^T couplings) or when some X has G(X, E) and G(X, F) both
// nonzero: along one axis k for the standard form (sum_k G_k^T M G_k), along
// any pair of axes for the viscous-stress form (G_j^T M G_i).
bool colouring_is_proper(const Level& L, int d, int scheme, int gamma, int64_t* bad_e) {
  std::vector<int> col(L.NE);
  for (int64_t E = 0; E < L.NE; ++E) {
    int c[3];
    coords(E, L.n, d, c);
    col[E] = colour_of(scheme, c, d);
  }
  const int nsets = gamma ? 1 : d;
  for (int si = 0; si < nsets; ++si) {
    const int kk = gamma ? -1 : si;
    std::vector<std::vector<int64_t>> lifts(L.NE);
    for (int64_t E = 0; E < L.NE; ++E) lift_set(L, d, E, kk, lifts[E], nullptr);
    std::vector<std::vector<int64_t>> rev(L.NE);
    for (int64_t E = 0; E < L.NE; ++E)
      for (int64_t X : lifts[E]) rev[X].push_back(E);
    for (int64_t E = 0; E < L.NE; ++E) {
      std::vector<int64_t> adj, l;
      lift_set(L, d, E, kk, l, &adj);
      for (int64_t F : adj)
        if (F != E && col[F] == col[E]) { *bad_e = E; return false; }
      for (int64_t X : lifts[E])
        for (int64_t F : rev[X])
          if (F != E && col[F] == col[E]) { *bad_e = E; return false; }
    }
  }
  return true;
}

void set_colouring(Level& L, int d, int scheme) {
  L.ncol = colour_count(scheme, d);
  L.colour.assign(L.NE, 0);
  L.elems.assign(L.ncol, {});
  for (int64_t E = 0; E < L.NE; ++E) {
    int c[3];
    coords(E, L.n, d, c);
    int col = colour_of(scheme, c, d);
    L.colour[E] = col;
    L.elems[col].push_back((int)E);
  }
}

}  // namespace ldgs
