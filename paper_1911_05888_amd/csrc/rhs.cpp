// Right-hand side of eq. (stokessystem), assembled on the host from the data
// callbacks of ldgs_rhs_data (appendix A of the paper):
//   momentum i: int f_i phi - sum_j G_j^T M_mu (J_g,ij + gamma J_g,ji) + J_h,i
//               + int_D tau_b g_i phi^- + int_Gij tau_ij g_ij,i [phi]
//   constraint: int f phi + J_{g.n}
// J_g, J_h and J_{g.n} are the boundary/interface data vectors of the
// appendix (definitions after eq. gsum, eq. wworkings and eq. ewv).  The
// product G_j^T M_mu J_g carries M_mu: substituting eq. (sigmaresult) into the
// adjoint form of w_i yields it (eq. wform prints the term without M_mu; the
// two agree for mu = 1).  Face integrals use p+3 Gauss points per axis.
#include <cmath>
#include <vector>

#include "build.hpp"
#include "host.hpp"

namespace ldgs {

static inline int ipow(int b, int e) {
  int v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}
static inline int digit(int a, int k, int m) { return (a / ipow(m, k)) % m; }
static inline int tang(int a, int k, int m) { return a % ipow(m, k) + ipow(m, k) * (a / ipow(m, k + 1)); }

void assemble_rhs_host(const ldgs_problem& P, const Geometry& g, const Basis& B, const Level& L,
                       const ldgs_rhs_data& data, double* out) {
  const int d = g.d, m = g.m, nq = g.nq, mt = g.mt, nb = g.nb, n = L.n;
  const double h = L.h;
  const int64_t NE = L.NE, S = NE * nq;
  const int q = P.degree + 3;
  std::vector<double> gx, gw;
  Basis::gauss(q, gx, gw);
  // ---- volume terms: int f phi = h^{d/2} sum_q w f(x_q) B(xi_q) ----
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
  std::vector<std::vector<double>> bu(d + 1, std::vector<double>(S, 0.0));
  const double vscale = std::pow(h, 0.5 * d);
  const int64_t chunk = 1 << 16;
  std::vector<double> X, F, Fd;
  std::vector<int> ph;
  for (int64_t E0 = 0; E0 < NE; E0 += chunk) {
    int64_t ne = std::min(chunk, NE - E0);
    X.assign(ne * nv * d, 0.0);
    ph.assign(ne * nv, 1);
    for (int64_t e = 0; e < ne; ++e) {
      int64_t E = E0 + e, r = E;
      int c[3];
      for (int j = 0; j < d; ++j) { c[j] = (int)(r % n); r /= n; }
      for (int i = 0; i < nv; ++i) {
        for (int j = 0; j < d; ++j) X[(e * nv + i) * d + j] = (c[j] + xi[i * d + j]) * h;
        ph[e * nv + i] = L.chi[E];
      }
    }
    if (data.f) {
      F.assign(ne * nv * d, 0.0);
      data.f(ne * nv, X.data(), ph.data(), nullptr, F.data(), data.user);
      for (int64_t e = 0; e < ne; ++e)
        for (int i = 0; i < d; ++i)
          for (int a = 0; a < nq; ++a) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) s += wv[k] * F[(e * nv + k) * d + i] * Bv[k * nq + a];
            bu[i][(E0 + e) * nq + a] += vscale * s;
          }
    }
    if (data.f_div) {
      Fd.assign(ne * nv, 0.0);
      data.f_div(ne * nv, X.data(), ph.data(), nullptr, Fd.data(), data.user);
      for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < nq; ++a) {
          double s = 0.0;
          for (int k = 0; k < nv; ++k) s += wv[k] * Fd[e * nv + k] * Bv[k * nq + a];
          bu[d][(E0 + e) * nq + a] += vscale * s;
        }
    }
  }
  // ---- face terms ----
  // tangential rule
  const int nt = ipow(q, d - 1);
  std::vector<double> tw(nt, 1.0), tp(nt * std::max(d - 1, 1));
  std::vector<double> Bt(nt * mt);
  for (int i = 0; i < nt; ++i) {
    for (int j = 0; j < d - 1; ++j) {
      int qi = (i / ipow(q, j)) % q;
      tp[i * (d - 1) + j] = gx[qi];
      tw[i] *= gw[qi];
    }
    for (int t = 0; t < mt; ++t) {
      double v = 1.0;
      for (int j = 0; j < d - 1; ++j) v *= Basis::leg(digit(t, j, m), tp[i * (d - 1) + j]);
      Bt[i * mt + t] = v;
    }
  }
  // int_face c phi_a = h^{d/2-1} e_side[a_k] sum_q w_q c(x_q) Bt[q][t(a)]
  const double fscale = std::pow(h, 0.5 * d - 1.0);
  std::vector<std::vector<double>> Jg(d * d, std::vector<double>(S, 0.0));
  std::vector<std::vector<double>> Jh(d, std::vector<double>(S, 0.0)), pen(d, std::vector<double>(S, 0.0));
  std::vector<double> Jgn(S, 0.0);
  auto add_face = [&](std::vector<double>& vec, int64_t E, int k, const double* e, const double* coef, double scale) {
    // coef: nt values at the face points
    for (int a = 0; a < nq; ++a) {
      double s = 0.0;
      int t = tang(a, k, m);
      for (int i = 0; i < nt; ++i) s += tw[i] * coef[i] * Bt[i * mt + t];
      vec[E * nq + a] += scale * fscale * e[digit(a, k, m)] * s;
    }
  };
  for (int k = 0; k < d; ++k) {
    const FaceSet& fs = L.faces[k];
    for (int64_t id = 0; id < fs.count; ++id) {
      unsigned char ty = fs.type[id];
      int c[3] = {0, 0, 0};
      int64_t r = id;
      int f = 0;
      for (int j = 0; j < d; ++j) {
        int ext = (j == k) ? fs.nfk : n;
        int v = (int)(r % ext);
        r /= ext;
        if (j == k) f = v;
        else c[j] = v;
      }
      const bool stress = P.bc[k] == LDGS_STRESS && fs.nfk != n && (f == 0 || f == n);
      if (ty != F_DIR_LO && ty != F_DIR_HI && ty != F_INTER && !stress) continue;
      int64_t eL, eR;
      face_elements(L, d, k, f, c, &eL, &eR);
      std::vector<double> Xf(nt * d), nrm(nt * d, 0.0), gv(nt * d, 0.0), hv(nt * d, 0.0), mu(nt), coef(nt);
      std::vector<int> phm(nt), php(nt);
      for (int i = 0; i < nt; ++i) {
        int jj = 0;
        for (int j = 0; j < d; ++j) Xf[i * d + j] = (j == k) ? f * h : (c[j] + tp[i * (d - 1) + jj++]) * h;
      }
      if (stress) {
        // J_h: int_wall phi h_i with h = sigma n, n outward
        const bool lo = f == 0;
        const int64_t Em = lo ? eR : eL;
        const double s = lo ? -1.0 : 1.0;
        const double* e = lo ? B.e0.data() : B.e1.data();
        for (int i = 0; i < nt; ++i) {
          phm[i] = L.chi[Em];
          nrm[i * d + k] = s;
        }
        if (!data.h_stress) continue;
        data.h_stress(nt, Xf.data(), phm.data(), nrm.data(), hv.data(), data.user);
        for (int i = 0; i < d; ++i) {
          for (int qq = 0; qq < nt; ++qq) coef[qq] = hv[qq * d + i];
          add_face(Jh[i], Em, k, e, coef.data(), 1.0);
        }
      } else if (ty == F_DIR_LO || ty == F_DIR_HI) {
        const int64_t Em = (ty == F_DIR_LO) ? eR : eL;
        const double s = (ty == F_DIR_LO) ? -1.0 : 1.0;        // outward normal n_k
        const double* e = (ty == F_DIR_LO) ? B.e0.data() : B.e1.data();
        for (int i = 0; i < nt; ++i) {
          phm[i] = L.chi[Em];
          nrm[i * d + k] = s;
        }
        if (!data.g_dirichlet) continue;
        data.g_dirichlet(nt, Xf.data(), phm.data(), nrm.data(), gv.data(), data.user);
        eval_field(P.mu, d, nt, Xf.data(), phm.data(), mu.data());
        const double tb = P.tau_u_bdry_C * P.degree / h;
        for (int i = 0; i < d; ++i) {
          for (int qq = 0; qq < nt; ++qq) coef[qq] = gv[qq * d + i] * s;
          add_face(Jg[i * d + k], Em, k, e, coef.data(), 1.0);
          for (int qq = 0; qq < nt; ++qq) coef[qq] = tb * mu[qq] * gv[qq * d + i];
          add_face(pen[i], Em, k, e, coef.data(), 1.0);
        }
        for (int qq = 0; qq < nt; ++qq) coef[qq] = gv[qq * d + k] * s;
        add_face(Jgn, Em, k, e, coef.data(), 1.0);
      } else {
        // interphase: minus side = phase 1 (lower index), normal from phase 1 to phase 2
        const bool minusL = L.chi[eL] < L.chi[eR];
        const int64_t Em = minusL ? eL : eR, Ep = minusL ? eR : eL;
        const double s = minusL ? 1.0 : -1.0;
        const double* em = minusL ? B.e1.data() : B.e0.data();
        const double* ep = minusL ? B.e0.data() : B.e1.data();
        double wm = minusL ? fs.w[2 * id] : fs.w[2 * id + 1];   // (1 - lambda) on the minus side
        double lam = 1.0 - wm;
        for (int i = 0; i < nt; ++i) {
          phm[i] = L.chi[Em];
          php[i] = L.chi[Ep];
          nrm[i * d + k] = s;
        }
        if (data.g_jump) data.g_jump(nt, Xf.data(), phm.data(), nrm.data(), gv.data(), data.user);
        if (data.h_jump) data.h_jump(nt, Xf.data(), phm.data(), nrm.data(), hv.data(), data.user);
        std::vector<double> mup(nt);
        eval_field(P.mu, d, nt, Xf.data(), phm.data(), mu.data());
        eval_field(P.mu, d, nt, Xf.data(), php.data(), mup.data());
        const double ti = P.tau_u_inter_C * P.degree / h;
        for (int i = 0; i < d; ++i) {
          for (int qq = 0; qq < nt; ++qq) coef[qq] = gv[qq * d + i] * s;
          add_face(Jg[i * d + k], Em, k, em, coef.data(), 1.0 - lam);
          add_face(Jg[i * d + k], Ep, k, ep, coef.data(), lam);
          for (int qq = 0; qq < nt; ++qq) coef[qq] = hv[qq * d + i];
          add_face(Jh[i], Em, k, em, coef.data(), lam);
          add_face(Jh[i], Ep, k, ep, coef.data(), 1.0 - lam);
          for (int qq = 0; qq < nt; ++qq) coef[qq] = ti * std::min(mu[qq], mup[qq]) * gv[qq * d + i];
          add_face(pen[i], Em, k, em, coef.data(), 1.0);
          add_face(pen[i], Ep, k, ep, coef.data(), -1.0);
        }
        for (int qq = 0; qq < nt; ++qq) coef[qq] = gv[qq * d + k] * s;
        add_face(Jgn, Em, k, em, coef.data(), 1.0 - lam);
        add_face(Jgn, Ep, k, ep, coef.data(), lam);
      }
    }
  }
  // ---- combine ----
  std::vector<double> tau(S), sv(S), tmp(S);
  for (int i = 0; i < d; ++i) {
    for (int64_t qq = 0; qq < S; ++qq) bu[i][qq] += Jh[i][qq] + pen[i][qq];
    for (int j = 0; j < d; ++j) {
      for (int64_t qq = 0; qq < S; ++qq) tau[qq] = Jg[i * d + j][qq] + P.form * Jg[j * d + i][qq];
      host_mmu(L, g, tau.data(), sv.data());
      host_gradT(L, g, B, j, sv.data(), tmp.data());
      for (int64_t qq = 0; qq < S; ++qq) bu[i][qq] -= tmp[qq];
    }
  }
  for (int64_t qq = 0; qq < S; ++qq) bu[d][qq] += Jgn[qq];
  for (int64_t E = 0; E < NE; ++E)
    for (int f = 0; f <= d; ++f)
      for (int a = 0; a < nq; ++a) out[E * nb + f * nq + a] = bu[f][E * nq + a];
}

}  // namespace ldgs
