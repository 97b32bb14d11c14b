// Local HHO-dp operators on the host: quadrature, hierarchical orthonormal
// bases, scalar potential reconstruction (Section 2.2.1), face-residual
// stabilisation (Section 2.2.3), symmetric Nitsche terms and the
// pressure-velocity coupling of the local residuals (Section 2.3.1), written as
// the local algebraic system of eq. def:HHOAB.
//
// Readings taken where the paper is silent or inconsistent:
//  * the Dirichlet datum multiplies (n . grad P v) with the sign that keeps the
//    symmetric Nitsche terms consistent: the residual holds
//    -(u_F - g_D).(n . grad P v) + eta/h_F (u_F - g_D).v_F;
//  * g_N is the traction (grad u - p I) n;
//  * the coupling is evaluated in the integrated-by-parts form
//    (B v, q) = sum_c (v_T,c, d_c q)_T - sum_{F not Dirichlet} (v_F . n_TF, q)_F,
//    which equals the three terms of eq. HHOdiscrCNT for exact quadrature.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>

#include "internal.h"

namespace hho {
namespace {

// ---------------------------------------------------------------- quadrature
struct Rule {
  std::vector<double> x;  // [n*3]
  std::vector<double> w;
  int n() const { return (int)w.size(); }
  void add(const double *p, double wt) {
    x.insert(x.end(), p, p + 3);
    w.push_back(wt);
  }
};

// Gauss-Legendre on [0,1]: roots z of the Legendre polynomial P_n by Newton
// iteration from Chebyshev-like guesses, weights 2/((1-z^2) P_n'(z)^2) halved.
void gauss01(int n, std::vector<double> &t, std::vector<double> &w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double p0 = 1, p1 = z, dp = 1;
    for (int it = 0; it < 100; ++it) {
      p0 = 1;
      p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    p0 = 1;
    p1 = z;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) p0 = 1;
    dp = n * (z * p1 - p0) / (z * z - 1);
    t[i] = 0.5 * (1 + z);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);
  }
}

struct GL {
  std::vector<double> t, w;
};
const GL &gl(int n) {
  // built once, before any worker thread reads it (thread-safe static initialisation)
  static const std::vector<GL> cache = [] {
    std::vector<GL> c(40);
    for (int i = 1; i < 40; ++i) gauss01(i, c[i].t, c[i].w);
    return c;
  }();
  if (n < 1) n = 1;
  if (n >= 40) fail(HHO_E_INVALID_ARG, "quadrature degree too high");
  return cache[n];
}

void rule_segment(const double *a, const double *b, int deg, Rule &R) {
  const GL &g = gl((deg + 2) / 2);
  double L = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]));
  for (size_t i = 0; i < g.t.size(); ++i) {
    double p[3];
    for (int q = 0; q < 3; ++q) p[q] = a[q] + g.t[i] * (b[q] - a[q]);
    R.add(p, g.w[i] * L);
  }
}

// collapsed product rule x = v0 + s (v1 - v0) + s t (v2 - v1); |J| = s * |(v1-v0) x (v2-v1)|
void rule_triangle(const double *v0, const double *v1, const double *v2, int deg, Rule &R) {
  const GL &g = gl((deg + 3) / 2);
  double e1[3], e2[3], c[3];
  for (int q = 0; q < 3; ++q) {
    e1[q] = v1[q] - v0[q];
    e2[q] = v2[q] - v1[q];
  }
  c[0] = e1[1] * e2[2] - e1[2] * e2[1];
  c[1] = e1[2] * e2[0] - e1[0] * e2[2];
  c[2] = e1[0] * e2[1] - e1[1] * e2[0];
  double J = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  for (size_t i = 0; i < g.t.size(); ++i)
    for (size_t j = 0; j < g.t.size(); ++j) {
      double s = g.t[i], t = g.t[j], p[3];
      for (int q = 0; q < 3; ++q) p[q] = v0[q] + s * (e1[q] + t * e2[q]);
      R.add(p, g.w[i] * g.w[j] * s * J);
    }
}

void rule_tet(const double *v0, const double *v1, const double *v2, const double *v3, int deg, Rule &R) {
  const GL &g = gl((deg + 4) / 2);
  double e1[3], e2[3], e3[3];
  for (int q = 0; q < 3; ++q) {
    e1[q] = v1[q] - v0[q];
    e2[q] = v2[q] - v1[q];
    e3[q] = v3[q] - v2[q];
  }
  double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
               e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
  det = std::fabs(det);
  size_t n = g.t.size();
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j)
      for (size_t l = 0; l < n; ++l) {
        double s = g.t[i], t = g.t[j], u = g.t[l], p[3];
        for (int q = 0; q < 3; ++q) p[q] = v0[q] + s * (e1[q] + t * (e2[q] + u * e3[q]));
        R.add(p, g.w[i] * g.w[j] * g.w[l] * s * s * t * det);
      }
}

void rule_box(const double *lo, const double *hi, int deg, Rule &R) {
  const GL &g = gl((deg + 2) / 2);
  size_t n = g.t.size();
  double vol = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j)
      for (size_t l = 0; l < n; ++l) {
        double p[3] = {lo[0] + g.t[i] * (hi[0] - lo[0]), lo[1] + g.t[j] * (hi[1] - lo[1]), lo[2] + g.t[l] * (hi[2] - lo[2])};
        R.add(p, g.w[i] * g.w[j] * g.w[l] * vol);
      }
}

const double *vx(const hho_mesh *m, int64_t v, double *buf) {
  for (int q = 0; q < 3; ++q) buf[q] = q < m->dim ? m->verts[v * m->dim + q] : 0.0;
  return buf;
}

void cell_rule(const hho_mesh *m, int64_t c, int deg, Rule &R) {
  double a[3], b[3], d0[3], apex[3];
  if (m->dim == 2) {
    const auto &ring = m->cring[c];  // counter-clockwise, convex: fan from the first vertex
    vx(m, ring[0], a);
    for (size_t i = 1; i + 1 < ring.size(); ++i) rule_triangle(a, vx(m, ring[i], b), vx(m, ring[i + 1], d0), deg, R);
    return;
  }
  if (m->cbox[c]) {
    rule_box(&m->clo[3 * c], &m->chi[3 * c], deg, R);
    return;
  }
  std::vector<int64_t> vs;
  for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
    int64_t f = m->cface[e];
    for (int64_t t = m->fptr[f]; t < m->fptr[f + 1]; ++t) vs.push_back(m->fvtx[t]);
  }
  std::sort(vs.begin(), vs.end());
  vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
  apex[0] = apex[1] = apex[2] = 0;
  for (int64_t v : vs) {
    vx(m, v, a);
    for (int q = 0; q < 3; ++q) apex[q] += a[q] / vs.size();
  }
  for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
    int64_t f = m->cface[e];
    const int64_t *fv = &m->fvtx[m->fptr[f]];
    int nvf = (int)(m->fptr[f + 1] - m->fptr[f]);
    double p0[3];
    vx(m, fv[0], p0);
    for (int i = 1; i + 1 < nvf; ++i) rule_tet(apex, p0, vx(m, fv[i], a), vx(m, fv[i + 1], b), deg, R);
  }
}

void face_rule(const hho_mesh *m, int64_t f, int deg, Rule &R) {
  const int64_t *fv = &m->fvtx[m->fptr[f]];
  int nvf = (int)(m->fptr[f + 1] - m->fptr[f]);
  double a[3], b[3], c[3];
  if (m->dim == 2) {
    rule_segment(vx(m, fv[0], a), vx(m, fv[1], b), deg, R);
    return;
  }
  vx(m, fv[0], a);
  for (int i = 1; i + 1 < nvf; ++i) rule_triangle(a, vx(m, fv[i], b), vx(m, fv[i + 1], c), deg, R);
}

// ---------------------------------------------------------------- bases
// exponents of the monomials of total degree <= deg, graded, first exponent decreasing
std::vector<int> exponents(int nvar, int deg) {
  std::vector<int> E;
  for (int n = 0; n <= deg; ++n) {
    if (nvar == 1) {
      E.push_back(n);
    } else if (nvar == 2) {
      for (int a = n; a >= 0; --a) {
        E.push_back(a);
        E.push_back(n - a);
      }
    } else {
      for (int a = n; a >= 0; --a)
        for (int b = n - a; b >= 0; --b) {
          E.push_back(a);
          E.push_back(b);
          E.push_back(n - a - b);
        }
    }
  }
  return E;
}

inline double ipow(double x, int e) {
  double r = 1;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

// Values M[q*N + i] of the monomials at the local coordinates xi[q*nvar + v].
void eval_monomials(const std::vector<int> &E, int nvar, const double *xi, int nq, double *M) {
  int N = (int)E.size() / nvar;
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < N; ++i) {
      double v = 1;
      for (int a = 0; a < nvar; ++a) v *= ipow(xi[q * nvar + a], E[i * nvar + a]);
      M[q * N + i] = v;
    }
}

// Gram-Schmidt (modified, two passes) of the columns of M [nq x N] in the
// weighted inner product; returns C [N x N] with phi_i = sum_j C[i][j] m_j.
void gram_schmidt(const double *M, const double *w, int nq, int N, std::vector<double> &C) {
  C.assign((size_t)N * N, 0.0);
  std::vector<double> V((size_t)nq * N), v(nq), c(N);
  for (int i = 0; i < N; ++i) {
    for (int q = 0; q < nq; ++q) v[q] = M[q * N + i];
    std::fill(c.begin(), c.end(), 0.0);
    c[i] = 1;
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < i; ++j) {
        double r = 0;
        for (int q = 0; q < nq; ++q) r += w[q] * v[q] * V[(size_t)q * N + j];
        for (int q = 0; q < nq; ++q) v[q] -= r * V[(size_t)q * N + j];
        for (int t = 0; t < N; ++t) c[t] -= r * C[(size_t)j * N + t];
      }
    double nv = 0;
    for (int q = 0; q < nq; ++q) nv += w[q] * v[q] * v[q];
    nv = std::sqrt(nv);
    if (!(nv > 0)) fail(HHO_E_MESH, "basis: degenerate element (Gram-Schmidt breakdown)");
    for (int q = 0; q < nq; ++q) V[(size_t)q * N + i] = v[q] / nv;
    for (int t = 0; t < N; ++t) C[(size_t)i * N + t] = c[t] / nv;
  }
}

struct CellBasis {
  int d, N;
  double x0[3], h;
  std::vector<int> E;
  std::vector<double> C;  // [N x N]
  // phi [nq x N]
  void values(const double *x, int nq, double *phi) const {
    std::vector<double> xi((size_t)nq * d), M((size_t)nq * N);
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a) xi[q * d + a] = (x[3 * q + a] - x0[a]) / h;
    eval_monomials(E, d, xi.data(), nq, M.data());
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < N; ++i) {
        double s = 0;
        for (int j = 0; j <= i; ++j) s += C[(size_t)i * N + j] * M[(size_t)q * N + j];
        phi[(size_t)q * N + i] = s;
      }
  }
  // grad [nq x N x d]
  void grads(const double *x, int nq, double *g) const {
    std::vector<double> xi((size_t)nq * d), dm((size_t)N);
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a) xi[q * d + a] = (x[3 * q + a] - x0[a]) / h;
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a) {
        for (int j = 0; j < N; ++j) {
          int ea = E[j * d + a];
          if (ea == 0) {
            dm[j] = 0;
            continue;
          }
          double v = ea / h;
          for (int b = 0; b < d; ++b) v *= ipow(xi[q * d + b], E[j * d + b] - (b == a ? 1 : 0));
          dm[j] = v;
        }
        for (int i = 0; i < N; ++i) {
          double s = 0;
          for (int j = 0; j <= i; ++j) s += C[(size_t)i * N + j] * dm[j];
          g[((size_t)q * N + i) * d + a] = s;
        }
      }
  }
};

struct FaceBasis {
  int nvar, N;
  double x0[3], t1[3], t2[3], h;
  std::vector<int> E;
  std::vector<double> C;
  void values(const double *x, int nq, double *psi) const {
    std::vector<double> xi((size_t)nq * nvar), M((size_t)nq * N);
    for (int q = 0; q < nq; ++q) {
      double r[3] = {x[3 * q] - x0[0], x[3 * q + 1] - x0[1], x[3 * q + 2] - x0[2]};
      xi[q * nvar] = (r[0] * t1[0] + r[1] * t1[1] + r[2] * t1[2]) / h;
      if (nvar == 2) xi[q * nvar + 1] = (r[0] * t2[0] + r[1] * t2[1] + r[2] * t2[2]) / h;
    }
    eval_monomials(E, nvar, xi.data(), nq, M.data());
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < N; ++i) {
        double s = 0;
        for (int j = 0; j <= i; ++j) s += C[(size_t)i * N + j] * M[(size_t)q * N + j];
        psi[(size_t)q * N + i] = s;
      }
  }
};

// ---------------------------------------------------------------- dense helpers
// in-place Cholesky of the SPD matrix A [n x n] (lower triangle); false if not SPD
bool cholesky(double *A, int n, int lda) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * lda + j];
    for (int t = 0; t < j; ++t) s -= A[j * lda + t] * A[j * lda + t];
    if (!(s > 0)) return false;
    double ljj = std::sqrt(s);
    A[j * lda + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * lda + j];
      for (int t = 0; t < j; ++t) v -= A[i * lda + t] * A[j * lda + t];
      A[i * lda + j] = v / ljj;
    }
  }
  return true;
}
// solve L L^T X = B for nrhs columns of B [n x nrhs] (row-major, ldb)
void chol_solve(const double *L, int n, int lda, double *B, int nrhs, int ldb) {
  for (int r = 0; r < nrhs; ++r) {
    for (int i = 0; i < n; ++i) {
      double v = B[i * ldb + r];
      for (int t = 0; t < i; ++t) v -= L[i * lda + t] * B[t * ldb + r];
      B[i * ldb + r] = v / L[i * lda + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = B[i * ldb + r];
      for (int t = i + 1; t < n; ++t) v -= L[t * lda + i] * B[t * ldb + r];
      B[i * ldb + r] = v / L[i * lda + i];
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- driver
namespace {
// Inputs shared by the local builds: quadrature rules, face basis values and
// the data at the data points.
struct LocalInputs {
  std::vector<Rule> crule, frule, corule, forule;         // data / operator rules of cells and faces
  std::vector<std::vector<double>> fpsi, fpsio;           // face basis values at the data / operator points
  std::vector<int64_t> coff, dof_, nof;                   // offsets of the cell / Dirichlet / Neumann data points
  std::vector<double> fval, dval, nval;                   // f, g_D, g_N at those points
};
void prepare_local_inputs(const hho_mesh *m, int k, int qdeg, hho_field_fn f_fn, hho_field_fn gD_fn,
                          hho_field_fn gN_fn, void *ctx, const char *who, LocalInputs &I) {
  const int d = m->dim, nF = dim_poly(d - 1, k);
  const int64_t nc = m->nc, nf = m->nf;
  // quadrature rules: the data integrals (f, g_D, g_N) use rules exact to qdeg;
  // every other integrand (Gram matrices of the bases, stiffness, reconstruction
  // right-hand side, trace projections, coupling) is a polynomial of degree at
  // most 2k + 2, integrated exactly by the cheaper operator rules
  const int odeg = std::min(qdeg, 2 * k + 2);
  I.crule.resize(nc);
  I.corule.resize(nc);
  I.frule.resize(nf);
  I.forule.resize(nf);
  auto &crule = I.crule, &frule = I.frule, &corule = I.corule, &forule = I.forule;
  parallel_for(nc, [&](int64_t c) {
    cell_rule(m, c, qdeg, crule[c]);
    cell_rule(m, c, odeg, corule[c]);
  });
  parallel_for(nf, [&](int64_t f) {
    face_rule(m, f, qdeg, frule[f]);
    face_rule(m, f, odeg, forule[f]);
  });

  // face bases (shared by the two cells of a face)
  std::vector<FaceBasis> fb(nf);
  I.fpsi.resize(nf);
  I.fpsio.resize(nf);
  auto &fpsi = I.fpsi, &fpsio = I.fpsio;  // values at the data / operator points
  const std::vector<int> EF = exponents(d - 1, k);
  parallel_for(nf, [&](int64_t f) {
    FaceBasis &B = fb[f];
    B.nvar = d - 1;
    B.N = nF;
    B.E = EF;
    B.h = m->fdiam[f];
    for (int q = 0; q < 3; ++q) {
      B.x0[q] = m->fcen[3 * f + q];
      B.t1[q] = m->ft1[3 * f + q];
      B.t2[q] = m->ft2[3 * f + q];
    }
    const Rule &R = forule[f];
    int nq = R.n();
    std::vector<double> xi((size_t)nq * B.nvar), M((size_t)nq * nF);
    for (int q = 0; q < nq; ++q) {
      const double *x = &R.x[3 * q];
      double r[3] = {x[0] - B.x0[0], x[1] - B.x0[1], x[2] - B.x0[2]};
      xi[q * B.nvar] = (r[0] * B.t1[0] + r[1] * B.t1[1] + r[2] * B.t1[2]) / B.h;
      if (B.nvar == 2) xi[q * B.nvar + 1] = (r[0] * B.t2[0] + r[1] * B.t2[1] + r[2] * B.t2[2]) / B.h;
    }
    eval_monomials(B.E, B.nvar, xi.data(), nq, M.data());
    gram_schmidt(M.data(), R.w.data(), nq, nF, B.C);
    fpsio[f].resize((size_t)nq * nF);
    B.values(R.x.data(), nq, fpsio[f].data());
    fpsi[f].resize((size_t)frule[f].n() * nF);
    B.values(frule[f].x.data(), frule[f].n(), fpsi[f].data());
  });

  // data at the quadrature points: body force on cells, Dirichlet / Neumann data on faces
  I.coff.assign(nc + 1, 0);
  I.dof_.assign(nf + 1, 0);
  I.nof.assign(nf + 1, 0);
  auto &coff = I.coff, &dof_ = I.dof_, &nof = I.nof;
  for (int64_t c = 0; c < nc; ++c) coff[c + 1] = coff[c] + crule[c].n();
  for (int64_t f = 0; f < nf; ++f) {
    dof_[f + 1] = dof_[f] + (m->fbc[f] == HHO_FACE_DIRICHLET ? frule[f].n() : 0);
    nof[f + 1] = nof[f] + (m->fbc[f] == HHO_FACE_NEUMANN ? frule[f].n() : 0);
  }
  std::vector<double> fx(coff[nc] * d);
  I.fval.assign(coff[nc] * d, 0.0);
  auto &fval = I.fval;
  for (int64_t c = 0; c < nc; ++c)
    for (int q = 0; q < crule[c].n(); ++q)
      for (int a = 0; a < d; ++a) fx[(coff[c] + q) * d + a] = crule[c].x[3 * q + a];
  if (f_fn && coff[nc]) f_fn(fx.data(), coff[nc], nullptr, fval.data(), ctx);
  std::vector<double> dx(dof_[nf] * d), dn(dof_[nf] * d);
  I.dval.assign(dof_[nf] * d, 0.0);
  auto &dval = I.dval;
  std::vector<double> nx(nof[nf] * d), nn(nof[nf] * d);
  I.nval.assign(nof[nf] * d, 0.0);
  auto &nval = I.nval;
  for (int64_t f = 0; f < nf; ++f) {
    if (m->fbc[f] == HHO_FACE_INTERIOR) continue;
    int64_t c = m->fcell[0][f];
    double sg = m->csign[m->cptr[c] + m->flocal[0][f]];
    bool isD = m->fbc[f] == HHO_FACE_DIRICHLET;
    int64_t o = isD ? dof_[f] : nof[f];
    for (int q = 0; q < frule[f].n(); ++q)
      for (int a = 0; a < d; ++a) {
        (isD ? dx : nx)[(o + q) * d + a] = frule[f].x[3 * q + a];
        (isD ? dn : nn)[(o + q) * d + a] = sg * m->fnrm[3 * f + a];
      }
  }
  if (gD_fn && dof_[nf]) gD_fn(dx.data(), dof_[nf], dn.data(), dval.data(), ctx);
  if (nof[nf]) {
    if (!gN_fn) fail(HHO_E_INVALID_ARG, std::string(who) + ": the mesh has Neumann faces but gN is NULL");
    gN_fn(nx.data(), nof[nf], nn.data(), nval.data(), ctx);
  }

}
}  // namespace

void build_local(const hho_mesh *m, int k, double eta, const double *cell_eta, int qdeg, hho_field_fn f_fn,
                 hho_field_fn gD_fn, hho_field_fn gN_fn, void *ctx, LocalData *out) {
  const int d = m->dim;
  const int N1 = dim_poly(d, k + 1), nT = dim_poly(d, k), nF = dim_poly(d - 1, k);
  out->k = k;
  out->d = d;
  out->nT = nT;
  out->nF = nF;
  out->N1 = N1;
  const int64_t nc = m->nc, nf = m->nf;

  LocalInputs I;
  prepare_local_inputs(m, k, qdeg, f_fn, gD_fn, gN_fn, ctx, "set_data", I);
  const std::vector<Rule> &crule = I.crule, &frule = I.frule, &corule = I.corule, &forule = I.forule;
  const std::vector<std::vector<double>> &fpsi = I.fpsi, &fpsio = I.fpsio;
  const std::vector<int64_t> &coff = I.coff, &dof_ = I.dof_, &nof = I.nof;
  const std::vector<double> &fval = I.fval, &dval = I.dval, &nval = I.nval;

  // record layout
  out->off.assign(nc + 1, 0);
  out->nloc.assign(nc, 0);
  for (int64_t c = 0; c < nc; ++c) {
    int nfc = (int)(m->cptr[c + 1] - m->cptr[c]);
    int nloc = nT + nfc * nF;
    out->nloc[c] = nloc;
    out->off[c + 1] = out->off[c] + (int64_t)nloc * nloc + (int64_t)d * nT * nloc + (int64_t)d * nloc + nT;
  }
  out->rec.assign(out->off[nc], 0.0);
  const std::vector<int> EC = exponents(d, k + 1);

  parallel_for(nc, [&](int64_t c) {
    const double eta_c = cell_eta ? cell_eta[c] : eta;  // Nitsche penalty of this cell
    const Rule &R = corule[c];
    const int nq = R.n();
    const int nfc = (int)(m->cptr[c + 1] - m->cptr[c]);
    const int nloc = nT + nfc * nF;
    CellBasis cb;
    cb.d = d;
    cb.N = N1;
    cb.E = EC;
    cb.h = m->cdiam[c];
    for (int q = 0; q < 3; ++q) cb.x0[q] = m->ccen[3 * c + q];
    {
      std::vector<double> xi((size_t)nq * d), M((size_t)nq * N1);
      for (int q = 0; q < nq; ++q)
        for (int a = 0; a < d; ++a) xi[q * d + a] = (R.x[3 * q + a] - cb.x0[a]) / cb.h;
      eval_monomials(cb.E, d, xi.data(), nq, M.data());
      gram_schmidt(M.data(), R.w.data(), nq, N1, cb.C);
    }
    std::vector<double> phi((size_t)nq * N1), gphi((size_t)nq * N1 * d);
    cb.values(R.x.data(), nq, phi.data());
    cb.grads(R.x.data(), nq, gphi.data());

    // stiffness K_ij = (grad phi_i, grad phi_j)_T
    std::vector<double> K((size_t)N1 * N1, 0.0);
    for (int q = 0; q < nq; ++q)
      for (int i = 1; i < N1; ++i)
        for (int j = 1; j <= i; ++j) {
          double s = 0;
          for (int a = 0; a < d; ++a) s += gphi[((size_t)q * N1 + i) * d + a] * gphi[((size_t)q * N1 + j) * d + a];
          K[(size_t)i * N1 + j] += R.w[q] * s;
        }
    for (int i = 1; i < N1; ++i)
      for (int j = 1; j < i; ++j) K[(size_t)j * N1 + i] = K[(size_t)i * N1 + j];

    // reconstruction right-hand side G [N1 x nloc]
    std::vector<double> G((size_t)N1 * nloc, 0.0);
    for (int i = 0; i < N1; ++i)
      for (int j = 0; j < nT; ++j) G[(size_t)i * nloc + j] = K[(size_t)i * N1 + j];
    struct FaceLoc {
      int64_t f;
      double n[3];
      int nq;
      std::vector<double> phif, gn;  // [nqf x N1]
    };
    std::vector<FaceLoc> FL(nfc);
    for (int i = 0; i < nfc; ++i) {
      int64_t e = m->cptr[c] + i, f = m->cface[e];
      FaceLoc &L = FL[i];
      L.f = f;
      for (int q = 0; q < 3; ++q) L.n[q] = m->csign[e] * m->fnrm[3 * f + q];
      const Rule &Rf = forule[f];
      L.nq = Rf.n();
      L.phif.resize((size_t)L.nq * N1);
      L.gn.resize((size_t)L.nq * N1);
      cb.values(Rf.x.data(), L.nq, L.phif.data());
      std::vector<double> g((size_t)L.nq * N1 * d);
      cb.grads(Rf.x.data(), L.nq, g.data());
      for (int q = 0; q < L.nq; ++q)
        for (int t = 0; t < N1; ++t) {
          double s = 0;
          for (int a = 0; a < d; ++a) s += g[((size_t)q * N1 + t) * d + a] * L.n[a];
          L.gn[(size_t)q * N1 + t] = s;
        }
      const double *psi = fpsio[f].data();
      for (int q = 0; q < L.nq; ++q) {
        double w = Rf.w[q];
        for (int t = 1; t < N1; ++t) {
          double gw = w * L.gn[(size_t)q * N1 + t];
          for (int j = 0; j < nT; ++j) G[(size_t)t * nloc + j] -= gw * L.phif[(size_t)q * N1 + j];
          for (int j = 0; j < nF; ++j) G[(size_t)t * nloc + nT + i * nF + j] += gw * psi[(size_t)q * nF + j];
        }
      }
    }
    // R = [e_0 ; K11^{-1} G1]
    std::vector<double> Rm((size_t)N1 * nloc, 0.0);
    Rm[0] = 1.0;
    {
      int n1 = N1 - 1;
      std::vector<double> L((size_t)n1 * n1);
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) L[(size_t)i * n1 + j] = K[(size_t)(i + 1) * N1 + (j + 1)];
      if (!cholesky(L.data(), n1, n1))
        fail(HHO_E_LOCAL_SINGULAR, "reconstruction stiffness not SPD in cell " + std::to_string(c));
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < nloc; ++j) Rm[(size_t)(i + 1) * nloc + j] = G[(size_t)(i + 1) * nloc + j];
      chol_solve(L.data(), n1, n1, &Rm[nloc], nloc, nloc);
    }

    double *rec = &out->rec[out->off[c]];
    double *A = rec;
    double *Bm = A + (size_t)nloc * nloc;
    double *ru = Bm + (size_t)d * nT * nloc;
    double *rp = ru + (size_t)d * nloc;
    // consistency: R^T K R = R1^T G1 (K R1 = G1 on the non-constant rows)
    for (int a = 0; a < nloc; ++a)
      for (int b = 0; b < nloc; ++b) {
        double s = 0;
        for (int t = 1; t < N1; ++t) s += Rm[(size_t)t * nloc + a] * G[(size_t)t * nloc + b];
        A[(size_t)a * nloc + b] = s;
      }
    // symmetrise the consistency term
    for (int a = 0; a < nloc; ++a)
      for (int b = 0; b < a; ++b) {
        double s = 0.5 * (A[(size_t)a * nloc + b] + A[(size_t)b * nloc + a]);
        A[(size_t)a * nloc + b] = A[(size_t)b * nloc + a] = s;
      }

    std::vector<double> Pi((size_t)nF * N1), D((size_t)nF * nloc), Nn((size_t)nF * N1);
    for (int i = 0; i < nfc; ++i) {
      const FaceLoc &L = FL[i];
      const int64_t f = L.f;
      const Rule &Rf = forule[f];
      const double *psi = fpsio[f].data();
      const double hF = m->fdiam[f];
      const int bc = m->fbc[f];
      // Pi[j][t] = (psi_j, phi_t)_F ; Nn[j][t] = (psi_j, grad phi_t . n)_F
      std::fill(Pi.begin(), Pi.end(), 0.0);
      std::fill(Nn.begin(), Nn.end(), 0.0);
      for (int q = 0; q < L.nq; ++q)
        for (int j = 0; j < nF; ++j) {
          double wp = Rf.w[q] * psi[(size_t)q * nF + j];
          for (int t = 0; t < N1; ++t) {
            Pi[(size_t)j * N1 + t] += wp * L.phif[(size_t)q * N1 + t];
            Nn[(size_t)j * N1 + t] += wp * L.gn[(size_t)q * N1 + t];
          }
        }
      // face residual D = E_F - Pi R - Pi_k (E_T - R_k)
      for (int j = 0; j < nF; ++j)
        for (int b = 0; b < nloc; ++b) {
          double s = (b == nT + i * nF + j) ? 1.0 : 0.0;
          for (int t = 0; t < N1; ++t) s -= Pi[(size_t)j * N1 + t] * Rm[(size_t)t * nloc + b];
          for (int t = 0; t < nT; ++t) {
            double et = (b == t) ? 1.0 : 0.0;
            s -= Pi[(size_t)j * N1 + t] * (et - Rm[(size_t)t * nloc + b]);
          }
          D[(size_t)j * nloc + b] = s;
        }
      for (int a = 0; a < nloc; ++a)
        for (int b = 0; b < nloc; ++b) {
          double s = 0;
          for (int j = 0; j < nF; ++j) s += D[(size_t)j * nloc + a] * D[(size_t)j * nloc + b];
          A[(size_t)a * nloc + b] += s / hF;
        }
      if (bc == HHO_FACE_DIRICHLET) {
        // -(n.grad P u, v_F) - (u_F, n.grad P v) + eta/h (u_F, v_F)
        std::vector<double> NR((size_t)nF * nloc, 0.0);
        for (int j = 0; j < nF; ++j)
          for (int b = 0; b < nloc; ++b) {
            double s = 0;
            for (int t = 0; t < N1; ++t) s += Nn[(size_t)j * N1 + t] * Rm[(size_t)t * nloc + b];
            NR[(size_t)j * nloc + b] = s;
          }
        for (int j = 0; j < nF; ++j) {
          int r = nT + i * nF + j;
          for (int b = 0; b < nloc; ++b) {
            A[(size_t)r * nloc + b] -= NR[(size_t)j * nloc + b];
            A[(size_t)b * nloc + r] -= NR[(size_t)j * nloc + b];
          }
          A[(size_t)r * nloc + r] += eta_c / hF;
        }
        // data: -(g_D, n.grad P v) + eta/h (g_D, v_F); mass: (g_D . n, q), at the
        // data points
        const double *g = &dval[dof_[f] * d];
        const Rule &Rd = frule[f];
        const int nqd = Rd.n();
        const double *psid = fpsi[f].data();
        std::vector<double> phid((size_t)nqd * N1), gnd((size_t)nqd * N1);
        {
          std::vector<double> gd((size_t)nqd * N1 * d);
          cb.values(Rd.x.data(), nqd, phid.data());
          cb.grads(Rd.x.data(), nqd, gd.data());
          for (int q = 0; q < nqd; ++q)
            for (int t = 0; t < N1; ++t) {
              double s = 0;
              for (int a = 0; a < d; ++a) s += gd[((size_t)q * N1 + t) * d + a] * L.n[a];
              gnd[(size_t)q * N1 + t] = s;
            }
        }
        for (int cc = 0; cc < d; ++cc) {
          std::vector<double> gt(N1, 0.0), gp(nF, 0.0);
          for (int q = 0; q < nqd; ++q) {
            double wg = Rd.w[q] * g[q * d + cc];
            for (int t = 0; t < N1; ++t) gt[t] += wg * gnd[(size_t)q * N1 + t];
            for (int j = 0; j < nF; ++j) gp[j] += wg * psid[(size_t)q * nF + j];
          }
          for (int b = 0; b < nloc; ++b) {
            double s = 0;
            for (int t = 0; t < N1; ++t) s += Rm[(size_t)t * nloc + b] * gt[t];
            ru[cc * nloc + b] -= s;
          }
          for (int j = 0; j < nF; ++j) ru[cc * nloc + nT + i * nF + j] += eta_c / hF * gp[j];
        }
        for (int q = 0; q < nqd; ++q) {
          double gn = 0;
          for (int a = 0; a < d; ++a) gn += g[q * d + a] * L.n[a];
          for (int t = 0; t < nT; ++t) rp[t] += Rd.w[q] * gn * phid[(size_t)q * N1 + t];
        }
      } else if (bc == HHO_FACE_NEUMANN) {
        const double *g = &nval[nof[f] * d];
        const Rule &Rd = frule[f];
        const double *psid = fpsi[f].data();
        for (int cc = 0; cc < d; ++cc)
          for (int q = 0; q < Rd.n(); ++q)
            for (int j = 0; j < nF; ++j)
              ru[cc * nloc + nT + i * nF + j] += Rd.w[q] * g[q * d + cc] * psid[(size_t)q * nF + j];
      }
      // coupling, face part: -(v_F . n, q)_F on non-Dirichlet faces
      if (bc != HHO_FACE_DIRICHLET)
        for (int cc = 0; cc < d; ++cc)
          for (int t = 0; t < nT; ++t)
            for (int j = 0; j < nF; ++j) {
              double s = 0;
              for (int q = 0; q < L.nq; ++q) s += Rf.w[q] * psi[(size_t)q * nF + j] * L.phif[(size_t)q * N1 + t];
              Bm[((size_t)cc * nT + t) * nloc + nT + i * nF + j] -= L.n[cc] * s;
            }
    }
    // coupling, cell part: (v_T,c, d_c q)_T
    for (int q = 0; q < nq; ++q) {
      double w = R.w[q];
      for (int cc = 0; cc < d; ++cc)
        for (int j = 0; j < nT; ++j) {
          double pj = w * phi[(size_t)q * N1 + j];
          for (int t = 0; t < nT; ++t) Bm[((size_t)cc * nT + t) * nloc + j] += pj * gphi[((size_t)q * N1 + t) * d + cc];
        }
    }
    // body force (f_c, v_T) at the data points
    {
      const Rule &Rd = crule[c];
      const int nqd = Rd.n();
      std::vector<double> phid((size_t)nqd * N1);
      cb.values(Rd.x.data(), nqd, phid.data());
      for (int q = 0; q < nqd; ++q)
        for (int cc = 0; cc < d; ++cc) {
          const double fv = Rd.w[q] * fval[(coff[c] + q) * d + cc];
          for (int j = 0; j < nT; ++j) ru[cc * nloc + j] += fv * phid[(size_t)q * N1 + j];
        }
    }
  });
}

// Local operators of the HHO scheme with hybrid pressure (Section 2.3.2,
// Scheme 2): cell velocity in P^{k+1}(T) (all N1 modes of the cell basis), face
// velocity and face pressure in P^k(F), cell pressure in P^k(T).  The viscous
// part is Scheme 1's with k' = k + 1, its face residual
// pi_F^k(v_F - p v) - (v_T - p v)|_F (degree k + 1 on the face) integrated at
// the face's quadrature points; the coupling is the hybrid one,
//   (B v, q) = -(div v_T, q_T)_T + sum_F ((v_T - v_F) . n_TF, q_F)_F
//              + sum_{F Dirichlet} (v_F . n_TF, q_F)_F,
// used for the momentum and (transposed, with the datum (g_D . n_TF, q_F)_F on
// Dirichlet faces) for the mass balance, so that the system is symmetric.
// Record of a cell: a [nloc x nloc], B [d][npl][nloc], rhs_u [d][nloc],
// rhs_p [npl], with nloc = N1 + card(F_T) nF and npl = nT + card(F_T) nF.
void build_local_hp(const hho_mesh *m, int k, double eta, int qdeg, hho_field_fn f_fn, hho_field_fn gD_fn,
                    hho_field_fn gN_fn, void *ctx, LocalDataHP *out) {
  const int d = m->dim;
  const int N1 = dim_poly(d, k + 1), nT = dim_poly(d, k), nF = dim_poly(d - 1, k);
  out->k = k;
  out->d = d;
  out->N1 = N1;
  out->nT = nT;
  out->nF = nF;
  const int64_t nc = m->nc, nf = m->nf;
  LocalInputs I;
  prepare_local_inputs(m, k, qdeg, f_fn, gD_fn, gN_fn, ctx, "local_hp", I);
  const std::vector<Rule> &crule = I.crule, &frule = I.frule, &corule = I.corule, &forule = I.forule;
  const std::vector<std::vector<double>> &fpsi = I.fpsi, &fpsio = I.fpsio;
  const std::vector<int64_t> &coff = I.coff, &dof_ = I.dof_, &nof = I.nof;
  const std::vector<double> &fval = I.fval, &dval = I.dval, &nval = I.nval;

  out->off.assign(nc + 1, 0);
  out->nloc.assign(nc, 0);
  out->npl.assign(nc, 0);
  for (int64_t c = 0; c < nc; ++c) {
    const int nfc = (int)(m->cptr[c + 1] - m->cptr[c]);
    const int nloc = N1 + nfc * nF, npl = nT + nfc * nF;
    out->nloc[c] = nloc;
    out->npl[c] = npl;
    out->off[c + 1] = out->off[c] + (int64_t)nloc * nloc + (int64_t)d * npl * nloc + (int64_t)d * nloc + npl;
  }
  out->rec.assign(out->off[nc], 0.0);
  const std::vector<int> EC = exponents(d, k + 1);

  parallel_for(nc, [&](int64_t c) {
    const Rule &R = corule[c];
    const int nq = R.n();
    const int nfc = (int)(m->cptr[c + 1] - m->cptr[c]);
    const int nloc = N1 + nfc * nF, npl = nT + nfc * nF;
    CellBasis cb;
    cb.d = d;
    cb.N = N1;
    cb.E = EC;
    cb.h = m->cdiam[c];
    for (int q = 0; q < 3; ++q) cb.x0[q] = m->ccen[3 * c + q];
    {
      std::vector<double> xi((size_t)nq * d), M((size_t)nq * N1);
      for (int q = 0; q < nq; ++q)
        for (int a = 0; a < d; ++a) xi[q * d + a] = (R.x[3 * q + a] - cb.x0[a]) / cb.h;
      eval_monomials(cb.E, d, xi.data(), nq, M.data());
      gram_schmidt(M.data(), R.w.data(), nq, N1, cb.C);
    }
    std::vector<double> phi((size_t)nq * N1), gphi((size_t)nq * N1 * d);
    cb.values(R.x.data(), nq, phi.data());
    cb.grads(R.x.data(), nq, gphi.data());
    std::vector<double> K((size_t)N1 * N1, 0.0);
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < N1; ++i)
        for (int j = 0; j <= i; ++j) {
          double s = 0;
          for (int a = 0; a < d; ++a) s += gphi[((size_t)q * N1 + i) * d + a] * gphi[((size_t)q * N1 + j) * d + a];
          K[(size_t)i * N1 + j] += R.w[q] * s;
        }
    for (int i = 0; i < N1; ++i)
      for (int j = 0; j < i; ++j) K[(size_t)j * N1 + i] = K[(size_t)i * N1 + j];
    // reconstruction right-hand side: (grad v_T, grad w)_T + sum_F (v_F - v_T, grad w . n)_F
    std::vector<double> G((size_t)N1 * nloc, 0.0);
    for (int i = 0; i < N1; ++i)
      for (int j = 0; j < N1; ++j) G[(size_t)i * nloc + j] = K[(size_t)i * N1 + j];
    std::vector<std::vector<double>> phif(nfc), gnf(nfc);
    std::vector<std::array<double, 3>> nrm(nfc);
    for (int i = 0; i < nfc; ++i) {
      const int64_t e = m->cptr[c] + i, f = m->cface[e];
      for (int q = 0; q < 3; ++q) nrm[i][q] = m->csign[e] * m->fnrm[3 * f + q];
      const Rule &Rf = forule[f];
      const int nqf = Rf.n();
      phif[i].resize((size_t)nqf * N1);
      gnf[i].resize((size_t)nqf * N1);
      cb.values(Rf.x.data(), nqf, phif[i].data());
      std::vector<double> g((size_t)nqf * N1 * d);
      cb.grads(Rf.x.data(), nqf, g.data());
      for (int q = 0; q < nqf; ++q)
        for (int t = 0; t < N1; ++t) {
          double s = 0;
          for (int a = 0; a < d; ++a) s += g[((size_t)q * N1 + t) * d + a] * nrm[i][a];
          gnf[i][(size_t)q * N1 + t] = s;
        }
      const double *psi = fpsio[f].data();
      for (int q = 0; q < nqf; ++q)
        for (int t = 1; t < N1; ++t) {
          const double gw = Rf.w[q] * gnf[i][(size_t)q * N1 + t];
          for (int j = 0; j < N1; ++j) G[(size_t)t * nloc + j] -= gw * phif[i][(size_t)q * N1 + j];
          for (int j = 0; j < nF; ++j) G[(size_t)t * nloc + N1 + i * nF + j] += gw * psi[(size_t)q * nF + j];
        }
    }
    std::vector<double> Rm((size_t)N1 * nloc, 0.0);
    Rm[0] = 1.0;  // same mean as v_T
    {
      const int n1 = N1 - 1;
      std::vector<double> L((size_t)n1 * n1);
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) L[(size_t)i * n1 + j] = K[(size_t)(i + 1) * N1 + (j + 1)];
      if (!cholesky(L.data(), n1, n1))
        fail(HHO_E_LOCAL_SINGULAR, "reconstruction stiffness not SPD in cell " + std::to_string(c));
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < nloc; ++j) Rm[(size_t)(i + 1) * nloc + j] = G[(size_t)(i + 1) * nloc + j];
      chol_solve(L.data(), n1, n1, &Rm[nloc], nloc, nloc);
    }
    double *A = &out->rec[out->off[c]];
    double *Bm = A + (size_t)nloc * nloc;
    double *ru = Bm + (size_t)d * npl * nloc;
    double *rp = ru + (size_t)d * nloc;
    // consistency (grad p u, grad p v)_T = R1^T G1, symmetrised
    for (int a = 0; a < nloc; ++a)
      for (int b = 0; b < nloc; ++b) {
        double s = 0;
        for (int t = 1; t < N1; ++t) s += Rm[(size_t)t * nloc + a] * G[(size_t)t * nloc + b];
        A[(size_t)a * nloc + b] = s;
      }
    for (int a = 0; a < nloc; ++a)
      for (int b = 0; b < a; ++b) {
        const double s = 0.5 * (A[(size_t)a * nloc + b] + A[(size_t)b * nloc + a]);
        A[(size_t)a * nloc + b] = A[(size_t)b * nloc + a] = s;
      }
    std::vector<double> Pi((size_t)nF * N1), Nn((size_t)nF * N1), PR((size_t)nF * nloc);
    for (int i = 0; i < nfc; ++i) {
      const int64_t f = m->cface[m->cptr[c] + i];
      const Rule &Rf = forule[f];
      const int nqf = Rf.n();
      const double *psi = fpsio[f].data();
      const double hF = m->fdiam[f];
      const int bc = m->fbc[f];
      const int fc0 = N1 + i * nF, pc0 = nT + i * nF;  // this face's velocity column / pressure row
      std::fill(Pi.begin(), Pi.end(), 0.0);
      std::fill(Nn.begin(), Nn.end(), 0.0);
      for (int q = 0; q < nqf; ++q)
        for (int j = 0; j < nF; ++j) {
          const double wp = Rf.w[q] * psi[(size_t)q * nF + j];
          for (int t = 0; t < N1; ++t) {
            Pi[(size_t)j * N1 + t] += wp * phif[i][(size_t)q * N1 + t];
            Nn[(size_t)j * N1 + t] += wp * gnf[i][(size_t)q * N1 + t];
          }
        }
      // coefficients of pi_F(v_F - p v): PR = E_F - Pi R
      for (int j = 0; j < nF; ++j)
        for (int b = 0; b < nloc; ++b) {
          double s = (b == fc0 + j) ? 1.0 : 0.0;
          for (int t = 0; t < N1; ++t) s -= Pi[(size_t)j * N1 + t] * Rm[(size_t)t * nloc + b];
          PR[(size_t)j * nloc + b] = s;
        }
      // face residual at each quadrature point, its square integrated / h_F
      std::vector<double> rq(nloc);
      for (int q = 0; q < nqf; ++q) {
        for (int b = 0; b < nloc; ++b) {
          double s = 0;
          for (int j = 0; j < nF; ++j) s += psi[(size_t)q * nF + j] * PR[(size_t)j * nloc + b];
          for (int t = 0; t < N1; ++t)
            s -= phif[i][(size_t)q * N1 + t] * (((b == t) ? 1.0 : 0.0) - Rm[(size_t)t * nloc + b]);
          rq[b] = s;
        }
        const double wq = Rf.w[q] / hF;
        for (int a = 0; a < nloc; ++a) {
          const double ra = wq * rq[a];
          if (ra == 0.0) continue;
          for (int b = 0; b < nloc; ++b) A[(size_t)a * nloc + b] += ra * rq[b];
        }
      }
      if (bc == HHO_FACE_DIRICHLET) {
        std::vector<double> NR((size_t)nF * nloc, 0.0);
        for (int j = 0; j < nF; ++j)
          for (int b = 0; b < nloc; ++b) {
            double s = 0;
            for (int t = 0; t < N1; ++t) s += Nn[(size_t)j * N1 + t] * Rm[(size_t)t * nloc + b];
            NR[(size_t)j * nloc + b] = s;
          }
        for (int j = 0; j < nF; ++j) {
          const int r = fc0 + j;
          for (int b = 0; b < nloc; ++b) {
            A[(size_t)r * nloc + b] -= NR[(size_t)j * nloc + b];
            A[(size_t)b * nloc + r] -= NR[(size_t)j * nloc + b];
          }
          A[(size_t)r * nloc + r] += eta / hF;
        }
        const double *g = &dval[dof_[f] * d];
        const Rule &Rd = frule[f];
        const int nqd = Rd.n();
        const double *psid = fpsi[f].data();
        std::vector<double> gd((size_t)nqd * N1 * d), gnd((size_t)nqd * N1);
        cb.grads(Rd.x.data(), nqd, gd.data());
        for (int q = 0; q < nqd; ++q)
          for (int t = 0; t < N1; ++t) {
            double s = 0;
            for (int a = 0; a < d; ++a) s += gd[((size_t)q * N1 + t) * d + a] * nrm[i][a];
            gnd[(size_t)q * N1 + t] = s;
          }
        for (int cc = 0; cc < d; ++cc) {
          std::vector<double> gt(N1, 0.0), gp(nF, 0.0);
          for (int q = 0; q < nqd; ++q) {
            const double wg = Rd.w[q] * g[q * d + cc];
            for (int t = 0; t < N1; ++t) gt[t] += wg * gnd[(size_t)q * N1 + t];
            for (int j = 0; j < nF; ++j) gp[j] += wg * psid[(size_t)q * nF + j];
          }
          for (int b = 0; b < nloc; ++b) {
            double s = 0;
            for (int t = 0; t < N1; ++t) s += Rm[(size_t)t * nloc + b] * gt[t];
            ru[cc * nloc + b] -= s;
          }
          for (int j = 0; j < nF; ++j) ru[cc * nloc + fc0 + j] += eta / hF * gp[j];
        }
        for (int q = 0; q < nqd; ++q) {  // mass datum (g_D . n, q_F)_F
          double gn = 0;
          for (int a = 0; a < d; ++a) gn += g[q * d + a] * nrm[i][a];
          for (int j = 0; j < nF; ++j) rp[pc0 + j] += Rd.w[q] * gn * psid[(size_t)q * nF + j];
        }
      } else if (bc == HHO_FACE_NEUMANN) {
        const double *g = &nval[nof[f] * d];
        const Rule &Rd = frule[f];
        const double *psid = fpsi[f].data();
        for (int cc = 0; cc < d; ++cc)
          for (int q = 0; q < Rd.n(); ++q)
            for (int j = 0; j < nF; ++j) ru[cc * nloc + fc0 + j] += Rd.w[q] * g[q * d + cc] * psid[(size_t)q * nF + j];
      }
      // hybrid coupling: (q_F, v_T . n)_F, and -(q_F, v_F . n)_F off Dirichlet faces
      for (int cc = 0; cc < d; ++cc)
        for (int j = 0; j < nF; ++j) {
          double *row = Bm + ((size_t)cc * npl + pc0 + j) * nloc;
          for (int t = 0; t < N1; ++t) row[t] += nrm[i][cc] * Pi[(size_t)j * N1 + t];
          if (bc != HHO_FACE_DIRICHLET)
            for (int l = 0; l < nF; ++l) {
              double s = 0;
              for (int q = 0; q < nqf; ++q) s += Rf.w[q] * psi[(size_t)q * nF + j] * psi[(size_t)q * nF + l];
              row[fc0 + l] -= nrm[i][cc] * s;
            }
        }
    }
    // -(q_T, div v_T)_T
    for (int q = 0; q < nq; ++q)
      for (int cc = 0; cc < d; ++cc)
        for (int t = 0; t < nT; ++t) {
          const double pt = R.w[q] * phi[(size_t)q * N1 + t];
          double *row = Bm + ((size_t)cc * npl + t) * nloc;
          for (int j = 0; j < N1; ++j) row[j] -= pt * gphi[((size_t)q * N1 + j) * d + cc];
        }
    // body force (f_c, v_T) on all N1 cell modes
    {
      const Rule &Rd = crule[c];
      const int nqd = Rd.n();
      std::vector<double> phid((size_t)nqd * N1);
      cb.values(Rd.x.data(), nqd, phid.data());
      for (int q = 0; q < nqd; ++q)
        for (int cc = 0; cc < d; ++cc) {
          const double fv = Rd.w[q] * fval[(coff[c] + q) * d + cc];
          for (int j = 0; j < N1; ++j) ru[cc * nloc + j] += fv * phid[(size_t)q * N1 + j];
        }
    }
  });
}

// v&p-cond of the HHO-hp scheme (Section 4.1.2 applied to Scheme 2): every
// cell's velocity (d N1) and pressure (nT) unknowns are eliminated from its
// local saddle-point system [[A (x) I_d, B^T], [B, 0]], leaving the face
// velocities and face pressures.  The cell block is solved through the
// Cholesky factor of the scalar a_TT and the SPD pressure Schur complement
// S_p = sum_c B_c a_TT^{-1} B_c^T (nonsingular: the divergence maps
// P^{k+1}(T)^d onto P^k(T)).  Skeletal unknown of face f, component c (c = d:
// the pressure), mode j: (f (d + 1) + c) nF + j.  Output: CSR (rows sorted, every
// block of a pair of faces of a common cell stored in full, explicit zeros
// included) and the right-hand side.
void build_skeleton_hp(const hho_mesh *m, const LocalDataHP &L, std::vector<int64_t> &rowptr,
                       std::vector<int64_t> &colidx, std::vector<double> &val, std::vector<double> &rhs) {
  const int d = L.d, N1 = L.N1, nT = L.nT, nF = L.nF, bs = (d + 1) * nF;
  const int64_t nc = m->nc, nf = m->nf, n = nf * bs;
  std::vector<std::vector<double>> Sc(nc), gc(nc);
  parallel_for(nc, [&](int64_t c) {
    const int nfc = (int)(m->cptr[c + 1] - m->cptr[c]);
    const int nloc = L.nloc[c], npl = L.npl[c];
    const double *a = &L.rec[L.off[c]];
    const double *B = a + (size_t)nloc * nloc;
    const double *ru = B + (size_t)d * npl * nloc;
    const double *rp = ru + (size_t)d * nloc;
    auto Bc = [&](int cc, int r, int col) { return B[((size_t)cc * npl + r) * nloc + col]; };
    // Cholesky of a_TT
    std::vector<double> La((size_t)N1 * N1);
    for (int i = 0; i < N1; ++i)
      for (int j = 0; j < N1; ++j) La[(size_t)i * N1 + j] = a[(size_t)i * nloc + j];
    if (!cholesky(La.data(), N1, N1)) fail(HHO_E_LOCAL_SINGULAR, "hp: a_TT not SPD in cell " + std::to_string(c));
    // W_c = a_TT^{-1} B_c^T (cell pressure rows), S_p = sum_c B_c W_c
    std::vector<double> W((size_t)d * N1 * nT), Sp((size_t)nT * nT, 0.0);
    for (int cc = 0; cc < d; ++cc) {
      double *Wc = &W[(size_t)cc * N1 * nT];
      for (int i = 0; i < N1; ++i)
        for (int t = 0; t < nT; ++t) Wc[(size_t)i * nT + t] = Bc(cc, t, i);
      chol_solve(La.data(), N1, N1, Wc, nT, nT);
      for (int t = 0; t < nT; ++t)
        for (int u = 0; u < nT; ++u) {
          double s = 0;
          for (int i = 0; i < N1; ++i) s += Bc(cc, t, i) * Wc[(size_t)i * nT + u];
          Sp[(size_t)t * nT + u] += s;
        }
    }
    if (!cholesky(Sp.data(), nT, nT)) fail(HHO_E_LOCAL_SINGULAR, "hp: pressure Schur complement not SPD in cell " + std::to_string(c));
    // the cell's skeletal unknowns: velocity (face i, component cc, mode j), then pressure (face i, mode j)
    const int nk = nfc * bs;
    auto kcol = [&](int kk, int cc) -> int {  // local velocity column of skeletal unknown kk for component cc (-1: none)
      const int nv = nfc * d * nF;
      if (kk >= nv) return -1;
      const int i = kk / (d * nF), c2 = (kk / nF) % d, j = kk % nF;
      return c2 == cc ? N1 + i * nF + j : -1;
    };
    auto krow = [&](int kk) -> int {  // local pressure row of skeletal unknown kk (-1: a velocity)
      const int nv = nfc * d * nF;
      return kk < nv ? -1 : nT + (kk - nv);
    };
    // columns: M_IK (one per skeletal unknown) and the interior right-hand side
    const int nI = d * N1 + nT, ncol = nk + 1;
    std::vector<double> X((size_t)nI * ncol, 0.0);  // rows: cell velocity (cc, i), then cell pressure t
    for (int kk = 0; kk <= nk; ++kk) {
      std::vector<double> fu((size_t)d * N1, 0.0), fp(nT, 0.0);
      if (kk < nk) {
        const int pr = krow(kk);
        for (int cc = 0; cc < d; ++cc) {
          const int vc = kcol(kk, cc);
          for (int i = 0; i < N1; ++i)
            fu[(size_t)cc * N1 + i] = vc >= 0 ? a[(size_t)i * nloc + vc] : (pr >= 0 ? Bc(cc, pr, i) : 0.0);
          if (vc >= 0)
            for (int t = 0; t < nT; ++t) fp[t] += Bc(cc, t, vc);
        }
      } else {
        for (int cc = 0; cc < d; ++cc)
          for (int i = 0; i < N1; ++i) fu[(size_t)cc * N1 + i] = ru[cc * nloc + i];
        for (int t = 0; t < nT; ++t) fp[t] = rp[t];
      }
      // saddle solve: g_c = a^{-1} f_c; S_p x_p = sum_c B_c g_c - f_p; x_c = g_c - W_c x_p
      std::vector<double> g(fu), xp(nT, 0.0);
      for (int cc = 0; cc < d; ++cc) chol_solve(La.data(), N1, N1, &g[(size_t)cc * N1], 1, 1);
      for (int t = 0; t < nT; ++t) {
        double s = -fp[t];
        for (int cc = 0; cc < d; ++cc)
          for (int i = 0; i < N1; ++i) s += Bc(cc, t, i) * g[(size_t)cc * N1 + i];
        xp[t] = s;
      }
      chol_solve(Sp.data(), nT, nT, xp.data(), 1, 1);
      for (int cc = 0; cc < d; ++cc)
        for (int i = 0; i < N1; ++i) {
          double s = g[(size_t)cc * N1 + i];
          for (int t = 0; t < nT; ++t) s -= W[((size_t)cc * N1 + i) * nT + t] * xp[t];
          X[((size_t)cc * N1 + i) * ncol + kk] = s;
        }
      for (int t = 0; t < nT; ++t) X[((size_t)d * N1 + t) * ncol + kk] = xp[t];
    }
    // S = M_KK - M_KI X_K, g = rhs_K - M_KI X_rhs; M_KI row kk is column kk of M_IK
    std::vector<double> &S = Sc[c];
    std::vector<double> &gl = gc[c];
    S.assign((size_t)nk * nk, 0.0);
    gl.assign(nk, 0.0);
    for (int r = 0; r < nk; ++r) {
      const int pr = krow(r);
      std::vector<double> mki(nI, 0.0);  // row r of M_KI
      for (int cc = 0; cc < d; ++cc) {
        const int vc = kcol(r, cc);
        for (int i = 0; i < N1; ++i)
          mki[(size_t)cc * N1 + i] = vc >= 0 ? a[(size_t)vc * nloc + i] : (pr >= 0 ? Bc(cc, pr, i) : 0.0);
        if (vc >= 0)
          for (int t = 0; t < nT; ++t) mki[(size_t)d * N1 + t] += Bc(cc, t, vc);
      }
      for (int s2 = 0; s2 <= nk; ++s2) {
        double v = 0;
        if (s2 < nk) {  // M_KK entry
          const int ps = krow(s2);
          for (int cc = 0; cc < d; ++cc) {
            const int vr = kcol(r, cc), vs = kcol(s2, cc);
            if (vr >= 0 && vs >= 0) v += a[(size_t)vr * nloc + vs];
            if (pr >= 0 && vs >= 0) v += Bc(cc, pr, vs);
            if (vr >= 0 && ps >= 0) v += Bc(cc, ps, vr);
          }
        } else {        // right-hand side entry
          if (pr >= 0) v = rp[pr];
          else
            for (int cc = 0; cc < d; ++cc)
              if (kcol(r, cc) >= 0) v = ru[cc * nloc + kcol(r, cc)];
        }
        for (int q = 0; q < nI; ++q) v -= mki[q] * X[(size_t)q * ncol + s2];
        if (s2 < nk) S[(size_t)r * nk + s2] = v;
        else gl[r] = v;
      }
    }
  });
  // global index of each of a cell's skeletal unknowns
  auto gidx = [&](int64_t c, int kk) -> int64_t {
    const int nv = (int)(m->cptr[c + 1] - m->cptr[c]) * d * nF;
    if (kk < nv) {
      const int i = kk / (d * nF), cc = (kk / nF) % d, j = kk % nF;
      return (m->cface[m->cptr[c] + i] * (d + 1) + cc) * nF + j;
    }
    const int i = (kk - nv) / nF, j = (kk - nv) % nF;
    return (m->cface[m->cptr[c] + i] * (d + 1) + d) * nF + j;
  };
  // face-face pattern: faces of a common cell, sorted
  std::vector<std::vector<int64_t>> nb(nf);
  for (int64_t c = 0; c < nc; ++c)
    for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e)
      for (int64_t e2 = m->cptr[c]; e2 < m->cptr[c + 1]; ++e2) nb[m->cface[e]].push_back(m->cface[e2]);
  for (auto &v : nb) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  rowptr.assign(n + 1, 0);
  for (int64_t f = 0; f < nf; ++f)
    for (int r = 0; r < bs; ++r) rowptr[f * bs + r + 1] = (int64_t)nb[f].size() * bs;
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
  colidx.assign(rowptr[n], 0);
  val.assign(rowptr[n], 0.0);
  rhs.assign(n, 0.0);
  for (int64_t f = 0; f < nf; ++f)
    for (int r = 0; r < bs; ++r) {
      int64_t o = rowptr[f * bs + r];
      for (int64_t g2 : nb[f])
        for (int cidx = 0; cidx < bs; ++cidx) colidx[o++] = g2 * bs + cidx;
    }
  for (int64_t c = 0; c < nc; ++c) {
    const int nk = (int)(m->cptr[c + 1] - m->cptr[c]) * bs;
    for (int r = 0; r < nk; ++r) {
      const int64_t gr = gidx(c, r);
      rhs[gr] += gc[c][r];
      const int64_t *cb = &colidx[rowptr[gr]], *ce = &colidx[rowptr[gr + 1]];
      for (int s2 = 0; s2 < nk; ++s2) {
        const int64_t gs = gidx(c, s2);
        const int64_t pos = std::lower_bound(cb, ce, gs) - colidx.data();
        val[pos] += Sc[c][(size_t)r * nk + s2];
      }
    }
  }
}

void build_data_moments(const hho_mesh *m, int k, int qdeg, hho_field_fn f_fn, hho_field_fn gD_fn,
                        hho_field_fn gN_fn, void *ctx, DataMoments *out, LocalData *lay) {
  const int d = m->dim;
  const int N1 = dim_poly(d, k + 1), nT = dim_poly(d, k), nF = dim_poly(d - 1, k);
  const int64_t nc = m->nc, nf = m->nf;
  lay->k = k;
  lay->d = d;
  lay->nT = nT;
  lay->nF = nF;
  lay->N1 = N1;
  lay->off.assign(nc + 1, 0);
  lay->nloc.assign(nc, 0);
  for (int64_t c = 0; c < nc; ++c) {
    const int nloc = nT + (int)(m->cptr[c + 1] - m->cptr[c]) * nF;
    lay->nloc[c] = nloc;
    lay->off[c + 1] = lay->off[c] + (int64_t)nloc * nloc + (int64_t)d * nT * nloc + (int64_t)d * nloc + nT;
  }
  lay->rec.clear();

  std::vector<Rule> crule(nc), frule(nf);
  parallel_for(nc, [&](int64_t c) { cell_rule(m, c, qdeg, crule[c]); });
  parallel_for(nf, [&](int64_t f) {
    if (m->fbc[f] != HHO_FACE_INTERIOR) face_rule(m, f, qdeg, frule[f]);
  });
  // data at the points
  std::vector<int64_t> coff(nc + 1, 0), boff(nf + 1, 0);
  for (int64_t c = 0; c < nc; ++c) coff[c + 1] = coff[c] + crule[c].n();
  for (int64_t f = 0; f < nf; ++f) boff[f + 1] = boff[f] + frule[f].n();
  std::vector<double> fx(coff[nc] * d), fval(coff[nc] * d, 0.0);
  for (int64_t c = 0; c < nc; ++c)
    for (int q = 0; q < crule[c].n(); ++q)
      for (int a = 0; a < d; ++a) fx[(coff[c] + q) * d + a] = crule[c].x[3 * q + a];
  if (f_fn && coff[nc]) f_fn(fx.data(), coff[nc], nullptr, fval.data(), ctx);
  std::vector<double> nrm(nf * 3, 0.0);
  std::vector<int64_t> dsel, nsel;  // Dirichlet / Neumann faces
  for (int64_t f = 0; f < nf; ++f) {
    if (m->fbc[f] == HHO_FACE_INTERIOR) continue;
    const int64_t c = m->fcell[0][f];
    const double sg = m->csign[m->cptr[c] + m->flocal[0][f]];
    for (int a = 0; a < 3; ++a) nrm[3 * f + a] = sg * m->fnrm[3 * f + a];
    (m->fbc[f] == HHO_FACE_DIRICHLET ? dsel : nsel).push_back(f);
  }
  auto gather = [&](const std::vector<int64_t> &sel, hho_field_fn fn, bool need, std::vector<double> &val,
                    std::vector<int64_t> &at) {
    int64_t n = 0;
    at.assign(nf, -1);
    for (int64_t f : sel) {
      at[f] = n;
      n += frule[f].n();
    }
    std::vector<double> x(n * d), nn(n * d);
    val.assign(n * d, 0.0);
    for (int64_t f : sel)
      for (int q = 0; q < frule[f].n(); ++q)
        for (int a = 0; a < d; ++a) {
          x[(at[f] + q) * d + a] = frule[f].x[3 * q + a];
          nn[(at[f] + q) * d + a] = nrm[3 * f + a];
        }
    if (n && !fn && need) fail(HHO_E_INVALID_ARG, "set_data: the mesh has Neumann faces but gN is NULL");
    if (n && fn) fn(x.data(), n, nn.data(), val.data(), ctx);
  };
  std::vector<double> dval, nval;
  std::vector<int64_t> dat, nat;
  gather(dsel, gD_fn, false, dval, dat);
  gather(nsel, gN_fn, true, nval, nat);

  // record offsets of the face data
  out->foff.assign(nf, -1);
  int64_t nfd = 0;
  for (int64_t f = 0; f < nf; ++f) {
    if (m->fbc[f] == HHO_FACE_DIRICHLET) {
      out->foff[f] = nfd;
      nfd += (int64_t)d * N1 + (int64_t)d * nF + nT;
    } else if (m->fbc[f] == HHO_FACE_NEUMANN) {
      out->foff[f] = nfd;
      nfd += (int64_t)d * nF;
    }
  }
  out->fd.assign(nfd, 0.0);
  out->mf.assign(nc * d * nT, 0.0);
  const std::vector<int> EC = exponents(d, k + 1), EF = exponents(d - 1, k);
  // cells: (f_a, M_j)_T
  parallel_for(nc, [&](int64_t c) {
    const Rule &R = crule[c];
    const int nq = R.n();
    const double h = m->cdiam[c], *x0 = &m->ccen[3 * c];
    std::vector<double> xi((size_t)nq * d), M((size_t)nq * N1);
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a) xi[q * d + a] = (R.x[3 * q + a] - x0[a]) / h;
    eval_monomials(EC, d, xi.data(), nq, M.data());
    double *o = &out->mf[c * d * nT];
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a) {
        const double wf = R.w[q] * fval[(coff[c] + q) * d + a];
        for (int j = 0; j < nT; ++j) o[a * nT + j] += wf * M[(size_t)q * N1 + j];
      }
  });
  // boundary faces
  parallel_for(nf, [&](int64_t f) {
    if (m->fbc[f] == HHO_FACE_INTERIOR) return;
    const bool isD = m->fbc[f] == HHO_FACE_DIRICHLET;
    const Rule &R = frule[f];
    const int nq = R.n();
    const double *g = isD ? &dval[dat[f] * d] : &nval[nat[f] * d];
    double *o = &out->fd[out->foff[f]];
    // face monomials
    const double hF = m->fdiam[f], *xf = &m->fcen[3 * f], *t1 = &m->ft1[3 * f], *t2 = &m->ft2[3 * f];
    const int nv = d - 1;
    std::vector<double> xi((size_t)nq * nv), Mf((size_t)nq * nF);
    for (int q = 0; q < nq; ++q) {
      const double r[3] = {R.x[3 * q] - xf[0], R.x[3 * q + 1] - xf[1], R.x[3 * q + 2] - xf[2]};
      xi[q * nv] = (r[0] * t1[0] + r[1] * t1[1] + r[2] * t1[2]) / hF;
      if (nv == 2) xi[q * nv + 1] = (r[0] * t2[0] + r[1] * t2[1] + r[2] * t2[2]) / hF;
    }
    eval_monomials(EF, nv, xi.data(), nq, Mf.data());
    double *gp = isD ? o + (int64_t)d * N1 : o;
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a)
        for (int j = 0; j < nF; ++j) gp[a * nF + j] += R.w[q] * g[q * d + a] * Mf[(size_t)q * nF + j];
    if (!isD) return;
    // cell monomials of the face's cell and their normal derivatives
    const int64_t c = m->fcell[0][f];
    const double h = m->cdiam[c], *x0 = &m->ccen[3 * c], *n = &nrm[3 * f];
    std::vector<double> xc((size_t)nq * d), M((size_t)nq * N1);
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < d; ++a) xc[q * d + a] = (R.x[3 * q + a] - x0[a]) / h;
    eval_monomials(EC, d, xc.data(), nq, M.data());
    double *gt = o, *gn = o + (int64_t)d * N1 + (int64_t)d * nF;
    for (int q = 0; q < nq; ++q) {
      double gdotn = 0;
      for (int a = 0; a < d; ++a) gdotn += g[q * d + a] * n[a];
      for (int t = 0; t < N1; ++t) {
        // n . grad M_t = sum_b n_b E_tb / h prod_c xi_c^(E_tc - [c == b])
        double dn = 0;
        for (int b = 0; b < d; ++b) {
          const int eb = EC[t * d + b];
          if (eb == 0) continue;
          double v = eb / h;
          for (int cc = 0; cc < d; ++cc) v *= ipow(xc[q * d + cc], EC[t * d + cc] - (cc == b ? 1 : 0));
          dn += n[b] * v;
        }
        for (int a = 0; a < d; ++a) gt[a * N1 + t] += R.w[q] * g[q * d + a] * dn;
      }
      for (int t = 0; t < nT; ++t) gn[t] += R.w[q] * gdotn * M[(size_t)q * N1 + t];
    }
  });
}

void build_local_geometry(const hho_mesh *m, int k, int qdeg, LocalGeomHost *g) {
  const int d = m->dim;
  const int64_t nc = m->nc, nf = m->nf;
  g->odeg = std::min(qdeg, 2 * k + 2);
  const int od = g->odeg;
  g->rptr.assign(1, 0);
  g->ring.clear();
  g->apex.assign(3 * nc, 0.0);
  int max_nq = 0, max_nqf = 0;
  const int n2 = (od + 3) / 2, n3b = (od + 2) / 2, n3t = (od + 4) / 2, nseg = (od + 2) / 2;
  if (n2 >= kGlMax || n3t >= kGlMax) fail(HHO_E_INVALID_ARG, "device local build: quadrature degree too high");
  for (int64_t c = 0; c < nc; ++c) {
    int nq = 0;
    if (d == 2) {
      const auto &r = m->cring[c];
      g->ring.insert(g->ring.end(), r.begin(), r.end());
      nq = (int)(r.size() - 2) * n2 * n2;
    } else if (m->cbox[c]) {
      nq = n3b * n3b * n3b;
    } else {
      std::vector<int64_t> vs;
      for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
        const int64_t f = m->cface[e];
        for (int64_t t = m->fptr[f]; t < m->fptr[f + 1]; ++t) vs.push_back(m->fvtx[t]);
        nq += (int)(m->fptr[f + 1] - m->fptr[f] - 2) * n3t * n3t * n3t;
      }
      std::sort(vs.begin(), vs.end());
      vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
      for (int64_t v : vs)
        for (int q = 0; q < 3; ++q) g->apex[3 * c + q] += m->verts[v * 3 + q] / vs.size();
    }
    g->rptr.push_back((int64_t)g->ring.size());
    max_nq = std::max(max_nq, nq);
  }
  for (int64_t f = 0; f < nf; ++f) {
    const int nvf = (int)(m->fptr[f + 1] - m->fptr[f]);
    max_nqf = std::max(max_nqf, d == 2 ? nseg : (nvf - 2) * n2 * n2);
  }
  g->max_nq = max_nq;
  g->max_nqf = max_nqf;
  g->glt.assign(kGlMax * kGlMax, 0.0);
  g->glw.assign(kGlMax * kGlMax, 0.0);
  for (int n = 1; n < kGlMax; ++n) {
    const GL &r = gl(n);
    for (int i = 0; i < n; ++i) {
      g->glt[n * kGlMax + i] = r.t[i];
      g->glw[n * kGlMax + i] = r.w[i];
    }
  }
  const std::vector<int> EC = exponents(d, k + 1), EF = exponents(d - 1, k);
  g->EC.assign(EC.begin(), EC.end());
  g->EF.assign(EF.begin(), EF.end());
}

}  // namespace hho
