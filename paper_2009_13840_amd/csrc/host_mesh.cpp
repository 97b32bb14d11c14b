// Mesh import, topology and geometry (Section 2.1 discrete setting).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <thread>

#include "internal.h"

namespace hho {

void parallel_for(int64_t n, const std::function<void(int64_t)> &fn) {
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  unsigned nt = (unsigned)std::min<int64_t>(hw, std::max<int64_t>(1, n / 16));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  std::vector<std::string> errs(nt);
  std::vector<int> codes(nt, 0);
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        for (;;) {
          int64_t i = next.fetch_add(1);
          if (i >= n) break;
          fn(i);
        }
      } catch (const Error &e) {
        codes[t] = e.code;
        errs[t] = e.msg;
        next.store(n);
      }
    });
  for (auto &x : th) x.join();
  for (unsigned t = 0; t < nt; ++t)
    if (codes[t]) throw Error{codes[t], errs[t]};
}

static void cross(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

void build_mesh(const hho_mesh_desc *d, hho_mesh *m) {
  if (!d || (d->dim != 2 && d->dim != 3)) fail(HHO_E_INVALID_ARG, "mesh: dim must be 2 or 3");
  if (d->n_verts <= 0 || d->n_faces <= 0 || d->n_cells <= 0) fail(HHO_E_INVALID_ARG, "mesh: empty mesh");
  if (!d->verts || !d->face_ptr || !d->face_vtx || !d->cell_ptr || !d->cell_face || !d->face_bc)
    fail(HHO_E_INVALID_ARG, "mesh: NULL array");
  const int D = d->dim;
  m->dim = D;
  m->nv = d->n_verts;
  m->nf = d->n_faces;
  m->nc = d->n_cells;
  m->verts.assign(d->verts, d->verts + m->nv * D);
  m->fptr.assign(d->face_ptr, d->face_ptr + m->nf + 1);
  m->cptr.assign(d->cell_ptr, d->cell_ptr + m->nc + 1);
  if (m->fptr[0] != 0 || m->cptr[0] != 0) fail(HHO_E_MESH, "mesh: CSR pointers must start at 0");
  for (int64_t f = 0; f < m->nf; ++f) {
    int64_t n = m->fptr[f + 1] - m->fptr[f];
    if ((D == 2 && n != 2) || (D == 3 && n < 3)) fail(HHO_E_MESH, "mesh: face " + std::to_string(f) + " has a bad vertex count");
  }
  for (int64_t c = 0; c < m->nc; ++c) {
    int64_t n = m->cptr[c + 1] - m->cptr[c];
    if (n < D + 1) fail(HHO_E_MESH, "mesh: cell " + std::to_string(c) + " has too few faces");
    m->max_faces = std::max<int>(m->max_faces, (int)n);
  }
  m->fvtx.assign(d->face_vtx, d->face_vtx + m->fptr[m->nf]);
  m->cface.assign(d->cell_face, d->cell_face + m->cptr[m->nc]);
  m->fbc.assign(d->face_bc, d->face_bc + m->nf);
  for (int64_t v : m->fvtx)
    if (v < 0 || v >= m->nv) fail(HHO_E_MESH, "mesh: face vertex out of range");
  for (int64_t f : m->cface)
    if (f < 0 || f >= m->nf) fail(HHO_E_MESH, "mesh: cell face out of range");

  // face -> cells
  for (int s = 0; s < 2; ++s) {
    m->fcell[s].assign(m->nf, -1);
    m->flocal[s].assign(m->nf, -1);
  }
  for (int64_t c = 0; c < m->nc; ++c)
    for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
      int64_t f = m->cface[e];
      int s = m->fcell[0][f] < 0 ? 0 : (m->fcell[1][f] < 0 ? 1 : 2);
      if (s == 2) fail(HHO_E_MESH, "mesh: face " + std::to_string(f) + " belongs to more than two cells");
      m->fcell[s][f] = c;
      m->flocal[s][f] = (int32_t)(e - m->cptr[c]);
    }
  for (int64_t f = 0; f < m->nf; ++f) {
    bool bnd = m->fcell[1][f] < 0;
    if (m->fcell[0][f] < 0) fail(HHO_E_MESH, "mesh: face " + std::to_string(f) + " belongs to no cell");
    if (bnd && m->fbc[f] != HHO_FACE_DIRICHLET && m->fbc[f] != HHO_FACE_NEUMANN)
      fail(HHO_E_MESH, "mesh: boundary face " + std::to_string(f) + " needs a Dirichlet or Neumann flag");
    if (!bnd && m->fbc[f] != HHO_FACE_INTERIOR)
      fail(HHO_E_MESH, "mesh: interior face " + std::to_string(f) + " has a boundary flag");
    if (m->fbc[f] == HHO_FACE_NEUMANN) m->has_neumann = true;
  }

  // face geometry
  m->farea.assign(m->nf, 0);
  m->fdiam.assign(m->nf, 0);
  m->fcen.assign(3 * m->nf, 0);
  m->fnrm.assign(3 * m->nf, 0);
  m->ft1.assign(3 * m->nf, 0);
  m->ft2.assign(3 * m->nf, 0);
  auto X = [&](int64_t v, int j) { return j < D ? m->verts[v * D + j] : 0.0; };
  for (int64_t f = 0; f < m->nf; ++f) {
    const int64_t *fv = &m->fvtx[m->fptr[f]];
    int nvf = (int)(m->fptr[f + 1] - m->fptr[f]);
    double dm = 0;
    for (int i = 0; i < nvf; ++i)
      for (int j = i + 1; j < nvf; ++j) {
        double s = 0;
        for (int q = 0; q < 3; ++q) s += (X(fv[i], q) - X(fv[j], q)) * (X(fv[i], q) - X(fv[j], q));
        dm = std::max(dm, std::sqrt(s));
      }
    m->fdiam[f] = dm;
    double t1[3] = {X(fv[1], 0) - X(fv[0], 0), X(fv[1], 1) - X(fv[0], 1), X(fv[1], 2) - X(fv[0], 2)};
    double l1 = norm3(t1);
    if (!(l1 > 0)) fail(HHO_E_MESH, "mesh: degenerate face " + std::to_string(f));
    for (int q = 0; q < 3; ++q) t1[q] /= l1;
    if (D == 2) {
      m->farea[f] = l1;
      for (int q = 0; q < 2; ++q) m->fcen[3 * f + q] = 0.5 * (X(fv[0], q) + X(fv[1], q));
      m->fnrm[3 * f + 0] = t1[1];
      m->fnrm[3 * f + 1] = -t1[0];
      m->ft1[3 * f + 0] = t1[0];
      m->ft1[3 * f + 1] = t1[1];
    } else {
      double nw[3] = {0, 0, 0};
      for (int i = 0; i < nvf; ++i) {
        double a[3] = {X(fv[i], 0), X(fv[i], 1), X(fv[i], 2)};
        int i2 = (i + 1) % nvf;
        double b[3] = {X(fv[i2], 0), X(fv[i2], 1), X(fv[i2], 2)};
        double c[3];
        cross(a, b, c);
        for (int q = 0; q < 3; ++q) nw[q] += c[q];
      }
      double ln = norm3(nw);
      if (!(ln > 0)) fail(HHO_E_MESH, "mesh: degenerate face " + std::to_string(f));
      double area = 0, cen[3] = {0, 0, 0};
      for (int i = 1; i + 1 < nvf; ++i) {  // fan from vertex 0
        double e1[3], e2[3], c[3];
        for (int q = 0; q < 3; ++q) {
          e1[q] = X(fv[i], q) - X(fv[0], q);
          e2[q] = X(fv[i + 1], q) - X(fv[0], q);
        }
        cross(e1, e2, c);
        double ar = 0.5 * (c[0] * nw[0] + c[1] * nw[1] + c[2] * nw[2]) / ln;
        area += ar;
        for (int q = 0; q < 3; ++q) cen[q] += ar * (X(fv[0], q) + X(fv[i], q) + X(fv[i + 1], q)) / 3.0;
      }
      m->farea[f] = area;
      for (int q = 0; q < 3; ++q) {
        m->fcen[3 * f + q] = cen[q] / area;
        m->fnrm[3 * f + q] = nw[q] / ln;
        m->ft1[3 * f + q] = t1[q];
      }
      cross(&m->fnrm[3 * f], t1, &m->ft2[3 * f]);
    }
  }

  // cell geometry
  m->cvol.assign(m->nc, 0);
  m->cdiam.assign(m->nc, 0);
  m->ccen.assign(3 * m->nc, 0);
  m->clo.assign(3 * m->nc, 0);
  m->chi.assign(3 * m->nc, 0);
  m->cbox.assign(m->nc, 0);
  m->csign.assign(m->cface.size(), 0);
  if (D == 2) m->cring.resize(m->nc);
  for (int64_t c = 0; c < m->nc; ++c) {
    std::vector<int64_t> vs;
    for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
      int64_t f = m->cface[e];
      for (int64_t t = m->fptr[f]; t < m->fptr[f + 1]; ++t) vs.push_back(m->fvtx[t]);
    }
    std::sort(vs.begin(), vs.end());
    vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
    double dm = 0;
    for (size_t i = 0; i < vs.size(); ++i)
      for (size_t j = i + 1; j < vs.size(); ++j) {
        double s = 0;
        for (int q = 0; q < D; ++q) s += (X(vs[i], q) - X(vs[j], q)) * (X(vs[i], q) - X(vs[j], q));
        dm = std::max(dm, std::sqrt(s));
      }
    m->cdiam[c] = dm;
    for (int q = 0; q < 3; ++q) {
      double lo = 1e300, hi = -1e300;
      for (int64_t v : vs) {
        lo = std::min(lo, X(v, q));
        hi = std::max(hi, X(v, q));
      }
      m->clo[3 * c + q] = lo;
      m->chi[3 * c + q] = hi;
    }
    if (D == 2) {
      // chain the segments into a ring
      int nfc = (int)(m->cptr[c + 1] - m->cptr[c]);
      std::vector<int64_t> ring;
      std::vector<char> used(nfc, 0);
      int64_t f0 = m->cface[m->cptr[c]];
      ring.push_back(m->fvtx[m->fptr[f0]]);
      int64_t cur = m->fvtx[m->fptr[f0] + 1];
      used[0] = 1;
      for (int it = 1; it < nfc; ++it) {
        ring.push_back(cur);
        bool found = false;
        for (int i = 0; i < nfc && !found; ++i) {
          if (used[i]) continue;
          int64_t f = m->cface[m->cptr[c] + i];
          int64_t a = m->fvtx[m->fptr[f]], b = m->fvtx[m->fptr[f] + 1];
          if (a == cur || b == cur) {
            used[i] = 1;
            cur = (a == cur) ? b : a;
            found = true;
          }
        }
        if (!found) fail(HHO_E_MESH, "mesh: cell " + std::to_string(c) + " boundary is not closed");
      }
      if (cur != ring[0]) fail(HHO_E_MESH, "mesh: cell " + std::to_string(c) + " boundary is not closed");
      double a2 = 0, cx = 0, cy = 0;
      int n = (int)ring.size();
      for (int i = 0; i < n; ++i) {
        double x0 = X(ring[i], 0), y0 = X(ring[i], 1), x1 = X(ring[(i + 1) % n], 0), y1 = X(ring[(i + 1) % n], 1);
        double cr = x0 * y1 - x1 * y0;
        a2 += cr;
        cx += (x0 + x1) * cr;
        cy += (y0 + y1) * cr;
      }
      if (a2 < 0) std::reverse(ring.begin(), ring.end());
      if (std::fabs(a2) <= 0) fail(HHO_E_MESH, "mesh: cell " + std::to_string(c) + " has zero area");
      m->cvol[c] = std::fabs(a2) / 2;
      m->ccen[3 * c] = cx / (3 * a2);
      m->ccen[3 * c + 1] = cy / (3 * a2);
      m->cring[c] = ring;
    } else {
      // volume and centroid from pyramids (vertex average apex) over face fans
      double apex[3] = {0, 0, 0};
      for (int64_t v : vs)
        for (int q = 0; q < 3; ++q) apex[q] += X(v, q) / vs.size();
      double vol = 0, cen[3] = {0, 0, 0};
      for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
        int64_t f = m->cface[e];
        const int64_t *fv = &m->fvtx[m->fptr[f]];
        int nvf = (int)(m->fptr[f + 1] - m->fptr[f]);
        for (int i = 1; i + 1 < nvf; ++i) {
          double a[3], b[3], cc[3], x[3];
          for (int q = 0; q < 3; ++q) {
            a[q] = X(fv[0], q) - apex[q];
            b[q] = X(fv[i], q) - apex[q];
            cc[q] = X(fv[i + 1], q) - apex[q];
          }
          cross(b, cc, x);
          double v6 = std::fabs(a[0] * x[0] + a[1] * x[1] + a[2] * x[2]) / 6.0;
          vol += v6;
          for (int q = 0; q < 3; ++q) cen[q] += v6 * (apex[q] + X(fv[0], q) + X(fv[i], q) + X(fv[i + 1], q)) / 4.0;
        }
      }
      if (!(vol > 0)) fail(HHO_E_MESH, "mesh: cell " + std::to_string(c) + " has zero volume");
      m->cvol[c] = vol;
      for (int q = 0; q < 3; ++q) m->ccen[3 * c + q] = cen[q] / vol;
      // axis-aligned box?
      bool box = true;
      for (int64_t v : vs)
        for (int q = 0; q < 3 && box; ++q) {
          double x = X(v, q), lo = m->clo[3 * c + q], hi = m->chi[3 * c + q], tol = 1e-12 * (hi - lo);
          if (std::fabs(x - lo) > tol && std::fabs(x - hi) > tol) box = false;
        }
      double bv = (m->chi[3 * c] - m->clo[3 * c]) * (m->chi[3 * c + 1] - m->clo[3 * c + 1]) * (m->chi[3 * c + 2] - m->clo[3 * c + 2]);
      m->cbox[c] = box && std::fabs(bv - vol) <= 1e-10 * vol;
    }
    for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) {
      int64_t f = m->cface[e];
      double s = 0;
      for (int q = 0; q < 3; ++q) s += (m->fcen[3 * f + q] - m->ccen[3 * c + q]) * m->fnrm[3 * f + q];
      m->csign[e] = s > 0 ? 1.0 : -1.0;
    }
  }
}

}  // namespace hho
