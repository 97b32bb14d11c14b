// Internal declarations of the HHO p-multilevel library (not part of the ABI).
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/hho_pmg.h"

namespace hho {

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};
void set_error(const std::string &msg);
[[noreturn]] void fail(int code, const std::string &msg);

// ---------------------------------------------------------------- small utils
inline int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
// dim P^deg in `nvar` variables
inline int dim_poly(int nvar, int deg) { return deg < 0 ? 0 : (int)binom(deg + nvar, nvar); }

void parallel_for(int64_t n, const std::function<void(int64_t)> &fn);

}  // namespace hho

// ---------------------------------------------------------------- mesh
struct hho_mesh {
  int dim = 0;
  int64_t nv = 0, nf = 0, nc = 0;
  std::vector<double> verts;
  std::vector<int64_t> fptr, fvtx, cptr, cface;
  std::vector<int8_t> fbc;
  // topology
  std::vector<int64_t> fcell[2];    // adjacent cells, -1 if none
  std::vector<int32_t> flocal[2];   // position of the face in the cell's face list
  std::vector<double> csign;        // per cell_face entry: +1 if n_F points out of the cell
  // geometry (xyz padded to 3)
  std::vector<double> farea, fdiam, fcen, fnrm, ft1, ft2;
  std::vector<double> cvol, cdiam, ccen, clo, chi;
  std::vector<uint8_t> cbox;
  std::vector<std::vector<int64_t>> cring;  // d=2: counter-clockwise vertex ring per cell
  int max_faces = 0;
  bool has_neumann = false;
};

namespace hho {
void build_mesh(const hho_mesh_desc *d, hho_mesh *m);

// Local HHO operators of every cell, packed per cell as
//   [a (nloc*nloc) | B (d*nT*nloc) | rhs_u (d*nloc) | rhs_p (nT)]
struct LocalData {
  int k = 0, d = 0, nT = 0, nF = 0, N1 = 0;
  std::vector<int64_t> off;   // [nc+1] record offsets (doubles)
  std::vector<int32_t> nloc;  // [nc]
  std::vector<double> rec;
};
// eta: Nitsche penalty of every cell, or, when cell_eta is not NULL, cell_eta[c] per cell
void build_local(const hho_mesh *m, int k, double eta, const double *cell_eta, int qdeg, hho_field_fn f,
                 hho_field_fn gD, hho_field_fn gN, void *ctx, LocalData *out);

// The HHO-hp scheme's local operators (Section 2.3.2), host only; per cell the
// record a [nloc^2], B [d][npl][nloc], rhs_u [d][nloc], rhs_p [npl].
struct LocalDataHP {
  int k = 0, d = 0, nT = 0, nF = 0, N1 = 0;
  std::vector<int64_t> off;                // [nc+1] record offsets (doubles)
  std::vector<int32_t> nloc, npl;          // [nc]
  std::vector<double> rec;
};
void build_local_hp(const hho_mesh *m, int k, double eta, int qdeg, hho_field_fn f, hho_field_fn gD,
                    hho_field_fn gN, void *ctx, LocalDataHP *out);
// its v&p-cond skeleton (face velocities and face pressures) as CSR + right-hand side
void build_skeleton_hp(const hho_mesh *m, const LocalDataHP &L, std::vector<int64_t> &rowptr,
                       std::vector<int64_t> &col, std::vector<double> &val, std::vector<double> &rhs);

// The data of the device build of the local operators: integrals of the data
// against scaled monomials, which the device maps onto the orthonormal bases.
//   mf   [nc][d][nT]   (f_a, M_j)_T, M_j the cell monomials of degree <= k at
//                      (x - x_T) / h_T in the graded order of the cell basis
//   fd   per boundary face f from foff[f] (-1: interior face); n the outward
//        normal of the face's cell T:
//        Dirichlet: [d][N1] (g_a, n . grad M_t)_F, t < N1 (monomials of T)
//                   [d][nF] (g_a, m_j)_F, m_j the face monomials
//                   [nT]    (g . n, M_t)_F
//        Neumann:   [d][nF] (g_a, m_j)_F
// Also fills the record layout of `lay` (off, nloc and the sizes; no records).
struct DataMoments {
  std::vector<double> mf, fd;
  std::vector<int64_t> foff;
};
void build_data_moments(const hho_mesh *m, int k, int qdeg, hho_field_fn f, hho_field_fn gD, hho_field_fn gN,
                        void *ctx, DataMoments *out, LocalData *lay);
// Geometry tables of the device build: counter-clockwise vertex rings of 2D
// cells (CSR), the vertex mean of every 3D cell (apex of its tetrahedra),
// Gauss-Legendre nodes and weights on [0, 1] for n = 1 .. kGlMax - 1 points
// ([n][i], stride kGlMax), and the point counts of the operator rules.
constexpr int kGlMax = 16;
struct LocalGeomHost {
  std::vector<int64_t> rptr, ring;
  std::vector<double> apex, glt, glw;
  std::vector<int32_t> EC, EF;
  int odeg = 0, max_nq = 0, max_nqf = 0;
};
void build_local_geometry(const hho_mesh *m, int k, int qdeg, LocalGeomHost *g);
}  // namespace hho
