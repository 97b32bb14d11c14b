// Local HHO-dp operators on the device, one workgroup per cell (Sections 2.2.1,
// 2.2.3 and 2.3.1): the cell's quadrature, the hierarchical orthonormal bases of
// the cell (degree k + 1) and of its faces (degree k), the scalar potential
// reconstruction, the face-residual stabilisation, the symmetric Nitsche terms,
// the pressure-velocity coupling and the right-hand side, written into the cell
// record [a | B | rhs_u | rhs_p] that the static condensation reads.  The data
// enter as integrals against scaled monomials (computed with the user's
// callbacks on the host); the bases' coefficients map them onto the bases.
//
// The face bases are formed first, one wave per face (k_face_bases), and read by
// both cells of a face.  Differences from the host build, all within rounding:
// the bases come from classical Gram-Schmidt applied twice (the host uses the
// modified form twice;
// both give the unique lower-triangular orthonormalisation of the graded
// monomials), the consistency term is Y^T Y with Y = L^{-1} G (L the Cholesky
// factor of the stiffness on the non-constant functions) instead of the
// symmetrised R^T G, and the stabilisation's face residual is written
//   D = E_F - [b < nT] Pi_F,b - sum_{t >= nT} Pi_F,t R_t
// (the same expression with the cancelling terms of degree <= k removed).
#include <algorithm>
#include <mutex>

#include "dev_common.h"
#include "device.h"
#include "internal.h"

namespace hho {
namespace {


__device__ inline void lvtx(const LocalGeom &g, int64_t v, double p[3]) {
  for (int q = 0; q < 3; ++q) p[q] = q < g.d ? g.verts[v * g.d + q] : 0.0;
}

__device__ inline double ipowd(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

// monomial j of the exponent table E (nv variables) at local coordinates xi
__device__ inline double mono(const int32_t *E, int nv, const double *xi, int j) {
  double v = 1.0;
  for (int a = 0; a < nv; ++a) v *= ipowd(xi[a], E[j * nv + a]);
  return v;
}
// d/dx_a of cell monomial j at xi = (x - x0) / h
__device__ inline double dmono(const int32_t *E, int d, const double *xi, double h, int j, int a) {
  const int ea = E[j * d + a];
  if (ea == 0) return 0.0;
  double v = ea / h;
  for (int b = 0; b < d; ++b) v *= ipowd(xi[b], E[j * d + b] - (b == a ? 1 : 0));
  return v;
}

// block-wide sum returned to every thread (red: 32 doubles; slots 0..15 take the
// waves' partials, slot 31 carries the result)
__device__ inline double lsum(double v, double *red) {
  const double r = block_sum(v, red);
  if (threadIdx.x == 0) red[31] = r;
  __syncthreads();
  return red[31];
}

// Operator quadrature point q of cell c: position and weight (the rules of the
// host build: triangle fans in 2D, a tensor rule on boxes, tetrahedra from the
// vertex mean over the fanned faces otherwise).
__device__ void cell_point(const LocalGeom &g, int c, int q, double x[3], double *w) {
  const int od = g.odeg;
  if (g.d == 2) {
    const int n = (od + 3) / 2, ppp = n * n;
    const int piece = q / ppp, i = (q % ppp) / n, j = q % n;
    const int64_t *r = g.ring + g.rptr[c];
    double v0[3], v1[3], v2[3];
    lvtx(g, r[0], v0);
    lvtx(g, r[piece + 1], v1);
    lvtx(g, r[piece + 2], v2);
    const double e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e2x = v2[0] - v1[0], e2y = v2[1] - v1[1];
    const double J = fabs(e1x * e2y - e1y * e2x);
    const double s = g.glt[n * kGlTable + i], t = g.glt[n * kGlTable + j];
    x[0] = v0[0] + s * (e1x + t * e2x);
    x[1] = v0[1] + s * (e1y + t * e2y);
    x[2] = 0.0;
    *w = g.glw[n * kGlTable + i] * g.glw[n * kGlTable + j] * s * J;
    return;
  }
  if (g.cbox[c]) {
    const int n = (od + 2) / 2;
    const int i = q / (n * n), j = (q / n) % n, l = q % n;
    const double *lo = g.clo + 3 * c, *hi = g.chi + 3 * c;
    const double vol = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    x[0] = lo[0] + g.glt[n * kGlTable + i] * (hi[0] - lo[0]);
    x[1] = lo[1] + g.glt[n * kGlTable + j] * (hi[1] - lo[1]);
    x[2] = lo[2] + g.glt[n * kGlTable + l] * (hi[2] - lo[2]);
    *w = g.glw[n * kGlTable + i] * g.glw[n * kGlTable + j] * g.glw[n * kGlTable + l] * vol;
    return;
  }
  const int n = (od + 4) / 2, ppp = n * n * n;
  int piece = q / ppp;
  const int lq = q % ppp, i = lq / (n * n), j = (lq / n) % n, l = lq % n;
  for (int e = g.cptr[c]; e < g.cptr[c + 1]; ++e) {
    const int f = g.cface[e];
    const int64_t f0 = g.fptr[f];
    const int ntri = (int)(g.fptr[f + 1] - f0) - 2;
    if (piece >= ntri) {
      piece -= ntri;
      continue;
    }
    double v0[3], v1[3], v2[3], v3[3];
    for (int a = 0; a < 3; ++a) v0[a] = g.apex[3 * c + a];
    lvtx(g, g.fvtx[f0], v1);
    lvtx(g, g.fvtx[f0 + piece + 1], v2);
    lvtx(g, g.fvtx[f0 + piece + 2], v3);
    double e1[3], e2[3], e3[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = v1[a] - v0[a];
      e2[a] = v2[a] - v1[a];
      e3[a] = v3[a] - v2[a];
    }
    const double det = fabs(e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                            e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]));
    const double s = g.glt[n * kGlTable + i], t = g.glt[n * kGlTable + j], u = g.glt[n * kGlTable + l];
    for (int a = 0; a < 3; ++a) x[a] = v0[a] + s * (e1[a] + t * (e2[a] + u * e3[a]));
    *w = g.glw[n * kGlTable + i] * g.glw[n * kGlTable + j] * g.glw[n * kGlTable + l] * s * s * t * det;
    return;
  }
  x[0] = x[1] = x[2] = 0.0;
  *w = 0.0;
}

__device__ int cell_npoints(const LocalGeom &g, int c) {
  const int od = g.odeg;
  if (g.d == 2) {
    const int n = (od + 3) / 2;
    return (int)(g.rptr[c + 1] - g.rptr[c] - 2) * n * n;
  }
  if (g.cbox[c]) {
    const int n = (od + 2) / 2;
    return n * n * n;
  }
  const int n = (od + 4) / 2;
  int t = 0;
  for (int e = g.cptr[c]; e < g.cptr[c + 1]; ++e) {
    const int f = g.cface[e];
    t += (int)(g.fptr[f + 1] - g.fptr[f] - 2);
  }
  return t * n * n * n;
}

// face rule: Gauss-Legendre on a segment (2D), triangle fan (3D)
__device__ int face_npoints(const LocalGeom &g, int f) {
  const int od = g.odeg;
  if (g.d == 2) return (od + 2) / 2;
  const int n = (od + 3) / 2;
  return (int)(g.fptr[f + 1] - g.fptr[f] - 2) * n * n;
}
__device__ void face_point(const LocalGeom &g, int f, int q, double x[3], double *w) {
  const int od = g.odeg;
  const int64_t f0 = g.fptr[f];
  if (g.d == 2) {
    const int n = (od + 2) / 2;
    double a[3], b[3];
    lvtx(g, g.fvtx[f0], a);
    lvtx(g, g.fvtx[f0 + 1], b);
    const double L = sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
    const double t = g.glt[n * kGlTable + q];
    for (int k = 0; k < 3; ++k) x[k] = a[k] + t * (b[k] - a[k]);
    *w = g.glw[n * kGlTable + q] * L;
    return;
  }
  const int n = (od + 3) / 2, ppp = n * n;
  const int piece = q / ppp, i = (q % ppp) / n, j = q % n;
  double v0[3], v1[3], v2[3];
  lvtx(g, g.fvtx[f0], v0);
  lvtx(g, g.fvtx[f0 + piece + 1], v1);
  lvtx(g, g.fvtx[f0 + piece + 2], v2);
  double e1[3], e2[3], cr[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = v1[a] - v0[a];
    e2[a] = v2[a] - v1[a];
  }
  cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
  cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
  cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double J = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  const double s = g.glt[n * kGlTable + i], t = g.glt[n * kGlTable + j];
  for (int a = 0; a < 3; ++a) x[a] = v0[a] + s * (e1[a] + t * e2[a]);
  *w = g.glw[n * kGlTable + i] * g.glw[n * kGlTable + j] * s * J;
}

// Classical Gram-Schmidt, applied twice, of the N columns of V [nq][ldv] in the
// weights W: on return the columns are orthonormal and row i of C [N][N] holds
// the coefficients of basis function i in the original columns (lower
// triangular).  `r` is LDS scratch of N doubles.  Returns false (on every
// thread) if a column is numerically zero.
__device__ bool cgs2(double *V, int ldv, const double *W, int nq, int N, double *C, double *r, double *red) {
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) C[e] = (e / N == e % N) ? 1.0 : 0.0;
  __syncthreads();
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int i = 0; i < N; ++i) {
    for (int pass = 0; pass < 2 && i > 0; ++pass) {
      for (int j = wid; j < i; j += nw) {  // r_j = (v, V_j)_W
        double s = 0;
        for (int q = lane; q < nq; q += kWave) s += W[q] * V[q * ldv + i] * V[q * ldv + j];
        s = wave_sum(s);
        if (lane == 0) r[j] = s;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        double v = V[q * ldv + i];
        for (int j = 0; j < i; ++j) v -= r[j] * V[q * ldv + j];
        V[q * ldv + i] = v;
      }
      for (int t = threadIdx.x; t < N; t += blockDim.x) {
        double v = C[i * N + t];
        for (int j = 0; j < i; ++j) v -= r[j] * C[j * N + t];
        C[i * N + t] = v;
      }
      __syncthreads();
    }
    double s = 0;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) s += W[q] * V[q * ldv + i] * V[q * ldv + i];
    const double nv = sqrt(lsum(s, red));
    if (!(nv > 0)) return false;
    const double inv = 1.0 / nv;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) V[q * ldv + i] *= inv;
    for (int t = threadIdx.x; t < N; t += blockDim.x) C[i * N + t] *= inv;
    __syncthreads();
  }
  return true;
}

// Orders the LDS accesses of one wave's lanes: what a lane wrote before is seen by
// every lane's later reads (a wave runs in order; this keeps the compiler's order).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// cgs2 for a small basis on few points (a face's) by one wave alone, lane j
// forming the product with column j, so the column steps need no workgroup
// barrier; N <= 64.  Every lane returns false if a column is numerically zero.
__device__ bool cgs2_one_wave(double *V, int ldv, const double *W, int nq, int N, double *C, double *r, int lane) {
  {
    for (int e = lane; e < N * N; e += kWave) C[e] = (e / N == e % N) ? 1.0 : 0.0;
    wave_sync();
    int bad = 0;
    for (int i = 0; i < N; ++i) {
      for (int pass = 0; pass < 2 && i > 0; ++pass) {
        if (lane < i) {  // r_j = (v, V_j)_W
          double s = 0;
          for (int q = 0; q < nq; ++q) s += W[q] * V[q * ldv + i] * V[q * ldv + lane];
          r[lane] = s;
        }
        wave_sync();
        for (int q = lane; q < nq; q += kWave) {
          double v = V[q * ldv + i];
          for (int j = 0; j < i; ++j) v -= r[j] * V[q * ldv + j];
          V[q * ldv + i] = v;
        }
        if (lane < N) {
          double v = C[i * N + lane];
          for (int j = 0; j < i; ++j) v -= r[j] * C[j * N + lane];
          C[i * N + lane] = v;
        }
        wave_sync();
      }
      double s = 0;
      for (int q = lane; q < nq; q += kWave) s += W[q] * V[q * ldv + i] * V[q * ldv + i];
      s = __shfl(wave_sum(s), 0, kWave);
      const double nv = sqrt(s);
      if (!(nv > 0)) {
        bad = 1;
        break;
      }
      const double inv = 1.0 / nv;
      for (int q = lane; q < nq; q += kWave) V[q * ldv + i] *= inv;
      if (lane < N) C[i * N + lane] *= inv;
      wave_sync();
    }
    return bad == 0;
  }
}

// Orthonormal basis of every face (its coefficients on the face monomials,
// CF[f][j][m], lower triangular), one wave per face: a face's basis is shared by
// its two cells, so it is formed once, here, with many faces in flight.
constexpr int kFaceWaves = 4;
__global__ void __launch_bounds__(kFaceWaves * kWave) k_face_bases(LocalGeom g, int max_nqf, double *CFall) {
  extern __shared__ double lds[];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int f = blockIdx.x * kFaceWaves + w;
  const int nF = g.nF;
  const int per = 4 * max_nqf + max_nqf * nF + nF * nF + nF + 1;
  double *X = lds + (int64_t)w * per, *W = X + 3 * max_nqf, *V = W + max_nqf, *C = V + (int64_t)max_nqf * nF,
         *r = C + nF * nF;
  if (f >= g.nf) return;
  const int nqf = face_npoints(g, f);
  for (int q = lane; q < nqf; q += kWave) {
    double x[3], wq;
    face_point(g, f, q, x, &wq);
    X[3 * q] = x[0];
    X[3 * q + 1] = x[1];
    X[3 * q + 2] = x[2];
    W[q] = wq;
  }
  wave_sync();
  const double hF = g.fdiam[f];
  for (int e = lane; e < nqf * nF; e += kWave) {
    const int q = e / nF, j = e % nF;
    const double rr[3] = {X[3 * q] - g.fcen[3 * f], X[3 * q + 1] - g.fcen[3 * f + 1], X[3 * q + 2] - g.fcen[3 * f + 2]};
    double xi[2];
    xi[0] = (rr[0] * g.ft1[3 * f] + rr[1] * g.ft1[3 * f + 1] + rr[2] * g.ft1[3 * f + 2]) / hF;
    xi[1] = (rr[0] * g.ft2[3 * f] + rr[1] * g.ft2[3 * f + 1] + rr[2] * g.ft2[3 * f + 2]) / hF;
    V[e] = mono(g.EF, g.d - 1, xi, j);
  }
  wave_sync();
  if (!cgs2_one_wave(V, nF, W, nqf, nF, C, r, lane)) {
    if (lane == 0) g.err[0] = -(f + 1);
    return;
  }
  double *out = CFall + (int64_t)f * nF * nF;
  for (int e = lane; e < nF * nF; e += kWave) out[e] = C[e];
}

__global__ void __launch_bounds__(kLocalThreads) k_local(LocalGeom g, LocalLds L) {
  extern __shared__ double lds[];
  const int c = blockIdx.x;
  const int d = g.d, N1 = g.N1, nT = g.nT, nF = g.nF;
  const int e0 = g.cptr[c], nfc = g.cptr[c + 1] - e0;
  const int nloc = nT + nfc * nF;
  double *Cc = lds + L.C, *K = lds + L.K, *Bc = lds + L.Bc, *G = lds + L.G, *Pi = lds + L.Pi, *Nn = lds + L.Nn,
         *gpo = lds + L.gpo, *red = lds + L.red, *rv = lds + L.rv, *gto = lds + L.gto, *S = lds + L.scr;
  __shared__ int fail_flag;
  if (threadIdx.x == 0) fail_flag = 0;
  const double h = g.cdiam[c];
  double x0[3];
  for (int a = 0; a < 3; ++a) x0[a] = g.ccen[3 * c + a];
  double *rec = g.rec + g.roff[c];
  double *A = rec, *Bg = A + (int64_t)nloc * nloc, *ru = Bg + (int64_t)d * nT * nloc, *rp = ru + (int64_t)d * nloc;

  // ---- cell phase: points, orthonormal cell basis, stiffness and the cell part of the coupling
  const int nq = cell_npoints(g, c);
  double *X = S, *W = X + 3 * L.max_nq, *M = W + L.max_nq, *GBm = M + (int64_t)L.max_nq * N1,
         *GB = GBm + (int64_t)L.chunk * N1 * d;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    double x[3], w;
    cell_point(g, c, q, x, &w);
    X[3 * q] = x[0];
    X[3 * q + 1] = x[1];
    X[3 * q + 2] = x[2];
    W[q] = w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nq * N1; e += blockDim.x) {
    const int q = e / N1, j = e % N1;
    double xi[3];
    for (int a = 0; a < d; ++a) xi[a] = (X[3 * q + a] - x0[a]) / h;
    M[e] = mono(g.EC, d, xi, j);
  }
  __syncthreads();
  if (!cgs2(M, N1, W, nq, N1, Cc, rv, red)) {
    if (threadIdx.x == 0) g.err[0] = c + 1;
    return;
  }
  // M now holds phi_i at the points
  for (int e = threadIdx.x; e < N1 * N1; e += blockDim.x) K[e] = 0.0;
  for (int e = threadIdx.x; e < d * nT * nT; e += blockDim.x) Bc[e] = 0.0;
  __syncthreads();
  const int P = L.chunk;
  for (int q0 = 0; q0 < nq; q0 += P) {
    const int np = min(P, nq - q0);
    // monomial gradients, then the basis gradients (every thread takes entries)
    for (int e = threadIdx.x; e < np * N1 * d; e += blockDim.x) {
      const int qq = e / (N1 * d), j = (e / d) % N1, a = e % d;
      double xi[3];
      for (int b = 0; b < d; ++b) xi[b] = (X[3 * (q0 + qq) + b] - x0[b]) / h;
      GBm[e] = dmono(g.EC, d, xi, h, j, a);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < np * N1 * d; e += blockDim.x) {
      const int qq = e / (N1 * d), i = (e / d) % N1, a = e % d;
      const double *row = GBm + (int64_t)qq * N1 * d + a, *ci = Cc + i * N1;
      double s0 = 0, s1 = 0;
      int m = 0;
      for (; m + 1 <= i; m += 2) {
        s0 += ci[m] * row[m * d];
        s1 += ci[m + 1] * row[(m + 1) * d];
      }
      if (m <= i) s0 += ci[m] * row[m * d];
      GB[e] = s0 + s1;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N1 * N1; e += blockDim.x) {
      const int i = e / N1, j = e % N1;
      double s = 0;
      for (int qq = 0; qq < np; ++qq) {
        const double *gi = GB + ((int64_t)qq * N1 + i) * d, *gj = GB + ((int64_t)qq * N1 + j) * d;
        double dot = 0;
        for (int a = 0; a < d; ++a) dot += gi[a] * gj[a];
        s += W[q0 + qq] * dot;
      }
      K[e] += s;
    }
    // (v_T,cc, d_cc q)_T: Bc[cc][t][j] = (phi_j, d_cc phi_t)
    for (int e = threadIdx.x; e < d * nT * nT; e += blockDim.x) {
      const int cc = e / (nT * nT), t = (e / nT) % nT, j = e % nT;
      double s = 0;
      for (int qq = 0; qq < np; ++qq)
        s += W[q0 + qq] * M[(int64_t)(q0 + qq) * N1 + j] * GB[((int64_t)qq * N1 + t) * d + cc];
      Bc[e] += s;
    }
    __syncthreads();
  }
  // reconstruction right-hand side, cell columns: G[i][j] = K[i][j], j < nT
  for (int e = threadIdx.x; e < N1 * nloc; e += blockDim.x) {
    const int i = e / nloc, j = e % nloc;
    G[e] = (j < nT) ? K[i * N1 + j] : 0.0;
  }
  __syncthreads();

  // ---- face phase: face bases, traces of the cell basis, reconstruction and stabilisation pieces
  for (int fi = 0; fi < nfc; ++fi) {
    const int e = e0 + fi, f = g.cface[e];
    const double sg = g.csign[e];
    double n[3];
    for (int a = 0; a < 3; ++a) n[a] = sg * g.fnrm[3 * f + a];
    const int nqf = face_npoints(g, f);
    double *Xf = S, *Wf = Xf + 3 * L.max_nqf, *Psi = Wf + L.max_nqf, *Phf = Psi + (int64_t)L.max_nqf * nF,
           *Gn = Phf + (int64_t)L.max_nqf * N1, *Mf = Gn + (int64_t)L.max_nqf * N1,
           *Mm = Mf + (int64_t)L.max_nqf * nF, *Dmm = Mm + (int64_t)L.max_nqf * N1;
    const double *CF = g.CF + (int64_t)f * nF * nF;  // the face's basis (k_face_bases)
    const double hF = g.fdiam[f];
    double xF[3], t1[3], t2[3];
    for (int a = 0; a < 3; ++a) {
      xF[a] = g.fcen[3 * f + a];
      t1[a] = g.ft1[3 * f + a];
      t2[a] = g.ft2[3 * f + a];
    }
    for (int q = threadIdx.x; q < nqf; q += blockDim.x) {
      double x[3], w;
      face_point(g, f, q, x, &w);
      Xf[3 * q] = x[0];
      Xf[3 * q + 1] = x[1];
      Xf[3 * q + 2] = x[2];
      Wf[q] = w;
    }
    __syncthreads();
    // face monomials, cell monomials and their normal derivatives at the face points
    for (int e2 = threadIdx.x; e2 < nqf * (nF + N1); e2 += blockDim.x) {
      const int q = e2 / (nF + N1), j = e2 % (nF + N1);
      if (j < nF) {
        const double r[3] = {Xf[3 * q] - xF[0], Xf[3 * q + 1] - xF[1], Xf[3 * q + 2] - xF[2]};
        double xi[2];
        xi[0] = (r[0] * t1[0] + r[1] * t1[1] + r[2] * t1[2]) / hF;
        xi[1] = (r[0] * t2[0] + r[1] * t2[1] + r[2] * t2[2]) / hF;
        Mf[q * nF + j] = mono(g.EF, d - 1, xi, j);
      } else {
        const int t = j - nF;
        double xc[3];
        for (int a = 0; a < d; ++a) xc[a] = (Xf[3 * q + a] - x0[a]) / h;
        Mm[(int64_t)q * N1 + t] = mono(g.EC, d, xc, t);
        double dn = 0;
        for (int b = 0; b < d; ++b) dn += n[b] * dmono(g.EC, d, xc, h, t, b);
        Dmm[(int64_t)q * N1 + t] = dn;
      }
    }
    __syncthreads();
    // the face basis at the face points
    for (int e2 = threadIdx.x; e2 < nqf * nF; e2 += blockDim.x) {
      const int q = e2 / nF, j = e2 % nF;
      double s1 = 0;
      for (int m = 0; m <= j; ++m) s1 += CF[j * nF + m] * Mf[q * nF + m];
      Psi[e2] = s1;
    }
    // the cell basis and its normal derivative at the face points
    for (int e2 = threadIdx.x; e2 < nqf * N1; e2 += blockDim.x) {
      const int q = e2 / N1, t = e2 % N1;
      const double *ct = Cc + t * N1, *mq = Mm + (int64_t)q * N1, *dq = Dmm + (int64_t)q * N1;
      double s1 = 0, s2 = 0;
      for (int m = 0; m <= t; ++m) {
        s1 += ct[m] * mq[m];
        s2 += ct[m] * dq[m];
      }
      Phf[e2] = s1;
      Gn[e2] = s2;
    }
    __syncthreads();
    // G[t][F_j] += (grad phi_t . n, psi_j)_F ; G[t][j'] -= (grad phi_t . n, phi_j')_F  (t >= 1)
    for (int e2 = threadIdx.x; e2 < N1 * (nF + nT); e2 += blockDim.x) {
      const int t = e2 / (nF + nT), col = e2 % (nF + nT);
      if (t == 0) continue;
      double s = 0;
      if (col < nF) {
        for (int q = 0; q < nqf; ++q) s += Wf[q] * Gn[(int64_t)q * N1 + t] * Psi[q * nF + col];
        G[t * nloc + nT + fi * nF + col] += s;
      } else {
        const int j = col - nF;
        for (int q = 0; q < nqf; ++q) s += Wf[q] * Gn[(int64_t)q * N1 + t] * Phf[(int64_t)q * N1 + j];
        G[t * nloc + j] -= s;
      }
    }
    // Pi[j][t] = (psi_j, phi_t)_F, Nn[j][t] = (psi_j, grad phi_t . n)_F
    double *Pif = Pi + (int64_t)fi * nF * N1, *Nnf = Nn + (int64_t)fi * nF * N1;
    for (int e2 = threadIdx.x; e2 < nF * N1; e2 += blockDim.x) {
      const int j = e2 / N1, t = e2 % N1;
      double s1 = 0, s2 = 0;
      for (int q = 0; q < nqf; ++q) {
        const double wp = Wf[q] * Psi[q * nF + j];
        s1 += wp * Phf[(int64_t)q * N1 + t];
        s2 += wp * Gn[(int64_t)q * N1 + t];
      }
      Pif[e2] = s1;
      Nnf[e2] = s2;
    }
    // boundary data against the face basis
    if (g.fbc[f] != HHO_FACE_INTERIOR) {
      const double *src = g.fd + g.foff[f] + (g.fbc[f] == HHO_FACE_DIRICHLET ? (int64_t)d * N1 : 0);
      for (int e2 = threadIdx.x; e2 < d * nF; e2 += blockDim.x) {
        const int a = e2 / nF, j = e2 % nF;
        double s = 0;
        for (int m = 0; m <= j; ++m) s += CF[j * nF + m] * src[a * nF + m];
        gpo[((int64_t)fi * d + a) * nF + j] = s;
      }
    }
    __syncthreads();
  }

  // ---- reconstruction: L L^T = K restricted to the non-constant functions
  const int n1 = N1 - 1;
  for (int j = 0; j < n1; ++j) {
    if (threadIdx.x == 0) {
      double s = K[(j + 1) * N1 + (j + 1)];
      for (int t = 0; t < j; ++t) s -= K[(j + 1) * N1 + (t + 1)] * K[(j + 1) * N1 + (t + 1)];
      if (!(s > 0)) {
        fail_flag = 1;
        s = 1.0;
      }
      K[(j + 1) * N1 + (j + 1)] = sqrt(s);
    }
    __syncthreads();
    const double ljj = K[(j + 1) * N1 + (j + 1)];
    for (int i = j + 1 + threadIdx.x; i < n1; i += blockDim.x) {
      double v = K[(i + 1) * N1 + (j + 1)];
      for (int t = 0; t < j; ++t) v -= K[(i + 1) * N1 + (t + 1)] * K[(j + 1) * N1 + (t + 1)];
      K[(i + 1) * N1 + (j + 1)] = v / ljj;
    }
    __syncthreads();
  }
  if (fail_flag) {
    if (threadIdx.x == 0) g.err[0] = c + 1;
    return;
  }
  // Y = L^{-1} G (rows 1..N1-1), one column per thread
  for (int b = threadIdx.x; b < nloc; b += blockDim.x) {
    for (int i = 0; i < n1; ++i) {
      double v = G[(i + 1) * nloc + b];
      for (int t = 0; t < i; ++t) v -= K[(i + 1) * N1 + (t + 1)] * G[(t + 1) * nloc + b];
      G[(i + 1) * nloc + b] = v / K[(i + 1) * N1 + (i + 1)];
    }
  }
  __syncthreads();
  // consistency term (grad R u, grad R v)_T = Y^T Y, kept in LDS until the record is written
  double *Al = S + 2LL * nF * L.nloc_max;
  for (int e = threadIdx.x; e < nloc * nloc; e += blockDim.x) {
    const int a = e / nloc, b = e % nloc;
    double s = 0;
    for (int t = 1; t < N1; ++t) s += G[t * nloc + a] * G[t * nloc + b];
    Al[e] = s;
  }
  __syncthreads();
  // R = L^{-T} Y; the constant function's row is e_0
  for (int b = threadIdx.x; b < nloc; b += blockDim.x) {
    for (int i = n1 - 1; i >= 0; --i) {
      double v = G[(i + 1) * nloc + b];
      for (int t = i + 1; t < n1; ++t) v -= K[(t + 1) * N1 + (i + 1)] * G[(t + 1) * nloc + b];
      G[(i + 1) * nloc + b] = v / K[(i + 1) * N1 + (i + 1)];
    }
    G[b] = (b == 0) ? 1.0 : 0.0;
  }
  __syncthreads();

  // ---- stabilisation, Nitsche terms and data, face by face
  const double eta = g.eta[c];
  double acc_u = 0.0, acc_p = 0.0;  // rhs_u entry threadIdx.x (< d nloc), rhs_p entry (< nT)
  const int ua = threadIdx.x / max(nloc, 1), ub = threadIdx.x % max(nloc, 1);
  if (threadIdx.x < d * nloc && ub < nT) {  // body force against the cell basis
    const double *mf = g.mf + ((int64_t)c * d + ua) * nT;
    for (int m = 0; m <= ub; ++m) acc_u += Cc[ub * N1 + m] * mf[m];
  }
  double *Dm = S, *NR = S + (int64_t)nF * L.nloc_max;
  for (int fi = 0; fi < nfc; ++fi) {
    const int e = e0 + fi, f = g.cface[e];
    const int bc = g.fbc[f];
    const double hF = g.fdiam[f];
    const double *Pif = Pi + (int64_t)fi * nF * N1, *Nnf = Nn + (int64_t)fi * nF * N1;
    for (int e2 = threadIdx.x; e2 < nF * nloc; e2 += blockDim.x) {
      const int j = e2 / nloc, b = e2 % nloc;
      double s = (b == nT + fi * nF + j) ? 1.0 : 0.0;
      if (b < nT) s -= Pif[j * N1 + b];
      for (int t = nT; t < N1; ++t) s -= Pif[j * N1 + t] * G[t * nloc + b];
      Dm[e2] = s;
      if (bc == HHO_FACE_DIRICHLET) {
        double r = 0;
        for (int t = 0; t < N1; ++t) r += Nnf[j * N1 + t] * G[t * nloc + b];
        NR[e2] = r;
      }
    }
    if (bc == HHO_FACE_DIRICHLET) {
      const double *gt = g.fd + g.foff[f];
      for (int e2 = threadIdx.x; e2 < d * N1; e2 += blockDim.x) {
        const int a = e2 / N1, t = e2 % N1;
        double s = 0;
        for (int m = 0; m <= t; ++m) s += Cc[t * N1 + m] * gt[a * N1 + m];
        gto[e2] = s;
      }
    }
    __syncthreads();
    const double ih = 1.0 / hF;
    for (int e2 = threadIdx.x; e2 < nloc * nloc; e2 += blockDim.x) {
      const int a = e2 / nloc, b = e2 % nloc;
      double s = 0;
      for (int j = 0; j < nF; ++j) s += Dm[j * nloc + a] * Dm[j * nloc + b];
      double v = Al[e2] + s / hF;
      if (bc == HHO_FACE_DIRICHLET) {
        const int fa = a - nT - fi * nF, fb = b - nT - fi * nF;
        if (fa >= 0 && fa < nF) v -= NR[fa * nloc + b];
        if (fb >= 0 && fb < nF) v -= NR[fb * nloc + a];
        if (fa >= 0 && fa < nF && a == b) v += eta * ih;
      }
      Al[e2] = v;
    }
    if (threadIdx.x < d * nloc) {
      const int fj = ub - nT - fi * nF;
      if (bc == HHO_FACE_DIRICHLET) {
        double s = 0;
        for (int t = 0; t < N1; ++t) s += G[t * nloc + ub] * gto[ua * N1 + t];
        acc_u -= s;
        if (fj >= 0 && fj < nF) acc_u += eta * ih * gpo[((int64_t)fi * d + ua) * nF + fj];
      } else if (bc == HHO_FACE_NEUMANN) {
        if (fj >= 0 && fj < nF) acc_u += gpo[((int64_t)fi * d + ua) * nF + fj];
      }
    }
    if (bc == HHO_FACE_DIRICHLET && threadIdx.x < nT) {
      const double *gn = g.fd + g.foff[f] + (int64_t)d * N1 + (int64_t)d * nF;
      const int t = threadIdx.x;
      for (int m = 0; m <= t; ++m) acc_p += Cc[t * N1 + m] * gn[m];
    }
    __syncthreads();
  }
  if (threadIdx.x < d * nloc) ru[threadIdx.x] = acc_u;
  if (threadIdx.x < nT) rp[threadIdx.x] = acc_p;
  for (int e = threadIdx.x; e < nloc * nloc; e += blockDim.x) A[e] = Al[e];

  // ---- coupling: cell part (v_T,cc, d_cc q)_T, face part -(v_F . n, q)_F off Dirichlet faces
  for (int e = threadIdx.x; e < d * nT * nloc; e += blockDim.x) {
    const int cc = e / (nT * nloc), t = (e / nloc) % nT, b = e % nloc;
    double v;
    if (b < nT) {
      v = Bc[(cc * nT + t) * nT + b];
    } else {
      const int fi = (b - nT) / nF, j = (b - nT) % nF;
      const int f = g.cface[e0 + fi];
      const double nc_ = g.csign[e0 + fi] * g.fnrm[3 * f + cc];
      v = (g.fbc[f] == HHO_FACE_DIRICHLET) ? 0.0 : -nc_ * Pi[((int64_t)fi * nF + j) * N1 + t];
    }
    Bg[e] = v;
  }
}

}  // namespace

void launch_local(const LocalGeom &g, const LocalLds &L, int nc, hipStream_t s) {
  if (nc <= 0) return;
  if (g.nf > 0) {  // the faces' bases first (read by every cell's face phase)
    const int per = 4 * L.max_nqf + L.max_nqf * g.nF + g.nF * g.nF + g.nF + 1;
    const size_t lds = (size_t)kFaceWaves * per * sizeof(double);
    hipLaunchKernelGGL(k_face_bases, dim3((g.nf + kFaceWaves - 1) / kFaceWaves), dim3(kFaceWaves * kWave), lds, s, g,
                       L.max_nqf, g.CF);
  }
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    attr = hipFuncSetAttribute((const void *)k_local, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMaxLdsBytes - 1024));
  });
  if (attr != hipSuccess) fail(HHO_E_DEVICE, "local build: cannot reserve LDS");
  hipLaunchKernelGGL(k_local, dim3(nc), dim3(L.threads), L.bytes, s, g, L);
}

static int64_t choose(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

LocalLds local_lds(int d, int k, int max_faces, int max_nq, int max_nqf) {
  const int N1 = (int)choose(k + 1 + d, d), nT = (int)choose(k + d, d), nF = (int)choose(k + d - 1, d - 1);
  LocalLds L{};
  const int nlocmax = nT + max_faces * nF;
  L.max_nq = max_nq;
  L.max_nqf = max_nqf;
  L.nloc_max = nlocmax;
  L.chunk = 16;
  int64_t o = 0;
  auto take = [&](int64_t n) {
    const int64_t r = o;
    o += n;
    return (int)r;
  };
  L.C = take((int64_t)N1 * N1);
  L.K = take((int64_t)N1 * N1);
  L.Bc = take((int64_t)d * nT * nT);
  L.G = take((int64_t)N1 * nlocmax);
  L.Pi = take((int64_t)max_faces * nF * N1);
  L.Nn = take((int64_t)max_faces * nF * N1);
  L.gpo = take((int64_t)max_faces * d * nF);
  L.red = take(32);
  L.rv = take(N1);
  L.gto = take((int64_t)d * N1);
  const int64_t cell = 4LL * max_nq + (int64_t)max_nq * N1 + 2LL * L.chunk * N1 * d;
  const int64_t face = 4LL * max_nqf + 2LL * max_nqf * nF + 4LL * max_nqf * N1;
  const int64_t stab = 2LL * nF * nlocmax + (int64_t)nlocmax * nlocmax;
  L.scr = take(std::max(cell, std::max(face, stab)));
  L.bytes = (size_t)o * sizeof(double);
  // Latency decides the speed (every phase is a chain of short LDS-bound loops):
  // a cell whose work arrays leave room for a second workgroup on the compute
  // unit runs with 512 threads, two or more cells per unit (measured on 2D
  // k = 3 Voronoi cells: 6.1 ms against 6.7 ms with 256 threads, 11.1 ms with
  // 768 and more with 1024); a cell that takes the unit alone gets 1024 threads
  // (16 waves) to hide
  // the latency itself.  Every rhs_u entry needs its own thread.
  L.threads = L.bytes > kMaxLdsBytes / 2 ? 1024 : 512;
  while (L.threads < d * nlocmax && L.threads < kLocalThreads) L.threads *= 2;
  return L;
}

}  // namespace hho
