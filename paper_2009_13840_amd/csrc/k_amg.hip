// Coarsest-level block preconditioner (FP64): numeric smoothed-aggregation
// setup from host-built gather lists, the AMG V-cycle on d right-hand sides
// (vectors stored [row][component]), and the pressure / velocity split of the
// block-triangular Stokes preconditioner
//   y = -g / S_T,   x = AMG(f - C y).
#include <algorithm>
#include <cmath>

#include "dev_common.h"
#include "dev_dense.h"
#include "device.h"
#include "k_amg.h"

namespace hho {
namespace {

inline int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

// scalar face operator of the coarsest level: (1/d) sum_c S[(f,c),(g,c)]
__global__ void k_amg_extract0(int64_t nnzb, int bs, int d, int cond, const double *bsr, double *val) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnzb; e += (int64_t)gridDim.x * blockDim.x) {
    if (cond == 1) {
      val[e] = bsr[e];
    } else {
      double s = 0;
      for (int c = 0; c < d; ++c) s += bsr[e * bs * bs + c * bs + c];
      val[e] = s / d;
    }
  }
}

// D^{-1} and lambda = max_i sum_j |A_ij| / A_ii (Gershgorin bound of D^{-1} A)
__global__ void __launch_bounds__(kBlock) k_amg_diag(int n, const int32_t *rp, const int32_t *diag,
                                                      const double *val, double *dinv, double *partial,
                                                      double *lam, int *counter) {
  __shared__ double red[kBlock];
  double mx = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double a = val[diag[i]];
    double s = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += fabs(val[e]);
    dinv[i] = 1.0 / a;
    mx = fmax(mx, s / a);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
  if (last_block_arrived(counter)) {
    if (threadIdx.x < kWave) {
      double m = 0;
      for (unsigned b = threadIdx.x; b < gridDim.x; b += kWave) m = fmax(m, vload(&partial[b]));
      m = wave_max(m);
      if (threadIdx.x == 0) *lam = m;
    }
  }
}

// P = T - (omega / lambda) D^{-1} A T
__global__ void k_amg_p(int64_t npe, const int32_t *prow, const int32_t *pgp, const int32_t *pgi,
                        const int32_t *pself, const double *val, const double *dinv, const double *lam,
                        double *pval) {
  const double w = kAmgOmegaSA / lam[0];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npe; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int k = pgp[e]; k < pgp[e + 1]; ++k) s += val[pgi[k]];
    pval[e] = (pself[e] ? 1.0 : 0.0) - w * dinv[prow[e]] * s;
  }
}

// out[e] = sum_{k in [pp[e], pp[e+1])} X[pa[k]] * Y[pb[k]]
__global__ void k_amg_pairs(int64_t nout, const int32_t *pp, const int32_t *pa, const int32_t *pb,
                            const double *X, const double *Y, double *out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nout; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int k = pp[e]; k < pp[e + 1]; ++k) s += X[pa[k]] * Y[pb[k]];
    out[e] = s;
  }
}

// coarsest level: dense inverse of the (small, SPD) CSR matrix in one block
__global__ void __launch_bounds__(kBlock) k_amg_coarsest(int n, const int32_t *rp, const int32_t *ci,
                                                          const double *val, double *L, double *Ainv, int *err) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) L[i] = 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int e = rp[i]; e < rp[i + 1]; ++e) L[i * n + ci[e]] = val[e];
  __syncthreads();
  blk_chol(L, n, n, &bad);
  __syncthreads();
  blk_chol_inverse(L, n, n, Ainv, n);
  if (threadIdx.x == 0 && bad) atomicMax(err, 1);
}

// pressure Schur approximation S_T = sum_{(f,c) in T} C[(f,c),T]^2 / S[(f,c),(f,c)]
__global__ void k_bp_setup(DTopo tp, int cond, const int32_t *fdiag, const double *bsr, const double *cpl,
                           double *Sd) {
  const int d = tp.d;
  const int bs = (cond == 1) ? 1 : d;
  for (int T = blockIdx.x * blockDim.x + threadIdx.x; T < tp.nc; T += gridDim.x * blockDim.x) {
    double s = 0;
    for (int e = tp.cptr[T]; e < tp.cptr[T + 1]; ++e) {
      const int f = tp.cface[e];
      for (int c = 0; c < d; ++c) {
        // v-cond: one scalar block for every component; v&p: component diagonal of the d x d block
        const double a = (cond == 1) ? bsr[fdiag[f]] : bsr[(int64_t)fdiag[f] * bs * bs + c * bs + c];
        const double cc = cpl[(int64_t)e * d + c];
        s += cc * cc / a;
      }
    }
    Sd[T] = (s > 0) ? s : 1.0;
  }
}

// split of the block preconditioner: z_T = -v_T / S_T on cells; the AMG
// right-hand side f - C y on faces ([face][component] = the k = 0 face layout)
__global__ void k_bp_rhs(DTopo tp, int64_t nface, const double *cpl, const double *Sd, const double *v,
                         double *rhs, double *z) {
  const int d = tp.d;
  const int64_t total = nface + tp.nc;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    if (o < nface) {
      const int f = (int)(o / d), c = (int)(o % d);
      double s = v[o];
      for (int k = 0; k < 2; ++k) {
        const int T = tp.fcell[2 * f + k];
        if (T < 0) continue;
        const int64_t e = (int64_t)tp.cptr[T] + tp.floc[2 * f + k];
        s += cpl[e * d + c] * v[nface + T] / Sd[T];
      }
      rhs[o] = s;
    } else {
      const int64_t T = o - nface;
      z[o] = -v[o] / Sd[T];
    }
  }
}

// xout = xin + w D^{-1} (r - A xin)   (xin == null: xout = w D^{-1} r)
__global__ void k_amg_jacobi(int n, int d, const int32_t *rp, const int32_t *ci, const double *val,
                             const double *dinv, const double *r, const double *xin, double *xout) {
  const int64_t total = (int64_t)n * d;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / d), c = (int)(o % d);
    double t = r[o];
    double x0 = 0;
    if (xin) {
      for (int e = rp[i]; e < rp[i + 1]; ++e) t -= val[e] * xin[(int64_t)ci[e] * d + c];
      x0 = xin[o];
    }
    xout[o] = x0 + kAmgOmegaJac * dinv[i] * t;
  }
}

__global__ void k_amg_residual(int n, int d, const int32_t *rp, const int32_t *ci, const double *val,
                               const double *r, const double *x, double *res) {
  const int64_t total = (int64_t)n * d;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / d), c = (int)(o % d);
    double t = r[o];
    for (int e = rp[i]; e < rp[i + 1]; ++e) t -= val[e] * x[(int64_t)ci[e] * d + c];
    res[o] = t;
  }
}

// rc = P^T res; one wavefront per coarse row, lanes split the row's entries
__global__ void __launch_bounds__(kBlock) k_amg_restrict(int nc, int d, const int32_t *ptp, const int32_t *pti,
                                                          const int32_t *pte, const double *pval, const double *res,
                                                          double *rc) {
  const int lane = threadIdx.x % kWave;
  const int64_t nwave = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave; I < nc; I += nwave) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int k = ptp[I] + lane; k < ptp[I + 1]; k += kWave) {
      const double pv = pval[pte[k]];
      const double *rr = res + (int64_t)pti[k] * d;
      s0 += pv * rr[0];
      if (d > 1) s1 += pv * rr[1];
      if (d > 2) s2 += pv * rr[2];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      rc[I * d] = s0;
      if (d > 1) rc[I * d + 1] = s1;
      if (d > 2) rc[I * d + 2] = s2;
    }
  }
}

// xout = xin + P xc (xout may alias xin: every entry is read and written by one thread)
__global__ void k_amg_prolong(int n, int d, const int32_t *prp, const int32_t *pci, const double *pval,
                              const double *xc, const double *xin, double *xout) {
  const int64_t total = (int64_t)n * d;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / d), c = (int)(o % d);
    double s = 0;
    for (int e = prp[i]; e < prp[i + 1]; ++e) s += pval[e] * xc[(int64_t)pci[e] * d + c];
    xout[o] = xin[o] + s;
  }
}

// x = Ainv r (dense, n <= 128), one thread per output
__global__ void k_amg_dense(int n, int d, const double *Ainv, const double *r, double *x) {
  const int64_t total = (int64_t)n * d;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / d), c = (int)(o % d);
    double s = 0;
    for (int j = 0; j < n; ++j) s += Ainv[(int64_t)i * n + j] * r[(int64_t)j * d + c];
    x[o] = s;
  }
}

}  // namespace

void amg_numeric_setup(const AmgDev &A, int cond, int d, int bs, int64_t nnzb0, const double *bsr0, int *err,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_amg_extract0, dim3(grid_for(nnzb0)), dim3(kBlock), 0, s, nnzb0, bs, d, cond, bsr0,
                     A.lev[0].val);
  for (int l = 0; l < A.nlev; ++l) {
    const AmgDevLevel &L = A.lev[l];
    if (l == A.nlev - 1) {
      hipLaunchKernelGGL(k_amg_coarsest, dim3(1), dim3(kBlock), 0, s, L.n, L.rp, L.ci, L.val, A.dense_scratch,
                         A.ainv, err);
      break;
    }
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((L.n + kBlock - 1) / kBlock, 256));
    hipLaunchKernelGGL(k_amg_diag, dim3(nb), dim3(kBlock), 0, s, L.n, L.rp, L.diag, L.val, L.dinv, A.partial,
                       L.lam, A.counter);
    hipLaunchKernelGGL(k_amg_p, dim3(grid_for(L.npe)), dim3(kBlock), 0, s, L.npe, L.prow, L.pgp, L.pgi, L.pself,
                       L.val, L.dinv, L.lam, L.pval);
    hipLaunchKernelGGL(k_amg_pairs, dim3(grid_for(L.nbe)), dim3(kBlock), 0, s, L.nbe, L.bpp, L.bpa, L.bpb,
                       (const double *)L.val, (const double *)L.pval, L.bval);
    const AmgDevLevel &N = A.lev[l + 1];
    hipLaunchKernelGGL(k_amg_pairs, dim3(grid_for(N.nnz)), dim3(kBlock), 0, s, N.nnz, L.cpp, L.cpa, L.cpb,
                       (const double *)L.pval, (const double *)L.bval, N.val);
  }
}

void bp_setup(const DTopo &tp, int cond, const int32_t *fdiag, const double *bsr, const double *cpl, double *Sd,
              hipStream_t s) {
  hipLaunchKernelGGL(k_bp_setup, dim3(grid_for(tp.nc)), dim3(kBlock), 0, s, tp, cond, fdiag, bsr, cpl, Sd);
}

// V-cycle on level l: x = AMG_l(r); x, r are [n_l][d]
static void vcycle(const AmgDev &A, int l, int d, int nu, const double *r, double *x, hipStream_t s) {
  const AmgDevLevel &L = A.lev[l];
  const int64_t nd = (int64_t)L.n * d;
  if (l == A.nlev - 1) {
    hipLaunchKernelGGL(k_amg_dense, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, (const double *)A.ainv, r, x);
    return;
  }
  // pre-smoothing (from zero): ends in x
  if (nu == 1) {
    hipLaunchKernelGGL(k_amg_jacobi, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, L.rp, L.ci,
                       (const double *)L.val, (const double *)L.dinv, r, (const double *)nullptr, x);
  } else {
    hipLaunchKernelGGL(k_amg_jacobi, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, L.rp, L.ci,
                       (const double *)L.val, (const double *)L.dinv, r, (const double *)nullptr, L.tmp);
    hipLaunchKernelGGL(k_amg_jacobi, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, L.rp, L.ci,
                       (const double *)L.val, (const double *)L.dinv, r, (const double *)L.tmp, x);
  }
  hipLaunchKernelGGL(k_amg_residual, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, L.rp, L.ci,
                     (const double *)L.val, r, (const double *)x, L.res);
  const AmgDevLevel &N = A.lev[l + 1];
  hipLaunchKernelGGL(k_amg_restrict, dim3(grid_for((int64_t)N.n * kWave)), dim3(kBlock), 0, s, N.n, d, L.ptp, L.pti,
                     L.pte, (const double *)L.pval, (const double *)L.res, N.r);
  vcycle(A, l + 1, d, nu, N.r, N.x, s);
  // prolongation, then nu post-smoothing sweeps alternating between tmp and x, ending in x
  double *cur = (nu % 2 == 1) ? L.tmp : x;
  hipLaunchKernelGGL(k_amg_prolong, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, L.prp, L.pci,
                     (const double *)L.pval, (const double *)N.x, (const double *)x, cur);
  for (int it = 0; it < nu; ++it) {
    double *nxt = (cur == x) ? L.tmp : x;
    hipLaunchKernelGGL(k_amg_jacobi, dim3(grid_for(nd)), dim3(kBlock), 0, s, L.n, d, L.rp, L.ci,
                       (const double *)L.val, (const double *)L.dinv, r, (const double *)cur, nxt);
    cur = nxt;
  }
}

void bp_apply(const DTopo &tp, const AmgDev &A, int64_t nface, const double *cpl, const double *Sd, const double *v,
              double *z, int nu, hipStream_t s) {
  const int d = tp.d;
  hipLaunchKernelGGL(k_bp_rhs, dim3(grid_for(nface + tp.nc)), dim3(kBlock), 0, s, tp, nface, cpl, Sd, v,
                     A.lev[0].r, z);
  vcycle(A, 0, d, nu, A.lev[0].r, z, s);
}

}  // namespace hho
